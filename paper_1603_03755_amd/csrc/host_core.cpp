// Host-side construction of embedded Hamiltonians, device layouts and
// acceptance tables.
#include "host_core.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace sqa {

// ------------------------------------------------------------- errors
static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

sqa_status fail(sqa_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

sqa_status hip_fail(hipError_t e, const char *what) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
  g_last_error = buf;
  return e == hipErrorOutOfMemory ? SQA_ERR_OOM : SQA_ERR_DEVICE;
}

const char *last_error_cstr() { return g_last_error.c_str(); }

// ------------------------------------------------------ device memory
sqa_status device_alloc(const sqa_allocator *a, void **p, size_t bytes, const char *what) {
  *p = nullptr;
  if (a && a->alloc) {
    *p = a->alloc(bytes, a->ctx);
    if (!*p) return fail(SQA_ERR_OOM, std::string(what) + ": the allocator returned NULL");
    return SQA_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return hip_fail(e, what);
  }
  return SQA_OK;
}

void device_free(const sqa_allocator *a, void *p) {
  if (!p) return;
  if (a && a->alloc) a->free(p, a->ctx);
  else (void)hipFree(p);
}

// -------------------------------------------------------- embeddings
static int32_t me_index(int32_t N, int32_t chain, int32_t slot) { return chain * (N - 1) + slot; }

static int32_t lhz_index(int32_t N, int32_t i, int32_t j) { return i * (2 * N - i - 1) / 2 + (j - i - 1); }

static void push_term(Embedded *e, int32_t w, std::initializer_list<int32_t> sites) {
  Term t{};
  t.w = w;
  t.arity = static_cast<int32_t>(sites.size());
  int q = 0;
  for (int32_t s : sites) t.s[q++] = s;
  for (; q < 4; ++q) t.s[q] = -1;
  e->terms.push_back(t);
}

// ME (Sec. II A), clique-chain layout: chain i = sites i(N-1)..i(N-1)+N-2 joined
// by J_F bonds along the chain; J_ij (i<j) joins slot j-1 of chain i and slot i
// of chain j; a logical field h_i sits on slot 0 of chain i.
// LHZ (Sec. II B, Eq. (3)): site per logical pair with field J_ij; constraint
// terms C*prod on the plaquettes {(i,j),(i,j+1),(i+1,j),(i+1,j+1)} (i+2<=j<=N-2)
// and on the diagonal triangles {(i,i+1),(i,i+2),(i+1,i+2)} (i<=N-3).
// Colours: ME (slot&1)|((chain&1)<<1), LHZ (i&1)|((j&1)<<1); no term joins two
// sites of one colour.
sqa_status build_embedding(const sqa_problem &p, const sqa_embedding &em, Embedded *out) {
  Embedded e;
  e.kind = em.kind;
  e.N = p.n;
  const int32_t N = p.n;
  if (em.kind == SQA_EMB_ME) {
    if (N < 2 || N > 256) return fail(SQA_ERR_INVALID, "ME needs 2 <= n <= 256");
    e.n = N * (N - 1);
    e.h.assign(e.n, 0);
    e.colour.assign(e.n, 0);
    for (int32_t i = 0; i < N; ++i)
      for (int32_t r = 0; r < N - 1; ++r) e.colour[me_index(N, i, r)] = (r & 1) | ((i & 1) << 1);
    for (int32_t i = 0; i < N; ++i)
      for (int32_t r = 0; r + 2 < N; ++r) push_term(&e, em.penalty, {me_index(N, i, r), me_index(N, i, r + 1)});
    for (int32_t i = 0; i < N; ++i)
      for (int32_t j = i + 1; j < N; ++j) push_term(&e, p.J[i * N + j], {me_index(N, i, j - 1), me_index(N, j, i)});
    if (p.h)
      for (int32_t i = 0; i < N; ++i) e.h[me_index(N, i, 0)] = p.h[i];
  } else if (em.kind == SQA_EMB_LHZ) {
    if (N < 3 || N > 256) return fail(SQA_ERR_INVALID, "LHZ needs 3 <= n <= 256");
    if (p.h)
      for (int32_t i = 0; i < N; ++i)
        if (p.h[i] != 0) return fail(SQA_ERR_UNSUPPORTED, "LHZ with logical fields needs an ancilla (not supported)");
    e.n = N * (N - 1) / 2;
    e.h.assign(e.n, 0);
    e.colour.assign(e.n, 0);
    for (int32_t i = 0; i < N; ++i)
      for (int32_t j = i + 1; j < N; ++j) {
        const int32_t k = lhz_index(N, i, j);
        e.h[k] = p.J[i * N + j];
        e.colour[k] = (i & 1) | ((j & 1) << 1);
      }
    for (int32_t i = 0; i + 2 < N; ++i)
      push_term(&e, em.penalty, {lhz_index(N, i, i + 1), lhz_index(N, i, i + 2), lhz_index(N, i + 1, i + 2)});
    for (int32_t i = 0; i < N; ++i)
      for (int32_t j = i + 2; j + 1 < N; ++j)
        push_term(&e, em.penalty,
                  {lhz_index(N, i, j), lhz_index(N, i, j + 1), lhz_index(N, i + 1, j), lhz_index(N, i + 1, j + 1)});
  } else if (em.kind == SQA_EMB_ME_CHIMERA) {
    // ME on Chimera C_m, m = ceil(N/4) (Sec. II A): logical spin i, block b = i/4,
    // k = i%4, is the chain of m+1 qubits H(b, 0..b, k) then V(b..m-1, b, k);
    // site i(m+1)+t is its slot t (t <= b: H(b, t, k); t > b: V(t-1, b, k)).
    // Chain bonds J_F between consecutive slots; the chains of i < j (blocks
    // a <= b) meet in cell (b, a), where J_ij couples V(b, a, k_i) (slot b+1 of
    // chain i) with H(b, a, k_j) (slot a of chain j).  h_i on slot 0.
    // Colour (row + column + side) & 1, side H = 1: Chimera is bipartite.
    if (N < 2 || N > 256) return fail(SQA_ERR_INVALID, "ME on Chimera needs 2 <= n <= 256");
    const int32_t m = (N + 3) / 4, len = m + 1;
    e.n = N * len;
    e.h.assign(e.n, 0);
    e.colour.assign(e.n, 0);
    for (int32_t i = 0; i < N; ++i) {
      const int32_t b = i / 4;
      for (int32_t t = 0; t < len; ++t) {
        const bool horiz = t <= b;
        const int32_t row = horiz ? b : t - 1, col = horiz ? t : b;
        e.colour[i * len + t] = (row + col + (horiz ? 1 : 0)) & 1;
      }
      for (int32_t t = 0; t + 1 < len; ++t) push_term(&e, em.penalty, {i * len + t, i * len + t + 1});
    }
    for (int32_t i = 0; i < N; ++i)
      for (int32_t j = i + 1; j < N; ++j) push_term(&e, p.J[i * N + j], {i * len + j / 4 + 1, j * len + i / 4});
    if (p.h)
      for (int32_t i = 0; i < N; ++i) e.h[i * len] = p.h[i];
  } else {
    return fail(SQA_ERR_INVALID, "unknown embedding kind");
  }
  if (e.n > 65535) return fail(SQA_ERR_UNSUPPORTED, "more than 65535 physical sites");
  std::vector<int32_t> fsite(e.n, 0);
  for (int32_t k = 0; k < e.n; ++k) fsite[k] = std::abs(e.h[k]);
  long long emax = 0;
  for (int32_t k = 0; k < e.n; ++k) emax += std::abs(e.h[k]);
  for (const Term &t : e.terms) {
    emax += std::abs(t.w);
    for (int q = 0; q < t.arity; ++q) fsite[t.s[q]] += std::abs(t.w);
  }
  e.fmax = 0;
  for (int32_t f : fsite) e.fmax = std::max(e.fmax, f);
  if (e.fmax > kLargeF) return fail(SQA_ERR_UNSUPPORTED, "sum of |coefficients| at one site exceeds 255");
  if (emax > (1ll << 30)) return fail(SQA_ERR_INVALID, "energy range too large");
  e.emax = static_cast<int32_t>(emax);
  *out = std::move(e);
  return SQA_OK;
}

sqa_status build_layout(const Embedded &emb, int32_t F, RecordLayout layout, DeviceLayout *out) {
  DeviceLayout L;
  const int32_t n = emb.n;
  const bool me = emb.kind == SQA_EMB_ME, mec = emb.kind == SQA_EMB_ME_CHIMERA;
  const int T = me ? 3 : (mec ? 6 : 4), P = (me || mec) ? 1 : 3;
  L.rec_words = me ? kRecWordsME : (mec ? kRecWordsMEC : kRecWordsLHZ);
  // colour-sorted device order, increasing physical index within a class
  L.phys_of.reserve(n);
  for (int c = 0; c < 4; ++c) {
    L.cls[c] = static_cast<int32_t>(L.phys_of.size());
    for (int32_t k = 0; k < n; ++k)
      if (emb.colour[k] == c) L.phys_of.push_back(k);
  }
  L.cls[4] = n;
  L.dev_of.assign(n, 0);
  for (int32_t d = 0; d < n; ++d) L.dev_of[L.phys_of[d]] = static_cast<uint16_t>(d);
  // incident terms per site
  std::vector<std::vector<int32_t>> inc(n);
  for (size_t t = 0; t < emb.terms.size(); ++t)
    for (int q = 0; q < emb.terms[t].arity; ++q) inc[emb.terms[t].s[q]].push_back(static_cast<int32_t>(t));
  const uint32_t zero = static_cast<uint32_t>(n);  // index of the all-zero lattice word
  if (8u * zero + 7u > 0xFFFFu) return fail(SQA_ERR_UNSUPPORTED, "lattice byte offsets exceed 16 bits");
  L.rec.assign(static_cast<size_t>(n) * L.rec_words, 0u);
  L.hfield.assign(n, 0);
  for (int32_t d = 0; d < n; ++d) {
    const int32_t k = L.phys_of[d];
    if (static_cast<int>(inc[k].size()) > T) return fail(SQA_ERR_UNSUPPORTED, "site with too many terms");
    uint32_t aw[6] = {0, 0, 0, 0, 0, 0};
    uint32_t neg = 0;
    uint32_t part[12];   // byte offsets of the partners' lattice words
    for (int q = 0; q < 12; ++q) part[q] = 8u * zero;
    int32_t fs = std::abs(emb.h[k]);
    for (size_t a = 0; a < inc[k].size(); ++a) {
      const Term &t = emb.terms[inc[k][a]];
      aw[a] = static_cast<uint32_t>(std::abs(t.w));
      fs += std::abs(t.w);
      if (t.w < 0) neg |= 1u << a;
      int q = 0;
      for (int z = 0; z < t.arity; ++z)
        if (t.s[z] != k) part[P * a + (q++)] = 8u * L.dev_of[t.s[z]];
      if (q > P) return fail(SQA_ERR_UNSUPPORTED, "term arity above the kernel limit");
    }
    if (emb.h[k] < 0) neg |= 1u << (mec ? kFieldSignMEC : 4);
    uint32_t ah = static_cast<uint32_t>(std::abs(emb.h[k]));
    uint32_t *r = &L.rec[static_cast<size_t>(d) * L.rec_words];
    const bool metro = layout == kLayoutMetropolis && F <= kSmallF;
    const bool wolff = layout == kLayoutWolff && F <= kMidF;
    const bool ptb = layout == kLayoutPT && F <= kPTByteF;
    if (metro || wolff || ptb) {
      // Signed-weight layout: each term (and h) enters as W y with y the plain
      // product bit (own spin ^ partners; the own spin for h), and a constant.
      // Metropolis (small fields): the sum is c + 6 A (A: agreeing weight,
      // c = 3 (F - F_site)); a term agrees when its product bit equals its sign
      // bit, so W = -6|w| and the constant takes 6|w| where w >= 0, W = +6|w|
      // where w < 0.  c' <= 3 F + 3 F_site <= 60.
      // Wolff: the sum is S = sum |w| X (X: the term disagrees, its product bit
      // differs from its sign bit), so W = +|w| where w >= 0 and W = -|w|, with
      // |w| in the constant, where w < 0.  c' <= F_site <= 63.
      // PT: like Wolff with 2|w| and c' = F - F_site + those 2|w| (at most 2F).
      // The kernels accumulate 4 (c' + sum W y) per byte, so 4c' fits a byte.
      const uint32_t s = metro ? 6u : (ptb ? 2u : 1u);
      uint32_t W[7];
      int32_t cc = metro ? 3 * (F - fs) : (ptb ? F - fs : 0);
      auto put = [&](uint32_t a, bool negative_weight, int slot) {
        const bool flip = metro ? !negative_weight : negative_weight;   // weight enters as s|w| (1 - y)
        W[slot] = flip ? ((0x10000u - s * a) & 0xFFFFu) : s * a;
        if (flip) cc += static_cast<int32_t>(s * a);
      };
      for (int a = 0; a < T; ++a) put(aw[a], (neg >> a) & 1u, a);
      put(ah, emb.h[k] < 0, T);
      const uint32_t c4 = 4u * static_cast<uint32_t>(cc);
      // Wolff: F_site (PT does not read it: ME's last partner offset is then the whole word)
      const uint32_t fsh = (metro || ptb) ? 0u : (static_cast<uint32_t>(fs) << 16);
      r[0] = static_cast<uint32_t>(k) | ((c4 | (c4 << 8)) << 16);
      if (me) {
        r[1] = W[0] | (W[1] << 16);
        r[2] = W[2] | (W[3] << 16);
        r[3] = part[0] | (part[1] << 16);
        r[4] = part[2] | fsh;
      } else if (mec) {
        for (int q = 0; q < 3; ++q) r[1 + q] = W[2 * q] | (W[2 * q + 1] << 16);
        r[4] = W[6] | fsh;
        for (int q = 0; q < 3; ++q) r[5 + q] = part[2 * q] | (part[2 * q + 1] << 16);
      } else {
        r[1] = W[0] | (W[1] << 16);
        r[2] = W[2] | (W[3] << 16);
        r[3] = W[4] | fsh;
        for (int q = 0; q < 6; ++q) r[4 + q] = part[2 * q] | (part[2 * q + 1] << 16);
      }
      L.hfield[d] = emb.h[k];
      continue;
    }
    const uint32_t base = static_cast<uint32_t>(3 * (fs + F) + 2);
    r[0] = static_cast<uint32_t>(k) | (base << 16);
    if (me) {
      r[1] = aw[0] | (aw[1] << 8) | (aw[2] << 16) | (ah << 24);
      r[2] = neg | (part[0] << 16);
      r[3] = part[1] | (part[2] << 16);
    } else if (mec) {
      r[1] = aw[0] | (aw[1] << 8) | (aw[2] << 16) | (aw[3] << 24);
      r[2] = aw[4] | (aw[5] << 8) | (ah << 16) | (neg << 24);
      for (int q = 0; q < 3; ++q) r[3 + q] = part[2 * q] | (part[2 * q + 1] << 16);
    } else {
      r[1] = aw[0] | (aw[1] << 8) | (aw[2] << 16) | (aw[3] << 24);
      r[2] = ah | (neg << 8);
      r[3] = 0;
      for (int q = 0; q < 6; ++q) r[4 + q] = part[2 * q] | (part[2 * q + 1] << 16);
    }
    L.hfield[d] = emb.h[k];
  }
  L.term_w.resize(emb.terms.size());
  L.term_s.resize(2 * emb.terms.size());
  for (size_t t = 0; t < emb.terms.size(); ++t) {
    const Term &x = emb.terms[t];
    uint32_t s[4];
    for (int q = 0; q < 4; ++q) s[q] = (q < x.arity) ? L.dev_of[x.s[q]] : zero;
    L.term_w[t] = x.w;
    L.term_s[2 * t] = s[0] | (s[1] << 16);
    L.term_s[2 * t + 1] = s[2] | (s[3] << 16);
  }
  *out = std::move(L);
  return SQA_OK;
}

// ---------------------------------------------------------- tables
// Metropolis threshold for log acceptance ratio x: always-accept code for
// x >= 0, else floor(e^x 2^32) capped at 2^32 - 2.  Accept iff the 32-bit
// random word u satisfies min(u, 2^32 - 2) < threshold.
uint32_t threshold_from_log(double x) {
  if (x >= 0.0) return kAlways;
  const double scaled = std::floor(std::ldexp(std::exp(x), 32));
  return scaled >= 4294967294.0 ? 0xFFFFFFFEu : static_cast<uint32_t>(scaled);
}

std::vector<double> linear_gamma(double g0, double g1, int32_t M) {
  std::vector<double> g(M);
  for (int32_t m = 0; m < M; ++m) {
    if (M == 1) {
      g[m] = g0;
      continue;
    }
    const double t = static_cast<double>(m) / static_cast<double>(M - 1);
    g[m] = g0 * (1.0 - t) + g1 * t;
  }
  return g;
}

// Trotterised action of Eq. (2) with L slices: flipping s with a = s*f and
// b = s*(neighbour-slice sum) has log acceptance 2 (beta B/L * a - J_perp * b),
// J_perp = -ln(tanh(beta Gamma / L)) / 2; L = 1 has no time term.
std::vector<uint32_t> sqa_threshold_table(double beta, int32_t L, const std::vector<double> &gamma,
                                          const std::vector<double> *bscale, int32_t F) {
  const int32_t M = static_cast<int32_t>(gamma.size());
  const int32_t width = 2 * F + 1;
  std::vector<uint32_t> T(static_cast<size_t>(M) * width * 3);
  for (int32_t m = 0; m < M; ++m) {
    const double B = bscale ? (*bscale)[m] : 1.0;
    const double bl = beta * B / static_cast<double>(L);
    const double jperp = (L > 1) ? -0.5 * std::log(std::tanh(beta * gamma[m] / static_cast<double>(L))) : 0.0;
    for (int32_t a = -F; a <= F; ++a)
      for (int32_t bi = 0; bi < 3; ++bi) {
        const int32_t b = 2 * bi - 2;
        const double tb = (b == 0) ? 0.0 : jperp * static_cast<double>(b);
        const double x = 2.0 * (bl * static_cast<double>(a) - tb);
        T[(static_cast<size_t>(m) * width + (a + F)) * 3 + bi] = threshold_from_log(x);
      }
  }
  return T;
}

// Sec. III, time-like Wolff moves on the same Trotter action: an aligned ring
// bond joins the cluster with probability 1 - exp(-2 J_perp) = 1 - tanh(beta
// Gamma / L) (no bonds with L = 1); a cluster whose spins carry sum s f = A
// flips with min(1, exp(2 beta B / L * A)).
std::vector<uint32_t> wolff_join_table(double beta, int32_t L, const std::vector<double> &gamma) {
  std::vector<uint32_t> T(gamma.size(), 0u);
  if (L > 1)
    for (size_t m = 0; m < gamma.size(); ++m)
      T[m] = threshold_from_log(std::log(1.0 - std::tanh(beta * gamma[m] / static_cast<double>(L))));
  return T;
}

std::vector<uint32_t> wolff_accept_table(double beta, int32_t L, const std::vector<double> *bscale, int32_t F,
                                         int32_t *rows) {
  const int32_t nrows = bscale ? static_cast<int32_t>(bscale->size()) : 1;
  const int32_t width = 2 * L * F + 1;
  std::vector<uint32_t> T(static_cast<size_t>(nrows) * width);
  for (int32_t r = 0; r < nrows; ++r) {
    const double bl = beta * (bscale ? (*bscale)[r] : 1.0) / static_cast<double>(L);
    for (int32_t a = -L * F; a <= L * F; ++a)
      T[static_cast<size_t>(r) * width + (a + L * F)] = threshold_from_log(2.0 * (bl * static_cast<double>(a)));
  }
  *rows = nrows;
  return T;
}

// Appendix B, Eq. (B2): geometric ladder, slot 0 coldest.
std::vector<double> pt_betas(double beta_min, double beta_max, int32_t R) {
  std::vector<double> b(R);
  for (int32_t r = 0; r < R; ++r)
    b[r] = (R == 1) ? beta_max
                    : beta_max * std::pow(beta_min / beta_max, static_cast<double>(r) / static_cast<double>(R - 1));
  return b;
}

// Classical Metropolis at beta_r: flip of a site with a = s*f has log ratio 2 beta_r a.
std::vector<uint32_t> pt_metropolis_table(const std::vector<double> &betas, int32_t F) {
  const int32_t width = 2 * F + 1;
  std::vector<uint32_t> T(betas.size() * width);
  for (size_t r = 0; r < betas.size(); ++r)
    for (int32_t a = -F; a <= F; ++a)
      T[r * width + (a + F)] = threshold_from_log(2.0 * (betas[r] * static_cast<double>(a)));
  return T;
}

// Eq. (B1): swap slots r, r+1 with probability min(1, exp(D (beta_{r+1} - beta_r))),
// D = E_{r+1} - E_r; T[r][D], D = 0..Dmax.
std::vector<uint32_t> pt_swap_table(const std::vector<double> &betas, int32_t Dmax) {
  const size_t R = betas.size();
  std::vector<uint32_t> T((R > 1 ? R - 1 : 1) * static_cast<size_t>(Dmax + 1), 0u);
  for (size_t r = 0; r + 1 < R; ++r)
    for (int32_t D = 0; D <= Dmax; ++D)
      T[r * (Dmax + 1) + D] = threshold_from_log(static_cast<double>(D) * (betas[r + 1] - betas[r]));
  return T;
}

std::vector<uint32_t> pt_swap_pack(const std::vector<uint32_t> &stab, int32_t R, int32_t Dmax) {
  const int pairs = R > 1 ? R - 1 : 0;
  std::vector<uint32_t> out(static_cast<size_t>(std::max(R, 1)), 0u);
  for (int r = 0; r < pairs; ++r) {
    const uint32_t *row = stab.data() + static_cast<size_t>(r) * (Dmax + 1);
    int len = Dmax + 1;
    while (len > 0 && row[len - 1] == 0u) --len;
    out[r] = static_cast<uint32_t>(out.size());
    out.insert(out.end(), row, row + len);
  }
  out[std::max(pairs, 0)] = static_cast<uint32_t>(out.size());
  return out;
}

// ---------------------------------------------------------- host Philox
void host_philox4x32(const uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4]) {
  uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  for (int round = 0; round < 10; ++round) {
    const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * x[0];
    const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * x[2];
    const uint32_t y0 = static_cast<uint32_t>(pb >> 32) ^ x[1] ^ k0;
    const uint32_t y2 = static_cast<uint32_t>(pa >> 32) ^ x[3] ^ k1;
    x[1] = static_cast<uint32_t>(pb);
    x[3] = static_cast<uint32_t>(pa);
    x[0] = y0;
    x[2] = y2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  for (int q = 0; q < 4; ++q) out[q] = x[q];
}

// --------------------------------------------------------- occupancy
int device_cu_count() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
    cus = prop.multiProcessorCount;
  }
  return cus;
}

// Resident groups per CU: the runtime's occupancy calculation for the sweep
// kernel (registers, LDS, wave slots), else an LDS / wave-slot estimate.
int occupancy_groups_per_cu(const LaunchShape &s) {
  const int rt = sqa_anneal_occupancy(s.move, s.waves, s.lds_bytes(), s.team);
  if (rt > 0) return rt;
  const size_t lds = s.lds_bytes() + 64;
  int by_lds = static_cast<int>(kMaxLds / std::max<size_t>(lds, 1));
  int by_waves = 32 / s.waves;  // 8 waves per SIMD x 4 SIMDs
  int g = std::min(by_lds, by_waves);
  return std::max(g, 1);
}

}  // namespace sqa

sqa::HandleDev sqa_handle::dev(int m0, int m1, int flags) const {
  sqa::HandleDev H{};
  H.rec = arena.at<uint32_t>(off_rec);
  H.dev_of = arena.at<uint16_t>(off_devof);
  H.hfield = arena.at<int32_t>(off_hfield);
  H.term_w = arena.at<int32_t>(off_tw);
  H.term_s = arena.at<uint32_t>(off_ts);
  H.table = arena.at<uint32_t>(off_table);
  H.wacc = (move == sqa::kMoveWolff) ? arena.at<uint32_t>(off_wacc) : nullptr;
  H.move = move;
  H.wrows = wrows;
  H.wwidth = wwidth;
  H.spins = arena.at<int8_t>(off_spins);
  H.energy = arena.at<int32_t>(off_energy);
  H.kind = emb.kind;
  H.n = emb.n;
  H.n_terms = static_cast<int32_t>(emb.terms.size());
  H.L = L;
  H.M = M;
  H.R = R;
  H.F = F;
  H.tw = tw;
  H.m0 = m0;
  H.m1 = m1;
  H.flags = flags;
  H.seed_lo = static_cast<uint32_t>(seed);
  H.seed_hi = static_cast<uint32_t>(seed >> 32);
  for (int c = 0; c < 5; ++c) H.cls[c] = lay.cls[c];
  return H;
}
