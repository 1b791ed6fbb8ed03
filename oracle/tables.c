/*
 * Annealing schedule and Metropolis acceptance tables for the oracle
 * (test infrastructure only).  All transcendental functions are evaluated
 * here, on the host, in double precision with the C library's exp/log/tanh/
 * pow; the stochastic part only ever compares a 32-bit random word with a
 * tabulated 32-bit threshold.
 *
 * Acceptance rule (Metropolis).  For a proposed flip whose log acceptance
 * ratio is x (accept with probability min(1, e^x)):
 *   x >= 0  -> threshold 0xFFFFFFFF, meaning "always accept";
 *   x <  0  -> threshold R = min(floor(e^x * 2^32), 0xFFFFFFFE);
 * and a flip with random word u is accepted iff R == 0xFFFFFFFF or u < R.
 * The acceptance probability is R / 2^32, below e^x by less than 2^-32.
 *
 * SQA (Eq. (2), Sec. II; Appendix B).  The paper anneals H(t) = A(t) H_X +
 * B(t) H_P with H_X = -sum sigma^x, using discrete-time path-integral Monte
 * Carlo with L Trotter slices.  The standard Suzuki-Trotter mapping (the
 * paper cites it, it prints no formula) gives the classical action
 *   S = (beta B / L) sum_tau H_P(s^tau) - J_perp sum_tau sum_k s_k^tau s_k^{tau+1},
 *   J_perp = -1/2 ln tanh(beta Gamma / L),   Gamma = A,
 * periodic in tau.  Flipping s = s_k^tau, with a = s * f_k^tau (local field
 * f) and b = s * (s_k^{tau-1} + s_k^{tau+1}), changes S by
 *   dS = 2 (J_perp b - (beta B / L) a),   so   x = -dS = 2 (bl*a - jp*b).
 * With L = 1 there is no time coupling (b = 0): classical Metropolis at beta.
 * The schedule shape A(t), B(t) is only shown in a figure; the reading used
 * is Gamma linear from Gamma_0 (sweep 0) to Gamma_1 (last sweep), B = 1,
 * unless explicit per-sweep arrays are given.
 *
 * Table layout: T[m][a + F][(b + 2) / 2], a in [-F, F], b in {-2, 0, 2}.
 */
#include <math.h>
#include "oracle.h"

uint32_t oracle_threshold(double x) {
  if (x >= 0.0) return 0xFFFFFFFFu;
  double s = ldexp(exp(x), 32);
  double f = floor(s);
  if (f >= 4294967294.0) return 0xFFFFFFFEu;
  return (uint32_t)f;
}

/* Gamma_m = Gamma_0 (1 - t) + Gamma_1 t with t = m / (M - 1): exact at both ends. */
void oracle_gamma_schedule(double g0, double g1, int32_t M, double *out) {
  for (int m = 0; m < M; ++m) {
    if (M == 1) {
      out[m] = g0;
    } else {
      double t = (double)m / (double)(M - 1);
      out[m] = g0 * (1.0 - t) + g1 * t;
    }
  }
}

void oracle_sqa_table(double beta, int32_t L, int32_t M, const double *gamma,
                      const double *bscale, int32_t F, uint32_t *out) {
  int width = 2 * F + 1;
  for (int m = 0; m < M; ++m) {
    double B = bscale ? bscale[m] : 1.0;
    double bl = beta * B / (double)L;
    double jp = 0.0;
    if (L > 1) jp = -0.5 * log(tanh(beta * gamma[m] / (double)L));
    for (int a = -F; a <= F; ++a) {
      for (int bi = 0; bi < 3; ++bi) {
        int b = 2 * bi - 2;
        double tb = (b == 0) ? 0.0 : jp * (double)b;  /* J_perp may be +inf at Gamma = 0 */
        double x = 2.0 * (bl * (double)a - tb);
        out[((size_t)m * width + (a + F)) * 3 + bi] = oracle_threshold(x);
      }
    }
  }
}

/* Appendix B, Eq. (B2): beta_r = beta_max (beta_min / beta_max)^(r / (R-1)),
 * slot 0 coldest.  (The paper: 64 temperatures, beta from 20 down to 0.1.) */
void oracle_pt_ladder(double beta_min, double beta_max, int32_t R, double *out) {
  for (int r = 0; r < R; ++r) {
    if (R == 1) out[r] = beta_max;
    else out[r] = beta_max * pow(beta_min / beta_max, (double)r / (double)(R - 1));
  }
}

/* Classical single-spin Metropolis at beta_r: flip changes E by -2a, so x = 2 beta_r a.
 * Layout T[r][a + F]. */
void oracle_pt_table(const double *betas, int32_t R, int32_t F, uint32_t *out) {
  int width = 2 * F + 1;
  for (int r = 0; r < R; ++r)
    for (int a = -F; a <= F; ++a)
      out[(size_t)r * width + (a + F)] = oracle_threshold(2.0 * (betas[r] * (double)a));
}

/* Appendix B, Eq. (B1): p_swap = min{1, exp[(E_{r+1} - E_r)(beta_{r+1} - beta_r)]}.
 * Layout T[r][D] for D = E_{r+1} - E_r in [0, Dmax]; D <= 0 always accepts. */
void oracle_swap_table(const double *betas, int32_t R, int32_t Dmax, uint32_t *out) {
  for (int r = 0; r + 1 < R; ++r)
    for (int D = 0; D <= Dmax; ++D)
      out[(size_t)r * (Dmax + 1) + D] =
          oracle_threshold((double)D * (betas[r + 1] - betas[r]));
}
