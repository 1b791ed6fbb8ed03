/*
 * CPU oracle for path-integral simulated quantum annealing (SQA) and parallel
 * tempering (PT) over minor-embedded (ME) and LHZ-embedded Ising problems.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, deliberately slow statement of
 * what the GPU library computes, used to check it element by element.  The
 * GPU library never includes, links or calls anything in this directory, and
 * this directory shares no code, header, table or constant generator with it.
 *
 * Paper: T. Albash, W. Vinci, D. A. Lidar, "Simulated Quantum Annealing
 * Comparison between All-to-All Connectivity Schemes" (arXiv:1603.03755).
 * Every function cites the section / equation it follows.  Where the paper is
 * silent, the reading taken is stated at the function.
 *
 * Conventions
 *   spins            int8_t, value +1 or -1
 *   SQA lattice      [replica][slice][site]   (slice-major)
 *   PT lattice       [replica][site]
 *   couplings J      int32_t, N*N row-major; only entries i<j are read
 */
#ifndef SQA_ORACLE_H
#define SQA_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* RNG streams of the counter layout. */
enum { OR_STREAM_INIT = 1, OR_STREAM_SQA = 2, OR_STREAM_PT = 3,
       OR_STREAM_SWAP = 4, OR_STREAM_TREE = 5, OR_STREAM_PT_INIT = 6, OR_STREAM_WOLFF = 7,
       OR_STREAM_SQA_LO = 8, OR_STREAM_WOLFF_LO = 9, OR_STREAM_PT_LO = 10 };

enum { OR_ME = 0, OR_LHZ = 1, OR_MEC = 2 };

/* A physical Hamiltonian: integer fields on sites plus k-body terms, k<=4. */
typedef struct {
  int32_t kind;       /* OR_ME, OR_LHZ or OR_MEC */
  int32_t N;          /* logical spins */
  int32_t n_sites;
  int32_t n_terms;
  int32_t fmax;       /* max over sites of |h_k| + sum over incident terms |w_t| */
  int32_t emax;       /* sum |h_k| + sum |w_t|: bound on |E| */
  int32_t *h;         /* [n_sites] */
  int32_t *colour;    /* [n_sites], 0..3 */
  int32_t *w;         /* [n_terms] */
  int32_t *arity;     /* [n_terms], 2..4 */
  int32_t *tsite;     /* [n_terms][4], unused slots -1 */
  int32_t *row;       /* [n_sites+1]  incident-term lists (CSR) */
  int32_t *inc;       /* [row[n_sites]] term ids */
} OEmb;

/* ---- Philox (Salmon, Moraes, Dror, Shaw, SC'11), 10 rounds -------------- */
void oracle_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
uint32_t oracle_sqa_word(uint64_t seed, uint32_t stream, uint32_t replica,
                         uint32_t site, uint32_t slice, uint32_t sweep);
uint32_t oracle_sqa_uniform(uint64_t seed, uint32_t replica, uint32_t site, uint32_t slice, uint32_t sweep);
uint32_t oracle_pt_word(uint64_t seed, uint32_t stream, uint32_t replica,
                        uint32_t site, uint32_t sweep);
uint32_t oracle_pt_uniform(uint64_t seed, uint32_t replica, uint32_t site, uint32_t sweep);

/* ---- embeddings ---------------------------------------------------------- */
int  oracle_embed(int32_t kind, int32_t N, const int32_t *J, const int32_t *h,
                  int32_t penalty, OEmb *out);
void oracle_emb_free(OEmb *e);
int32_t oracle_me_site(int32_t N, int32_t i, int32_t r);
int32_t oracle_lhz_site(int32_t N, int32_t i, int32_t j);
int32_t oracle_chimera_m(int32_t N);
int32_t oracle_chimera_site(int32_t N, int32_t i, int32_t t);
void oracle_chimera_qubit(int32_t N, int32_t i, int32_t t, int32_t *row, int32_t *col, int32_t *side, int32_t *k);
int32_t oracle_local_field(const OEmb *e, const int8_t *s, int32_t k);
int32_t oracle_energy(const OEmb *e, const int8_t *s);
int32_t oracle_logical_energy(int32_t N, const int32_t *J, const int32_t *h, const int8_t *sigma);

/* ---- schedule and acceptance tables -------------------------------------- */
uint32_t oracle_threshold(double x);
void oracle_gamma_schedule(double g0, double g1, int32_t M, double *out);
void oracle_sqa_table(double beta, int32_t L, int32_t M, const double *gamma,
                      const double *bscale, int32_t F, uint32_t *out);
void oracle_pt_ladder(double beta_min, double beta_max, int32_t R, double *out);
void oracle_pt_table(const double *betas, int32_t R, int32_t F, uint32_t *out);
void oracle_swap_table(const double *betas, int32_t R, int32_t Dmax, uint32_t *out);

/* ---- SQA ----------------------------------------------------------------- */
void oracle_sqa_init(const OEmb *e, int32_t L, int32_t R, uint64_t seed, int8_t *spins);
void oracle_sqa_init_from(const OEmb *e, int32_t L, int32_t r0, int32_t R, uint64_t seed, int8_t *spins);
int32_t oracle_sqa_sweep_order(const OEmb *e, int32_t L, int32_t *site_out, int32_t *slice_out);
uint32_t oracle_sqa_attempt_threshold(const OEmb *e, int32_t L, const uint32_t *table,
                                      int32_t F, const int8_t *lat, int32_t k,
                                      int32_t tau, int32_t m);
void oracle_sqa_run(const OEmb *e, int32_t L, int32_t R, int32_t m0, int32_t m1,
                    const uint32_t *table, int32_t F, uint64_t seed,
                    int8_t *spins, int32_t nthreads);
void oracle_sqa_run_from(const OEmb *e, int32_t L, int32_t r0, int32_t R, int32_t m0, int32_t m1,
                         const uint32_t *table, int32_t F, uint64_t seed,
                         int8_t *spins, int32_t nthreads);
void oracle_sqa_energies(const OEmb *e, int32_t L, int32_t R, const int8_t *spins,
                         int32_t *E);

/* ---- SQA with time-like Wolff cluster updates (Sec. III) ------------------ */
uint32_t oracle_wolff_bond_uniform(uint64_t seed, uint32_t r, uint32_t k, uint32_t b, uint32_t m);
void oracle_wolff_site_words(uint64_t seed, uint32_t r, uint32_t k, uint32_t m, uint32_t *u_seed,
                             uint32_t *u_acc);
void oracle_wolff_tables(double beta, int32_t L, int32_t M, const double *gamma,
                         const double *bscale, int32_t F, uint32_t *padd, uint32_t *acc);
void oracle_wolff_move(const OEmb *e, int32_t L, int32_t count, int8_t *lats, int32_t k, int32_t tau0,
                       const uint32_t *bond_u, uint32_t u_acc, uint32_t padd, const uint32_t *acc_row,
                       int32_t F, uint32_t *thr_out, uint64_t *cl_out);
int32_t oracle_wolff_site_order(const OEmb *e, int32_t *site_out);
void oracle_wolff_run(const OEmb *e, int32_t L, int32_t r0, int32_t R, int32_t m0, int32_t m1,
                      const uint32_t *padd, const uint32_t *acc, int32_t rows, int32_t F,
                      uint64_t seed, int8_t *spins, int32_t nthreads);

/* ---- PT ------------------------------------------------------------------ */
void oracle_pt_init(const OEmb *e, int32_t R, uint64_t seed, int8_t *spins);
void oracle_pt_run(const OEmb *e, int32_t R, int32_t sweeps, int32_t sweeps_per_swap,
                   const uint32_t *mtab, int32_t F, const uint32_t *stab, int32_t Dmax,
                   uint64_t seed, int8_t *spins, int32_t *E, int32_t *rep_at,
                   uint64_t *swap_acc);

/* ---- decoders ------------------------------------------------------------ */
void oracle_me_majority(const OEmb *e, const int8_t *slice, int8_t *logical);
void oracle_lhz_tree_decode(int32_t N, const int8_t *slice, const int32_t *parents,
                            int32_t n_trees, int8_t *logical);
int  oracle_random_trees(uint64_t seed, int32_t N, int32_t n_trees, int32_t *parents);
void oracle_lhz_mwd(int32_t N, const int8_t *slice, int8_t *logical);
void oracle_lhz_bp(int32_t N, const int8_t *slice, double error_rate, int32_t iterations,
                   const int32_t *parents, int32_t n_trees, int8_t *logical, int8_t *pairs_out);
void oracle_lhz_mld(int32_t N, const int8_t *slice, double error_rate, int8_t *logical, int64_t *corr_out);
int32_t oracle_ground_states(int32_t N, const int32_t *J, const int32_t *h,
                             int8_t *states, int32_t max_states, int32_t *n_found);

#ifdef __cplusplus
}
#endif
#endif
