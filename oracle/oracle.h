/*
 * CPU oracle for the IRLS undirected s-t min-cut (Zhu & Gleich, "A Parallel
 * Min-Cut Algorithm using Iteratively Reweighted Least Squares").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain FP64 statement
 * of what the GPU library computes.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it.  It shares no source with
 * the GPU library and must never be linked into it.
 *
 * All entry points take the graph as an undirected edge list over node ids
 * 0..n-1 with capacities c > 0 (Section 2, problem statement), a source s
 * and a sink t.  Self loops are dropped and parallel edges merged by summing
 * their capacities in ascending input order.
 *
 * Return codes (shared meaning with the GPU library, defined separately):
 *   0 ok, 1 null pointer, 2 range, 3 bad capacity, 4 disconnected,
 *   5 bad options, 7 CG breakdown, 100 CG hit maxit (result usable).
 */
#ifndef IRLS_ORACLE_H
#define IRLS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0, ORC_ERR_NULL = 1, ORC_ERR_RANGE = 2, ORC_ERR_CAPACITY = 3,
  ORC_ERR_DISCONNECTED = 4, ORC_ERR_OPTIONS = 5, ORC_ERR_BREAKDOWN = 7,
  ORC_ERR_NOMEM = 9, ORC_WARN_MAXIT = 100
};

typedef struct {
  int32_t rounds;        /* T: reweighted rounds after round 0 */
  double  eps0;          /* smoothing of round 1 */
  double  eps_factor;    /* eps_{l+1} = eps_l * eps_factor */
  int32_t weight_form;   /* 0: c/sqrt(d^2+eps); 1: c^2/sqrt((c d)^2+eps) */
  int32_t init;          /* 0: round 0 solves with W0=C; 1: x=1/2; 2: caller x0 */
  int32_t warm_start;    /* 1: CG starts from the previous round's v */
  double  cg_rtol;       /* stop when ||r||_2 <= rtol ||b||_2 */
  int64_t cg_maxit;
  int32_t threads;       /* OpenMP threads, 0 = runtime default */
  int32_t precond;       /* 0: Jacobi (diagonal); block-Jacobi over blocks of rows (the
                            principal submatrices of L~), each solved 1: exactly (dense
                            Cholesky) or 2: by ILU(0) in ascending row order */
  int32_t block_size;    /* rows per block for precond 1, 2 when no block ids are given
                            (blocks of consecutive non-terminal rows; >= 1) */
} orc_options;

typedef struct {
  double  eps;           /* smoothing used to build this round's weights (0 in round 0) */
  int64_t cg_iters;
  double  rel_res;       /* recursive ||r||/||b|| at exit */
  double  true_rel_res;  /* ||b - A v||/||b|| recomputed at exit */
  double  s_eps;         /* smoothed objective at this round's x, eps of the next round */
  double  l1;            /* ||C B x||_1 */
  double  flow;          /* x^T L x with this round's conductances */
  double  flow_s;        /* flow leaving s */
  double  flow_t;        /* flow entering t */
  double  vmin, vmax;    /* range of the non-terminal potentials */
  int32_t status;
  double  lower_bound;   /* with f_e = w_e (x_u - x_v), F = max(flow_s, flow_t) -
                            ||b - A v||_1 and rho = max_e |f_e| / c_e:
                            max(F / max(1, rho), F - sum_e max(0, |f_e| - c_e)),
                            a lower bound on the minimum cut */
} orc_round;

void orc_options_default(orc_options *o);

/* Full IRLS: round 0 (or the chosen start) then rounds 1..T.
 * x0: n potentials used when init==2 (entries of s and t ignored), else NULL.
 * x_out: n potentials of the last round (x_s = 1, x_t = 0).
 * rounds_out: T+1 records (NULL allowed). */
int orc_irls(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
             const double *cap, int64_t s, int64_t t, const orc_options *opt,
             const double *x0, double *x_out, orc_round *rounds_out);

/* orc_irls with the block-Jacobi blocks given by block_of (n entries, >= 0,
 * indexed by node id; entries of s and t ignored): rows with equal ids form a
 * block.  block_of NULL: blocks of block_size consecutive rows. */
int orc_irls_blocks(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
                    const double *cap, int64_t s, int64_t t, const orc_options *opt,
                    const int64_t *block_of, const double *x0, double *x_out,
                    orc_round *rounds_out);

/* One application z = M^-1 r of the block-Jacobi preconditioner of a round's
 * system (x, eps, weight_form as for orc_reduced_system): blocks from
 * block_of (n entries) or of block_size consecutive rows, each factored by
 * kind 1 (exact, dense Cholesky) or 2 (ILU(0)).  r and z: n_nonterminal
 * entries, non-terminal nodes in ascending id. */
int orc_block_apply(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
                    const double *cap, int64_t s, int64_t t, const double *x, double eps,
                    int32_t weight_form, int32_t kind, int64_t block_size, const int64_t *block_of,
                    const double *r, double *z);

/* Reduced Laplacian of one round (pattern + values) for tests.
 * x: n potentials, or NULL for round 0 (conductance = capacity).
 * Call first with rowptr != NULL and col == NULL to get nnz in *nnz_out
 * (rowptr filled); then again with col/val/b/diag sized.  Rows are the
 * non-terminal nodes in ascending id; each row lists its neighbours and
 * itself in ascending order. */
int orc_reduced_system(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
                       const double *cap, int64_t s, int64_t t, const double *x,
                       double eps, int32_t weight_form, int64_t *rowptr, int64_t *col,
                       double *val, double *b, int64_t *nnz_out);

/* Sweep cut over x (n entries; those of s and t ignored).  Nodes are ordered
 * by x descending, ties by id ascending; S_k = {s} + first k nodes,
 * k = 0..n_nonterminal; the smallest k of minimum cut value wins.  Cut values
 * are exact sums in 128-bit fixed point; *value is the exact minimum
 * rounded to double.  in_S (n bytes), kstar, scale may be NULL. */
int orc_sweep(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
              const double *cap, int64_t s, int64_t t, const double *x,
              uint8_t *in_S, double *value, int64_t *kstar, int32_t *scale);

/* Exact value of the cut (S, V\S) given by in_S (in_S[s]=1, in_S[t]=0). */
int orc_cut_value(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
                  const double *cap, int64_t s, int64_t t, const uint8_t *in_S,
                  double *value);

/* Exact minimum s-t cut by FIFO push-relabel (global relabel + gap) on
 * 64-bit fixed-point capacities.  in_S: source side; value: exact value
 * (128-bit) of that cut rounded to double. */
int orc_maxflow(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
                const double *cap, int64_t s, int64_t t, uint8_t *in_S, double *value);

/* Exhaustive minimum s-t cut over all 2^(n-2) sets, n <= 24, exact 128-bit.
 * second: the smallest cut value strictly above the minimum (or -1). */
int orc_bruteforce(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
                   const double *cap, int64_t s, int64_t t, uint8_t *in_S,
                   double *value, double *second);

int orc_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
