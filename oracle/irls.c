/*
 * Oracle IRLS rounds (test infrastructure only).
 *
 * Section 2.1: each round computes conductances from the previous
 * potentials (Step 1, eq. define-reweight-vector with the reweighted
 * Laplacian of eq. reweighted-laplacian), then solves the weighted least
 * squares problem (Step 2, eq. constrained-wls) through the reduced
 * Laplacian system L~ v = b of eq. reduced-laplacian-system, where L~ drops
 * the rows and columns of s and t and b_u is the conductance of edge {u,s}.
 * Round 0 uses W = C, i.e. conductance = capacity.
 *
 * Section 3.1: the system is solved by preconditioned CG (Saad's PCG),
 * warm-started from the previous round's solution when requested, with the
 * paper's block-Jacobi preconditioner (eq. block-jacobi-subsystem): M =
 * blockdiag of the principal submatrices of L~ over a partition of the rows
 * into blocks, each block's rows taken in ascending order.  Blocks of size one
 * (precond 0) are the Jacobi preconditioner.  The blocks are consecutive rows
 * (block_size of them), or a caller's block id per node.  Each block is
 * factored once per round and applied by forward and back substitution, by
 * the paper's two strategies: precond 1 solves it exactly (its dense Cholesky
 * factorisation, the symmetric form of LU), precond 2 by ILU(0) (Saad's
 * incomplete LU with no fill: L unit lower and U upper triangular, both on
 * the pattern of the block, with (LU)_ij = A_ij on that pattern).
 *
 * Two conductance forms are provided:
 *   form 0: g = c / sqrt(d^2 + eps)
 *   form 1: g = c^2 / sqrt((c d)^2 + eps)   (paper's w with eps^2 -> eps)
 * with d = x_u - x_v.
 *
 * Dot products are summed in fixed chunks of 4096 entries, chunk partials in
 * chunk order, so the result does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "ograph.h"

#define CHUNK 4096

void orc_options_default(orc_options *o) {
  o->rounds = 30;
  o->eps0 = 0.1;
  o->eps_factor = 0.5;
  o->weight_form = 0;
  o->init = 0;
  o->warm_start = 1;
  o->cg_rtol = 1e-10;
  o->cg_maxit = 100000;
  o->threads = 0;
  o->precond = 0;
  o->block_size = 1;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static double cond(double c, double d, double eps, int form) {
  if (form == 0) return c / sqrt(d * d + eps);
  return (c * c) / sqrt((c * d) * (c * d) + eps);
}

static double dot(const double *a, const double *b, int64_t n) {
  int64_t nc = (n + CHUNK - 1) / CHUNK;
  double *part = (double *)malloc(sizeof(double) * (size_t)(nc ? nc : 1));
  #pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nc; c++) {
    int64_t lo = c * CHUNK, hi = lo + CHUNK < n ? lo + CHUNK : n;
    double acc = 0.0;
    for (int64_t i = lo; i < hi; i++) acc += a[i] * b[i];
    part[c] = acc;
  }
  double tot = 0.0;
  for (int64_t c = 0; c < nc; c++) tot += part[c];
  free(part);
  return tot;
}

/* one round's reduced system: conductances, diagonal and right-hand side */
typedef struct {
  double *w;          /* conductance per interior adjacency entry */
  double *ws, *wt;    /* conductance of the s-edge / t-edge per row */
  double  wst;        /* conductance of the s-t edge */
  double *D, *b;
} osys;

static void assemble(const ograph *g, osys *S, const double *v, int round0,
                     double eps, int form) {
  int64_t nt = g->nt;
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nt; i++) {
    double diag = 0.0;
    for (int64_t a = g->rp[i]; a < g->rp[i + 1]; a++) {
      double c = g->nc[a];
      S->w[a] = round0 ? c : cond(c, v[i] - v[g->nb[a]], eps, form);
      diag += S->w[a];
    }
    double cs = g->cs[i], ct = g->ct[i];
    S->ws[i] = cs > 0.0 ? (round0 ? cs : cond(cs, 1.0 - v[i], eps, form)) : 0.0;
    S->wt[i] = ct > 0.0 ? (round0 ? ct : cond(ct, v[i] - 0.0, eps, form)) : 0.0;
    S->D[i] = diag + S->ws[i] + S->wt[i];
    S->b[i] = S->ws[i];
  }
  S->wst = g->cst > 0.0 ? (round0 ? g->cst : cond(g->cst, 1.0, eps, form)) : 0.0;
}

/* q = L~ p */
static void spmv(const ograph *g, const osys *S, const double *p, double *q) {
  int64_t nt = g->nt;
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nt; i++) {
    double acc = S->D[i] * p[i];
    for (int64_t a = g->rp[i]; a < g->rp[i + 1]; a++) acc -= S->w[a] * p[g->nb[a]];
    q[i] = acc;
  }
}

/* block-Jacobi preconditioner.  Block k holds the rows rows[ptr[k] ..
 * ptr[k+1]) in ascending order; F + off[k] is its dense nb x nb factor
 * (row-major): the Cholesky factor L (lower) for precond 1, or L (strictly
 * lower, unit diagonal implied) and U (upper) in one array for precond 2. */
typedef struct {
  int32_t kind;       /* 1 exact (Cholesky), 2 ILU(0) */
  int64_t nblk;
  int64_t *ptr;       /* [nblk + 1] */
  int64_t *rows;      /* [nt] */
  int64_t *off;       /* [nblk] offsets into F */
  double *F;
  uint8_t *pat;       /* ILU(0): the block's pattern, same layout as F */
} oprec;

static void prec_free(oprec *P) {
  free(P->ptr); free(P->rows); free(P->off); free(P->F); free(P->pat);
}

static int cmp_pair(const void *a, const void *b) {
  const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
  if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
  return (x[1] > y[1]) - (x[1] < y[1]);
}

/* Blocks from block ids (NULL: consecutive runs of bs rows); returns 0 or
 * ORC_ERR_NOMEM. */
static int prec_setup(const ograph *g, const int64_t *block_of, int64_t bs, int32_t kind, oprec *P) {
  const int64_t nt = g->nt;
  memset(P, 0, sizeof(*P));
  P->kind = kind;
  /* (block id, row) pairs sorted: rows of a block are consecutive and
     ascending, blocks in ascending id (their order does not matter: they are
     independent) */
  int64_t (*pr)[2] = malloc(sizeof(*pr) * (size_t)(nt ? nt : 1));
  int64_t *bid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nt ? nt : 1));
  if (!pr || !bid) { free(pr); free(bid); return ORC_ERR_NOMEM; }
  for (int64_t i = 0; i < nt; i++) {
    pr[i][0] = block_of ? block_of[g->orig[i]] : i / bs;
    pr[i][1] = i;
  }
  qsort(pr, (size_t)nt, sizeof(*pr), cmp_pair);
  int64_t nb = 0;
  for (int64_t i = 0; i < nt; i++) {
    if (i == 0 || pr[i][0] != pr[i - 1][0]) nb++;
    bid[pr[i][1]] = nb - 1;
  }
  free(pr);
  P->nblk = nb;
  P->ptr = (int64_t *)calloc((size_t)nb + 1, sizeof(int64_t));
  P->rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nt ? nt : 1));
  P->off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb ? nb : 1));
  if (!P->ptr || !P->rows || !P->off) { free(bid); prec_free(P); return ORC_ERR_NOMEM; }
  for (int64_t i = 0; i < nt; i++) P->ptr[bid[i] + 1]++;
  for (int64_t k = 0; k < nb; k++) P->ptr[k + 1] += P->ptr[k];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb ? nb : 1));
  if (!fill) { free(bid); prec_free(P); return ORC_ERR_NOMEM; }
  for (int64_t k = 0; k < nb; k++) fill[k] = P->ptr[k];
  for (int64_t i = 0; i < nt; i++) P->rows[fill[bid[i]]++] = i;   /* ascending within each block */
  size_t tot = 0;
  for (int64_t k = 0; k < nb; k++) {
    const int64_t m = P->ptr[k + 1] - P->ptr[k];
    P->off[k] = (int64_t)tot;
    tot += (size_t)(m * m);
  }
  P->F = (double *)malloc(sizeof(double) * (tot ? tot : 1));
  if (kind == 2) P->pat = (uint8_t *)malloc(tot ? tot : 1);
  free(bid); free(fill);
  if (!P->F || (kind == 2 && !P->pat)) { prec_free(P); return ORC_ERR_NOMEM; }
  return ORC_OK;
}

/* The block's principal submatrix of L~ = D - W (dense), and its pattern. */
static void prec_gather(const ograph *g, const osys *S, const oprec *P, int64_t k, double *A, uint8_t *pat) {
  const int64_t b0 = P->ptr[k], m = P->ptr[k + 1] - b0;
  const int64_t *rows = P->rows + b0;
  for (int64_t i = 0; i < m * m; i++) { A[i] = 0.0; if (pat) pat[i] = 0; }
  for (int64_t i = 0; i < m; i++) {
    const int64_t r = rows[i];
    A[i * m + i] = S->D[r];
    if (pat) pat[i * m + i] = 1;
    for (int64_t a = g->rp[r]; a < g->rp[r + 1]; a++) {
      const int64_t j = g->nb[a];
      int64_t lo = 0, hi = m;                               /* position of row j in the block */
      while (lo < hi) { int64_t mid = (lo + hi) / 2; if (rows[mid] < j) lo = mid + 1; else hi = mid; }
      if (lo < m && rows[lo] == j) {
        A[i * m + lo] -= S->w[a];
        if (pat) pat[i * m + lo] = 1;
      }
    }
  }
}

static void prec_factor(const ograph *g, const osys *S, oprec *P) {
  #pragma omp parallel for schedule(dynamic)
  for (int64_t k = 0; k < P->nblk; k++) {
    const int64_t m = P->ptr[k + 1] - P->ptr[k];
    double *A = P->F + P->off[k];
    uint8_t *pat = P->kind == 2 ? P->pat + P->off[k] : NULL;
    prec_gather(g, S, P, k, A, pat);
    if (P->kind == 1) {
      for (int64_t j = 0; j < m; j++) {           /* Cholesky A = L L^T, in place */
        double d = A[j * m + j];
        for (int64_t c = 0; c < j; c++) d -= A[j * m + c] * A[j * m + c];
        d = sqrt(d);
        A[j * m + j] = d;
        for (int64_t i = j + 1; i < m; i++) {
          double x = A[i * m + j];
          for (int64_t c = 0; c < j; c++) x -= A[i * m + c] * A[j * m + c];
          A[i * m + j] = x / d;
        }
      }
    } else {
      /* ILU(0), row by row (Saad's IKJ form): for each pattern entry (i, k)
         left of the diagonal, a_ik /= a_kk, then a_ij -= a_ik a_kj for the
         pattern entries (i, j) right of k; nothing outside the pattern. */
      for (int64_t i = 1; i < m; i++) {
        for (int64_t kk = 0; kk < i; kk++) {
          if (!pat[i * m + kk]) continue;
          A[i * m + kk] /= A[kk * m + kk];
          const double l = A[i * m + kk];
          for (int64_t j = kk + 1; j < m; j++)
            if (pat[i * m + j]) A[i * m + j] -= l * A[kk * m + j];
        }
      }
    }
  }
}

/* z = M^-1 r */
static void prec_apply(const ograph *g, const osys *S, const oprec *P, const double *r, double *z) {
  const int64_t nt = g->nt;
  if (!P) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nt; i++) z[i] = r[i] / S->D[i];
    return;
  }
  #pragma omp parallel for schedule(dynamic)
  for (int64_t k = 0; k < P->nblk; k++) {
    const int64_t m = P->ptr[k + 1] - P->ptr[k];
    const int64_t *rows = P->rows + P->ptr[k];
    const double *F = P->F + P->off[k];
    if (P->kind == 1) {
      for (int64_t i = 0; i < m; i++) {           /* L y = r */
        double x = r[rows[i]];
        for (int64_t c = 0; c < i; c++) x -= F[i * m + c] * z[rows[c]];
        z[rows[i]] = x / F[i * m + i];
      }
      for (int64_t i = m - 1; i >= 0; i--) {      /* L^T z = y */
        double x = z[rows[i]];
        for (int64_t c = i + 1; c < m; c++) x -= F[c * m + i] * z[rows[c]];
        z[rows[i]] = x / F[i * m + i];
      }
    } else {
      const uint8_t *pat = P->pat + P->off[k];
      for (int64_t i = 0; i < m; i++) {           /* L y = r, L unit lower */
        double x = r[rows[i]];
        for (int64_t c = 0; c < i; c++)
          if (pat[i * m + c]) x -= F[i * m + c] * z[rows[c]];
        z[rows[i]] = x;
      }
      for (int64_t i = m - 1; i >= 0; i--) {      /* U z = y */
        double x = z[rows[i]];
        for (int64_t c = i + 1; c < m; c++)
          if (pat[i * m + c]) x -= F[i * m + c] * z[rows[c]];
        z[rows[i]] = x / F[i * m + i];
      }
    }
  }
}

/* PCG from the initial guess in v; returns status, fills iters/res.
 * P == NULL: Jacobi. */
static int pcg(const ograph *g, const osys *S, const oprec *P, double *v, double rtol, int64_t maxit,
               double *r, double *z, double *p, double *q, int64_t *iters, double *relres) {
  int64_t nt = g->nt;
  double bnorm = sqrt(dot(S->b, S->b, nt));
  *iters = 0;
  if (bnorm == 0.0) {                   /* b = 0: the unique solution is v = 0 */
    for (int64_t i = 0; i < nt; i++) v[i] = 0.0;
    *relres = 0.0;
    return ORC_OK;
  }
  spmv(g, S, v, q);
  for (int64_t i = 0; i < nt; i++) r[i] = S->b[i] - q[i];
  double rnorm = sqrt(dot(r, r, nt));
  if (rnorm <= rtol * bnorm) { *relres = rnorm / bnorm; return ORC_OK; }
  prec_apply(g, S, P, r, z);
  for (int64_t i = 0; i < nt; i++) p[i] = z[i];
  double rho = dot(r, z, nt);
  int64_t k = 0;
  while (k < maxit) {
    spmv(g, S, p, q);
    double pq = dot(p, q, nt);
    if (!(pq > 0.0) || !isfinite(pq)) { *iters = k; *relres = rnorm / bnorm; return ORC_ERR_BREAKDOWN; }
    double alpha = rho / pq;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nt; i++) { v[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
    k++;
    rnorm = sqrt(dot(r, r, nt));
    if (rnorm <= rtol * bnorm) break;
    prec_apply(g, S, P, r, z);
    double rho_new = dot(r, z, nt);
    double beta = rho_new / rho;
    rho = rho_new;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nt; i++) p[i] = z[i] + beta * p[i];
  }
  *iters = k;
  *relres = rnorm / bnorm;
  if (!isfinite(rnorm)) return ORC_ERR_BREAKDOWN;
  return rnorm <= rtol * bnorm ? ORC_OK : ORC_WARN_MAXIT;
}

/* per-round diagnostics at potentials v (x_s = 1, x_t = 0) */
static void round_stats(const ograph *g, const osys *S, const double *v, double eps_next,
                        int form, double *q, orc_round *R) {
  int64_t nt = g->nt;
  double se = 0.0, l1 = 0.0, fl = 0.0, fs = 0.0, ft = 0.0;
  double rho = 0.0;                                     /* max over edges of |w d| / c */
  double over = 0.0;                                    /* sum over edges of max(0, |w d| - c) */
  double vmin = nt ? v[0] : 0.0, vmax = nt ? v[0] : 0.0;
  for (int64_t i = 0; i < nt; i++) {
    for (int64_t a = g->rp[i]; a < g->rp[i + 1]; a++) {
      if (g->nb[a] <= i) continue;                      /* each interior edge once */
      double c = g->nc[a], d = v[i] - v[g->nb[a]];
      se += form == 0 ? c * sqrt(d * d + eps_next) : sqrt((c * d) * (c * d) + eps_next);
      l1 += c * fabs(d);
      fl += S->w[a] * d * d;
      if (S->w[a] * fabs(d) / c > rho) rho = S->w[a] * fabs(d) / c;
      if (S->w[a] * fabs(d) > c) over += S->w[a] * fabs(d) - c;
    }
    if (g->cs[i] > 0.0) {
      double c = g->cs[i], d = 1.0 - v[i];
      se += form == 0 ? c * sqrt(d * d + eps_next) : sqrt((c * d) * (c * d) + eps_next);
      l1 += c * fabs(d);
      fl += S->ws[i] * d * d;
      fs += S->ws[i] * d;
      if (S->ws[i] * fabs(d) / c > rho) rho = S->ws[i] * fabs(d) / c;
      if (S->ws[i] * fabs(d) > c) over += S->ws[i] * fabs(d) - c;
    }
    if (g->ct[i] > 0.0) {
      double c = g->ct[i], d = v[i];
      se += form == 0 ? c * sqrt(d * d + eps_next) : sqrt((c * d) * (c * d) + eps_next);
      l1 += c * fabs(d);
      fl += S->wt[i] * d * d;
      ft += S->wt[i] * d;
      if (S->wt[i] * fabs(d) / c > rho) rho = S->wt[i] * fabs(d) / c;
      if (S->wt[i] * fabs(d) > c) over += S->wt[i] * fabs(d) - c;
    }
    if (v[i] < vmin) vmin = v[i];
    if (v[i] > vmax) vmax = v[i];
  }
  if (g->cst > 0.0) {
    double c = g->cst;
    se += form == 0 ? c * sqrt(1.0 + eps_next) : sqrt(c * c + eps_next);
    l1 += c;
    fl += S->wst;
    fs += S->wst;
    ft += S->wst;
    if (S->wst / c > rho) rho = S->wst / c;
    if (S->wst > c) over += S->wst - c;
  }
  R->s_eps = se; R->l1 = l1; R->flow = fl; R->flow_s = fs; R->flow_t = ft;
  R->vmin = vmin; R->vmax = vmax;
  /* true residual of this round's system */
  double r1 = 0.0;                                      /* ||b - A v||_1 */
  if (nt > 0) {
    spmv(g, S, v, q);
    for (int64_t i = 0; i < nt; i++) q[i] = S->b[i] - q[i];
    double bn = sqrt(dot(S->b, S->b, nt));
    R->true_rel_res = bn > 0.0 ? sqrt(dot(q, q, nt)) / bn : 0.0;
    for (int64_t i = 0; i < nt; i++) r1 += fabs(q[i]);
  } else {
    R->true_rel_res = 0.0;
  }
  /* The electrical flow f_e = w_e d_e leaves node u's balance off by the
     residual r_u, so its net flow across any s-t cut is at least
     F = max(flow_s, flow_t) - ||r||_1.  Two lower bounds on the minimum cut
     follow: divided by max(1, rho) it respects every capacity, so F / max(1,
     rho) is at most the cut's capacity; and across any cut it carries at most
     the cut's capacity plus the overload sum(max(0, |f_e| - c_e)) of the
     cut's edges, hence of all edges (max-flow / min-cut duality). */
  double F = (fs > ft ? fs : ft) - r1;
  double lb1 = F / (rho > 1.0 ? rho : 1.0), lb2 = F - over;
  R->lower_bound = lb1 > lb2 ? lb1 : lb2;
}

int orc_irls(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
             const double *cap, int64_t s, int64_t t, const orc_options *opt,
             const double *x0, double *x_out, orc_round *rounds_out) {
  return orc_irls_blocks(n, m, eu, ev, cap, s, t, opt, NULL, x0, x_out, rounds_out);
}

int orc_irls_blocks(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
                    const double *cap, int64_t s, int64_t t, const orc_options *opt,
                    const int64_t *block_of, const double *x0, double *x_out, orc_round *rounds_out) {
  orc_options o;
  if (opt) o = *opt; else orc_options_default(&o);
  if (!x_out) return ORC_ERR_NULL;
  if (o.rounds < 0 || o.weight_form < 0 || o.weight_form > 1 || o.init < 0 || o.init > 2 ||
      !(o.cg_rtol > 0.0) || o.cg_maxit < 1 || (o.rounds > 0 && !(o.eps0 > 0.0)) ||
      !(o.eps_factor > 0.0) || o.eps_factor > 1.0 || o.precond < 0 || o.precond > 2 ||
      (o.precond >= 1 && !block_of && o.block_size < 1))
    return ORC_ERR_OPTIONS;
  if (o.init == 2 && !x0) return ORC_ERR_NULL;
#ifdef _OPENMP
  if (o.threads > 0) omp_set_num_threads(o.threads);
#endif
  ograph g;
  int rc = og_build(&g, n, m, eu, ev, cap, s, t);
  if (rc) return rc;
  int64_t nt = g.nt, na = g.rp[nt];
  size_t nv = (size_t)(nt ? nt : 1);
  osys S;
  S.w = (double *)malloc(sizeof(double) * (size_t)(na ? na : 1));
  S.ws = (double *)malloc(sizeof(double) * nv);
  S.wt = (double *)malloc(sizeof(double) * nv);
  S.D = (double *)malloc(sizeof(double) * nv);
  S.b = (double *)malloc(sizeof(double) * nv);
  double *v = (double *)calloc(nv, sizeof(double));
  double *r = (double *)malloc(sizeof(double) * nv);
  double *z = (double *)malloc(sizeof(double) * nv);
  double *p = (double *)malloc(sizeof(double) * nv);
  double *q = (double *)malloc(sizeof(double) * nv);
  oprec Pr, *P = NULL;
  memset(&Pr, 0, sizeof(Pr));
  int status = ORC_OK;
  if (!S.w || !S.ws || !S.wt || !S.D || !S.b || !v || !r || !z || !p || !q) { status = ORC_ERR_NOMEM; goto done; }
  if (o.precond >= 1 && nt > 0) {
    if (block_of)
      for (int64_t u = 0; u < n; u++)
        if (block_of[u] < 0) { status = ORC_ERR_RANGE; goto done; }
    status = prec_setup(&g, block_of, o.block_size < nt ? o.block_size : nt, o.precond, &Pr);
    if (status) goto done;
    P = &Pr;
  }

  if (o.init == 2) {
    for (int64_t i = 0; i < nt; i++) {
      v[i] = x0[g.orig[i]];
      if (!isfinite(v[i])) { status = ORC_ERR_RANGE; goto done; }
    }
  } else if (o.init == 1) {
    for (int64_t i = 0; i < nt; i++) v[i] = 0.5;
  }

  double eps = o.eps0;
  for (int32_t l = 0; l <= o.rounds; l++) {
    orc_round R;
    memset(&R, 0, sizeof(R));
    int64_t it = 0;
    double rel = 0.0;
    int st = ORC_OK;
    if (l == 0) {
      assemble(&g, &S, v, 1, 0.0, o.weight_form);
      if (P) prec_factor(&g, &S, P);
      if (o.init == 0) {                          /* x(0): WLS with W0 = C, cold start */
        for (int64_t i = 0; i < nt; i++) v[i] = 0.0;
        st = nt ? pcg(&g, &S, P, v, o.cg_rtol, o.cg_maxit, r, z, p, q, &it, &rel) : ORC_OK;
      }
      R.eps = 0.0;
    } else {
      assemble(&g, &S, v, 0, eps, o.weight_form);
      if (P) prec_factor(&g, &S, P);
      if (!o.warm_start) for (int64_t i = 0; i < nt; i++) v[i] = 0.0;
      st = nt ? pcg(&g, &S, P, v, o.cg_rtol, o.cg_maxit, r, z, p, q, &it, &rel) : ORC_OK;
      R.eps = eps;
    }
    R.cg_iters = it;
    R.rel_res = rel;
    R.status = st;
    double eps_next = l == 0 ? o.eps0 : eps * o.eps_factor;
    round_stats(&g, &S, v, eps_next, o.weight_form, q, &R);
    if (rounds_out) rounds_out[l] = R;
    if (st == ORC_ERR_BREAKDOWN) { status = st; goto done; }
    if (st == ORC_WARN_MAXIT) status = ORC_WARN_MAXIT;
    if (l >= 1) eps = eps * o.eps_factor;
  }
  for (int64_t u = 0; u < n; u++) x_out[u] = 0.0;
  for (int64_t i = 0; i < nt; i++) x_out[g.orig[i]] = v[i];
  x_out[s] = 1.0;
  x_out[t] = 0.0;
done:
  free(S.w); free(S.ws); free(S.wt); free(S.D); free(S.b);
  free(v); free(r); free(z); free(p); free(q);
  prec_free(&Pr);
  og_free(&g);
  return status;
}

int orc_reduced_system(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
                       const double *cap, int64_t s, int64_t t, const double *x,
                       double eps, int32_t weight_form, int64_t *rowptr, int64_t *col,
                       double *val, double *b, int64_t *nnz_out) {
  if (!rowptr || !nnz_out) return ORC_ERR_NULL;
  ograph g;
  int rc = og_build(&g, n, m, eu, ev, cap, s, t);
  if (rc) return rc;
  int64_t nt = g.nt;
  rowptr[0] = 0;
  for (int64_t i = 0; i < nt; i++) rowptr[i + 1] = rowptr[i] + (g.rp[i + 1] - g.rp[i]) + 1;
  *nnz_out = rowptr[nt];
  if (!col) { og_free(&g); return ORC_OK; }
  if (!val || !b) { og_free(&g); return ORC_ERR_NULL; }
  size_t nv = (size_t)(nt ? nt : 1);
  double *v = (double *)calloc(nv, sizeof(double));
  osys S;
  S.w = (double *)malloc(sizeof(double) * (size_t)(g.rp[nt] ? g.rp[nt] : 1));
  S.ws = (double *)malloc(sizeof(double) * nv);
  S.wt = (double *)malloc(sizeof(double) * nv);
  S.D = (double *)malloc(sizeof(double) * nv);
  S.b = (double *)malloc(sizeof(double) * nv);
  if (x) for (int64_t i = 0; i < nt; i++) v[i] = x[g.orig[i]];
  assemble(&g, &S, v, x == NULL, eps, weight_form);
  for (int64_t i = 0; i < nt; i++) {
    int64_t o = rowptr[i];
    int placed = 0;
    for (int64_t a = g.rp[i]; a < g.rp[i + 1]; a++) {
      if (!placed && g.nb[a] > i) { col[o] = i; val[o] = S.D[i]; o++; placed = 1; }
      col[o] = g.nb[a]; val[o] = -S.w[a]; o++;
    }
    if (!placed) { col[o] = i; val[o] = S.D[i]; o++; }
    b[i] = S.b[i];
  }
  free(v); free(S.w); free(S.ws); free(S.wt); free(S.D); free(S.b);
  og_free(&g);
  return ORC_OK;
}

int orc_block_apply(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
                    const double *cap, int64_t s, int64_t t, const double *x, double eps,
                    int32_t weight_form, int32_t kind, int64_t block_size, const int64_t *block_of,
                    const double *r, double *z) {
  if (!r || !z) return ORC_ERR_NULL;
  if (kind < 1 || kind > 2 || (!block_of && block_size < 1)) return ORC_ERR_OPTIONS;
  ograph g;
  int rc = og_build(&g, n, m, eu, ev, cap, s, t);
  if (rc) return rc;
  int64_t nt = g.nt;
  size_t nv = (size_t)(nt ? nt : 1);
  double *v = (double *)calloc(nv, sizeof(double));
  osys S;
  S.w = (double *)malloc(sizeof(double) * (size_t)(g.rp[nt] ? g.rp[nt] : 1));
  S.ws = (double *)malloc(sizeof(double) * nv);
  S.wt = (double *)malloc(sizeof(double) * nv);
  S.D = (double *)malloc(sizeof(double) * nv);
  S.b = (double *)malloc(sizeof(double) * nv);
  oprec P;
  memset(&P, 0, sizeof(P));
  if (!v || !S.w || !S.ws || !S.wt || !S.D || !S.b) rc = ORC_ERR_NOMEM;
  if (!rc && nt > 0) {
    if (x) for (int64_t i = 0; i < nt; i++) v[i] = x[g.orig[i]];
    assemble(&g, &S, v, x == NULL, eps, weight_form);
    rc = prec_setup(&g, block_of, block_size < nt ? block_size : nt, kind, &P);
    if (!rc) {
      prec_factor(&g, &S, &P);
      prec_apply(&g, &S, &P, r, z);
    }
  }
  prec_free(&P);
  free(v); free(S.w); free(S.ws); free(S.wt); free(S.D); free(S.b);
  og_free(&g);
  return rc;
}
