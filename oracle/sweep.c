/*
 * Oracle sweep cut and exact cut values (test infrastructure only).
 *
 * The paper rounds the final voltage vector by a sweep cut (Section 3.4):
 * order the nodes by potential and take the best prefix set.  Reading used
 * here: nodes ordered by x descending with ties broken by ascending id;
 * candidate sets S_k = {s} + first k non-terminals for k = 0..n_nt; the
 * smallest k attaining the minimum cut wins.
 *
 * Cut values are sums of capacities.  To make the choice of k independent
 * of summation order, every capacity is mapped to a 128-bit integer
 * round-half-even(c * 2^k) with one scale k per graph, chosen so that the
 * sum of all capacities stays below 2^125.  For any capacity >= 2^(52-k)
 * the mapping is exact, so the sums are the exact sums of the doubles.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "ograph.h"

int fx_scale(const ograph *g) {
  double cmax = 0.0;
  for (int64_t e = 0; e < g->ne; e++) if (g->ec[e] > cmax) cmax = g->ec[e];
  int e2 = 0;
  if (cmax > 0.0) frexp(cmax, &e2);              /* cmax = f 2^e2, f in [0.5, 1) */
  int L = 0;                                     /* smallest L with 2^L >= ne + 1 */
  while (((int64_t)1 << L) < g->ne + 1) L++;
  return 125 - e2 - L;
}

i128 fx_quant(double c, int k) {
  if (c == 0.0) return 0;
  int e = 0;
  double f = frexp(c, &e);                       /* c = f 2^e */
  int64_t mant = (int64_t)ldexp(f, 53);          /* exact: f has 53 significant bits */
  int sh = e - 53 + k;                           /* c 2^k = mant 2^sh */
  if (sh >= 0) return (i128)mant << sh;
  int r = -sh;
  if (r >= 63) return 0;                         /* mant < 2^53 <= half of 2^r */
  int64_t q = mant >> r;
  int64_t rem = mant & (((int64_t)1 << r) - 1);
  int64_t half = (int64_t)1 << (r - 1);
  if (rem > half || (rem == half && (q & 1))) q++;
  return (i128)q;
}

double fx_to_double(i128 v, int k) {
  return ldexp((double)v, -k);                   /* int128 -> double rounds to nearest even */
}

typedef struct { double x; int64_t i; } okey;

static int cmp_okey(const void *a, const void *b) {
  const okey *p = (const okey *)a, *q = (const okey *)b;
  if (p->x > q->x) return -1;
  if (p->x < q->x) return 1;
  return p->i < q->i ? -1 : (p->i > q->i);
}

int orc_sweep(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
              const double *cap, int64_t s, int64_t t, const double *x,
              uint8_t *in_S, double *value, int64_t *kstar, int32_t *scale) {
  if (!x) return ORC_ERR_NULL;
  ograph g;
  int rc = og_build(&g, n, m, eu, ev, cap, s, t);
  if (rc) return rc;
  int64_t nt = g.nt;
  for (int64_t i = 0; i < nt; i++)
    if (!isfinite(x[g.orig[i]])) { og_free(&g); return ORC_ERR_RANGE; }
  okey *ord = (okey *)malloc(sizeof(okey) * (size_t)(nt ? nt : 1));
  int64_t *rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nt ? nt : 1));
  if (!ord || !rank) { free(ord); free(rank); og_free(&g); return ORC_ERR_NOMEM; }
  for (int64_t i = 0; i < nt; i++) { ord[i].x = x[g.orig[i]]; ord[i].i = i; }
  qsort(ord, (size_t)nt, sizeof(okey), cmp_okey);
  for (int64_t j = 0; j < nt; j++) rank[ord[j].i] = j + 1;

  int k = fx_scale(&g);
  /* S_0 = {s}: every edge at s is cut, including the s-t edge */
  i128 cur = fx_quant(g.cst, k);
  for (int64_t i = 0; i < nt; i++) cur += fx_quant(g.cs[i], k);
  i128 best = cur;
  int64_t kb = 0;
  for (int64_t j = 1; j <= nt; j++) {
    int64_t u = ord[j - 1].i;
    /* moving u into S: its s-edge stops being cut, its t-edge starts; an
     * interior edge stops being cut if the neighbour is already in S */
    i128 d = fx_quant(g.ct[u], k) - fx_quant(g.cs[u], k);
    for (int64_t a = g.rp[u]; a < g.rp[u + 1]; a++) {
      i128 q = fx_quant(g.nc[a], k);
      if (rank[g.nb[a]] > rank[u]) d += q; else d -= q;
    }
    cur += d;
    if (cur < best) { best = cur; kb = j; }
  }
  if (in_S) {
    for (int64_t v = 0; v < n; v++) in_S[v] = 0;
    in_S[s] = 1;
    for (int64_t i = 0; i < nt; i++) if (rank[i] <= kb) in_S[g.orig[i]] = 1;
  }
  if (value) *value = fx_to_double(best, k);
  if (kstar) *kstar = kb;
  if (scale) *scale = k;
  free(ord); free(rank); og_free(&g);
  return ORC_OK;
}

int orc_cut_value(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
                  const double *cap, int64_t s, int64_t t, const uint8_t *in_S,
                  double *value) {
  if (!in_S || !value) return ORC_ERR_NULL;
  ograph g;
  int rc = og_build(&g, n, m, eu, ev, cap, s, t);
  if (rc) return rc;
  if (!in_S[s] || in_S[t]) { og_free(&g); return ORC_ERR_RANGE; }
  int k = fx_scale(&g);
  i128 acc = 0;
  for (int64_t e = 0; e < g.ne; e++)
    if ((in_S[g.ea[e]] != 0) != (in_S[g.eb[e]] != 0)) acc += fx_quant(g.ec[e], k);
  *value = fx_to_double(acc, k);
  og_free(&g);
  return ORC_OK;
}
