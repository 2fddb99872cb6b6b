/*
 * Exact minimum s-t cut for checking (test infrastructure only).
 *
 * The paper measures the quality of a rounded cut by delta = (mu - mu*)/mu*
 * (Section 5, Table 4), with mu* from an exact combinatorial solver, and
 * names push-relabel as the fastest combinatorial family (Section 4).
 * This is a FIFO push-relabel (Goldberg-Tarjan) with periodic global
 * relabelling by backward BFS from t, on capacities mapped to 64-bit fixed
 * point round(c 2^k) with k chosen so that all capacities sum below 2^62.
 * Only the first phase (maximum preflow) is run: afterwards the nodes that
 * cannot reach t in the residual graph form a minimum cut's source side.
 *
 * orc_bruteforce enumerates every source side on graphs of <= 24 nodes and
 * sums exact 128-bit fixed-point capacities.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "ograph.h"

static int scale64(const ograph *g) {
  double cmax = 0.0;
  for (int64_t e = 0; e < g->ne; e++) if (g->ec[e] > cmax) cmax = g->ec[e];
  int e2 = 0;
  if (cmax > 0.0) frexp(cmax, &e2);
  int L = 0;
  while (((int64_t)1 << L) < g->ne + 1) L++;
  return 62 - e2 - L;
}

typedef struct {
  int64_t n, s, t;
  int64_t *first;     /* [n+1] arcs of node v: first[v] .. first[v+1]-1 */
  int64_t *head;      /* [2ne] arc target */
  int64_t *mate;      /* [2ne] reverse arc */
  int64_t *res;       /* [2ne] residual capacity */
  int64_t *h, *ex, *cur, *queue, *bfs;
  char *inq;
} pr_state;

static void global_relabel(pr_state *P) {
  int64_t n = P->n;
  for (int64_t v = 0; v < n; v++) P->h[v] = n;
  int64_t qh = 0, qt = 0;
  P->h[P->t] = 0;
  P->bfs[qt++] = P->t;
  while (qh < qt) {
    int64_t w = P->bfs[qh++];
    for (int64_t a = P->first[w]; a < P->first[w + 1]; a++) {
      int64_t x = P->head[a];
      /* arc x -> w is mate(a); usable when it has residual capacity */
      if (P->res[P->mate[a]] > 0 && P->h[x] == n && x != P->s) {
        P->h[x] = P->h[w] + 1;
        P->bfs[qt++] = x;
      }
    }
  }
  P->h[P->s] = n;
  for (int64_t v = 0; v < n; v++) P->cur[v] = P->first[v];
}

int orc_maxflow(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
                const double *cap, int64_t s, int64_t t, uint8_t *in_S, double *value) {
  if (!in_S || !value) return ORC_ERR_NULL;
  ograph g;
  int rc = og_build(&g, n, m, eu, ev, cap, s, t);
  if (rc) return rc;
  int k64 = scale64(&g);
  int64_t na = 2 * g.ne;
  pr_state P;
  memset(&P, 0, sizeof(P));
  P.n = n; P.s = s; P.t = t;
  P.first = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  P.head = (int64_t *)malloc(sizeof(int64_t) * (size_t)(na ? na : 1));
  P.mate = (int64_t *)malloc(sizeof(int64_t) * (size_t)(na ? na : 1));
  P.res = (int64_t *)malloc(sizeof(int64_t) * (size_t)(na ? na : 1));
  P.h = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  P.ex = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  P.cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  P.queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  P.bfs = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  P.inq = (char *)calloc((size_t)n, 1);
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int status = ORC_OK;
  if (!P.first || !P.head || !P.mate || !P.res || !P.h || !P.ex || !P.cur || !P.queue ||
      !P.bfs || !P.inq || !fill) { status = ORC_ERR_NOMEM; goto done; }

  /* each undirected edge {a,b} gives arcs a->b and b->a of equal capacity */
  for (int64_t e = 0; e < g.ne; e++) { P.first[g.ea[e] + 1]++; P.first[g.eb[e] + 1]++; }
  for (int64_t v = 0; v < n; v++) P.first[v + 1] += P.first[v];
  memcpy(fill, P.first, sizeof(int64_t) * (size_t)n);
  for (int64_t e = 0; e < g.ne; e++) {
    int64_t a = g.ea[e], b = g.eb[e];
    int64_t qa = fill[a]++, qb = fill[b]++;
    int64_t c = (int64_t)fx_quant(g.ec[e], k64);
    P.head[qa] = b; P.res[qa] = c; P.mate[qa] = qb;
    P.head[qb] = a; P.res[qb] = c; P.mate[qb] = qa;
  }

  /* saturate the arcs leaving s */
  for (int64_t a = P.first[s]; a < P.first[s + 1]; a++) {
    int64_t w = P.head[a], d = P.res[a];
    P.res[a] = 0; P.res[P.mate[a]] += d; P.ex[w] += d; P.ex[s] -= d;
  }
  global_relabel(&P);
  int64_t qh = 0, qt = 0, qn = 0;           /* circular FIFO of active nodes */
  for (int64_t v = 0; v < n; v++)
    if (v != s && v != t && P.ex[v] > 0 && P.h[v] < n) { P.queue[qt] = v; qt = (qt + 1) % n; qn++; P.inq[v] = 1; }
  int64_t work = 0, threshold = 6 * n + g.ne;

  while (qn > 0) {
    int64_t v = P.queue[qh]; qh = (qh + 1) % n; qn--; P.inq[v] = 0;
    while (P.ex[v] > 0 && P.h[v] < n) {
      if (P.cur[v] == P.first[v + 1]) {
        /* relabel: one above the lowest neighbour reachable by a residual arc */
        int64_t nh = 2 * n;
        for (int64_t a = P.first[v]; a < P.first[v + 1]; a++)
          if (P.res[a] > 0 && P.h[P.head[a]] + 1 < nh) nh = P.h[P.head[a]] + 1;
        P.h[v] = nh < n ? nh : n;
        P.cur[v] = P.first[v];
        work += 12 + (P.first[v + 1] - P.first[v]);
        continue;
      }
      int64_t a = P.cur[v], w = P.head[a];
      if (P.res[a] > 0 && P.h[v] == P.h[w] + 1) {
        int64_t d = P.ex[v] < P.res[a] ? P.ex[v] : P.res[a];
        P.res[a] -= d; P.res[P.mate[a]] += d; P.ex[v] -= d; P.ex[w] += d;
        if (w != s && w != t && !P.inq[w] && P.h[w] < n) {
          P.queue[qt] = w; qt = (qt + 1) % n; qn++; P.inq[w] = 1;
        }
      } else {
        P.cur[v]++;
      }
    }
    if (work > threshold) {
      work = 0;
      global_relabel(&P);
      /* rebuild the queue: labels changed, some nodes are now cut off */
      qh = qt = qn = 0;
      for (int64_t u = 0; u < n; u++) P.inq[u] = 0;
      for (int64_t u = 0; u < n; u++)
        if (u != s && u != t && P.ex[u] > 0 && P.h[u] < n) { P.queue[qt] = u; qt = (qt + 1) % n; qn++; P.inq[u] = 1; }
    }
  }

  /* source side: nodes that cannot reach t through residual arcs */
  global_relabel(&P);
  for (int64_t v = 0; v < n; v++) in_S[v] = P.h[v] >= n ? 1 : 0;
  in_S[s] = 1; in_S[t] = 0;
  {
    int k = fx_scale(&g);
    i128 acc = 0;
    for (int64_t e = 0; e < g.ne; e++)
      if (in_S[g.ea[e]] != in_S[g.eb[e]]) acc += fx_quant(g.ec[e], k);
    *value = fx_to_double(acc, k);
  }
done:
  free(P.first); free(P.head); free(P.mate); free(P.res); free(P.h); free(P.ex);
  free(P.cur); free(P.queue); free(P.bfs); free(P.inq); free(fill);
  og_free(&g);
  return status;
}

int orc_bruteforce(int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
                   const double *cap, int64_t s, int64_t t, uint8_t *in_S,
                   double *value, double *second) {
  if (!in_S || !value || !second) return ORC_ERR_NULL;
  if (n > 24) return ORC_ERR_RANGE;
  ograph g;
  int rc = og_build(&g, n, m, eu, ev, cap, s, t);
  if (rc) return rc;
  int k = fx_scale(&g);
  i128 *q = (i128 *)malloc(sizeof(i128) * (size_t)(g.ne ? g.ne : 1));
  for (int64_t e = 0; e < g.ne; e++) q[e] = fx_quant(g.ec[e], k);
  uint8_t side[24];
  int64_t nt = g.nt;
  i128 best = -1, sec = -1;
  uint64_t bestmask = 0;
  for (uint64_t mask = 0; mask < ((uint64_t)1 << nt); mask++) {
    for (int64_t v = 0; v < n; v++) side[v] = 0;
    side[s] = 1;
    for (int64_t i = 0; i < nt; i++) if (mask >> i & 1) side[g.orig[i]] = 1;
    i128 acc = 0;
    for (int64_t e = 0; e < g.ne; e++) if (side[g.ea[e]] != side[g.eb[e]]) acc += q[e];
    if (best < 0 || acc < best) {
      if (best >= 0) sec = best;
      best = acc; bestmask = mask;
    } else if (acc > best && (sec < 0 || acc < sec)) {
      sec = acc;
    }
  }
  for (int64_t v = 0; v < n; v++) in_S[v] = 0;
  in_S[s] = 1;
  for (int64_t i = 0; i < nt; i++) if (bestmask >> i & 1) in_S[g.orig[i]] = 1;
  *value = fx_to_double(best, k);
  *second = sec >= 0 ? fx_to_double(sec, k) : -1.0;
  free(q);
  og_free(&g);
  return ORC_OK;
}
