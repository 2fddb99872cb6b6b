/*
 * Oracle graph set-up: validation, merging, connectivity, non-terminal
 * numbering (test infrastructure only).
 *
 * Problem statement (Section 2): G = (V, E) undirected, c({u,v}) > 0,
 * distinguished s and t, G assumed connected.  Connectivity also makes every
 * reduced system nonsingular (Proposition 1).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "ograph.h"

typedef struct { int64_t a, b, idx; } erec;

static int cmp_erec(const void *x, const void *y) {
  const erec *p = (const erec *)x, *q = (const erec *)y;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  if (p->b != q->b) return p->b < q->b ? -1 : 1;
  return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

void og_free(ograph *g) {
  free(g->nid); free(g->orig); free(g->ea); free(g->eb); free(g->ec);
  free(g->cs); free(g->ct); free(g->rp); free(g->nb); free(g->nc);
  memset(g, 0, sizeof(*g));
}

int og_build(ograph *g, int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
             const double *cap, int64_t s, int64_t t) {
  memset(g, 0, sizeof(*g));
  if (m > 0 && (!eu || !ev || !cap)) return ORC_ERR_NULL;
  if (n < 2 || m < 0 || s < 0 || s >= n || t < 0 || t >= n || s == t) return ORC_ERR_RANGE;
  for (int64_t e = 0; e < m; e++) {
    if (eu[e] < 0 || eu[e] >= n || ev[e] < 0 || ev[e] >= n) return ORC_ERR_RANGE;
    if (!(cap[e] > 0.0) || !isfinite(cap[e])) return ORC_ERR_CAPACITY;
  }
  g->n = n; g->s = s; g->t = t;

  /* merge: sort (min, max, input index); sum each run left to right */
  erec *r = (erec *)malloc(sizeof(erec) * (size_t)(m > 0 ? m : 1));
  if (!r) return ORC_ERR_NOMEM;
  int64_t k = 0;
  for (int64_t e = 0; e < m; e++) {
    if (eu[e] == ev[e]) continue;                       /* self loop */
    r[k].a = eu[e] < ev[e] ? eu[e] : ev[e];
    r[k].b = eu[e] < ev[e] ? ev[e] : eu[e];
    r[k].idx = e;
    k++;
  }
  qsort(r, (size_t)k, sizeof(erec), cmp_erec);
  g->ea = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k ? k : 1));
  g->eb = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k ? k : 1));
  g->ec = (double *)malloc(sizeof(double) * (size_t)(k ? k : 1));
  if (!g->ea || !g->eb || !g->ec) { free(r); og_free(g); return ORC_ERR_NOMEM; }
  int64_t ne = 0;
  for (int64_t i = 0; i < k; i++) {
    if (ne > 0 && g->ea[ne - 1] == r[i].a && g->eb[ne - 1] == r[i].b) {
      g->ec[ne - 1] = g->ec[ne - 1] + cap[r[i].idx];
    } else {
      g->ea[ne] = r[i].a; g->eb[ne] = r[i].b; g->ec[ne] = cap[r[i].idx]; ne++;
    }
  }
  free(r);
  g->ne = ne;

  /* connectivity: depth-first search from s over the merged edges */
  int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t *adj = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * ne + 1));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  char *seen = (char *)calloc((size_t)n, 1);
  int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!deg || !adj || !fill || !seen || !stack) {
    free(deg); free(adj); free(fill); free(seen); free(stack); og_free(g); return ORC_ERR_NOMEM;
  }
  for (int64_t e = 0; e < ne; e++) { deg[g->ea[e] + 1]++; deg[g->eb[e] + 1]++; }
  for (int64_t v = 0; v < n; v++) deg[v + 1] += deg[v];
  memcpy(fill, deg, sizeof(int64_t) * (size_t)n);
  for (int64_t e = 0; e < ne; e++) { adj[fill[g->ea[e]]++] = g->eb[e]; adj[fill[g->eb[e]]++] = g->ea[e]; }
  int64_t top = 0, reached = 1;
  stack[top++] = s; seen[s] = 1;
  while (top > 0) {
    int64_t u = stack[--top];
    for (int64_t j = deg[u]; j < deg[u + 1]; j++) {
      int64_t v = adj[j];
      if (!seen[v]) { seen[v] = 1; reached++; stack[top++] = v; }
    }
  }
  free(deg); free(adj); free(fill); free(seen); free(stack);
  if (reached != n) { og_free(g); return ORC_ERR_DISCONNECTED; }

  /* non-terminal numbering in ascending node id */
  g->nt = n - 2;
  g->nid = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  g->orig = (int64_t *)malloc(sizeof(int64_t) * (size_t)(g->nt > 0 ? g->nt : 1));
  g->cs = (double *)calloc((size_t)(g->nt > 0 ? g->nt : 1), sizeof(double));
  g->ct = (double *)calloc((size_t)(g->nt > 0 ? g->nt : 1), sizeof(double));
  g->rp = (int64_t *)calloc((size_t)g->nt + 1, sizeof(int64_t));
  if (!g->nid || !g->orig || !g->cs || !g->ct || !g->rp) { og_free(g); return ORC_ERR_NOMEM; }
  int64_t c = 0;
  for (int64_t v = 0; v < n; v++) {
    if (v == s || v == t) { g->nid[v] = -1; continue; }
    g->nid[v] = c; g->orig[c] = v; c++;
  }

  /* classify merged edges: interior, s-edge, t-edge, s-t edge */
  g->cst = 0.0;
  int64_t ninterior = 0;
  for (int64_t e = 0; e < ne; e++) {
    int64_t a = g->ea[e], b = g->eb[e];
    int sa = (a == s) || (b == s), ta = (a == t) || (b == t);
    if (sa && ta) { g->cst = g->ec[e]; continue; }
    if (sa) { g->cs[g->nid[a == s ? b : a]] = g->ec[e]; continue; }
    if (ta) { g->ct[g->nid[a == t ? b : a]] = g->ec[e]; continue; }
    g->rp[g->nid[a] + 1]++; g->rp[g->nid[b] + 1]++; ninterior++;
  }
  for (int64_t i = 0; i < g->nt; i++) g->rp[i + 1] += g->rp[i];
  g->nb = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * ninterior + 1));
  g->nc = (double *)malloc(sizeof(double) * (size_t)(2 * ninterior + 1));
  int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(g->nt + 1));
  if (!g->nb || !g->nc || !pos) { free(pos); og_free(g); return ORC_ERR_NOMEM; }
  memcpy(pos, g->rp, sizeof(int64_t) * (size_t)g->nt);
  /* merged edges are sorted by (min id, max id): filling in that order gives
   * every row its neighbours in ascending order */
  for (int64_t pass = 0; pass < 2; pass++) {
    for (int64_t e = 0; e < ne; e++) {
      int64_t a = g->ea[e], b = g->eb[e];
      if (a == s || a == t || b == s || b == t) continue;
      int64_t ia = g->nid[a], ib = g->nid[b];
      /* pass 0: rows get their smaller neighbours (row = b), pass 1 the larger (row = a) */
      if (pass == 0) { g->nb[pos[ib]] = ia; g->nc[pos[ib]] = g->ec[e]; pos[ib]++; }
      else           { g->nb[pos[ia]] = ib; g->nc[pos[ia]] = g->ec[e]; pos[ia]++; }
    }
  }
  free(pos);
  return ORC_OK;
}
