/* Internal graph form of the oracle (test infrastructure only). */
#ifndef IRLS_ORACLE_GRAPH_H
#define IRLS_ORACLE_GRAPH_H
#include <stdint.h>
#include "oracle.h"

/* The graph after validation: merged undirected edges, the non-terminal
 * numbering (Section 2: the non-terminal graph is G minus s and t) and the
 * interior adjacency in CSR form over non-terminal indices. */
typedef struct {
  int64_t n, s, t;
  int64_t nt;          /* number of non-terminal nodes */
  int64_t *nid;        /* [n]  non-terminal index of a node, -1 for s and t */
  int64_t *orig;       /* [nt] node id of non-terminal i (ascending) */
  int64_t ne;          /* merged edges (self loops removed) */
  int64_t *ea, *eb;    /* [ne] endpoints, ea < eb */
  double  *ec;         /* [ne] merged capacity */
  double  *cs, *ct;    /* [nt] capacity to s / to t (0 if no such edge) */
  double   cst;        /* capacity of the s-t edge (0 if none) */
  int64_t *rp;         /* [nt+1] interior adjacency row pointers */
  int64_t *nb;         /* neighbour non-terminal index, ascending per row */
  double  *nc;         /* capacity of that interior edge */
} ograph;

int  og_build(ograph *g, int64_t n, int64_t m, const int64_t *eu, const int64_t *ev,
              const double *cap, int64_t s, int64_t t);
void og_free(ograph *g);

/* 128-bit fixed point used for exact cut values. */
typedef __int128 i128;
int     fx_scale(const ograph *g);                /* k: values are round(c * 2^k) */
i128    fx_quant(double c, int k);                /* round-half-even(c * 2^k) */
double  fx_to_double(i128 v, int k);              /* v * 2^-k, correctly rounded */
#endif
