// Host-only parts of libirls_mincut that touch no GPU: graph validation and
// set-up (merging, connectivity, the diagonal-format test), the exact
// fixed-point conversions of the sweep cut, the exact max-flow of the
// two-level rounding's coarse graph, and option checks.  Built into the
// library, and on its own (with the host sanitizers) for the CPU tests.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/irls_mincut.h"

namespace irls_host {

typedef __int128 i128;

constexpr int kMaxDiag = 8;          // most index offsets the diagonal format stores

// exact fixed point for cut values: the scale exponent k for capacities up
// to cmax summed over merged_edges edges; round-half-even(c 2^k); and a
// 128-bit fixed-point value rounded once to double
int fx_scale_of(double cmax, int64_t merged_edges);
i128 fx_round_host(double c, int k);
double fx_to_double(i128 v, int k);

struct HostGraph {
  int64_t n = 0, s = 0, t = 0, nt = 0;
  std::vector<int32_t> rowptr, col;
  std::vector<double> ccap, cs, ct, dcap;
  double cst = 0.0, cmax = 0.0;
  int64_t merged = 0, interior = 0;
  int32_t K = 0;
  int32_t off[kMaxDiag] = {0};
  bool dia_ok = false;
  int32_t fx_k = 0;
  i128 D0 = 0;
  bool no_source_edges = true;
};

inline int64_t nid_of(int64_t u, int64_t s, int64_t t) { return u - (u > s) - (u > t); }
inline int64_t orig_of(int64_t i, int64_t s, int64_t t) {
  int64_t lo = std::min(s, t), hi = std::max(s, t);
  if (i >= lo) i++;
  if (i >= hi) i++;
  return i;
}

struct UnionFind {
  std::vector<int64_t> p;
  explicit UnionFind(int64_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
  int64_t find(int64_t x) {
    while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
    return x;
  }
  void unite(int64_t a, int64_t b) {
    a = find(a); b = find(b);
    if (a != b) p[std::max(a, b)] = std::min(a, b);
  }
};

// Validates the edge list (ids, capacities, connectivity), merges parallel
// edges, drops self-loops and builds the CSR and, for grids, the diagonal
// format of the non-terminal rows.
irls_status build_host_graph(HostGraph &g, int64_t n, int64_t m, const int64_t *eu,
                             const int64_t *ev, const double *cap, int64_t s, int64_t t,
                             std::string &err);

struct FlowGraph {
  int64_t n = 0;
  std::vector<int64_t> first;     // [n+1] arcs of node v
  std::vector<int64_t> to, mate;  // [arcs]
  std::vector<i128> res;          // residual capacity
};

FlowGraph flow_graph(int64_t n, const std::vector<int64_t> &a, const std::vector<int64_t> &b,
                     const std::vector<i128> &c);
i128 max_flow(FlowGraph &F, int64_t s, int64_t t, std::vector<uint8_t> &source_side);
i128 coarse_min_cut(int64_t nc, const std::vector<int32_t> &eu, const std::vector<int32_t> &ev,
                    const std::vector<i128> &ecap, const std::vector<i128> &ws, const std::vector<i128> &wt,
                    i128 st, std::vector<uint8_t> &side);
double total_capacity2(const HostGraph &g);
irls_status check_options(const irls_options &o, std::string &err);

}  // namespace irls_host
