// Host-only parts of libirls_mincut (see host_graph.h).
#include "host_graph.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <exception>
#include <limits>
#include <new>
#include <numeric>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

namespace irls_host {

// ----------------------------------------------------------------------------
// exact fixed point for cut values (host side of the sweep)
// ----------------------------------------------------------------------------
int fx_scale_of(double cmax, int64_t merged_edges) {
  int e2 = 0;
  if (cmax > 0.0) std::frexp(cmax, &e2);       // cmax = f 2^e2, f in [0.5, 1)
  int L = 0;
  while (L < 62 && ((int64_t)1 << L) < merged_edges + 1) L++;
  return 125 - e2 - L;                          // sum of all capacities < 2^125
}

i128 fx_round_host(double c, int k) {
  if (!(c > 0.0)) return 0;
  uint64_t bits;
  std::memcpy(&bits, &c, 8);
  int ef = (int)((bits >> 52) & 0x7FF);
  uint64_t mant = bits & ((1ull << 52) - 1);
  int e2;
  if (ef == 0) { e2 = -1074; } else { mant |= 1ull << 52; e2 = ef - 1075; }
  int sh = e2 + k;
  if (sh >= 0) return ((i128)mant) << sh;
  int r = -sh;
  if (r >= 64) return 0;
  uint64_t q = mant >> r, rem = mant & ((1ull << r) - 1), half = 1ull << (r - 1);
  if (rem > half || (rem == half && (q & 1ull))) q++;
  return (i128)q;
}

// round-to-nearest-even conversion of a 128-bit integer, then scaling by 2^-k
double fx_to_double(i128 v, int k) {
  bool neg = v < 0;
  unsigned __int128 a = neg ? (unsigned __int128)(-(v + 1)) + 1u : (unsigned __int128)v;
  if (a == 0) return 0.0;
  int msb = 127;
  while (!((a >> msb) & 1u)) msb--;
  double r;
  if (msb <= 52) {
    r = (double)(uint64_t)a;
  } else {
    int sh = msb - 52;
    unsigned __int128 mant = a >> sh;
    unsigned __int128 rem = a & ((((unsigned __int128)1) << sh) - 1u);
    unsigned __int128 half = ((unsigned __int128)1) << (sh - 1);
    if (rem > half || (rem == half && (mant & 1u))) mant++;
    if (mant >> 53) { mant >>= 1; sh++; }
    r = std::ldexp((double)(uint64_t)mant, sh);
  }
  r = std::ldexp(r, -k);
  return neg ? -r : r;
}

// ----------------------------------------------------------------------------
// host graph
// ----------------------------------------------------------------------------
irls_status build_host_graph(HostGraph &g, int64_t n, int64_t m, const int64_t *eu,
                             const int64_t *ev, const double *cap, int64_t s, int64_t t,
                             std::string &err) {
  if (m > 0 && (!eu || !ev || !cap)) { err = "edge arrays must not be NULL"; return IRLS_ERR_NULL; }
  if (n < 2 || m < 0 || s < 0 || s >= n || t < 0 || t >= n || s == t) {
    err = "need n >= 2, m >= 0, s and t distinct nodes in [0,n)";
    return IRLS_ERR_RANGE;
  }
  if (n - 2 >= (int64_t)INT32_MAX) { err = "too many nodes for 32-bit device indices"; return IRLS_ERR_RANGE; }
  g.n = n; g.s = s; g.t = t; g.nt = n - 2;
  const int64_t nt = g.nt;
  for (int64_t e = 0; e < m; e++) {
    if (eu[e] < 0 || eu[e] >= n || ev[e] < 0 || ev[e] >= n) {
      err = "edge " + std::to_string(e) + " has an endpoint outside [0,n)";
      return IRLS_ERR_RANGE;
    }
    if (!(cap[e] > 0.0) || !std::isfinite(cap[e])) {
      err = "edge " + std::to_string(e) + " has a capacity that is not finite and positive";
      return IRLS_ERR_CAPACITY;
    }
  }
  g.cs.assign(nt, 0.0);
  g.ct.assign(nt, 0.0);
  // terminal edges are merged per node by a left-to-right sum in input order;
  // interior edges are collected as (row a, row b), a < b
  std::vector<int32_t> ia, ib;
  std::vector<double> ic;
  ia.reserve(m); ib.reserve(m); ic.reserve(m);
  bool sorted = true;
  uint64_t last = 0;
  for (int64_t e = 0; e < m; e++) {
    int64_t u = eu[e], v = ev[e];
    if (u == v) continue;
    double c = cap[e];
    bool us = (u == s) || (v == s), ut = (u == t) || (v == t);
    if (us && ut) { g.cst += c; continue; }
    if (us) { g.cs[nid_of(u == s ? v : u, s, t)] += c; continue; }
    if (ut) { g.ct[nid_of(u == t ? v : u, s, t)] += c; continue; }
    int32_t a = (int32_t)nid_of(std::min(u, v), s, t), b = (int32_t)nid_of(std::max(u, v), s, t);
    uint64_t key = ((uint64_t)a << 32) | (uint32_t)b;
    if (!ia.empty() && key <= last) sorted = false;
    last = key;
    ia.push_back(a); ib.push_back(b); ic.push_back(c);
  }
  // merge parallel interior edges (stable by input order inside a key)
  if (!sorted) {
    std::vector<int64_t> idx(ia.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
      return ia[x] != ia[y] ? ia[x] < ia[y] : ib[x] < ib[y];
    });
    std::vector<int32_t> na, nb;
    std::vector<double> nc;
    na.reserve(idx.size()); nb.reserve(idx.size()); nc.reserve(idx.size());
    for (int64_t j : idx) {
      if (!na.empty() && na.back() == ia[j] && nb.back() == ib[j]) { nc.back() += ic[j]; continue; }
      na.push_back(ia[j]); nb.push_back(ib[j]); nc.push_back(ic[j]);
    }
    ia.swap(na); ib.swap(nb); ic.swap(nc);
  }
  const int64_t mi = (int64_t)ia.size();
  g.interior = mi;
  if (2 * mi >= (int64_t)INT32_MAX) { err = "too many edges for 32-bit device indices"; return IRLS_ERR_RANGE; }

  // connectivity (Proposition 1 needs G connected)
  {
    UnionFind uf(n);
    for (int64_t i = 0; i < nt; i++) {
      if (g.cs[i] > 0.0) uf.unite(orig_of(i, s, t), s);
      if (g.ct[i] > 0.0) uf.unite(orig_of(i, s, t), t);
    }
    if (g.cst > 0.0) uf.unite(s, t);
    for (int64_t e = 0; e < mi; e++) uf.unite(orig_of(ia[e], s, t), orig_of(ib[e], s, t));
    int64_t root = uf.find(s);
    for (int64_t u = 0; u < n; u++)
      if (uf.find(u) != root) { err = "graph is not connected"; return IRLS_ERR_DISCONNECTED; }
  }

  // CSR over non-terminal rows, columns ascending
  g.rowptr.assign(nt + 1, 0);
  for (int64_t e = 0; e < mi; e++) { g.rowptr[ia[e] + 1]++; g.rowptr[ib[e] + 1]++; }
  for (int64_t i = 0; i < nt; i++) g.rowptr[i + 1] += g.rowptr[i];
  g.col.resize(2 * mi);
  g.ccap.resize(2 * mi);
  {
    std::vector<int32_t> pos(g.rowptr.begin(), g.rowptr.end() - 1);
    for (int64_t e = 0; e < mi; e++) { int32_t r = ib[e]; g.col[pos[r]] = ia[e]; g.ccap[pos[r]++] = ic[e]; }
    for (int64_t e = 0; e < mi; e++) { int32_t r = ia[e]; g.col[pos[r]] = ib[e]; g.ccap[pos[r]++] = ic[e]; }
  }

  // diagonal format: few distinct offsets b - a and at least half of the slots used
  {
    int32_t offs[kMaxDiag + 1];
    int K = 0;
    bool ok = true;
    for (int64_t e = 0; e < mi && ok; e++) {
      int32_t d = ib[e] - ia[e];
      int k = 0;
      while (k < K && offs[k] != d) k++;
      if (k == K) {
        if (K == kMaxDiag) ok = false;
        else offs[K++] = d;
      }
    }
    if (ok && K > 0 && 2 * mi >= (int64_t)K * nt) {
      std::sort(offs, offs + K);
      g.K = K;
      for (int k = 0; k < K; k++) g.off[k] = offs[k];
      g.dia_ok = true;
    }
  }
  if (g.dia_ok) {
    g.dcap.assign((size_t)g.K * nt, 0.0);
    for (int64_t e = 0; e < mi; e++) {
      int32_t d = ib[e] - ia[e];
      int k = 0;
      while (g.off[k] != d) k++;
      g.dcap[(size_t)k * nt + ia[e]] = ic[e];
    }
  }

  // fixed-point scale of exact cut values and the cut of S_0 = {s}
  double cmax = g.cst;
  int64_t merged = mi + (g.cst > 0.0);
  for (int64_t e = 0; e < mi; e++) cmax = std::max(cmax, ic[e]);
  for (int64_t i = 0; i < nt; i++) {
    if (g.cs[i] > 0.0) { merged++; cmax = std::max(cmax, g.cs[i]); g.no_source_edges = false; }
    if (g.ct[i] > 0.0) { merged++; cmax = std::max(cmax, g.ct[i]); }
  }
  g.cmax = cmax;
  g.merged = merged;
  g.fx_k = fx_scale_of(cmax, merged);
  g.D0 = fx_round_host(g.cst, g.fx_k);
  for (int64_t i = 0; i < nt; i++) g.D0 += fx_round_host(g.cs[i], g.fx_k);
  return IRLS_OK;
}

// ----------------------------------------------------------------------------
// Exact maximum flow / minimum cut of an undirected graph with 128-bit
// integer capacities (the coarse graph of the two-level rounding): the first
// phase of push-relabel, which ends in a maximum preflow.  Active nodes are
// discharged highest label first; labels are reset to exact residual
// distances to t by a reverse breadth-first search at the start and after
// work proportional to the graph, and the gap heuristic lifts every node
// above an emptied label to n (such nodes cannot reach t).
// The returned source side is the set of nodes that cannot reach t in the
// residual graph of the preflow.  Nodes that reach t hold no excess at the
// end, so the preflow saturates every arc into that set and carries nothing
// out of it.  Returning the excess to s (the second phase) would only change
// arcs outside it, so it is also the set a maximum flow gives: the largest
// minimum-cut source side.
// ----------------------------------------------------------------------------

FlowGraph flow_graph(int64_t n, const std::vector<int64_t> &a, const std::vector<int64_t> &b,
                     const std::vector<i128> &c) {
  FlowGraph F;
  F.n = n;
  F.first.assign(n + 1, 0);
  for (size_t e = 0; e < a.size(); e++) { F.first[a[e] + 1]++; F.first[b[e] + 1]++; }
  for (int64_t v = 0; v < n; v++) F.first[v + 1] += F.first[v];
  const int64_t na = F.first[n];
  F.to.resize(na);
  F.mate.resize(na);
  F.res.resize(na);
  std::vector<int64_t> fill(F.first.begin(), F.first.end() - 1);
  for (size_t e = 0; e < a.size(); e++) {           // an undirected edge: two arcs of capacity c
    const int64_t x = fill[a[e]]++, y = fill[b[e]]++;
    F.to[x] = b[e]; F.res[x] = c[e]; F.mate[x] = y;
    F.to[y] = a[e]; F.res[y] = c[e]; F.mate[y] = x;
  }
  return F;
}

i128 max_flow(FlowGraph &F, int64_t s, int64_t t, std::vector<uint8_t> &source_side) {
  const int64_t n = F.n;
  std::vector<int64_t> d(n, n), cur(n), queue(n);
  std::vector<i128> ex(n, 0);
  std::vector<int64_t> anext(n, -1), ahead(n + 1, -1);               // active nodes by label
  std::vector<int64_t> lnext(n, -1), lprev(n, -1), lhead(n + 1, -1);  // all nodes by label (< n)
  int64_t amax = -1, lmax = -1;
  auto list_insert = [&](int64_t v) {
    const int64_t h = lhead[d[v]];
    lnext[v] = h;
    lprev[v] = -1;
    if (h >= 0) lprev[h] = v;
    lhead[d[v]] = v;
    lmax = std::max(lmax, d[v]);
  };
  auto list_remove = [&](int64_t v) {
    if (lprev[v] >= 0) lnext[lprev[v]] = lnext[v];
    else lhead[d[v]] = lnext[v];
    if (lnext[v] >= 0) lprev[lnext[v]] = lprev[v];
  };
  auto activate = [&](int64_t v) {
    anext[v] = ahead[d[v]];
    ahead[d[v]] = v;
    amax = std::max(amax, d[v]);
  };
  auto global_relabel = [&]() {
    std::fill(d.begin(), d.end(), n);
    std::fill(ahead.begin(), ahead.end(), -1);
    std::fill(lhead.begin(), lhead.end(), -1);
    amax = lmax = -1;
    int64_t qh = 0, qt = 0;
    d[t] = 0;
    queue[qt++] = t;
    while (qh < qt) {
      const int64_t y = queue[qh++];
      for (int64_t a = F.first[y]; a < F.first[y + 1]; a++) {
        const int64_t x = F.to[a];
        if (x != s && d[x] == n && F.res[F.mate[a]] > 0) { d[x] = d[y] + 1; queue[qt++] = x; }
      }
    }
    for (int64_t v = 0; v < n; v++) {
      if (v == s || v == t || d[v] >= n) continue;
      cur[v] = F.first[v];
      list_insert(v);
      if (ex[v] > 0) activate(v);
    }
  };
  for (int64_t a = F.first[s]; a < F.first[s + 1]; a++) {      // saturate every arc out of s
    const i128 c = F.res[a];
    if (c <= 0) continue;
    F.res[a] = 0;
    F.res[F.mate[a]] += c;
    ex[F.to[a]] += c;
  }
  global_relabel();
  int64_t work = 0;
  const int64_t work_limit = 6 * n + (int64_t)F.to.size();
  while (amax >= 0) {
    const int64_t v = ahead[amax];
    if (v < 0) { amax--; continue; }
    ahead[amax] = anext[v];
    if (d[v] != amax || ex[v] <= 0) continue;         // lifted by a gap after it was queued
    while (ex[v] > 0) {
      if (cur[v] == F.first[v + 1]) {                  // no admissible arc left: relabel
        const int64_t old = d[v];
        list_remove(v);
        if (lhead[old] < 0) {                          // gap at `old`
          for (int64_t L = old + 1; L <= lmax; L++) {
            for (int64_t x = lhead[L]; x >= 0; x = lnext[x]) d[x] = n;
            lhead[L] = -1;
          }
          lmax = old - 1;
          d[v] = n;
          break;
        }
        int64_t m = n;
        for (int64_t a = F.first[v]; a < F.first[v + 1]; a++)
          if (F.res[a] > 0) m = std::min(m, d[F.to[a]] + 1);
        work += 12 + (F.first[v + 1] - F.first[v]);
        d[v] = m;
        if (m >= n) break;
        cur[v] = F.first[v];
        list_insert(v);
        continue;
      }
      const int64_t a = cur[v], w = F.to[a];
      if (F.res[a] > 0 && d[w] == d[v] - 1) {          // push along an admissible arc
        const i128 delta = std::min(ex[v], F.res[a]);
        F.res[a] -= delta;
        F.res[F.mate[a]] += delta;
        ex[v] -= delta;
        if (w != t && ex[w] == 0) activate(w);
        ex[w] += delta;
      } else {
        cur[v]++;
      }
    }
    if (work > work_limit) {
      global_relabel();
      work = 0;
    }
  }
  // nodes that reach t through residual arcs form the sink side
  std::vector<uint8_t> reach(n, 0);
  int64_t qh = 0, qt = 0;
  reach[t] = 1;
  queue[qt++] = t;
  while (qh < qt) {
    const int64_t y = queue[qh++];
    for (int64_t a = F.first[y]; a < F.first[y + 1]; a++) {
      const int64_t x = F.to[a];
      if (!reach[x] && F.res[F.mate[a]] > 0) { reach[x] = 1; queue[qt++] = x; }
    }
  }
  source_side.assign(n, 0);
  for (int64_t v = 0; v < n; v++) source_side[v] = reach[v] ? 0 : 1;
  return ex[t];
}

// Minimum s_c-t_c cut of the coarse graph: nodes 0..nc-1 with capacity ws[u]
// to s_c = nc and wt[u] to t_c = nc + 1, edges (eu, ev, ecap) among them, and
// st between s_c and t_c.
//   * The flow along s_c - u - t_c (min(ws, wt) per node) and along s_c - t_c
//     is taken first, so each node keeps at most one terminal edge.  The arcs
//     into s_c and out of t_c this leaves out lie on no augmenting path.
//   * The rest splits into the connected components of the Sc-Sc edges:
//     they share only s_c and t_c, so each is a max-flow problem of its own
//     (a node reaching t_c through s_c would contradict maximality).  The
//     components run on host threads, largest first.
// Returns the flow (= the cut value) and the largest source side (nc + 2
// entries): the nodes that cannot reach t_c in the residual graph.
i128 coarse_min_cut(int64_t nc, const std::vector<int32_t> &eu, const std::vector<int32_t> &ev,
                    const std::vector<i128> &ecap, const std::vector<i128> &ws, const std::vector<i128> &wt,
                    i128 st, std::vector<uint8_t> &side) {
  i128 flow = st;
  std::vector<i128> rs(nc), rt(nc);
  for (int64_t u = 0; u < nc; u++) {
    const i128 d = std::min(ws[u], wt[u]);
    flow += d;
    rs[u] = ws[u] - d;
    rt[u] = wt[u] - d;
  }
  side.assign(nc + 2, 0);
  side[nc] = 1;
  if (nc == 0) return flow;
  UnionFind uf(nc);
  for (size_t e = 0; e < eu.size(); e++) uf.unite(eu[e], ev[e]);
  // components: dense ids, members in ascending order, edges grouped
  std::vector<int64_t> comp(nc), cstart, pos(nc);
  int64_t ncomp = 0;
  {
    std::vector<int64_t> id_of_root(nc, -1);
    for (int64_t u = 0; u < nc; u++) {
      const int64_t r = uf.find(u);
      if (id_of_root[r] < 0) id_of_root[r] = ncomp++;
      comp[u] = id_of_root[r];
    }
  }
  cstart.assign(ncomp + 1, 0);
  for (int64_t u = 0; u < nc; u++) cstart[comp[u] + 1]++;
  for (int64_t c = 0; c < ncomp; c++) cstart[c + 1] += cstart[c];
  std::vector<int64_t> members(nc), fillm(cstart.begin(), cstart.end() - 1);
  for (int64_t u = 0; u < nc; u++) { pos[u] = fillm[comp[u]] - cstart[comp[u]]; members[fillm[comp[u]]++] = u; }
  std::vector<int64_t> estart(ncomp + 1, 0), edges(eu.size());
  for (size_t e = 0; e < eu.size(); e++) estart[comp[eu[e]] + 1]++;
  for (int64_t c = 0; c < ncomp; c++) estart[c + 1] += estart[c];
  std::vector<int64_t> fille(estart.begin(), estart.end() - 1);
  for (size_t e = 0; e < eu.size(); e++) edges[fille[comp[eu[e]]]++] = (int64_t)e;
  std::vector<int64_t> order(ncomp);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    return cstart[x + 1] - cstart[x] > cstart[y + 1] - cstart[y];
  });
  auto solve = [&](int64_t c) -> i128 {
    const int64_t k = cstart[c + 1] - cstart[c];
    const int64_t *mem = members.data() + cstart[c];
    if (estart[c + 1] == estart[c]) {                 // a lone node: no path through it
      for (int64_t i = 0; i < k; i++) side[mem[i]] = rt[mem[i]] > 0 ? 0 : 1;
      return 0;
    }
    std::vector<int64_t> fa, fb;
    std::vector<i128> fc;
    for (int64_t q = estart[c]; q < estart[c + 1]; q++) {
      const int64_t e = edges[q];
      fa.push_back(pos[eu[e]]); fb.push_back(pos[ev[e]]); fc.push_back(ecap[e]);
    }
    for (int64_t i = 0; i < k; i++) {
      const int64_t u = mem[i];
      if (rs[u] > 0) { fa.push_back(k); fb.push_back(i); fc.push_back(rs[u]); }
      if (rt[u] > 0) { fa.push_back(i); fb.push_back(k + 1); fc.push_back(rt[u]); }
    }
    FlowGraph F = flow_graph(k + 2, fa, fb, fc);
    std::vector<uint8_t> ls;
    const i128 f = max_flow(F, k, k + 1, ls);
    for (int64_t i = 0; i < k; i++) side[mem[i]] = ls[i];
    return f;
  };
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nth = (int)std::min<int64_t>({(int64_t)std::min(hw, 16u), ncomp, nc / 4096 + 1});
  std::vector<i128> part(nth, 0);
  std::atomic<int64_t> next{0};
  // an exception in a worker (an allocation failure) stops the others from
  // taking more components and is rethrown here, after every thread joined
  std::vector<std::exception_ptr> errs(nth);
  auto worker = [&](int tid) {
    try {
      for (int64_t q; (q = next.fetch_add(1)) < ncomp;) part[tid] += solve(order[q]);
    } catch (...) {
      errs[tid] = std::current_exception();
      next.store(ncomp);
    }
  };
  std::vector<std::thread> pool;
  try {
    for (int tid = 1; tid < nth; tid++) pool.emplace_back(worker, tid);
  } catch (const std::system_error &) {
    // fewer threads than asked for: the running ones take the remaining work
  }
  worker(0);
  for (auto &th : pool) th.join();
  for (const std::exception_ptr &e : errs)
    if (e) std::rethrow_exception(e);
  for (const i128 f : part) flow += f;
  return flow;
}

// C = 2 * (sum of all merged capacities): interior edges are stored in both
// rows of the CSR, terminal edges once per node, and the s-t edge once.
double total_capacity2(const HostGraph &g) {
  double c = 0.0;
  for (double x : g.ccap) c += x;
  for (double x : g.cs) c += 2.0 * x;
  for (double x : g.ct) c += 2.0 * x;
  return c + 2.0 * g.cst;
}

irls_status check_options(const irls_options &o, std::string &err) {
  if (o.struct_size != (int32_t)sizeof(irls_options)) { err = "irls_options.struct_size mismatch"; return IRLS_ERR_OPTIONS; }
  if (o.rounds < 0 || o.weight_form < 0 || o.weight_form > 1 || o.init < 0 || o.init > 2 ||
      !(o.cg_rtol > 0.0) || o.cg_maxit < 1 || (o.rounds > 0 && !(o.eps0 > 0.0)) ||
      !(o.eps_factor > 0.0) || o.eps_factor > 1.0 || o.precision < 0 || o.precision > 1 ||
      o.refine_every < 0 || o.format < 0 || o.format > 2 || o.solver < 0 || o.solver > 2 ||
      o.chunk < 0 || (o.warm_start != 0 && o.warm_start != 1) ||
      (o.inputs_on_device != 0 && o.inputs_on_device != 1) || o.rows_per_wave < 0 ||
      o.rows_per_wave > 64 || (o.rows_per_wave & (o.rows_per_wave - 1)) != 0 || o.precond < 0 ||
      o.precond > 2 || o.block_size < 0 || o.block_size > 128 || (o.block_size & 1) != 0 ||
      (o.unscaled_cg != 0 && o.unscaled_cg != 1) || !(o.stop_gap >= 0.0) || !(o.stop_gap < 1.0)) {
    err = "an option is out of range";
    return IRLS_ERR_OPTIONS;
  }
  if (o.precision == 1 && o.solver == 2) { err = "the resident solver runs in FP64 only"; return IRLS_ERR_OPTIONS; }
  if (o.precond >= 1 && o.solver == 2) {
    err = "block-Jacobi runs on the multi-workgroup solver";
    return IRLS_ERR_OPTIONS;
  }
  if (o.precond == 1 && o.precision != 0) {
    err = "exact line blocks run in FP64";
    return IRLS_ERR_OPTIONS;
  }
  if (o.precond == 1 && o.format == 1) {
    err = "exact line blocks need the diagonal format";
    return IRLS_ERR_OPTIONS;
  }
  return IRLS_OK;
}


}  // namespace irls_host

extern "C" void irls_options_default(irls_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = (int32_t)sizeof(irls_options);
  o->rounds = 30;
  o->eps0 = 0.1;
  o->eps_factor = 0.5;
  o->weight_form = 0;
  o->init = 0;
  o->warm_start = 1;
  o->cg_rtol = 1e-10;
  o->cg_maxit = 100000;
  o->precision = 0;
  o->refine_every = 20;
  o->fp64_weights_below_eps = 1e-4;
  o->format = 0;
  o->solver = 0;
  o->chunk = 0;
  o->inputs_on_device = 0;
  o->rows_per_wave = 0;
  o->precond = 0;
  o->block_size = 0;
  o->unscaled_cg = 0;
  o->stop_gap = 0.0;
}
