// CPU sanitizer driver (test infrastructure).  Runs the library's host-only
// code (graph validation and set-up, the exact fixed-point conversions, the
// coarse max-flow of the two-level rounding, option checks) and the oracle on
// small seeded inputs, built with AddressSanitizer and
// UndefinedBehaviorSanitizer, and checks the max-flows against exhaustive
// search.  Exit status 0 when every check holds; the sanitizers abort on the
// first error they find.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_1501_03105_amd/csrc/host_graph.h"
extern "C" {
#include "../../oracle/oracle.h"
}

using namespace irls_host;

static uint64_t mix(uint64_t z) {                  // SplitMix64 finaliser
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double unif(uint64_t seed, uint64_t i) { return (mix(seed * 0x1000003ull + i) >> 11) * 0x1.0p-53; }

static int failures = 0;
#define CHECK(c, ...)                                \
  do {                                               \
    if (!(c)) {                                      \
      std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
      std::printf(__VA_ARGS__);                      \
      std::printf("\n");                             \
      failures++;                                    \
    }                                                \
  } while (0)

struct EdgeList {
  int64_t n = 0, s = 0, t = 0;
  std::vector<int64_t> u, v;
  std::vector<double> c;
};

// a connected random graph: a path through all nodes plus extra edges
static EdgeList random_graph(uint64_t seed, int64_t n, int extra) {
  EdgeList g;
  g.n = n;
  g.s = 0;
  g.t = n - 1;
  for (int64_t i = 0; i + 1 < n; i++) {
    g.u.push_back(i);
    g.v.push_back(i + 1);
    g.c.push_back(0.1 + unif(seed, 3 * i));
  }
  for (int k = 0; k < extra; k++) {
    g.u.push_back((int64_t)(unif(seed, 1000 + 2 * k) * n));
    g.v.push_back((int64_t)(unif(seed, 1001 + 2 * k) * n));     // self-loops and repeats allowed
    g.c.push_back(0.1 + unif(seed, 5000 + k));
  }
  return g;
}

// exhaustive minimum s-t cut in 128-bit fixed point
static i128 brute_min_cut(int64_t n, int64_t s, int64_t t, const std::vector<int64_t> &a,
                          const std::vector<int64_t> &b, const std::vector<i128> &c) {
  std::vector<int64_t> free_nodes;
  for (int64_t x = 0; x < n; x++)
    if (x != s && x != t) free_nodes.push_back(x);
  i128 best = -1;
  const int64_t k = (int64_t)free_nodes.size();
  std::vector<uint8_t> side(n);
  for (int64_t mask = 0; mask < ((int64_t)1 << k); mask++) {
    for (int64_t x = 0; x < n; x++) side[x] = 0;
    side[s] = 1;
    for (int64_t j = 0; j < k; j++) side[free_nodes[j]] = (mask >> j) & 1;
    i128 cut = 0;
    for (size_t e = 0; e < a.size(); e++)
      if (side[a[e]] != side[b[e]]) cut += c[e];
    if (best < 0 || cut < best) best = cut;
  }
  return best;
}

static void check_host_graph() {
  for (uint64_t seed = 1; seed <= 40; seed++) {
    EdgeList g = random_graph(seed, 6 + (int64_t)(seed % 9), (int)(seed % 17));
    HostGraph h;
    std::string err;
    const irls_status rc = build_host_graph(h, g.n, (int64_t)g.u.size(), g.u.data(), g.v.data(), g.c.data(),
                                            g.s, g.t, err);
    CHECK(rc == IRLS_OK, "build_host_graph seed %llu: %s", (unsigned long long)seed, err.c_str());
    CHECK(h.nt == g.n - 2, "row count");
    CHECK((int64_t)h.rowptr.size() == h.nt + 1 && h.rowptr[h.nt] == (int32_t)h.col.size(), "CSR shape");
    for (int64_t r = 0; r < h.nt; r++)
      for (int32_t e = h.rowptr[r]; e < h.rowptr[r + 1]; e++) {
        CHECK(h.col[e] >= 0 && h.col[e] < h.nt && h.col[e] != r, "column range");
        CHECK(e == h.rowptr[r] || h.col[e] > h.col[e - 1], "columns ascending and merged");
      }
  }
  // invalid inputs give their error codes, not a crash
  EdgeList g = random_graph(7, 8, 3);
  HostGraph h;
  std::string err;
  std::vector<double> bad = g.c;
  bad[2] = -1.0;
  CHECK(build_host_graph(h, g.n, (int64_t)g.u.size(), g.u.data(), g.v.data(), bad.data(), g.s, g.t, err) ==
            IRLS_ERR_CAPACITY, "negative capacity");
  bad[2] = NAN;
  CHECK(build_host_graph(h, g.n, (int64_t)g.u.size(), g.u.data(), g.v.data(), bad.data(), g.s, g.t, err) ==
            IRLS_ERR_CAPACITY, "NaN capacity");
  std::vector<int64_t> ids = g.v;
  ids[1] = g.n + 3;
  CHECK(build_host_graph(h, g.n, (int64_t)g.u.size(), g.u.data(), ids.data(), g.c.data(), g.s, g.t, err) ==
            IRLS_ERR_RANGE, "node id out of range");
  CHECK(build_host_graph(h, g.n, (int64_t)g.u.size(), g.u.data(), g.v.data(), g.c.data(), 2, 2, err) ==
            IRLS_ERR_RANGE, "s == t");
  CHECK(build_host_graph(h, g.n, (int64_t)g.u.size(), nullptr, g.v.data(), g.c.data(), g.s, g.t, err) ==
            IRLS_ERR_NULL, "NULL array");
  std::vector<int64_t> cu = {0, 2}, cv = {1, 3};
  std::vector<double> cc = {1.0, 1.0};
  CHECK(build_host_graph(h, 4, 2, cu.data(), cv.data(), cc.data(), 0, 3, err) == IRLS_ERR_DISCONNECTED,
        "disconnected graph");
  irls_options o;
  irls_options_default(&o);
  CHECK(check_options(o, err) == IRLS_OK, "default options");
  o.precond = 7;
  CHECK(check_options(o, err) == IRLS_ERR_OPTIONS, "precond out of range");
  // block-Jacobi: ILU(0) blocks also in the precision form (which blocks the
  // graph allows is decided at create); exact line blocks only in FP64;
  // neither on the resident solver
  irls_options_default(&o);
  o.precond = 2;
  o.precision = 1;
  CHECK(check_options(o, err) == IRLS_OK, "precision form with ILU(0) blocks");
  o.precond = 1;
  CHECK(check_options(o, err) == IRLS_ERR_OPTIONS, "precision form with exact line blocks");
  o.precision = 0;
  CHECK(check_options(o, err) == IRLS_OK, "exact line blocks in FP64");
  o.precond = 2;
  o.solver = 2;
  CHECK(check_options(o, err) == IRLS_ERR_OPTIONS, "block-Jacobi on the resident solver");
}

static void check_fixed_point() {
  for (uint64_t i = 0; i < 2000; i++) {
    const double c = std::ldexp(0.5 + unif(11, i), (int)(unif(12, i) * 40) - 20);
    const int k = fx_scale_of(1e6, 1000);
    const i128 q = fx_round_host(c, k);
    const double back = fx_to_double(q, k);
    CHECK(std::fabs(back - c) <= std::ldexp(1.0, -k), "fixed point round trip of %.17g", c);
  }
}

static void check_max_flow() {
  for (uint64_t seed = 1; seed <= 60; seed++) {
    const int64_t n = 4 + (int64_t)(seed % 9);
    std::vector<int64_t> a, b;
    std::vector<i128> c;
    for (int64_t i = 0; i + 1 < n; i++) {
      a.push_back(i);
      b.push_back(i + 1);
      c.push_back((i128)(1 + unif(seed, i) * 1000));
    }
    for (int k = 0; k < (int)(2 * n); k++) {
      const int64_t x = (int64_t)(unif(seed, 100 + 2 * k) * n), y = (int64_t)(unif(seed, 101 + 2 * k) * n);
      if (x == y) continue;
      a.push_back(x);
      b.push_back(y);
      c.push_back((i128)(1 + unif(seed, 300 + k) * 1000));
    }
    FlowGraph F = flow_graph(n, a, b, c);
    std::vector<uint8_t> side;
    const i128 f = max_flow(F, 0, n - 1, side);
    const i128 best = brute_min_cut(n, 0, n - 1, a, b, c);
    CHECK(f == best, "max_flow seed %llu", (unsigned long long)seed);
    i128 cut = 0;
    for (size_t e = 0; e < a.size(); e++)
      if (side[a[e]] != side[b[e]]) cut += c[e];
    CHECK(side[0] == 1 && side[n - 1] == 0 && cut == best, "max_flow side seed %llu", (unsigned long long)seed);
  }
  // the coarse graph form: nodes 0..nc-1 with terminal capacities to s_c, t_c
  for (uint64_t seed = 1; seed <= 40; seed++) {
    const int64_t nc = 2 + (int64_t)(seed % 8);
    std::vector<int32_t> eu, ev;
    std::vector<i128> ecap, ws(nc), wt(nc);
    for (int64_t u = 0; u < nc; u++) {
      ws[u] = (i128)(unif(seed, 700 + u) * 50);
      wt[u] = (i128)(unif(seed, 800 + u) * 50);
    }
    for (int k = 0; k < (int)(nc + seed % 5); k++) {
      const int32_t x = (int32_t)(unif(seed, 900 + 2 * k) * nc), y = (int32_t)(unif(seed, 901 + 2 * k) * nc);
      if (x == y) continue;
      eu.push_back(x);
      ev.push_back(y);
      ecap.push_back((i128)(1 + unif(seed, 950 + k) * 30));
    }
    const i128 st = (i128)(unif(seed, 999) * 10);
    std::vector<uint8_t> side;
    const i128 f = coarse_min_cut(nc, eu, ev, ecap, ws, wt, st, side);
    std::vector<int64_t> a, b;
    std::vector<i128> c;
    for (size_t e = 0; e < eu.size(); e++) { a.push_back(eu[e]); b.push_back(ev[e]); c.push_back(ecap[e]); }
    for (int64_t u = 0; u < nc; u++) {
      a.push_back(nc); b.push_back(u); c.push_back(ws[u]);
      a.push_back(u); b.push_back(nc + 1); c.push_back(wt[u]);
    }
    a.push_back(nc); b.push_back(nc + 1); c.push_back(st);
    CHECK(f == brute_min_cut(nc + 2, nc, nc + 1, a, b, c), "coarse_min_cut seed %llu", (unsigned long long)seed);
  }
}

static void check_oracle() {
  for (uint64_t seed = 1; seed <= 12; seed++) {
    EdgeList g = random_graph(100 + seed, 10 + (int64_t)(seed % 7), 12);
    const int64_t m = (int64_t)g.u.size();
    orc_options o;
    orc_options_default(&o);
    o.rounds = 8;
    o.cg_rtol = 1e-10;
    o.precond = (int32_t)(seed % 3);
    o.block_size = 3;
    std::vector<double> x(g.n);
    std::vector<orc_round> R(o.rounds + 1);
    int rc = orc_irls(g.n, m, g.u.data(), g.v.data(), g.c.data(), g.s, g.t, &o, nullptr, x.data(), R.data());
    CHECK(rc == 0 || rc == 100, "orc_irls seed %llu: %d", (unsigned long long)seed, rc);
    std::vector<uint8_t> in_s(g.n), in_b(g.n), in_f(g.n);
    double val = 0, mu = 0, mu2 = 0, second = 0;
    int64_t ks = 0;
    int32_t sc = 0;
    CHECK(orc_sweep(g.n, m, g.u.data(), g.v.data(), g.c.data(), g.s, g.t, x.data(), in_s.data(), &val, &ks, &sc) == 0,
          "orc_sweep");
    CHECK(orc_bruteforce(g.n, m, g.u.data(), g.v.data(), g.c.data(), g.s, g.t, in_b.data(), &mu, &second) == 0,
          "orc_bruteforce");
    CHECK(orc_maxflow(g.n, m, g.u.data(), g.v.data(), g.c.data(), g.s, g.t, in_f.data(), &mu2) == 0, "orc_maxflow");
    CHECK(mu == mu2 && val >= mu, "cut values seed %llu: sweep %.17g, brute %.17g, maxflow %.17g",
          (unsigned long long)seed, val, mu, mu2);
    std::vector<int64_t> blk(g.n);
    for (int64_t u = 0; u < g.n; u++) blk[u] = u % 3;
    std::vector<double> r(g.n - 2), z(g.n - 2);
    for (int64_t i = 0; i < g.n - 2; i++) r[i] = unif(seed, 4000 + i);
    for (int kind = 1; kind <= 2; kind++)
      CHECK(orc_block_apply(g.n, m, g.u.data(), g.v.data(), g.c.data(), g.s, g.t, x.data(), 1e-3, 0, kind, 1,
                            blk.data(), r.data(), z.data()) == 0, "orc_block_apply");
  }
}

int main() {
  check_host_graph();
  check_fixed_point();
  check_max_flow();
  check_oracle();
  std::printf("sanitizer driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
