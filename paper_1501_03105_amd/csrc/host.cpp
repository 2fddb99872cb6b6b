// Host side of libirls_mincut: the C ABI, argument validation, graph set-up
// (merging, connectivity, storage format), the IRLS round driver, the
// sweep-cut driver and the two-level rounding driver.  All arithmetic of the
// method runs in the HIP kernels, except the exact minimum cut of the small
// coarse graph of the two-level rounding (a max-flow, below).
#include <hip/hip_runtime.h>

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

#include "host_graph.h"
#include "internal.h"

using namespace irls;
using namespace irls_host;

namespace {

thread_local std::string g_thread_error;

// workgroups of the streaming kernels: a multiple of the 8 XCDs (see slab_rows)
int grid_for(int64_t rows) {
  int64_t g = (rows + kBlock - 1) / kBlock;
  g = (g + 7) / 8 * 8;
  if (g > kMaxGrid) g = kMaxGrid;
  return g < 8 ? 8 : (int)g;
}

constexpr int64_t kResidentMaxRows = 32768;

// SpMV lanes per row: the power of two at or above the mean row length
int lanes_for(int64_t rows, int64_t nnz) {
  double avg = rows > 0 ? (double)nnz / (double)rows : 1.0;
  int L = 1;
  while (L < 64 && L < avg) L <<= 1;
  return L;
}

// Heavy rows of one graph for the resident solver (rows with more than
// kHeavyRow entries, cut into kChunk-entry chunks), appended to the lists of a
// batch; also the lane count for the remaining (light) rows.
struct HeavyLists {
  std::vector<int32_t> crow, cbeg, cend, hrow, hc0, hc1;
  std::vector<int32_t> brow, bbeg, bend;          // light rows by bin, nt slots per graph
};

void add_heavy_rows(const std::vector<int32_t> &rowptr, int64_t nt, HeavyLists &H, BatchGraph &B) {
  B.chunk0 = (int64_t)H.crow.size();
  B.heavy0 = (int64_t)H.hrow.size();
  B.nnz = rowptr[nt];
  int32_t nchunks = 0, nheavy = 0;
  int64_t light_rows = 0, light_nnz = 0;
  // light rows by bin (stable within a bin), padded to nt slots per graph
  std::vector<int32_t> cnt(kBins + 1, 0);
  auto bin_of = [](int32_t d) {
    int b = 0;
    while (b < kBins - 1 && d > (2 << b)) b++;
    return b;
  };
  for (int64_t i = 0; i < nt; i++) {
    const int32_t d = rowptr[i + 1] - rowptr[i];
    if (d <= kHeavyRow) cnt[bin_of(d) + 1]++;
  }
  for (int b = 0; b < kBins; b++) cnt[b + 1] += cnt[b];
  for (int b = 0; b <= kBins; b++) B.bin[b] = cnt[b];
  const size_t base = H.brow.size();
  H.brow.resize(base + nt, 0);
  H.bbeg.resize(base + nt, 0);
  H.bend.resize(base + nt, 0);
  for (int64_t i = 0; i < nt; i++) {
    const int32_t d = rowptr[i + 1] - rowptr[i];
    if (d > kHeavyRow) continue;
    const int32_t j = cnt[bin_of(d)]++;
    H.brow[base + j] = (int32_t)i;
    H.bbeg[base + j] = rowptr[i];
    H.bend[base + j] = rowptr[i + 1];
  }
  for (int64_t i = 0; i < nt; i++) {
    const int32_t e0 = rowptr[i], e1 = rowptr[i + 1];
    if (e1 - e0 <= kHeavyRow) {
      light_rows++;
      light_nnz += e1 - e0;
      continue;
    }
    H.hrow.push_back((int32_t)i);
    H.hc0.push_back(nchunks);
    for (int32_t e = e0; e < e1; e += kChunk) {
      H.crow.push_back((int32_t)i);
      H.cbeg.push_back(e);
      H.cend.push_back(std::min(e + kChunk, e1));
      nchunks++;
    }
    H.hc1.push_back(nchunks);
    nheavy++;
  }
  B.nchunks = nchunks;
  B.nheavy = nheavy;
  B.lanes = lanes_for(light_rows, light_nnz);
}

}  // namespace

// ----------------------------------------------------------------------------
// handle
// ----------------------------------------------------------------------------
struct irls_mincut_s {
  irls_options opt;
  hipStream_t stream = nullptr;
  std::string err;
  bool solved = false;
  // Cheeger-type bracket: C = 2 * (total capacity), and the round-0 energy
  // E01 of the last solve whose round 0 used W = C
  double ctot = 0.0, e01 = 0.0;
  bool e01_valid = false;
  bool batch = false;
  GraphDev g;
  i128 D0 = 0;
  int solver = 1;
  int rpw = 8;
  int grid = 1;
  int32_t march_bs = 0, march_ty = 0;   // marching SpMV tile request (0, 0: the default)
  // FP64 state (both precisions)
  double *v = nullptr, *b = nullptr, *gt = nullptr;
  double *w64 = nullptr, *D64 = nullptr;
  // working-precision state (double for precision 0, float for 1)
  void *w = nullptr, *D = nullptr, *r = nullptr, *q = nullptr, *p0 = nullptr, *p1 = nullptr;
  void *wh = nullptr;               // scaled conductances (scaled form only)
  float *Dn = nullptr;              // FP64 scaled form: D in FP32 for the stopping norm
  double *wh64 = nullptr;           // their FP64 values (precision 1, scaled form)
  bool scaled = false;              // CG on D^-1/2 L~ D^-1/2 (Jacobi as symmetric scaling)
  double *partials = nullptr;
  double *vsave = nullptr;         // potentials saved across kernel timing
  Scalars *sc = nullptr, *sc_bench = nullptr;
  irls_round_stats *dstats = nullptr;
  int64_t stats_cap = 0;            // records dstats holds
  int64_t last_iters = 0;           // CG iterations of the last round solved (chunk sizing)
  int32_t bj_block = 0;             // block-Jacobi rows per block (0: Jacobi)
  int32_t bj_kind = 0, bj_tile = 0; // 1 line blocks (exact), 2 ILU(0) of cubic tiles,
                                    // 3 ILU(0) of CSR blocks of a breadth-first ordering
  int64_t nblk = 0;
  int32_t *blk_ptr = nullptr, *blk_rows = nullptr, *row_blk = nullptr;
  double *ilu_f = nullptr;
  void *bj_r = nullptr, *bj_im = nullptr;     // working precision (CGArgs::rbuf, bj_im)
  double *bj_f = nullptr, *bj_g = nullptr;
  // resident solver: heavy-row chunks (device) and the single graph's record
  int32_t *hv_crow = nullptr, *hv_cbeg = nullptr, *hv_cend = nullptr;
  int32_t *hv_hrow = nullptr, *hv_hc0 = nullptr, *hv_hc1 = nullptr;
  int32_t *hv_brow = nullptr, *hv_bbeg = nullptr, *hv_bend = nullptr;
  double *hv_part = nullptr;
  // multi-workgroup CSR SpMV: heavy rows cut into chunks (CGArgs::csr_*)
  int32_t csr_nheavy = 0, csr_nchunks = 0;
  int32_t *csr_hfirst = nullptr, *csr_cbeg = nullptr, *csr_cend = nullptr;
  double *csr_cpart = nullptr;
  BatchGraph res_graph;             // single-graph handles with solver 2
  uint32_t lane_code = kDefaultLaneCode;   // resident solver: lanes per light row by bin
  Scalars *pinned = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // resident solver (one graph, or every graph of a batch)
  int32_t G = 1;
  BatchGraph *rgraphs = nullptr;
  int32_t *rorder = nullptr;
  unsigned *rnext = nullptr;
  int grid_res = 1;
  // batch
  std::vector<BatchGraph> hgraphs;
  std::vector<i128> D0s;
  uint32_t *gid = nullptr;
  int64_t nodes_total = 0;
  SweepBatchBufs swb;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  SweepBufs sw;
  TwoLevelBufs tl;
  std::vector<void *> allocs;
  // in-solve timing of one CG kernel (irls_mincut_set_kernel_timing): an
  // event pair around each of its launches; per round, the first pair and the
  // round's converged iteration count, resolved after the solve
  int32_t prof_which = -1;
  int32_t prof_every = 1;           // time launches 0, every, 2*every, ... of each round
  std::vector<hipEvent_t> prof_ev;
  size_t prof_used = 0;
  struct ProfRound { size_t pair0, pair1; int64_t iters; };   // pair p times iteration (p - pair0) * every
  std::vector<ProfRound> prof_rounds;
  double prof_ms_work = 0.0, prof_ms_all = 0.0;
  int64_t prof_n_work = 0, prof_n_all = 0;

  template <typename T>
  hipError_t dalloc(T **p, size_t count) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    allocs.push_back(q);
    *p = (T *)q;
    return hipSuccess;
  }
  void release() {
    for (void *p : allocs) (void)hipFree(p);
    allocs.clear();
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    for (auto &e : ev) if (e) (void)hipEventDestroy(e);
    for (auto &e : prof_ev) (void)hipEventDestroy(e);
    prof_ev.clear();
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    gexec = nullptr;
    cap_stream = nullptr;
  }
};

namespace {

irls_status dev_fail(irls_mincut_t h, hipError_t e, const char *what) {
  h->err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? IRLS_ERR_OOM : IRLS_ERR_DEVICE;
}

#define HIPCHK(h, expr, what)                          \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return dev_fail(h, e_, what); \
  } while (0)

template <typename T>
CGArgs<T> make_args(irls_mincut_t h) {
  CGArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.nt = h->g.nt;
  a.rowptr = h->g.rowptr;
  a.col = h->g.col;
  a.ccap = h->g.ccap;
  a.K = h->g.format == 2 ? h->g.K : 0;
  for (int k = 0; k < kMaxDiag; k++) a.off[k] = h->g.off[k];
  a.dcap = h->g.dcap;
  a.cs = h->g.cs;
  a.ct = h->g.ct;
  a.w = (T *)h->w;
  a.D = (T *)h->D;
  a.w64 = h->w64;
  a.D64 = h->D64;
  a.b = h->b;
  a.gt = h->gt;
  a.v = h->v;
  a.z = (T *)h->r;
  a.q = (T *)h->q;
  a.p0 = (T *)h->p0;
  a.p1 = (T *)h->p1;
  a.partials = h->partials;
  a.sc = h->sc;
  a.form = h->opt.weight_form;
  a.cst = h->g.cst;
  a.rtol = h->opt.cg_rtol;
  a.weights_fp64 = 1;
  a.grid_main = h->grid;
  a.csr_lanes = h->rpw > 0 ? 64 / h->rpw : 64;
  a.march_bs = h->march_bs;
  a.march_ty = h->march_ty;
  a.csr_nheavy = h->csr_nheavy;
  a.csr_nchunks = h->csr_nchunks;
  a.csr_hfirst = h->csr_hfirst;
  a.csr_cbeg = h->csr_cbeg;
  a.csr_cend = h->csr_cend;
  a.csr_cpart = h->csr_cpart;
  spmv_layout(a, h->grid);
  a.bj_block = h->bj_block;
  a.bj_kind = h->bj_kind;
  a.bj_tile = h->bj_tile;
  a.nblk = h->nblk;
  a.blk_ptr = h->blk_ptr;
  a.blk_rows = h->blk_rows;
  a.row_blk = h->row_blk;
  a.ilu_f = h->ilu_f;
  a.rbuf = (T *)h->bj_r;
  a.bj_f = h->bj_f;
  a.bj_im = (T *)h->bj_im;
  a.bj_g = h->bj_g;
  a.wh = (T *)h->wh;
  a.wh64 = h->wh64;
  a.Dn = sizeof(T) == 4 ? (float *)h->D : h->Dn;
  a.scaled = h->scaled ? 1 : 0;
  return a;
}

// CG iterations first .. first + count - 1 of this round (the kernels learn
// the true iteration from the scalar block; the index only steers loads that
// are issued before they read it)
// The next event pair of the in-solve kernel timing (created on first use,
// reused by later solves).
hipError_t prof_pair(irls_mincut_t h, hipEvent_t *e0, hipEvent_t *e1) {
  while (h->prof_ev.size() < 2 * (h->prof_used + 1)) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    h->prof_ev.push_back(e);
  }
  *e0 = h->prof_ev[2 * h->prof_used];
  *e1 = h->prof_ev[2 * h->prof_used + 1];
  h->prof_used++;
  return hipSuccess;
}

// Launch one CG kernel (iteration `it` of the round), bracketed by an event
// pair when it is the kernel timed and `it` is a sampled iteration.
template <typename F>
hipError_t timed_launch(irls_mincut_t h, int which, int64_t it, F &&launch) {
  if (h->prof_which != which || it % h->prof_every != 0) return launch();
  hipEvent_t e0, e1;
  hipError_t e = prof_pair(h, &e0, &e1);
  if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
  return e;
}

template <typename T>
hipError_t launch_iterations(irls_mincut_t h, const CGArgs<T> &a0, int64_t first, int64_t count) {
  hipError_t e = hipSuccess;
  CGArgs<T> a = a0;
  for (int64_t i = 0; i < count && e == hipSuccess; i++) {
    a.it_hint = first + i;
    if (a.K == 0) e = launch_direction(a, h->grid, h->stream);
    if (e == hipSuccess)
      e = timed_launch(h, 0, a.it_hint, [&] { return launch_spmv(a, h->grid, h->rpw, a.K > 0, h->stream); });
    if (e == hipSuccess) e = timed_launch(h, 1, a.it_hint, [&] { return launch_update(a, h->grid, h->stream); });
    if (e == hipSuccess && a.bj_block > 0 && !bj_update_fused(a))
      e = timed_launch(h, 3, a.it_hint, [&] { return launch_bj_apply(a, h->grid, kPUpd, h->stream); });
    if (e == hipSuccess && h->opt.precision == 1)
      e = timed_launch(h, 2, a.it_hint, [&] { return launch_replace_residual(a, h->grid, h->stream); });
  }
  return e;
}

// After a solve has synchronised: add the timed launches of its rounds to the
// totals.  Launch i of a round did work when i < the round's CG iterations
// (launch `iters` finds CG stopped and returns; later ones too).  The pairs of
// a round time its launches 0, every, 2 * every, ... in order.
irls_status prof_resolve(irls_mincut_t h) {
  for (const auto &r : h->prof_rounds) {
    for (size_t p = r.pair0; p < r.pair1; p++) {
      float ms = 0.0f;
      HIPCHK(h, hipEventElapsedTime(&ms, h->prof_ev[2 * p], h->prof_ev[2 * p + 1]), "kernel timing");
      const bool work = (int64_t)(p - r.pair0) * h->prof_every < r.iters;
      h->prof_ms_all += ms;
      h->prof_n_all++;
      if (work) {
        h->prof_ms_work += ms;
        h->prof_n_work++;
      }
    }
  }
  h->prof_rounds.clear();
  h->prof_used = 0;
  return IRLS_OK;
}

// Run CG iterations in chunks until the device reports done.  The next chunk
// is queued before the previous chunk's state is read back, so the GPU never
// waits for the host; iterations queued after convergence return at once.
template <typename T>
irls_status run_cg(irls_mincut_t h, const CGArgs<T> &a, int64_t pred, int64_t *iters, int *status) {
  // the stopping test of iteration i runs at the start of iteration i + 1, so
  // cg_maxit iterations need cg_maxit + 1 direction launches
  const int64_t maxit = h->opt.cg_maxit + 1;
  // first chunk: the previous round's count (counts rarely fall between
  // rounds); then chunks of 8, so at most two chunks run past convergence.
  // A launch past convergence still issues its first loads, so the chunks
  // stay short; 8 iterations (hundreds of microseconds on large systems)
  // outlast the host's read-back and relaunch.
  int64_t first = pred > 0 ? std::max<int64_t>(8, pred) : 16;
  int64_t next = 8;
  if (h->opt.chunk > 0) first = next = h->opt.chunk;
  first = std::min(first, maxit);
  const size_t pair0 = h->prof_used;
  HIPCHK(h, launch_iterations(h, a, 0, first), "CG launch");
  HIPCHK(h, hipMemcpyAsync(&h->pinned[0], h->sc, sizeof(Scalars), hipMemcpyDeviceToHost, h->stream), "readback");
  HIPCHK(h, hipEventRecord(h->ev[0], h->stream), "event");
  int64_t launched = first;
  int slot = 0;
  for (;;) {
    bool queued = false;
    if (launched < maxit) {
      int64_t c = std::min(next, maxit - launched);
      HIPCHK(h, launch_iterations(h, a, launched, c), "CG launch");
      HIPCHK(h, hipMemcpyAsync(&h->pinned[1 - slot], h->sc, sizeof(Scalars), hipMemcpyDeviceToHost, h->stream), "readback");
      HIPCHK(h, hipEventRecord(h->ev[1 - slot], h->stream), "event");
      launched += c;
      queued = true;
    }
    HIPCHK(h, hipEventSynchronize(h->ev[slot]), "sync");
    if (h->pinned[slot].done) break;
    if (!queued) {
      HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
      slot = 1 - slot;
      if (!h->pinned[slot].done) { h->err = "CG did not stop at cg_maxit"; return IRLS_ERR_DEVICE; }
      break;
    }
    slot = 1 - slot;
  }
  *iters = h->pinned[slot].iter_b;
  *status = h->pinned[slot].status;
  if (h->prof_which >= 0) h->prof_rounds.push_back({pair0, h->prof_used, *iters});
  return IRLS_OK;
}

irls_status load_x0(irls_mincut_t h, const double *x0) {
  const int64_t n = h->g.n, nt = h->g.nt;
  std::vector<double> xh;
  const double *src = x0;
  if (h->opt.inputs_on_device) {
    xh.resize(n);
    HIPCHK(h, hipMemcpy(xh.data(), x0, n * sizeof(double), hipMemcpyDeviceToHost), "x0 copy");
    src = xh.data();
  }
  std::vector<double> vn(nt);
  for (int64_t i = 0; i < nt; i++) {
    vn[i] = src[orig_of(i, h->g.s, h->g.t)];
    if (!std::isfinite(vn[i])) { h->err = "x0 has a non-finite entry"; return IRLS_ERR_RANGE; }
  }
  if (nt > 0)
    HIPCHK(h, hipMemcpyAsync(h->v, vn.data(), nt * sizeof(double), hipMemcpyHostToDevice, h->stream), "x0 upload");
  HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
  return IRLS_OK;
}

template <typename T>
irls_status solve_multi(irls_mincut_t h, irls_round_stats *stats) {
  const irls_options &o = h->opt;
  const int64_t nt = h->g.nt;
  CGArgs<T> a = make_args<T>(h);
  const bool fp64 = sizeof(T) == 8;
  // chunk sizing: a continuation starts near the last round's CG count
  int64_t pred = o.init == 2 ? h->last_iters : 0;
  h->prof_rounds.clear();                          // pairs of a failed earlier solve are dropped
  h->prof_used = 0;
  double eps = o.eps0;
  irls_status result = IRLS_OK;
  for (int l = 0; l <= o.rounds; l++) {
    a.round0 = l == 0;
    a.eps = l == 0 ? 0.0 : eps;
    a.eps_next = l == 0 ? o.eps0 : eps * o.eps_factor;
    a.warm = (l > 0 && o.warm_start) ? 1 : 0;
    a.weights_fp64 = (fp64 || a.eps < o.fp64_weights_below_eps) ? 1 : 0;
    a.stat = h->dstats + l;
    const int32_t refine = o.refine_every > 0 ? o.refine_every : INT32_MAX;
    HIPCHK(h, launch_scalars_reset(h->sc, o.cg_maxit, fp64 ? 0 : refine, h->stream), "reset");
    if (nt > 0) HIPCHK(h, launch_assemble(a, h->grid, h->stream), "assemble");
    if (nt > 0 && a.bj_block > 0) HIPCHK(h, launch_bj_factor(a, h->grid, h->stream), "block-Jacobi factors");
    if (nt > 0 && a.scaled) HIPCHK(h, launch_scale_w(a, h->grid, h->stream), "scaling");
    bool solve = !(l == 0 && o.init != 0) && nt > 0;
    if (solve && h->g.no_source_edges) {
      HIPCHK(h, launch_fill(h->v, nt, 0.0, h->stream), "fill");
      solve = false;
    }
    if (solve) {
      HIPCHK(h, launch_cginit(a, h->grid, h->stream), "cg init");
      if (a.bj_block > 0) HIPCHK(h, launch_bj_apply(a, h->grid, kPInit, h->stream), "block-Jacobi apply");
      if (a.scaled) HIPCHK(h, launch_scale_v(a, +1, h->grid, h->stream), "scaling");
      int64_t it = 0;
      int st = IRLS_OK;
      irls_status rc = run_cg(h, a, pred, &it, &st);
      if (rc != IRLS_OK) return rc;
      if (a.scaled) HIPCHK(h, launch_scale_v(a, -1, h->grid, h->stream), "scaling");
      else if (bj_update_fused(a)) HIPCHK(h, launch_flush_v(a, h->grid, h->stream), "pending step");
      pred = it;
      h->last_iters = it;
      if (st == IRLS_ERR_DEVICE) {
        h->err = "CG kernels out of step with the host's iteration count in round " + std::to_string(l);
        return IRLS_ERR_DEVICE;
      }
      if (st == IRLS_ERR_CG_BREAKDOWN) {
        h->err = "CG breakdown in round " + std::to_string(l);
        result = IRLS_ERR_CG_BREAKDOWN;
      } else if (st == IRLS_WARN_CG_MAXIT && result == IRLS_OK) {
        result = IRLS_WARN_CG_MAXIT;
      }
    }
    if (nt > 0) HIPCHK(h, launch_stats(a, h->grid, h->stream), "stats");
    if (result == IRLS_ERR_CG_BREAKDOWN) break;
    if (o.stop_gap > 0.0 && nt > 0) {
      // the certified gap of this round: ||CBx||_1 - lower bound (both bound
      // the minimum cut); the records of rounds not run are cleared
      irls_round_stats r;
      HIPCHK(h, hipMemcpyAsync(&r, h->dstats + l, sizeof(r), hipMemcpyDeviceToHost, h->stream), "stats read");
      HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
      if (r.l1 - r.lower_bound <= o.stop_gap * r.l1) {
        if (l < o.rounds)
          HIPCHK(h, hipMemsetAsync(h->dstats + l + 1, 0, (size_t)(o.rounds - l) * sizeof(irls_round_stats),
                                   h->stream), "clear");
        break;
      }
    }
    if (l >= 1) eps *= o.eps_factor;
  }
  if (stats)
    HIPCHK(h, hipMemcpyAsync(stats, h->dstats, (o.rounds + 1) * sizeof(irls_round_stats),
                             hipMemcpyDeviceToHost, h->stream), "stats copy");
  HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
  if (h->prof_which >= 0) {
    irls_status pr = prof_resolve(h);
    if (pr != IRLS_OK) return pr;
  }
  return result;
}

ResidentArgs resident_args(irls_mincut_t h) {
  const irls_options &o = h->opt;
  ResidentArgs a;
  std::memset(&a, 0, sizeof(a));
  a.G = h->G;
  a.graphs = h->rgraphs;
  a.rowptr = h->g.rowptr;
  a.col = h->g.col;
  a.ccap = h->g.ccap;
  a.cs = h->g.cs;
  a.ct = h->g.ct;
  a.w = (double *)h->w;
  a.D = (double *)h->D;
  a.b = h->b;
  a.gt = h->gt;
  a.v = h->v;
  a.r = (double *)h->r;
  a.p = (double *)h->p0;
  a.q = (double *)h->q;
  a.stats = h->dstats;
  a.next_graph = h->rnext;
  a.order = h->rorder;
  a.chunk_row = h->hv_crow;
  a.chunk_beg = h->hv_cbeg;
  a.chunk_end = h->hv_cend;
  a.heavy_row = h->hv_hrow;
  a.heavy_c0 = h->hv_hc0;
  a.heavy_c1 = h->hv_hc1;
  a.chunk_part = h->hv_part;
  a.bin_row = h->hv_brow;
  a.bin_beg = h->hv_bbeg;
  a.bin_end = h->hv_bend;
  a.rounds = o.rounds;
  a.eps0 = o.eps0;
  a.eps_factor = o.eps_factor;
  a.form = o.weight_form;
  a.init = o.init;
  a.warm = o.warm_start;
  a.rtol = o.cg_rtol;
  a.maxit = o.cg_maxit;
  a.lane_code = h->lane_code;
  a.stop_gap = o.stop_gap;
  return a;
}

irls_status solve_resident(irls_mincut_t h, irls_round_stats *stats) {
  const irls_options &o = h->opt;
  const ResidentArgs a = resident_args(h);
  const int64_t nrec = (int64_t)h->G * (o.rounds + 1);
  if (h->batch) {
    // the whole batched solve (queue reset + one persistent launch running
    // every round of every graph) is captured once and replayed
    if (!h->gexec) {
      hipGraph_t graph = nullptr;
      HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "capture");
      hipError_t e1 = launch_resident_reset(h->rnext, h->dstats, nrec, h->cap_stream);
      hipError_t e2 = launch_resident(a, h->grid_res, 1024, h->cap_stream);
      hipError_t e3 = hipStreamEndCapture(h->cap_stream, &graph);
      if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return dev_fail(h, e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3), "graph capture");
      }
      hipError_t e4 = hipGraphInstantiate(&h->gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e4 != hipSuccess) { h->gexec = nullptr; return dev_fail(h, e4, "graph instantiate"); }
    }
    HIPCHK(h, hipGraphLaunch(h->gexec, h->stream), "graph launch");
  } else {
    HIPCHK(h, launch_resident_reset(h->rnext, h->dstats, nrec, h->stream), "reset");
    HIPCHK(h, launch_resident(a, h->grid_res, 1024, h->stream), "resident solve");
  }
  std::vector<irls_round_stats> hs(nrec);
  HIPCHK(h, hipMemcpyAsync(hs.data(), h->dstats, hs.size() * sizeof(irls_round_stats),
                           hipMemcpyDeviceToHost, h->stream), "stats copy");
  HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
  if (stats) std::memcpy(stats, hs.data(), hs.size() * sizeof(irls_round_stats));
  irls_status result = IRLS_OK;
  for (int64_t i = 0; i < nrec; i++) {
    if (hs[i].status == IRLS_ERR_CG_BREAKDOWN) {
      h->err = "CG breakdown in graph " + std::to_string(i / (o.rounds + 1)) + " round " +
               std::to_string(i % (o.rounds + 1));
      return IRLS_ERR_CG_BREAKDOWN;
    }
    if (hs[i].status == IRLS_WARN_CG_MAXIT) result = IRLS_WARN_CG_MAXIT;
  }
  return result;
}

// The graph record of a single-graph resident handle (heavy-row counts and
// lanes from create; the capacity-dependent fields from the graph).
// Light rows of the resident solver's graphs in each length bin.
void resident_bin_rows(irls_mincut_t h, int64_t (&rows)[kBins]) {
  for (int b = 0; b < kBins; b++) rows[b] = 0;
  auto add = [&](const BatchGraph &B) {
    for (int b = 0; b < kBins; b++) rows[b] += B.bin[b + 1] - B.bin[b];
  };
  if (h->batch) for (const BatchGraph &B : h->hgraphs) add(B);
  else add(h->res_graph);
}

uint32_t lane_code_with(uint32_t code, int b, int lg) {
  return (code & ~(7u << (3 * b))) | ((uint32_t)lg << (3 * b));
}

// One resident solve of `rounds` rounds, launched directly (not from the
// captured graph) under the given lane code and timed with the two events on
// the handle's stream.  It starts as a solve does: from x = 0.5 with init 1,
// else from the saved potentials (which round 0 ignores with init 0).
irls_status time_resident(irls_mincut_t h, int32_t rounds, uint32_t code, hipEvent_t e0, hipEvent_t e1,
                          float *ms) {
  ResidentArgs a = resident_args(h);
  a.rounds = rounds;
  a.lane_code = code;
  const int64_t nrec = (int64_t)h->G * (rounds + 1);
  if (h->opt.init == 1) HIPCHK(h, launch_fill(h->v, h->g.nt, 0.5, h->stream), "fill");
  else HIPCHK(h, hipMemcpyAsync(h->v, h->vsave, h->g.nt * sizeof(double), hipMemcpyDeviceToDevice, h->stream),
              "restore");
  HIPCHK(h, hipEventRecord(e0, h->stream), "event");
  HIPCHK(h, launch_resident_reset(h->rnext, h->dstats, nrec, h->stream), "reset");
  HIPCHK(h, launch_resident(a, h->grid_res, 1024, h->stream), "resident solve");
  HIPCHK(h, hipEventRecord(e1, h->stream), "event");
  HIPCHK(h, hipEventSynchronize(e1), "sync");
  HIPCHK(h, hipEventElapsedTime(ms, e0, e1), "event time");
  return IRLS_OK;
}

irls_status upload_res_record(irls_mincut_t h) {
  BatchGraph rg = h->res_graph;
  rg.node0 = 0;
  rg.nnz0 = 0;
  rg.node_off = 0;
  rg.nt = h->g.nt;
  rg.s = h->g.s;
  rg.t = h->g.t;
  rg.cst = h->g.cst;
  rg.fx_k = h->g.fx_k;
  rg.no_source_edges = h->g.no_source_edges ? 1 : 0;
  HIPCHK(h, hipMemcpy(h->rgraphs, &rg, sizeof(rg), hipMemcpyHostToDevice), "upload");
  return IRLS_OK;
}

irls_status alloc_state(irls_mincut_t h) {
  const int64_t nt = h->g.nt;
  const bool f32 = h->opt.precision == 1;
  const size_t ts = f32 ? sizeof(float) : sizeof(double);
  const int64_t nw = h->g.format == 2 ? (int64_t)h->g.K * nt : h->g.nnz;
  auto rawalloc = [&](void **p, size_t bytes) -> hipError_t {
    char *q = nullptr;
    hipError_t e = h->dalloc(&q, bytes);
    *p = q;
    return e;
  };
  HIPCHK(h, h->dalloc(&h->v, nt), "alloc");
  HIPCHK(h, h->dalloc(&h->b, nt), "alloc");
  if (h->bj_kind == 3) HIPCHK(h, h->dalloc(&h->ilu_f, h->g.nnz), "alloc");
  if (h->bj_block > 0) {
    HIPCHK(h, rawalloc(&h->bj_r, nt * ts), "alloc");
    HIPCHK(h, h->dalloc(&h->bj_f, nt), "alloc");
    HIPCHK(h, rawalloc(&h->bj_im, nt * ts), "alloc");
    HIPCHK(h, h->dalloc(&h->bj_g, nt), "alloc");
  }
  HIPCHK(h, h->dalloc(&h->gt, nt), "alloc");
  HIPCHK(h, rawalloc(&h->w, nw * ts), "alloc");
  HIPCHK(h, rawalloc(&h->D, nt * ts), "alloc");
  HIPCHK(h, rawalloc(&h->r, nt * ts), "alloc");
  HIPCHK(h, rawalloc(&h->q, nt * ts), "alloc");
  HIPCHK(h, rawalloc(&h->p0, nt * ts), "alloc");
  if (h->g.format == 2) HIPCHK(h, rawalloc(&h->p1, nt * ts), "alloc");
  if (h->scaled) HIPCHK(h, rawalloc(&h->wh, nw * ts), "alloc");
  if (h->scaled && !f32) HIPCHK(h, h->dalloc(&h->Dn, nt), "alloc");
  if (f32) {
    HIPCHK(h, h->dalloc(&h->w64, nw), "alloc");
    HIPCHK(h, h->dalloc(&h->D64, nt), "alloc");
    if (h->scaled) HIPCHK(h, h->dalloc(&h->wh64, nw), "alloc");
  }
  HIPCHK(h, h->dalloc(&h->partials, (size_t)kNumPSlots * kNumPartial * kMaxGrid), "alloc");
  HIPCHK(h, hipMemset(h->partials, 0, (size_t)kNumPSlots * kNumPartial * kMaxGrid * sizeof(double)), "memset");
  HIPCHK(h, h->dalloc(&h->sc, 1), "alloc");
  HIPCHK(h, h->dalloc(&h->sc_bench, 1), "alloc");
  HIPCHK(h, h->dalloc(&h->dstats, (int64_t)h->G * (h->opt.rounds + 1)), "alloc");
  h->stats_cap = (int64_t)h->G * (h->opt.rounds + 1);
  HIPCHK(h, hipMemset(h->v, 0, std::max<int64_t>(nt, 1) * sizeof(double)), "memset");
  HIPCHK(h, hipHostMalloc((void **)&h->pinned, 2 * sizeof(Scalars), hipHostMallocDefault), "pinned alloc");
  std::memset(h->pinned, 0, 2 * sizeof(Scalars));
  HIPCHK(h, hipEventCreateWithFlags(&h->ev[0], hipEventDisableTiming), "event");
  HIPCHK(h, hipEventCreateWithFlags(&h->ev[1], hipEventDisableTiming), "event");
  if (h->solver == 2 && !h->batch) {
    HIPCHK(h, h->dalloc(&h->rgraphs, 1), "alloc");
    HIPCHK(h, h->dalloc(&h->rorder, 1), "alloc");
    HIPCHK(h, h->dalloc(&h->rnext, 1), "alloc");
    int32_t zero = 0;
    HIPCHK(h, hipMemcpy(h->rorder, &zero, sizeof(zero), hipMemcpyHostToDevice), "upload");
    irls_status rc = upload_res_record(h);
    if (rc != IRLS_OK) return rc;
    h->rpw = 64 / h->res_graph.lanes;
  }
  return IRLS_OK;
}

template <typename T>
irls_status upload(irls_mincut_t h, T **dst, const std::vector<T> &src) {
  HIPCHK(h, h->dalloc(dst, src.size()), "alloc");
  if (!src.empty()) HIPCHK(h, hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice), "upload");
  return IRLS_OK;
}

irls_status upload_heavy(irls_mincut_t h, const HeavyLists &H) {
  irls_status rc;
  if ((rc = upload(h, &h->hv_crow, H.crow)) != IRLS_OK || (rc = upload(h, &h->hv_cbeg, H.cbeg)) != IRLS_OK ||
      (rc = upload(h, &h->hv_cend, H.cend)) != IRLS_OK || (rc = upload(h, &h->hv_hrow, H.hrow)) != IRLS_OK ||
      (rc = upload(h, &h->hv_hc0, H.hc0)) != IRLS_OK || (rc = upload(h, &h->hv_hc1, H.hc1)) != IRLS_OK ||
      (rc = upload(h, &h->hv_brow, H.brow)) != IRLS_OK || (rc = upload(h, &h->hv_bbeg, H.bbeg)) != IRLS_OK ||
      (rc = upload(h, &h->hv_bend, H.bend)) != IRLS_OK)
    return rc;
  HIPCHK(h, h->dalloc(&h->hv_part, H.crow.size() * kChunkQ), "alloc");
  return IRLS_OK;
}

}  // namespace

namespace irls {
// read-only views of a handle for the learned warm start (gnn_host.cpp)
const GraphDev *handle_graph(irls_mincut_t h) { return &h->g; }
bool handle_is_batch(irls_mincut_t h) { return h->batch; }
double *handle_potentials(irls_mincut_t h) { return h->solved ? h->v : nullptr; }
hipStream_t handle_stream(irls_mincut_t h) { return h->stream; }
}  // namespace irls

// ----------------------------------------------------------------------------
// C ABI
// ----------------------------------------------------------------------------
extern "C" {


irls_status irls_mincut_create(irls_mincut_t *out, int64_t n, int64_t m, const int64_t *edge_u,
                               const int64_t *edge_v, const double *cap, int64_t s, int64_t t,
                               const irls_options *opt, void *hip_stream) {
  if (!out) { g_thread_error = "out must not be NULL"; return IRLS_ERR_NULL; }
  *out = nullptr;
  irls_mincut_t h = nullptr;
  try {
    irls_options o;
    if (opt) o = *opt; else irls_options_default(&o);
    std::string err;
    irls_status rc = check_options(o, err);
    if (rc != IRLS_OK) { g_thread_error = err; return rc; }
    if (m > 0 && (!edge_u || !edge_v || !cap)) { g_thread_error = "edge arrays must not be NULL"; return IRLS_ERR_NULL; }
    // device-resident inputs are staged to the host for set-up
    std::vector<int64_t> hu, hv;
    std::vector<double> hc;
    if (o.inputs_on_device && m > 0) {
      if (n < 2 || m < 0) { g_thread_error = "need n >= 2 and m >= 0"; return IRLS_ERR_RANGE; }
      hu.resize(m); hv.resize(m); hc.resize(m);
      if (hipMemcpy(hu.data(), edge_u, m * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(hv.data(), edge_v, m * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(hc.data(), cap, m * 8, hipMemcpyDeviceToHost) != hipSuccess) {
        g_thread_error = "cannot read the device edge arrays";
        return IRLS_ERR_DEVICE;
      }
      edge_u = hu.data(); edge_v = hv.data(); cap = hc.data();
    }
    HostGraph hg;
    rc = build_host_graph(hg, n, m, edge_u, edge_v, cap, s, t, err);
    if (rc != IRLS_OK) { g_thread_error = err; return rc; }
    hu.clear(); hv.clear(); hc.clear();
    if (o.format == 2 && !hg.dia_ok) {
      g_thread_error = "graph does not fit the diagonal format";
      return IRLS_ERR_OPTIONS;
    }
    h = new irls_mincut_s();
    h->opt = o;
    h->stream = (hipStream_t)hip_stream;
    GraphDev &g = h->g;
    g.n = n; g.s = s; g.t = t; g.nt = hg.nt;
    g.nnz = (int64_t)hg.col.size();
    g.cst = hg.cst;
    g.fx_k = hg.fx_k;
    g.cmax = hg.cmax;
    g.no_source_edges = hg.no_source_edges;
    h->D0 = hg.D0;
    h->ctot = total_capacity2(hg);
    h->solver = o.solver ? o.solver
                         : ((o.precision == 0 && o.precond == 0 && hg.nt <= kResidentMaxRows) ? 2 : 1);
    if (h->solver == 2 && o.format == 2) {
      g_thread_error = "the resident solver stores the graph in CSR form";
      delete h;
      return IRLS_ERR_OPTIONS;
    }
    // the resident solver keeps one conductance per CSR entry
    const bool use_dia = hg.dia_ok && o.format != 1 && h->solver == 1;
    g.format = use_dia ? 2 : 1;
    g.K = use_dia ? hg.K : 0;
    for (int k = 0; k < kMaxDiag; k++) g.off[k] = hg.off[k];
    if (o.precond == 1) {
      // blocks of consecutive rows inside one line of offset-1 edges
      if (!use_dia || hg.off[0] != 1) {
        g_thread_error = "block-Jacobi needs a graph in the diagonal format with offset 1";
        delete h;
        return IRLS_ERR_OPTIONS;
      }
      const int32_t line = hg.K >= 2 ? hg.off[1] : 128;
      int32_t B = o.block_size ? o.block_size : std::min<int32_t>(line, 128) & ~1;
      if (B < 2 || B > line) {
        g_thread_error = "block_size must be even, at least 2 and at most the offset-1 line length";
        delete h;
        return IRLS_ERR_OPTIONS;
      }
      h->bj_block = B;
      h->bj_kind = 1;
    }
    std::vector<int32_t> blk_ptr, blk_rows, row_blk;
    if (o.precond == 2 && !use_dia) {
      // CSR: blocks of B consecutive positions of a breadth-first ordering
      // (from the smallest unvisited row, neighbours in ascending order), each
      // block's rows taken in ascending order
      const int32_t B = o.block_size ? o.block_size : 32;
      const int64_t nt = hg.nt;
      std::vector<int32_t> order;
      order.reserve(nt);
      std::vector<uint8_t> seen(nt, 0);
      for (int64_t r = 0; r < nt; r++) {
        if (seen[r]) continue;
        size_t head = order.size();
        seen[r] = 1;
        order.push_back((int32_t)r);
        while (head < order.size()) {
          const int32_t u = order[head++];
          for (int32_t e = hg.rowptr[u]; e < hg.rowptr[u + 1]; e++) {
            const int32_t v = hg.col[e];
            if (!seen[v]) { seen[v] = 1; order.push_back(v); }
          }
        }
      }
      const int64_t nb = (nt + B - 1) / B;
      blk_ptr.resize(nb + 1);
      row_blk.resize(nt);
      for (int64_t k = 0; k <= nb; k++) blk_ptr[k] = (int32_t)std::min<int64_t>(k * B, nt);
      blk_rows = order;
      for (int64_t k = 0; k < nb; k++) {
        std::sort(blk_rows.begin() + blk_ptr[k], blk_rows.begin() + blk_ptr[k + 1]);
        for (int32_t q = blk_ptr[k]; q < blk_ptr[k + 1]; q++) row_blk[blk_rows[q]] = (int32_t)k;
      }
      h->bj_block = B;
      h->bj_kind = 3;
      h->nblk = nb;
    }
    if (o.precond == 2 && use_dia) {
      // cubic tiles of a 3-D grid: offsets 1, N, P with N and P / N multiples
      // of the tile edge, and whole planes
      const int32_t B = o.block_size ? o.block_size : 4;
      const bool grid3 = (B == 2 || B == 4 || B == 8) && hg.K == 3 && hg.off[0] == 1 && hg.off[1] > 0 &&
                         hg.off[2] % hg.off[1] == 0 && hg.off[1] % B == 0 && (hg.off[2] / hg.off[1]) % B == 0 &&
                         hg.nt % hg.off[2] == 0;
      if (!grid3) {
        g_thread_error = "ILU(0) tiles need a tile edge of 2, 4 or 8 and a 3-D grid in the diagonal format "
                         "whose lines and planes are multiples of it, with whole planes (format 1 gives "
                         "CSR blocks instead)";
        delete h;
        return IRLS_ERR_OPTIONS;
      }
      h->bj_block = B * B * B;
      h->bj_kind = 2;
      h->bj_tile = B;
    }
    if (o.precond == 2 && o.precision == 1 && !(h->bj_kind == 2 && h->bj_tile == 4)) {
      g_thread_error = "the precision form takes ILU(0) of 4x4x4 tiles of a 3-D grid only";
      delete h;
      return IRLS_ERR_OPTIONS;
    }
    h->grid = grid_for(hg.nt);
    // the multi-workgroup CSR SpMV: rows of more than kCsrHeavy entries are
    // cut into chunks of kCsrChunk (a wavefront each)
    std::vector<int32_t> csr_hfirst, csr_cbeg, csr_cend;
    if (!use_dia && h->solver == 1) {
      for (int64_t i = 0; i < hg.nt; i++) {
        const int32_t e0 = hg.rowptr[i], e1 = hg.rowptr[i + 1];
        if (e1 - e0 <= kCsrHeavy) continue;
        if (csr_hfirst.empty()) csr_hfirst.assign(hg.nt, 0);
        csr_hfirst[i] = (int32_t)csr_cbeg.size() + 1;
        h->csr_nheavy++;
        for (int32_t e = e0; e < e1; e += kCsrChunk) {
          csr_cbeg.push_back(e);
          csr_cend.push_back(std::min(e + kCsrChunk, e1));
        }
      }
      h->csr_nchunks = (int32_t)csr_cbeg.size();
    }
    // Jacobi as symmetric scaling wherever the marching SpMV runs with point
    // Jacobi: that SpMV then reads no diagonal
    if (use_dia && o.precond == 0 && !o.unscaled_cg)
      h->scaled = (o.precision == 1 ? make_args<float>(h).march_planes : make_args<double>(h).march_planes) > 0;
    {
      double avg = hg.nt > 0 ? (double)hg.col.size() / (double)hg.nt : 1.0;
      int L = 1;
      while (L < 64 && L < avg) L <<= 1;
      h->rpw = o.rows_per_wave ? o.rows_per_wave : 64 / L;
    }
    HeavyLists H;
    std::memset(&h->res_graph, 0, sizeof(h->res_graph));
    if (h->solver == 2) add_heavy_rows(hg.rowptr, hg.nt, H, h->res_graph);
    if ((rc = upload(h, &g.rowptr, hg.rowptr)) != IRLS_OK ||
        (rc = upload(h, &g.col, hg.col)) != IRLS_OK ||
        (rc = upload(h, &g.ccap, hg.ccap)) != IRLS_OK ||
        (rc = upload(h, &g.cs, hg.cs)) != IRLS_OK ||
        (rc = upload(h, &g.ct, hg.ct)) != IRLS_OK ||
        (use_dia && (rc = upload(h, &g.dcap, hg.dcap)) != IRLS_OK) ||
        (h->bj_kind == 3 && ((rc = upload(h, &h->blk_ptr, blk_ptr)) != IRLS_OK ||
                             (rc = upload(h, &h->blk_rows, blk_rows)) != IRLS_OK ||
                             (rc = upload(h, &h->row_blk, row_blk)) != IRLS_OK)) ||
        (rc = upload_heavy(h, H)) != IRLS_OK ||
        (h->csr_nheavy > 0 && ((rc = upload(h, &h->csr_hfirst, csr_hfirst)) != IRLS_OK ||
                               (rc = upload(h, &h->csr_cbeg, csr_cbeg)) != IRLS_OK ||
                               (rc = upload(h, &h->csr_cend, csr_cend)) != IRLS_OK ||
                               (rc = upload(h, &h->csr_cpart, std::vector<double>(csr_cbeg.size(), 0.0))) != IRLS_OK)) ||
        (rc = alloc_state(h)) != IRLS_OK) {
      g_thread_error = h->err;
      h->release();
      delete h;
      return rc;
    }
    *out = h;
    return IRLS_OK;
  } catch (const std::bad_alloc &) {
    if (h) { h->release(); delete h; }
    g_thread_error = "host allocation failed";
    return IRLS_ERR_OOM;
  } catch (...) {
    if (h) { h->release(); delete h; }
    g_thread_error = "unexpected host exception";
    return IRLS_ERR_DEVICE;
  }
}

}  // extern "C"

namespace {

// one call of the round driver with (possibly) overridden start, first eps
// and round count; the handle's options are restored afterwards
irls_status solve_impl(irls_mincut_t h, int start, const double *x0, double eps_first, int32_t rounds,
                       irls_round_stats *stats) {
  const irls_options saved = h->opt;
  irls_options &o = h->opt;
  o.rounds = rounds;
  if (eps_first > 0.0) o.eps0 = eps_first;
  if (start != 0) o.init = 2;                       // no round-0 solve: round 0 reports the start
  irls_status rc = IRLS_OK;
  if ((int64_t)rounds + 1 > h->stats_cap) {
    irls_round_stats *ns = nullptr;
    hipError_t e = h->dalloc(&ns, rounds + 1);
    if (e != hipSuccess) { h->opt = saved; return dev_fail(h, e, "alloc"); }
    h->dstats = ns;
    h->stats_cap = rounds + 1;
  }
  if (start == 2 || (start == 0 && saved.init == 2)) {
    if (!x0) { h->opt = saved; h->err = "this start needs x0"; return IRLS_ERR_NULL; }
    rc = load_x0(h, x0);
  } else if (start == 0 && saved.init == 1 && h->g.nt > 0) {
    hipError_t e = launch_fill(h->v, h->g.nt, 0.5, h->stream);
    if (e != hipSuccess) rc = dev_fail(h, e, "fill");
  }
  if (rc == IRLS_OK) {
    if (h->solver == 2) rc = solve_resident(h, stats);
    else if (o.precision == 1) rc = solve_multi<float>(h, stats);
    else rc = solve_multi<double>(h, stats);
  }
  h->opt = saved;
  return rc;
}

}  // namespace

extern "C" {

// After a solve from round 0 with init 0: round 0's energy E01 = x^T L x at
// W = C, for the Cheeger-type bracket.  It depends on the graph alone, so it
// stays valid until the capacities change.
irls_status keep_round0_energy(irls_mincut_t h, int32_t start) {
  if (start != 0 || h->opt.init != 0) return IRLS_OK;
  if (h->g.nt == 0) {
    h->e01 = h->g.cst;                                 // only the s-t edge carries flow
  } else {
    irls_round_stats r0;
    HIPCHK(h, hipMemcpy(&r0, h->dstats, sizeof(r0), hipMemcpyDeviceToHost), "readback");
    h->e01 = r0.flow;
  }
  h->e01_valid = true;
  return IRLS_OK;
}

irls_status irls_mincut_solve(irls_mincut_t h, const double *x0, irls_round_stats *stats) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (h->batch) { h->err = "use irls_mincut_solve_batch for a batch handle"; return IRLS_ERR_OPTIONS; }
  try {
    h->solved = false;
    irls_status rc = solve_impl(h, 0, x0, -1.0, h->opt.rounds, stats);
    if (rc == IRLS_OK || rc == IRLS_WARN_CG_MAXIT) {
      h->solved = true;
      irls_status r2 = keep_round0_energy(h, 0);
      if (r2 != IRLS_OK) return r2;
    }
    return rc;
  } catch (...) {
    h->err = "unexpected host exception";
    return IRLS_ERR_DEVICE;
  }
}

irls_status irls_mincut_solve_range(irls_mincut_t h, int32_t start, const double *x0, double eps_first,
                                    int32_t rounds, irls_round_stats *stats) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (h->batch) { h->err = "not available for a batch handle"; return IRLS_ERR_OPTIONS; }
  if (start < 0 || start > 2 || rounds < 0 || (rounds > 0 && !(eps_first > 0.0) && start != 0)) {
    h->err = "need start in {0,1,2}, rounds >= 0 and eps_first > 0";
    return IRLS_ERR_OPTIONS;
  }
  if (start == 1 && !h->solved) { h->err = "no potentials to continue from"; return IRLS_ERR_NOT_SOLVED; }
  try {
    h->solved = false;
    irls_status rc = solve_impl(h, start, x0, eps_first, rounds, stats);
    if (rc == IRLS_OK || rc == IRLS_WARN_CG_MAXIT) {
      h->solved = true;
      irls_status r2 = keep_round0_energy(h, start);
      if (r2 != IRLS_OK) return r2;
    }
    return rc;
  } catch (...) {
    h->err = "unexpected host exception";
    return IRLS_ERR_DEVICE;
  }
}

// The sweep cut of the handle's potentials; its work buffers are the
// handle's (allocated on first use) or, with noalloc, the library's static
// scratch array.
static irls_status cut_impl(irls_mincut_t h, bool noalloc, uint8_t *in_source_side, double *cut_value,
                            int64_t *k_star) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (h->batch) { h->err = "use irls_mincut_cut_batch for a batch handle"; return IRLS_ERR_OPTIONS; }
  if (!h->solved) { h->err = "no potentials yet: call irls_mincut_solve first"; return IRLS_ERR_NOT_SOLVED; }
  if (noalloc && h->g.nt > IRLS_NOALLOC_MAX_NONTERMINAL) {
    h->err = "irls_mincut_cut_noalloc takes at most " + std::to_string(IRLS_NOALLOC_MAX_NONTERMINAL) +
             " non-terminal nodes (this graph has " + std::to_string(h->g.nt) + "): use irls_mincut_cut";
    return IRLS_ERR_OPTIONS;
  }
  try {
    GraphDev &g = h->g;
    i128 best = 0;
    int64_t ks = 0;
    SweepBufs sb_static;
    if (g.nt > 0) {
      if (noalloc) HIPCHK(h, sweep_noalloc_buffers(g.nt, g.n, sb_static), "static scratch");
      SweepBufs &b = noalloc ? sb_static : h->sw;
      if (!b.keyA) {
        const size_t nb = sweep_sort_blocks(g.nt), sb = sweep_scan_blocks(g.nt);
        HIPCHK(h, h->dalloc(&b.keyA, g.nt), "alloc");
        HIPCHK(h, h->dalloc(&b.keyB, g.nt), "alloc");
        HIPCHK(h, h->dalloc(&b.idA, g.nt), "alloc");
        HIPCHK(h, h->dalloc(&b.idB, g.nt), "alloc");
        HIPCHK(h, h->dalloc(&b.rank, g.nt), "alloc");
        HIPCHK(h, h->dalloc(&b.delta, g.nt), "alloc");
        HIPCHK(h, h->dalloc(&b.hist, 256 * nb + 256), "alloc");   // counts, then the 256 digit totals
        HIPCHK(h, h->dalloc(&b.bsum, sb), "alloc");
        HIPCHK(h, h->dalloc(&b.bmin, sb), "alloc");
        HIPCHK(h, h->dalloc(&b.barg, sb), "alloc");
        HIPCHK(h, h->dalloc(&b.best, 2), "alloc");
        HIPCHK(h, h->dalloc(&b.kstar, 1), "alloc");
        HIPCHK(h, h->dalloc(&b.mask, g.n), "alloc");
      }
      SweepArgs a;
      a.nt = g.nt; a.n = g.n; a.s = g.s; a.t = g.t;
      a.v = h->v;
      a.rowptr = g.rowptr; a.col = g.col; a.ccap = g.ccap; a.cs = g.cs; a.ct = g.ct;
      a.cst = g.cst;
      a.fx_k = g.fx_k;
      HIPCHK(h, sweep_run(a, b, h->stream), "sweep");
      HIPCHK(h, hipMemcpyAsync(&best, b.best, sizeof(i128), hipMemcpyDeviceToHost, h->stream), "readback");
      HIPCHK(h, hipMemcpyAsync(&ks, b.kstar, sizeof(int64_t), hipMemcpyDeviceToHost, h->stream), "readback");
      if (in_source_side)
        HIPCHK(h, hipMemcpyAsync(in_source_side, b.mask, g.n, hipMemcpyDeviceToHost, h->stream), "readback");
      HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
    } else if (in_source_side) {
      in_source_side[g.s] = 1;
      in_source_side[g.t] = 0;
    }
    if (cut_value) *cut_value = fx_to_double(h->D0 + best, g.fx_k);
    if (k_star) *k_star = ks;
    return IRLS_OK;
  } catch (...) {
    h->err = "unexpected host exception";
    return IRLS_ERR_DEVICE;
  }
}

irls_status irls_mincut_cut(irls_mincut_t h, uint8_t *in_source_side, double *cut_value, int64_t *k_star) {
  return cut_impl(h, false, in_source_side, cut_value, k_star);
}

irls_status irls_mincut_cut_noalloc(irls_mincut_t h, uint8_t *in_source_side, double *cut_value,
                                    int64_t *k_star) {
  return cut_impl(h, true, in_source_side, cut_value, k_star);
}

irls_status irls_mincut_cut_two_level(irls_mincut_t h, uint8_t *in_source_side, double *cut_value,
                                      irls_two_level_info *info) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (h->batch) { h->err = "two-level rounding runs on single-graph handles"; return IRLS_ERR_OPTIONS; }
  if (!h->solved) { h->err = "no potentials yet: call irls_mincut_solve first"; return IRLS_ERR_NOT_SOLVED; }
  try {
    GraphDev &g = h->g;
    const int64_t nt = g.nt, n = g.n;
    TwoLevelBufs &b = h->tl;
    if (!b.cls && nt > 0) {
      b.grid = (int)std::min<int64_t>(kMaxGrid, std::max<int64_t>(1, (nt + kBlock - 1) / kBlock));
      b.chunk = (nt + b.grid - 1) / b.grid;
      const int64_t ni = std::max<int64_t>(1, g.nnz / 2);
      HIPCHK(h, h->dalloc(&b.cls, nt), "alloc");
      HIPCHK(h, h->dalloc(&b.cid, nt), "alloc");
      HIPCHK(h, h->dalloc(&b.part, 3 * b.grid), "alloc");
      HIPCHK(h, h->dalloc(&b.bnodes, b.grid), "alloc");
      HIPCHK(h, h->dalloc(&b.bedges, b.grid), "alloc");
      HIPCHK(h, h->dalloc(&b.boff, b.grid), "alloc");
      HIPCHK(h, h->dalloc(&b.eoff, b.grid), "alloc");
      HIPCHK(h, h->dalloc(&b.bst, b.grid), "alloc");
      HIPCHK(h, h->dalloc(&b.eu, ni), "alloc");
      HIPCHK(h, h->dalloc(&b.ev, ni), "alloc");
      HIPCHK(h, h->dalloc(&b.ecap, ni), "alloc");
      HIPCHK(h, h->dalloc(&b.ws, nt), "alloc");
      HIPCHK(h, h->dalloc(&b.wt, nt), "alloc");
      HIPCHK(h, h->dalloc(&b.side, nt + 2), "alloc");
      HIPCHK(h, h->dalloc(&b.mask, n), "alloc");
    }
    hipStream_t st = h->stream;
    // 1. K-means with two centres on all n potentials (x_s = 1, x_t = 0)
    double c0 = 0.1, c1 = 0.9;
    double prev = -1.0;
    int32_t updates = 0;
    std::vector<double> part(3 * (size_t)std::max(b.grid, 1));
    while (updates < 100) {
      const double m = 0.5 * (c0 + c1);
      double cnt_hi = 0.0, sum_hi = 0.0, sum_lo = 0.0;
      if (nt > 0) {
        HIPCHK(h, launch_tl_kmeans(h->v, nt, m, b.part, b.grid, st), "K-means");
        HIPCHK(h, hipMemcpyAsync(part.data(), b.part, part.size() * sizeof(double), hipMemcpyDeviceToHost, st),
               "readback");
        HIPCHK(h, hipStreamSynchronize(st), "sync");
        for (int w = 0; w < b.grid; w++) { cnt_hi += part[3 * w]; sum_hi += part[3 * w + 1]; sum_lo += part[3 * w + 2]; }
      }
      for (double xt : {1.0, 0.0}) {                   // s and t
        if (xt > m) { cnt_hi += 1.0; sum_hi += xt; }
        else sum_lo += xt;
      }
      if (cnt_hi == prev) break;
      const double cnt_lo = (double)n - cnt_hi;
      if (cnt_lo > 0.0) c0 = sum_lo / cnt_lo;
      if (cnt_hi > 0.0) c1 = sum_hi / cnt_hi;
      prev = cnt_hi;
      updates++;
    }
    const double g0 = c0 + 0.05, g1 = c1 - 0.05;
    if (!(1.0 >= g1) || !(0.0 <= g0)) {
      h->err = "potentials outside [0, 1]: s or t would not be coalesced";
      return IRLS_ERR_RANGE;
    }
    // 2. split and compaction, 3. coarse capacities (exact fixed point)
    int64_t nc = 0, ne = 0, n_s1 = 1, n_s0 = 1;
    std::vector<int32_t> eu, ev;
    std::vector<i128> ecap, ws, wt;
    i128 st_cap = fx_round_host(g.cst, g.fx_k);
    if (nt > 0) {
      const int G = b.grid;
      HIPCHK(h, launch_tl_classify(h->v, nt, g0, g1, b.cls, G, st), "classify");
      HIPCHK(h, launch_tl_count(b.cls, g.rowptr, g.col, nt, b.chunk, b.bnodes, b.bedges, G, st), "count");
      std::vector<int64_t> bn(G), be(G), bo(G), eo(G);
      HIPCHK(h, hipMemcpyAsync(bn.data(), b.bnodes, G * sizeof(int64_t), hipMemcpyDeviceToHost, st), "readback");
      HIPCHK(h, hipMemcpyAsync(be.data(), b.bedges, G * sizeof(int64_t), hipMemcpyDeviceToHost, st), "readback");
      HIPCHK(h, hipStreamSynchronize(st), "sync");
      for (int w = 0; w < G; w++) { bo[w] = nc; eo[w] = ne; nc += bn[w]; ne += be[w]; }
      HIPCHK(h, hipMemcpyAsync(b.boff, bo.data(), G * sizeof(int64_t), hipMemcpyHostToDevice, st), "upload");
      HIPCHK(h, hipMemcpyAsync(b.eoff, eo.data(), G * sizeof(int64_t), hipMemcpyHostToDevice, st), "upload");
      HIPCHK(h, launch_tl_ids(b.cls, nt, b.chunk, b.boff, nc, b.cid, G, st), "ids");
      HIPCHK(h, launch_tl_edges(b.cls, b.cid, g.rowptr, g.col, g.ccap, g.cs, g.ct, nt, b.chunk, g.fx_k, b.eoff,
                                b.eu, b.ev, b.ecap, b.ws, b.wt, b.bst, G, st), "coarse edges");
      eu.resize(ne); ev.resize(ne); ecap.resize(ne); ws.resize(nc); wt.resize(nc);
      std::vector<i128> bst(G);
      if (ne > 0) {
        HIPCHK(h, hipMemcpyAsync(eu.data(), b.eu, ne * sizeof(int32_t), hipMemcpyDeviceToHost, st), "readback");
        HIPCHK(h, hipMemcpyAsync(ev.data(), b.ev, ne * sizeof(int32_t), hipMemcpyDeviceToHost, st), "readback");
        HIPCHK(h, hipMemcpyAsync(ecap.data(), b.ecap, ne * sizeof(i128), hipMemcpyDeviceToHost, st), "readback");
      }
      if (nc > 0) {
        HIPCHK(h, hipMemcpyAsync(ws.data(), b.ws, nc * sizeof(i128), hipMemcpyDeviceToHost, st), "readback");
        HIPCHK(h, hipMemcpyAsync(wt.data(), b.wt, nc * sizeof(i128), hipMemcpyDeviceToHost, st), "readback");
      }
      HIPCHK(h, hipMemcpyAsync(bst.data(), b.bst, G * sizeof(i128), hipMemcpyDeviceToHost, st), "readback");
      HIPCHK(h, hipStreamSynchronize(st), "sync");
      for (int w = 0; w < G; w++) st_cap += bst[w];
    }
    // 4. exact minimum cut of G_c: Sc = 0..nc-1, s_c = nc, t_c = nc + 1
    int64_t merged_edges = ne + (st_cap > 0);
    for (int64_t u = 0; u < nc; u++) merged_edges += (ws[u] > 0) + (wt[u] > 0);
    std::vector<uint8_t> side;
    const i128 flow = coarse_min_cut(nc, eu, ev, ecap, ws, wt, st_cap, side);
    // lift: S1 and the source side's part of Sc, in original node ids
    if (in_source_side) {
      if (nt > 0) {
        HIPCHK(h, hipMemcpyAsync(b.side, side.data(), nc + 2, hipMemcpyHostToDevice, st), "upload");
        HIPCHK(h, launch_tl_lift(b.cls, b.cid, b.side, nt, std::min(g.s, g.t), std::max(g.s, g.t), b.mask, b.grid, st),
               "lift");
        HIPCHK(h, hipMemcpyAsync(in_source_side, b.mask, n, hipMemcpyDeviceToHost, st), "readback");
        HIPCHK(h, hipStreamSynchronize(st), "sync");
      }
      in_source_side[g.s] = 1;
      in_source_side[g.t] = 0;
    }
    if (nt > 0) {
      std::vector<int8_t> cls(nt);
      HIPCHK(h, hipMemcpyAsync(cls.data(), b.cls, nt, hipMemcpyDeviceToHost, st), "readback");
      HIPCHK(h, hipStreamSynchronize(st), "sync");
      for (int64_t u = 0; u < nt; u++) { n_s0 += cls[u] == 0; n_s1 += cls[u] == 1; }
    }
    const double value = fx_to_double(flow, g.fx_k);
    if (cut_value) *cut_value = value;
    if (info) {
      info->c0 = c0;
      info->c1 = c1;
      info->gamma0 = g0;
      info->gamma1 = g1;
      info->kmeans_updates = updates;
      info->n_s0 = n_s0;
      info->n_s1 = n_s1;
      info->n_sc = nc;
      info->coarse_edges = merged_edges;
      info->coarse_value = value;
    }
    return IRLS_OK;
  } catch (const std::bad_alloc &) {
    h->err = "host allocation failed";
    return IRLS_ERR_OOM;
  } catch (...) {
    h->err = "unexpected host exception";
    return IRLS_ERR_DEVICE;
  }
}

irls_status irls_mincut_update_capacities(irls_mincut_t h, int64_t m, const int64_t *edge_u,
                                          const int64_t *edge_v, const double *cap) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (h->batch) { h->err = "capacity updates run on single-graph handles"; return IRLS_ERR_OPTIONS; }
  if (m > 0 && (!edge_u || !edge_v || !cap)) { h->err = "edge arrays must not be NULL"; return IRLS_ERR_NULL; }
  try {
    GraphDev &g = h->g;
    std::vector<int64_t> hu, hv;
    std::vector<double> hc;
    if (h->opt.inputs_on_device && m > 0) {
      hu.resize(m); hv.resize(m); hc.resize(m);
      if (hipMemcpy(hu.data(), edge_u, m * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(hv.data(), edge_v, m * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(hc.data(), cap, m * 8, hipMemcpyDeviceToHost) != hipSuccess) {
        h->err = "cannot read the device edge arrays";
        return IRLS_ERR_DEVICE;
      }
      edge_u = hu.data(); edge_v = hv.data(); cap = hc.data();
    }
    HostGraph hg;
    std::string err;
    irls_status rc = build_host_graph(hg, g.n, m, edge_u, edge_v, cap, g.s, g.t, err);
    if (rc != IRLS_OK) { h->err = err; return rc; }
    // the merged structure must be the handle's: same rows and neighbours
    bool same = hg.nt == g.nt && (int64_t)hg.col.size() == g.nnz;
    if (same && g.format == 2) {
      same = hg.dia_ok && hg.K == g.K;
      for (int k = 0; same && k < g.K; k++) same = hg.off[k] == g.off[k];
    }
    if (same && g.nt > 0) {
      std::vector<int32_t> rp(g.nt + 1), cl(g.nnz);
      HIPCHK(h, hipMemcpy(rp.data(), g.rowptr, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost), "readback");
      if (g.nnz > 0)
        HIPCHK(h, hipMemcpy(cl.data(), g.col, cl.size() * sizeof(int32_t), hipMemcpyDeviceToHost), "readback");
      same = rp == hg.rowptr && cl == hg.col;
    }
    if (!same) {
      h->err = "the edges do not have the handle's structure (create a new handle)";
      return IRLS_ERR_OPTIONS;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
    auto put = [&](double *dst, const std::vector<double> &src) -> hipError_t {
      return src.empty() ? hipSuccess : hipMemcpy(dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice);
    };
    HIPCHK(h, put(g.ccap, hg.ccap), "upload");
    HIPCHK(h, put(g.cs, hg.cs), "upload");
    HIPCHK(h, put(g.ct, hg.ct), "upload");
    if (g.format == 2) HIPCHK(h, put(g.dcap, hg.dcap), "upload");
    g.cst = hg.cst;
    g.cmax = hg.cmax;
    g.fx_k = hg.fx_k;
    g.no_source_edges = hg.no_source_edges;
    h->D0 = hg.D0;
    h->ctot = total_capacity2(hg);
    h->e01_valid = false;
    if (h->solver == 2) {
      rc = upload_res_record(h);
      if (rc != IRLS_OK) return rc;
    }
    return IRLS_OK;
  } catch (const std::bad_alloc &) {
    h->err = "host allocation failed";
    return IRLS_ERR_OOM;
  } catch (...) {
    h->err = "unexpected host exception";
    return IRLS_ERR_DEVICE;
  }
}

irls_status irls_mincut_cheeger_bracket(irls_mincut_t h, double *lower, double *upper) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (!lower || !upper) { h->err = "lower and upper must not be NULL"; return IRLS_ERR_NULL; }
  if (h->batch) { h->err = "not available for a batch handle"; return IRLS_ERR_OPTIONS; }
  if (!h->e01_valid) {
    h->err = "needs a solve from round 0 with init 0 (round 0 at W = C) since the capacities were set";
    return IRLS_ERR_NOT_SOLVED;
  }
  *lower = h->e01;
  *upper = 2.0 * std::sqrt(h->ctot * h->e01);
  return IRLS_OK;
}

irls_status irls_mincut_potentials(irls_mincut_t h, double *x) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (!x) { h->err = "x must not be NULL"; return IRLS_ERR_NULL; }
  if (!h->solved) { h->err = "no potentials yet"; return IRLS_ERR_NOT_SOLVED; }
  try {
    const int64_t nt = h->g.nt;
    std::vector<double> vn(nt);
    if (nt > 0) HIPCHK(h, hipMemcpyAsync(vn.data(), h->v, nt * sizeof(double), hipMemcpyDeviceToHost, h->stream), "readback");
    HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
    if (h->batch) {                 // every graph, laid out like node_off
      for (const BatchGraph &B : h->hgraphs) {
        for (int64_t i = 0; i < B.nt; i++) x[B.node_off + orig_of(i, B.s, B.t)] = vn[B.node0 + i];
        x[B.node_off + B.s] = 1.0;
        x[B.node_off + B.t] = 0.0;
      }
      return IRLS_OK;
    }
    for (int64_t i = 0; i < nt; i++) x[orig_of(i, h->g.s, h->g.t)] = vn[i];
    x[h->g.s] = 1.0;
    x[h->g.t] = 0.0;
    return IRLS_OK;
  } catch (...) {
    h->err = "unexpected host exception";
    return IRLS_ERR_DEVICE;
  }
}

irls_status irls_mincut_set_potentials(irls_mincut_t h, const double *x) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (!x) { h->err = "x must not be NULL"; return IRLS_ERR_NULL; }
  if (h->batch) { h->err = "not available for a batch handle"; return IRLS_ERR_OPTIONS; }
  try {
    irls_status rc = load_x0(h, x);
    if (rc != IRLS_OK) return rc;
    h->solved = true;
    return IRLS_OK;
  } catch (...) {
    h->err = "unexpected host exception";
    return IRLS_ERR_DEVICE;
  }
}

irls_status irls_mincut_info(irls_mincut_t h, int64_t *n_nonterminal, int64_t *nnz_offdiag,
                             int32_t *format, int32_t *n_diagonals, int32_t *solver,
                             int32_t *rows_per_wave) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (n_nonterminal) *n_nonterminal = h->g.nt;
  if (nnz_offdiag) *nnz_offdiag = h->g.nnz;
  if (format) *format = h->g.format;
  if (n_diagonals) *n_diagonals = h->g.K;
  if (solver) *solver = h->solver;
  if (rows_per_wave) *rows_per_wave = h->rpw;
  return IRLS_OK;
}

irls_status irls_mincut_spmv_kernel(irls_mincut_t h, int32_t *variant, int32_t *grid) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (h->batch || h->solver != 1) { h->err = "only the multi-workgroup solver has an SpMV kernel"; return IRLS_ERR_OPTIONS; }
  if (h->opt.precision == 1) {
    const CGArgs<float> a = make_args<float>(h);
    if (variant) *variant = spmv_variant(a);
    if (grid) *grid = a.grid_spmv;
  } else {
    const CGArgs<double> a = make_args<double>(h);
    if (variant) *variant = spmv_variant(a);
    if (grid) *grid = a.grid_spmv;
  }
  return IRLS_OK;
}

// The marching SpMV's tile shape on the handle's system: (bs, ty, planes per
// workgroup), or all 0 when the handle does not march.
static void march_shape(irls_mincut_t h, int32_t *bs, int32_t *ty, int32_t *planes) {
  if (h->opt.precision == 1) {
    const CGArgs<float> a = make_args<float>(h);
    *bs = a.march_bs; *ty = a.march_ty; *planes = a.march_planes;
  } else {
    const CGArgs<double> a = make_args<double>(h);
    *bs = a.march_bs; *ty = a.march_ty; *planes = a.march_planes;
  }
}

irls_status irls_mincut_set_march_tile(irls_mincut_t h, int32_t threads, int32_t lines) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (h->batch || h->solver != 1) { h->err = "only the multi-workgroup solver marches"; return IRLS_ERR_OPTIONS; }
  const int32_t rb = h->march_bs, rt = h->march_ty;
  h->march_bs = threads;
  h->march_ty = lines;
  if (threads == 0 && lines == 0) return IRLS_OK;
  int32_t bs, ty, pl;
  march_shape(h, &bs, &ty, &pl);
  if (pl == 0 || bs != threads || ty != lines) {
    h->march_bs = rb;
    h->march_ty = rt;
    h->err = "the marching SpMV cannot take this tile shape on this graph";
    return IRLS_ERR_OPTIONS;
  }
  return IRLS_OK;
}

irls_status irls_mincut_march_tile(irls_mincut_t h, int32_t *threads, int32_t *lines, int32_t *planes) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  int32_t bs = 0, ty = 0, pl = 0;
  if (!h->batch && h->solver == 1) march_shape(h, &bs, &ty, &pl);
  if (threads) *threads = bs;
  if (lines) *lines = ty;
  if (planes) *planes = pl;
  return IRLS_OK;
}

irls_status irls_mincut_time_kernel(irls_mincut_t h, int32_t which, int32_t reps, double *avg_ms) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (!avg_ms) { h->err = "avg_ms must not be NULL"; return IRLS_ERR_NULL; }
  if (which < 0 || which > 2 || reps < 1) { h->err = "which must be 0, 1 or 2, reps >= 1"; return IRLS_ERR_OPTIONS; }
  if (h->batch || h->solver != 1) { h->err = "kernel timing needs the multi-workgroup solver"; return IRLS_ERR_OPTIONS; }
  if (!h->solved) { h->err = "call irls_mincut_solve first"; return IRLS_ERR_NOT_SOLVED; }
  try {
    // The launches run on the live system of the last round with a private
    // scalar block (iteration 1, or 2 for which = 2; done = 0, no stopping);
    // the potentials are saved first and restored afterwards.
    const int64_t it = which == 2 ? 2 : 1;
    Scalars s;
    std::memset(&s, 0, sizeof(s));
    s.rho[0] = s.rho[1] = 1.0;
    s.iter_a = s.iter_b = it;
    s.maxit = std::numeric_limits<int64_t>::max();
    HIPCHK(h, hipMemcpy(h->sc_bench, &s, sizeof(s), hipMemcpyHostToDevice), "upload");
    if (!h->vsave) HIPCHK(h, h->dalloc(&h->vsave, h->g.nt), "alloc");
    HIPCHK(h, hipMemcpyAsync(h->vsave, h->v, h->g.nt * sizeof(double), hipMemcpyDeviceToDevice, h->stream), "save");
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0), "event");
    HIPCHK(h, hipEventCreate(&e1), "event");
    auto one = [&](void) -> hipError_t {
      if (h->opt.precision == 1) {
        CGArgs<float> a = make_args<float>(h);
        a.sc = h->sc_bench;
        a.it_hint = it;
        return which == 0 ? launch_spmv(a, h->grid, h->rpw, a.K > 0, h->stream) : launch_update(a, h->grid, h->stream);
      }
      CGArgs<double> a = make_args<double>(h);
      a.sc = h->sc_bench;
      a.it_hint = it;
      return which == 0 ? launch_spmv(a, h->grid, h->rpw, a.K > 0, h->stream) : launch_update(a, h->grid, h->stream);
    };
    hipError_t e = one();
    if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
    for (int i = 0; i < reps && e == hipSuccess; i++) e = one();
    if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return dev_fail(h, e, "kernel timing");
    HIPCHK(h, hipMemcpyAsync(h->v, h->vsave, h->g.nt * sizeof(double), hipMemcpyDeviceToDevice, h->stream), "restore");
    HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
    *avg_ms = (double)ms / reps;
    return IRLS_OK;
  } catch (...) {
    h->err = "unexpected host exception";
    return IRLS_ERR_DEVICE;
  }
}

irls_status irls_mincut_set_kernel_timing(irls_mincut_t h, int32_t which, int32_t every) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (which < -1 || which > 3) { h->err = "which must be -1, 0, 1, 2 or 3"; return IRLS_ERR_OPTIONS; }
  if (every < 1) { h->err = "every must be at least 1"; return IRLS_ERR_OPTIONS; }
  if (h->batch || h->solver != 1) { h->err = "kernel timing needs the multi-workgroup solver"; return IRLS_ERR_OPTIONS; }
  if (which == 2 && h->opt.precision != 1) { h->err = "which = 2 needs the precision form"; return IRLS_ERR_OPTIONS; }
  if (which == 3 && h->bj_block == 0) { h->err = "which = 3 needs a block-Jacobi preconditioner"; return IRLS_ERR_OPTIONS; }
  if (which == 3 && h->bj_kind == 2 && h->bj_tile == 4) {
    h->err = "with ILU(0) of 4x4x4 tiles the application runs inside the vector update: time which = 1";
    return IRLS_ERR_OPTIONS;
  }
  h->prof_which = which;
  h->prof_every = every;
  h->prof_rounds.clear();
  h->prof_used = 0;
  h->prof_ms_work = h->prof_ms_all = 0.0;
  h->prof_n_work = h->prof_n_all = 0;
  return IRLS_OK;
}

irls_status irls_mincut_kernel_timing(irls_mincut_t h, double *ms_working, int64_t *n_working,
                                      double *ms_all, int64_t *n_all) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (ms_working) *ms_working = h->prof_ms_work;
  if (n_working) *n_working = h->prof_n_work;
  if (ms_all) *ms_all = h->prof_ms_all;
  if (n_all) *n_all = h->prof_n_all;
  return IRLS_OK;
}

irls_status irls_stream_probe(int64_t rows, int32_t reads, int32_t writes, int32_t workgroups, int32_t reps,
                              void *hip_stream, double *avg_ms) {
  if (!avg_ms) { g_thread_error = "avg_ms must not be NULL"; return IRLS_ERR_NULL; }
  if (rows < 2 || rows % 2 != 0 || reads < 1 || reads > 6 || writes < 1 || writes > 2 || workgroups < 8 ||
      workgroups > kMaxGrid || workgroups % 8 != 0 || reps < 1 || reps > 1000) {
    g_thread_error = "need even rows >= 2, reads 1..6, writes 1..2, workgroups a multiple of 8 in 8..1024, reps 1..1000";
    return IRLS_ERR_OPTIONS;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  double *in = nullptr, *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&in, (size_t)reads * rows * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&out, (size_t)writes * rows * sizeof(double));
  if (e == hipSuccess) e = launch_fill(in, (int64_t)reads * rows, 1.0, st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // both forms of access, plain and streaming; the faster one counts
  double best = 0.0;
  for (int nt = 0; nt < 2 && e == hipSuccess; nt++) {
    e = launch_stream_probe(in, out, rows, reads, writes, workgroups, nt != 0, st);   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int i = 0; i < reps && e == hipSuccess; i++)
      e = launch_stream_probe(in, out, rows, reads, writes, workgroups, nt != 0, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && (nt == 0 || (double)ms / reps < best)) best = (double)ms / reps;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (in) (void)hipFree(in);
  if (out) (void)hipFree(out);
  if (e != hipSuccess) {
    g_thread_error = std::string("stream probe: ") + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? IRLS_ERR_OOM : IRLS_ERR_DEVICE;
  }
  *avg_ms = best;
  return IRLS_OK;
}

irls_status irls_mincut_set_row_lanes(irls_mincut_t h, const int32_t *lanes) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (!lanes) { h->err = "lanes must not be NULL"; return IRLS_ERR_NULL; }
  if (!h->batch && h->solver != 2) { h->err = "row lanes apply to the resident solver (solver 2 or a batch)"; return IRLS_ERR_OPTIONS; }
  uint32_t code = 0;
  for (int b = 0; b < kBins; b++) {
    int lg = 0;
    while (lg < 7 && (1 << lg) < lanes[b]) lg++;
    if (lanes[b] < 1 || (1 << lg) != lanes[b] || lg > bin_default_lg(b)) {
      h->err = "lanes[" + std::to_string(b) + "] must be a power of two from 1 to " +
               std::to_string(1 << bin_default_lg(b));
      return IRLS_ERR_OPTIONS;
    }
    code = lane_code_with(code, b, lg);
  }
  if (code != h->lane_code) {
    h->lane_code = code;
    if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; }   // captured with the old code
  }
  return IRLS_OK;
}

// The marching SpMV: its tile shape, measured by timing the SpMV on the last
// solve's system for every shape a launch can take (256 or 512 threads; 0,
// 1, 2, ..., 32 lines per tile).
static irls_status autotune_march(irls_mincut_t h, int32_t reps, int32_t *lanes) {
  int32_t bs0, ty0, pl;
  march_shape(h, &bs0, &ty0, &pl);
  if (pl == 0) { h->err = "the diagonal format without the marching SpMV has nothing to tune"; return IRLS_ERR_OPTIONS; }
  if (!h->solved) { h->err = "the SpMV is timed on a solved system: call irls_mincut_solve first"; return IRLS_ERR_NOT_SOLVED; }
  const int launches = 20 * reps;
  const int32_t rb = h->march_bs, rt = h->march_ty;
  double tcur = 0.0;
  irls_status rc = irls_mincut_time_kernel(h, 0, launches, &tcur);
  if (rc != IRLS_OK) return rc;
  int32_t best_bs = bs0, best_ty = ty0;
  double tbest = tcur;
  for (int32_t bs : {256, 512}) {
    for (int32_t ty : {0, 1, 2, 4, 8, 16, 32}) {
      h->march_bs = bs;
      h->march_ty = ty;
      int32_t b2, t2, p2;
      march_shape(h, &b2, &t2, &p2);
      if (b2 != bs || t2 != ty || (bs == bs0 && ty == ty0)) continue;      // not possible here, or the current one
      double t = 0.0;
      rc = irls_mincut_time_kernel(h, 0, launches, &t);
      if (rc != IRLS_OK) { h->march_bs = rb; h->march_ty = rt; return rc; }
      if (t < 0.98 * tcur && t < tbest) { best_bs = bs; best_ty = ty; tbest = t; }
    }
  }
  h->march_bs = best_bs;
  h->march_ty = best_ty;
  if (lanes) {
    lanes[0] = best_bs;
    lanes[1] = best_ty;
    for (int b = 2; b < kBins; b++) lanes[b] = 0;
  }
  return IRLS_OK;
}

// The multi-workgroup CSR path: rows per wavefront of its SpMV (and per-round
// CSR kernels), measured by timing the SpMV on the last solve's system.
static irls_status autotune_csr(irls_mincut_t h, int32_t reps, int32_t *lanes) {
  const int32_t K = h->opt.precision == 1 ? make_args<float>(h).K : make_args<double>(h).K;
  if (K > 0) return autotune_march(h, reps, lanes);
  if (!h->solved) { h->err = "the CSR SpMV is timed on a solved system: call irls_mincut_solve first"; return IRLS_ERR_NOT_SOLVED; }
  const int launches = 20 * reps;
  double tcur = 0.0;
  irls_status rc = irls_mincut_time_kernel(h, 0, launches, &tcur);
  if (rc != IRLS_OK) return rc;
  const int cur = h->rpw;
  int best = cur;
  double tbest = tcur;
  for (int rpw = 1; rpw <= 64; rpw *= 2) {
    if (rpw == cur) continue;
    h->rpw = rpw;
    double t = 0.0;
    rc = irls_mincut_time_kernel(h, 0, launches, &t);
    if (rc != IRLS_OK) { h->rpw = cur; return rc; }
    if (t < 0.98 * tcur && t < tbest) { best = rpw; tbest = t; }
  }
  h->rpw = best;
  if (lanes) {
    lanes[0] = 64 / best;
    for (int b = 1; b < kBins; b++) lanes[b] = 0;
  }
  return IRLS_OK;
}

irls_status irls_mincut_autotune(irls_mincut_t h, int32_t rounds, int32_t reps, int32_t *lanes) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (reps < 1 || reps > 100) { h->err = "reps must lie in 1..100"; return IRLS_ERR_OPTIONS; }
  if (!h->batch && h->solver == 1) {
    try {
      return autotune_csr(h, reps, lanes);
    } catch (...) {
      h->err = "unexpected host exception";
      return IRLS_ERR_DEVICE;
    }
  }
  if (!h->batch && h->solver != 2) { h->err = "autotuning applies to the resident solver (solver 2 or a batch)"; return IRLS_ERR_OPTIONS; }
  if (rounds < 0 || rounds > h->opt.rounds) {
    h->err = "rounds must lie in [0, the handle's rounds]";
    return IRLS_ERR_OPTIONS;
  }
  if (h->opt.init == 2 && !h->solved) {
    h->err = "init = 2 starts from the potentials: set them (or solve) first";
    return IRLS_ERR_NOT_SOLVED;
  }
  const bool was_solved = h->solved;
  h->solved = false;                   // until the potentials are back in place
  try {
    if (h->g.nt > 0) {
      if (!h->vsave) HIPCHK(h, h->dalloc(&h->vsave, h->g.nt), "alloc");
      HIPCHK(h, hipMemcpyAsync(h->vsave, h->v, h->g.nt * sizeof(double), hipMemcpyDeviceToDevice, h->stream),
             "save");
      struct Events {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events() {
          for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
        }
      } ev;
      for (hipEvent_t &e : ev.e) HIPCHK(h, hipEventCreate(&e), "event");
      int64_t rows[kBins];
      resident_bin_rows(h, rows);
      uint32_t code = h->lane_code;
      auto best_of = [&](uint32_t c, float &t) -> irls_status {
        t = std::numeric_limits<float>::infinity();
        for (int r = 0; r < reps; r++) {
          float ms = 0.0f;
          irls_status rc = time_resident(h, rounds, c, ev.e[0], ev.e[1], &ms);
          if (rc != IRLS_OK) return rc;
          t = std::min(t, ms);
        }
        return IRLS_OK;
      };
      // one sweep of coordinate descent over the bins that hold rows: the
      // lanes per row of bin b from its default down to an eighth of it; a
      // change must gain 2 % over the bin's current choice
      for (int b = 0; b < kBins; b++) {
        if (rows[b] == 0) continue;
        const int cur = (int)((code >> (3 * b)) & 7u);
        float tcur;
        irls_status rc = best_of(code, tcur);
        if (rc != IRLS_OK) return rc;
        int best = cur;
        float tbest = tcur;
        for (int lg = bin_default_lg(b); lg >= 0 && lg >= bin_default_lg(b) - 3; lg--) {
          if (lg == cur) continue;
          float t;
          rc = best_of(lane_code_with(code, b, lg), t);
          if (rc != IRLS_OK) return rc;
          if (t < 0.98f * tcur && t < tbest) { best = lg; tbest = t; }
        }
        code = lane_code_with(code, b, best);
      }
      HIPCHK(h, hipMemcpyAsync(h->v, h->vsave, h->g.nt * sizeof(double), hipMemcpyDeviceToDevice, h->stream),
             "restore");
      HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
      if (code != h->lane_code) {
        h->lane_code = code;
        if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; }
      }
    }
    h->solved = was_solved;
    if (lanes)
      for (int b = 0; b < kBins; b++) lanes[b] = 1 << ((h->lane_code >> (3 * b)) & 7u);
    return IRLS_OK;
  } catch (const std::bad_alloc &) {
    h->err = "host allocation failed";
    return IRLS_ERR_OOM;
  } catch (...) {
    h->err = "unexpected host exception";
    return IRLS_ERR_DEVICE;
  }
}

void irls_mincut_destroy(irls_mincut_t h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  h->release();
  delete h;
}

const char *irls_mincut_last_error(irls_mincut_t h) {
  return h ? h->err.c_str() : g_thread_error.c_str();
}

irls_status irls_mincut_create_batch(irls_mincut_t *out, int32_t G, const int64_t *node_off,
                                     const int64_t *edge_off, const int64_t *edge_u,
                                     const int64_t *edge_v, const double *cap, const int64_t *s,
                                     const int64_t *t, const irls_options *opt, void *hip_stream) {
  if (!out) { g_thread_error = "out must not be NULL"; return IRLS_ERR_NULL; }
  *out = nullptr;
  irls_mincut_t h = nullptr;
  try {
    irls_options o;
    if (opt) o = *opt; else irls_options_default(&o);
    std::string err;
    irls_status rc = check_options(o, err);
    if (rc != IRLS_OK) { g_thread_error = err; return rc; }
    if (o.precision != 0 || o.solver == 1 || o.init == 2) {
      g_thread_error = "the batched form runs the FP64 resident solver and starts from W = C or x = 1/2";
      return IRLS_ERR_OPTIONS;
    }
    if (G < 1 || G > 65536) { g_thread_error = "need 1 <= G <= 65536 graphs"; return IRLS_ERR_RANGE; }
    if (!node_off || !edge_off || !s || !t) { g_thread_error = "offset and terminal arrays must not be NULL"; return IRLS_ERR_NULL; }
    std::vector<int64_t> hno, heo, hs, ht, hu, hv;
    std::vector<double> hc;
    if (o.inputs_on_device) {
      hno.resize(G + 1); heo.resize(G + 1); hs.resize(G); ht.resize(G);
      if (hipMemcpy(hno.data(), node_off, (G + 1) * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(heo.data(), edge_off, (G + 1) * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(hs.data(), s, G * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(ht.data(), t, G * 8, hipMemcpyDeviceToHost) != hipSuccess) {
        g_thread_error = "cannot read the device arrays";
        return IRLS_ERR_DEVICE;
      }
      node_off = hno.data(); edge_off = heo.data(); s = hs.data(); t = ht.data();
    }
    if (node_off[0] != 0 || edge_off[0] != 0) { g_thread_error = "offsets must start at 0"; return IRLS_ERR_RANGE; }
    for (int32_t g = 0; g < G; g++)
      if (node_off[g + 1] < node_off[g] || edge_off[g + 1] < edge_off[g]) {
        g_thread_error = "offsets must not decrease";
        return IRLS_ERR_RANGE;
      }
    const int64_t M = edge_off[G];
    if (M > 0 && (!edge_u || !edge_v || !cap)) { g_thread_error = "edge arrays must not be NULL"; return IRLS_ERR_NULL; }
    if (o.inputs_on_device && M > 0) {
      hu.resize(M); hv.resize(M); hc.resize(M);
      if (hipMemcpy(hu.data(), edge_u, M * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(hv.data(), edge_v, M * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(hc.data(), cap, M * 8, hipMemcpyDeviceToHost) != hipSuccess) {
        g_thread_error = "cannot read the device edge arrays";
        return IRLS_ERR_DEVICE;
      }
      edge_u = hu.data(); edge_v = hv.data(); cap = hc.data();
    }
    // per-graph set-up, concatenated rows and CSR entries
    std::vector<int32_t> rowptr, col;
    std::vector<double> ccap, cs, ct;
    std::vector<BatchGraph> graphs(G);
    HeavyLists heavy;
    std::vector<uint32_t> gid;
    std::vector<i128> D0s(G);
    int64_t rows = 0, nnz = 0;
    for (int32_t g = 0; g < G; g++) {
      HostGraph hg;
      const int64_t e0 = edge_off[g];
      rc = build_host_graph(hg, node_off[g + 1] - node_off[g], edge_off[g + 1] - e0, edge_u + e0,
                            edge_v + e0, cap + e0, s[g], t[g], err);
      if (rc != IRLS_OK) { g_thread_error = "graph " + std::to_string(g) + ": " + err; return rc; }
      BatchGraph &B = graphs[g];
      std::memset(&B, 0, sizeof(B));
      B.node0 = rows;
      B.nt = hg.nt;
      B.nnz0 = nnz;
      B.node_off = node_off[g];
      B.s = s[g];
      B.t = t[g];
      B.cst = hg.cst;
      B.fx_k = hg.fx_k;
      add_heavy_rows(hg.rowptr, hg.nt, heavy, B);
      B.no_source_edges = hg.no_source_edges ? 1 : 0;
      D0s[g] = hg.D0;
      rowptr.insert(rowptr.end(), hg.rowptr.begin(), hg.rowptr.end());
      col.insert(col.end(), hg.col.begin(), hg.col.end());
      ccap.insert(ccap.end(), hg.ccap.begin(), hg.ccap.end());
      cs.insert(cs.end(), hg.cs.begin(), hg.cs.end());
      ct.insert(ct.end(), hg.ct.begin(), hg.ct.end());
      gid.insert(gid.end(), (size_t)hg.nt, (uint32_t)g);
      rows += hg.nt;
      nnz += (int64_t)hg.col.size();
    }
    if (rows >= (int64_t)INT32_MAX) { g_thread_error = "too many rows in the batch"; return IRLS_ERR_RANGE; }
    // largest graphs first, so the longest solves start first
    std::vector<int32_t> order(G);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
      int64_t wx = graphs[x].nt + (int64_t)(x + 1 < G ? graphs[x + 1].nnz0 : nnz) - graphs[x].nnz0;
      int64_t wy = graphs[y].nt + (int64_t)(y + 1 < G ? graphs[y + 1].nnz0 : nnz) - graphs[y].nnz0;
      return wx > wy;
    });
    h = new irls_mincut_s();
    h->opt = o;
    h->stream = (hipStream_t)hip_stream;
    h->batch = true;
    h->G = G;
    h->solver = 2;
    h->hgraphs = graphs;
    h->D0s = D0s;
    h->nodes_total = node_off[G];
    GraphDev &gd = h->g;
    gd.n = node_off[G];
    gd.nt = rows;
    gd.nnz = nnz;
    gd.format = 1;
    // as many workgroups as can be resident at once (the kernel's registers
    // allow one 1024-thread workgroup per CU), each taking graphs from the
    // queue until it is empty
    int cus = 256, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    h->grid_res = std::max(1, std::min(G, resident_blocks_per_cu() * cus));
    h->grid = grid_for(rows);
    if ((rc = upload(h, &gd.rowptr, rowptr)) != IRLS_OK || (rc = upload(h, &gd.col, col)) != IRLS_OK ||
        (rc = upload(h, &gd.ccap, ccap)) != IRLS_OK || (rc = upload(h, &gd.cs, cs)) != IRLS_OK ||
        (rc = upload(h, &gd.ct, ct)) != IRLS_OK || (rc = upload(h, &h->rgraphs, graphs)) != IRLS_OK ||
        (rc = upload(h, &h->rorder, order)) != IRLS_OK || (rc = upload(h, &h->gid, gid)) != IRLS_OK ||
        (rc = upload_heavy(h, heavy)) != IRLS_OK || (rc = alloc_state(h)) != IRLS_OK) {
      g_thread_error = h->err;
      h->release();
      delete h;
      return rc;
    }
    hipError_t e = h->dalloc(&h->rnext, 1);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      g_thread_error = std::string("batch set-up: ") + hipGetErrorString(e);
      h->release();
      delete h;
      return e == hipErrorOutOfMemory ? IRLS_ERR_OOM : IRLS_ERR_DEVICE;
    }
    *out = h;
    return IRLS_OK;
  } catch (const std::bad_alloc &) {
    if (h) { h->release(); delete h; }
    g_thread_error = "host allocation failed";
    return IRLS_ERR_OOM;
  } catch (...) {
    if (h) { h->release(); delete h; }
    g_thread_error = "unexpected host exception";
    return IRLS_ERR_DEVICE;
  }
}

irls_status irls_mincut_solve_batch(irls_mincut_t h, irls_round_stats *stats) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (!h->batch) { h->err = "not a batch handle"; return IRLS_ERR_OPTIONS; }
  try {
    h->solved = false;
    if (h->opt.init == 1 && h->g.nt > 0) HIPCHK(h, launch_fill(h->v, h->g.nt, 0.5, h->stream), "fill");
    irls_status rc = solve_resident(h, stats);
    if (rc == IRLS_OK || rc == IRLS_WARN_CG_MAXIT) h->solved = true;
    return rc;
  } catch (...) {
    h->err = "unexpected host exception";
    return IRLS_ERR_DEVICE;
  }
}

irls_status irls_mincut_cut_batch(irls_mincut_t h, uint8_t *in_source_side, double *cut_values) {
  if (!h) { g_thread_error = "handle must not be NULL"; return IRLS_ERR_NULL; }
  if (!h->batch) { h->err = "not a batch handle"; return IRLS_ERR_OPTIONS; }
  if (!h->solved) { h->err = "no potentials yet: call irls_mincut_solve_batch first"; return IRLS_ERR_NOT_SOLVED; }
  try {
    const int64_t rows = h->g.nt;
    SweepBufs &b = h->sw;
    if (!h->swb.kstar) {
      const size_t nb = sweep_sort_blocks(rows), sb = sweep_scan_blocks(rows);
      HIPCHK(h, h->dalloc(&b.keyA, rows), "alloc");
      HIPCHK(h, h->dalloc(&b.keyB, rows), "alloc");
      HIPCHK(h, h->dalloc(&b.idA, rows), "alloc");
      HIPCHK(h, h->dalloc(&b.idB, rows), "alloc");
      HIPCHK(h, h->dalloc(&b.rank, rows), "alloc");
      HIPCHK(h, h->dalloc(&b.delta, rows), "alloc");
      HIPCHK(h, h->dalloc(&b.hist, 256 * nb + 256), "alloc");   // counts, then the 256 digit totals
      HIPCHK(h, h->dalloc(&b.bsum, sb), "alloc");
      HIPCHK(h, h->dalloc(&h->swb.best, h->G), "alloc");
      HIPCHK(h, h->dalloc(&h->swb.mask, h->nodes_total), "alloc");
      HIPCHK(h, h->dalloc(&h->swb.kstar, h->G), "alloc");
    }
    SweepBatchArgs a;
    a.G = h->G;
    a.rows = rows;
    a.graphs = h->rgraphs;
    a.gid = h->gid;
    a.v = h->v;
    a.rowptr = h->g.rowptr;
    a.col = h->g.col;
    a.ccap = h->g.ccap;
    a.cs = h->g.cs;
    a.ct = h->g.ct;
    HIPCHK(h, sweep_batch_run(a, b, h->swb, h->stream), "batched sweep");
    std::vector<i128> best(h->G);
    HIPCHK(h, hipMemcpyAsync(best.data(), h->swb.best, h->G * sizeof(i128), hipMemcpyDeviceToHost, h->stream), "readback");
    if (in_source_side)
      HIPCHK(h, hipMemcpyAsync(in_source_side, h->swb.mask, h->nodes_total, hipMemcpyDeviceToHost, h->stream), "readback");
    HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
    if (cut_values)
      for (int32_t g = 0; g < h->G; g++) cut_values[g] = fx_to_double(h->D0s[g] + best[g], h->hgraphs[g].fx_k);
    return IRLS_OK;
  } catch (...) {
    h->err = "unexpected host exception";
    return IRLS_ERR_DEVICE;
  }
}

}  // extern "C"
