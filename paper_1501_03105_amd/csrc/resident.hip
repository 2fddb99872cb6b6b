// Resident IRLS solver: one workgroup of 1024 threads owns one graph and runs
// all of its rounds (reweight, Jacobi-PCG, diagnostics) inside one launch,
// synchronising with workgroup barriers only.  Workgroups take graphs from an
// atomic work queue (largest first), so one persistent launch solves a whole
// batch of independent graphs of uneven size.  The arithmetic follows the
// multi-workgroup kernels: Section 2.1 Steps 1-2 with round 0 at W = C, Jacobi
// PCG warm-started from the previous round (Section 3.1).
#include "device_common.h"

namespace irls {

constexpr int kResBlock = 1024;
constexpr int kResWaves = kResBlock / 64;

__device__ __forceinline__ double res_cond(double c, double d, double eps, int form, bool round0) {
  return round0 ? c : conductance<double>(c, d, eps, form);
}

// The rows of the graph a workgroup owns, and how its passes walk them.
struct ResRows {
  int64_t nt;
  int32_t nnz;                        // CSR entries of the graph
  const int32_t *col;
  const int32_t *brow, *bbeg, *bend;  // light rows by length bin: row, entry range
  const int32_t *bin;                 // [kBins + 1] bin boundaries (the graph's record)
  const int32_t *crow, *cbeg, *cend, *hrow, *hc0, *hc1;
  int32_t nchunks, nheavy;
  uint32_t lane_code;                 // log2 of the lanes per light row of bin b at bits 3b..3b+2
  double *cpart;
};

// Lanes per row of bin b are 2^lg (lg from the lane code, uniform across the
// workgroup); a row of the bin has at most bin_max(b) entries, so a lane
// takes at most bin_max(b) / 2^lg of them.
__device__ __forceinline__ int bin_lg(const ResRows &R, int b) { return (int)((R.lane_code >> (3 * b)) & 7u); }
__device__ __forceinline__ constexpr int bin_max(int b) { return b == kBins - 1 ? kHeavyRow : (2 << b); }

// Heavy rows of a pass: their 64-entry chunks spread over the wavefronts,
// each reduced across the wavefront, then after a barrier one wavefront per
// heavy row adds its chunk sums in a fixed order.
template <int NQ, typename F, typename Fin>
__device__ __forceinline__ void heavy_pass(const ResRows &R, F f, Fin fin) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll 1
  for (int32_t c = wid; c < R.nchunks; c += kResWaves) {
    const int64_t i = R.crow[c];
    const int32_t e = R.cbeg[c] + lane;
    double s[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) s[q] = 0.0;
    if (e < R.cend[c]) f(i, e, s);
#pragma unroll
    for (int q = 0; q < NQ; q++)
      for (int o = 32; o > 0; o >>= 1) s[q] += __shfl_xor(s[q], o, 64);
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < NQ; q++) R.cpart[(int64_t)c * kChunkQ + q] = s[q];
  }
  __syncthreads();
#pragma unroll 1
  for (int32_t hh = wid; hh < R.nheavy; hh += kResWaves) {
    const int64_t i = R.hrow[hh];
    double s[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) s[q] = 0.0;
#pragma unroll 1
    for (int32_t c = R.hc0[hh] + lane; c < R.hc1[hh]; c += 64)
#pragma unroll
      for (int q = 0; q < NQ; q++) s[q] += R.cpart[(int64_t)c * kChunkQ + q];
#pragma unroll
    for (int q = 0; q < NQ; q++)
      for (int o = 32; o > 0; o >>= 1) s[q] += __shfl_xor(s[q], o, 64);
    if (lane == 0) fin(i, s);
  }
}

// One pass of per-row sums over the CSR entries: f(i, e, s) adds entry e of
// row i into s[0..NQ); fin(i, s) receives each row's totals once, on one
// lane.  Light rows go by length bin, a group of 2^bin_lg(b) lanes per row;
// heavy rows by chunks.  Deterministic: no atomics.  Every thread of the
// workgroup must call it; the caller puts a barrier between two passes.
template <int NQ, typename F, typename Fin>
__device__ __forceinline__ void rows_pass(const ResRows &R, F f, Fin fin) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll 1
  for (int b = 0; b < kBins; b++) {
    const int lg = bin_lg(R, b), L = 1 << lg, rpw = 64 >> lg, sub = lane >> lg, lid = lane & (L - 1);
    const int32_t hi = R.bin[b + 1];
#pragma unroll 1
    for (int32_t j0 = R.bin[b] + wid * rpw; j0 < hi; j0 += kResWaves * rpw) {
      const int32_t j = j0 + sub;
      double s[NQ];
#pragma unroll
      for (int q = 0; q < NQ; q++) s[q] = 0.0;
      int64_t i = 0;
      if (j < hi) {
        i = R.brow[j];
        const int32_t e1 = R.bend[j];
        for (int32_t e = R.bbeg[j] + lid; e < e1; e += L) f(i, e, s);
      }
      for (int o = L >> 1; o > 0; o >>= 1)
#pragma unroll
        for (int q = 0; q < NQ; q++) s[q] += __shfl_xor(s[q], o, 64);
      if (j < hi && lid == 0) fin(i, s);
    }
  }
  if (R.nheavy > 0) heavy_pass<NQ>(R, f, fin);       // the same for the whole workgroup
}

// The CG loop's SpMV, q = D p - W p and the partial sums of p^T q, with the
// same row assignment and summation order as rows_pass, but with kSpmvRows
// row groups (light) or chunks (heavy) per wavefront in flight at once: their
// index and value loads are issued together (out-of-range lanes read entry 0
// and add nothing), so one workgroup keeps enough loads in flight for large
// graphs.  Two groups per pass measured faster than four on the 512-graph
// R-MAT batch: four need more registers than a 1024-thread workgroup allows
// and spill.
constexpr int kSpmvRows = 2;

__device__ __forceinline__ void spmv_pass(const ResRows &R, const double *w, const double *p, const double *D,
                                          double *q, double &x1) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  constexpr int U = kSpmvRows;
#pragma unroll 1
  for (int b = 0; b < kBins; b++) {
    const int lg = bin_lg(R, b), L = 1 << lg, rpw = 64 >> lg, sub = lane >> lg, lid = lane & (L - 1);
    const int steps = R.nnz > 0 ? bin_max(b) >> lg : 0;           // entry 0 must exist
    const int32_t hi = R.bin[b + 1];
    const int32_t step = kResWaves * rpw;
    // The next row groups' (row, entry range) triples are loaded one pass
    // ahead, and each row's own D and p with its entries, so a pass waits for
    // two dependent round trips (entries, then the gathered p) instead of four.
    int64_t i[U], in[U];
    int32_t e0[U], e1[U], e0n[U], e1n[U];
    auto meta = [&](int32_t j0, int64_t *ii, int32_t *b0, int32_t *b1) {
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int32_t j = j0 + u * step + sub;
        const bool ok = j < hi;
        ii[u] = ok ? R.brow[j] : 0;
        b0[u] = ok ? R.bbeg[j] : 0;
        b1[u] = ok ? R.bend[j] : 0;
      }
    };
    int32_t j0 = R.bin[b] + wid * rpw;
    if (j0 < hi) meta(j0, in, e0n, e1n);
#pragma unroll 1
    for (; j0 < hi; j0 += U * step) {
#pragma unroll
      for (int u = 0; u < U; u++) { i[u] = in[u]; e0[u] = e0n[u]; e1[u] = e1n[u]; }
      double acc[U], dii[U], pii[U];
#pragma unroll
      for (int u = 0; u < U; u++) acc[u] = 0.0;
#pragma unroll 1
      for (int t = 0; t < steps; t++) {
        int32_t c[U];
        double wv[U], pv[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
          const int32_t e = e0[u] + lid + t * L;
          ok[u] = e < e1[u];
          const int32_t ee = ok[u] ? e : 0;
          c[u] = R.col[ee];
          wv[u] = w[ee];
        }
        if (t == 0) {
          if (j0 + U * step < hi) meta(j0 + U * step, in, e0n, e1n);
#pragma unroll
          for (int u = 0; u < U; u++) { dii[u] = D[i[u]]; pii[u] = p[i[u]]; }
        }
#pragma unroll
        for (int u = 0; u < U; u++) pv[u] = p[c[u]];
#pragma unroll
        for (int u = 0; u < U; u++)
          if (ok[u]) acc[u] += wv[u] * pv[u];
      }
      if (R.nnz == 0) {
#pragma unroll
        for (int u = 0; u < U; u++) { dii[u] = D[i[u]]; pii[u] = p[i[u]]; }
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        for (int o = L >> 1; o > 0; o >>= 1) acc[u] += __shfl_xor(acc[u], o, 64);
        if (j0 + u * step + sub < hi && lid == 0) {
          const double qi = dii[u] * pii[u] - acc[u];
          q[i[u]] = qi;
          x1 += pii[u] * qi;
        }
      }
    }
  }
  if (R.nheavy > 0) {                                // the same for the whole workgroup
#pragma unroll 1
    for (int32_t c0 = wid; c0 < R.nchunks; c0 += U * kResWaves) {
      bool ok[U];
      int32_t c[U];
      double wv[U], pv[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int32_t cu = c0 + u * kResWaves;
        const bool valid = cu < R.nchunks;
        const int32_t ee0 = valid ? R.cbeg[cu] + lane : 0;
        ok[u] = valid && ee0 < R.cend[cu];
        const int32_t ee = ok[u] ? ee0 : 0;
        c[u] = R.col[ee];
        wv[u] = w[ee];
      }
#pragma unroll
      for (int u = 0; u < U; u++) pv[u] = p[c[u]];
#pragma unroll
      for (int u = 0; u < U; u++) {
        double sum = ok[u] ? wv[u] * pv[u] : 0.0;
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        const int32_t cu = c0 + u * kResWaves;
        if (lane == 0 && cu < R.nchunks) R.cpart[(int64_t)cu * kChunkQ] = sum;
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int32_t hh = wid; hh < R.nheavy; hh += kResWaves) {
      const int64_t i = R.hrow[hh];
      double sum = 0.0;
#pragma unroll 1
      for (int32_t c = R.hc0[hh] + lane; c < R.hc1[hh]; c += 64) sum += R.cpart[(int64_t)c * kChunkQ];
      for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
      if (lane == 0) {
        const double qi = D[i] * p[i] - sum;
        q[i] = qi;
        x1 += p[i] * qi;
      }
    }
  }
}

__global__ __launch_bounds__(kResBlock) void k_resident(ResidentArgs a) {
  __shared__ double lds[11 * (kResBlock / 64)];
  __shared__ double bc[11];
  __shared__ int gsh, stop_sh;
  const int tid = threadIdx.x, bd = blockDim.x;
  for (;;) {
    if (tid == 0) gsh = (int)atomicAdd(a.next_graph, 1u);
    __syncthreads();
    // uniform across the workgroup: readfirstlane lets the compiler keep the
    // graph's record and every pointer derived from it in scalar registers
    const int gi = __builtin_amdgcn_readfirstlane(gsh);
    __syncthreads();
    if (gi >= a.G) return;
    const int g = __builtin_amdgcn_readfirstlane(a.order[gi]);
    const BatchGraph gr = a.graphs[g];
    const int64_t nt = gr.nt;
    const int32_t *col = a.col + gr.nnz0;
    const double *cc = a.ccap + gr.nnz0;
    double *w = a.w + gr.nnz0;
    const double *cs = a.cs + gr.node0, *ct = a.ct + gr.node0;
    double *D = a.D + gr.node0, *b = a.b + gr.node0, *gtv = a.gt + gr.node0;
    double *v = a.v + gr.node0, *r = a.r + gr.node0, *p = a.p + gr.node0, *q = a.q + gr.node0;
    irls_round_stats *st = a.stats + (int64_t)g * (a.rounds + 1);
    ResRows R;
    R.nt = nt;
    R.nnz = gr.nnz;
    R.col = col;
    R.brow = a.bin_row + gr.node0;
    R.bbeg = a.bin_beg + gr.node0;
    R.bend = a.bin_end + gr.node0;
    R.bin = a.graphs[g].bin;
    R.crow = a.chunk_row + gr.chunk0;
    R.cbeg = a.chunk_beg + gr.chunk0;
    R.cend = a.chunk_end + gr.chunk0;
    R.hrow = a.heavy_row + gr.heavy0;
    R.hc0 = a.heavy_c0 + gr.heavy0;
    R.hc1 = a.heavy_c1 + gr.heavy0;
    R.nchunks = gr.nchunks;
    R.nheavy = gr.nheavy;
    R.lane_code = a.lane_code;
    R.cpart = a.chunk_part + gr.chunk0 * kChunkQ;
    double eps = a.eps0;
    for (int l = 0; l <= a.rounds; l++) {
      const bool round0 = l == 0;
      const double eps_l = round0 ? 0.0 : eps;
      const double eps_next = round0 ? a.eps0 : eps * a.eps_factor;
      // Step 1: conductances and the reduced system of this round
      rows_pass<1>(
          R,
          [&](int64_t i, int32_t e, auto &s) {
            const double gval = res_cond(cc[e], v[i] - v[col[e]], eps_l, a.form, round0);
            w[e] = gval;
            s[0] += gval;
          },
          [&](int64_t i, const auto &s) {
            const double vi = v[i];
            const double gs = cs[i] > 0.0 ? res_cond(cs[i], 1.0 - vi, eps_l, a.form, round0) : 0.0;
            const double gt = ct[i] > 0.0 ? res_cond(ct[i], vi, eps_l, a.form, round0) : 0.0;
            D[i] = s[0] + gs + gt;
            b[i] = gs;
            gtv[i] = gt;
          });
      __syncthreads();
      int64_t iters = 0;
      int status = IRLS_OK;
      double bb = 0.0, rr = 0.0;
      bool solve = !(round0 && a.init != 0);
      if (solve && gr.no_source_edges) {
        for (int64_t i = tid; i < nt; i += bd) v[i] = 0.0;
        solve = false;
      }
      if (solve) {
        // Step 2: Jacobi PCG on L~ v = b
        const bool warm = !round0 && a.warm;
        double x3[3] = {0.0, 0.0, 0.0};
        rows_pass<1>(
            R,
            [&](int64_t i, int32_t e, auto &s) {
              if (warm) s[0] += w[e] * v[col[e]];
            },
            [&](int64_t i, const auto &s) {
              const double ri = warm ? b[i] - (D[i] * v[i] - s[0]) : b[i];
              r[i] = ri;
              const double zi = ri / D[i];
              p[i] = zi;
              x3[0] += ri * zi;
              x3[1] += b[i] * b[i];
              x3[2] += ri * ri;
            });
        __syncthreads();                  // every row has read v before a cold start clears it
        if (!warm)
          for (int64_t i = tid; i < nt; i += bd) v[i] = 0.0;
        block_allreduce<3>(x3, lds, bc);
        double rho = x3[0];
        bb = x3[1];
        rr = x3[2];
        const double thr = a.rtol * sqrt(bb);
        bool done = sqrt(rr) <= thr;
        if (!isfinite(rho) || !isfinite(rr)) { status = IRLS_ERR_CG_BREAKDOWN; done = true; }
        while (!done) {
          double x1[1] = {0.0};
          spmv_pass(R, w, p, D, q, x1[0]);
          block_allreduce<1>(x1, lds, bc);
          const double pq = x1[0];
          if (!(pq > 0.0) || !isfinite(pq)) { status = IRLS_ERR_CG_BREAKDOWN; break; }
          const double alpha = rho / pq;
          double x2[2] = {0.0, 0.0};
#pragma unroll 4
          for (int64_t i = tid; i < nt; i += bd) {
            v[i] += alpha * p[i];
            double ri = r[i] - alpha * q[i];
            r[i] = ri;
            double zi = ri / D[i];
            x2[0] += ri * zi;
            x2[1] += ri * ri;
          }
          block_allreduce<2>(x2, lds, bc);
          iters++;
          rr = x2[1];
          if (!isfinite(x2[0]) || !isfinite(rr)) { status = IRLS_ERR_CG_BREAKDOWN; break; }
          if (sqrt(rr) <= thr) break;
          if (iters >= a.maxit) { status = IRLS_WARN_CG_MAXIT; break; }
          const double beta = x2[0] / rho;
          rho = x2[0];
#pragma unroll 4
          for (int64_t i = tid; i < nt; i += bd) p[i] = r[i] / D[i] + beta * p[i];
          __syncthreads();
        }
      }
      __syncthreads();
      // diagnostics of this round: x^T L x's off-diagonal part and, once per
      // edge (j > i), the smoothed objective, ||C B x||_1 and sum w d^2; for
      // the lower bound the largest w |d| / c, the overload max(0, w|d| - c)
      // and ||r||_1 (kept per thread, then reduced over the workgroup)
      double x[11] = {0, 0, 0, 0, 0, 0, -INFINITY, -INFINITY, 0, 0, 0};
      rows_pass<4>(
          R,
          [&](int64_t i, int32_t e, auto &s) {
            const int32_t j = col[e];
            const double vj = v[j];
            s[0] += w[e] * vj;
            if (j <= i) return;
            const double c = cc[e], d = v[i] - vj;
            s[1] += a.form == 0 ? c * sqrt(d * d + eps_next) : sqrt((c * d) * (c * d) + eps_next);
            s[2] += c * fabs(d);
            s[3] += w[e] * d * d;
            x[8] = fmax(x[8], w[e] * fabs(d) / c);
            x[9] += fmax(0.0, w[e] * fabs(d) - c);
          },
          [&](int64_t i, const auto &s) {
            const double vi = v[i];
            const double acc = D[i] * vi - s[0];
            x[0] += s[1];
            x[1] += s[2];
            x[2] += s[3];
            if (cs[i] > 0.0) {
              double c = cs[i], d = 1.0 - vi;
              x[0] += a.form == 0 ? c * sqrt(d * d + eps_next) : sqrt((c * d) * (c * d) + eps_next);
              x[1] += c * fabs(d);
              x[2] += b[i] * d * d;
              x[3] += b[i] * d;
              x[8] = fmax(x[8], b[i] * fabs(d) / c);
              x[9] += fmax(0.0, b[i] * fabs(d) - c);
            }
            if (ct[i] > 0.0) {
              double c = ct[i], d = vi;
              x[0] += a.form == 0 ? c * sqrt(d * d + eps_next) : sqrt((c * d) * (c * d) + eps_next);
              x[1] += c * fabs(d);
              x[2] += gtv[i] * d * d;
              x[4] += gtv[i] * d;
              x[8] = fmax(x[8], gtv[i] * fabs(d) / c);
              x[9] += fmax(0.0, gtv[i] * fabs(d) - c);
            }
            double res = b[i] - acc;
            x[5] += res * res;
            x[10] += fabs(res);
            x[6] = fmax(x[6], -vi);
            x[7] = fmax(x[7], vi);
          });
      block_reduce<11, 0x1C0u>(x, lds);
      if (tid == 0) {
        double gst = 0.0, sst = 0.0;
        if (gr.cst > 0.0) {
          gst = res_cond(gr.cst, 1.0, eps_l, a.form, round0);
          sst = a.form == 0 ? gr.cst * sqrt(1.0 + eps_next) : sqrt(gr.cst * gr.cst + eps_next);
        }
        irls_round_stats RS;
        RS.eps = eps_l;
        RS.cg_iters = iters;
        RS.rel_res = bb > 0.0 ? sqrt(rr / bb) : 0.0;
        RS.true_rel_res = bb > 0.0 ? sqrt(x[5] / bb) : 0.0;
        RS.s_eps = x[0] + sst;
        RS.l1 = x[1] + gr.cst;
        RS.flow = x[2] + gst;
        RS.flow_s = x[3] + gst;
        RS.flow_t = x[4] + gst;
        RS.vmin = nt > 0 ? -x[6] : 0.0;
        RS.vmax = nt > 0 ? x[7] : 0.0;
        RS.status = status;
        // lower bound on the minimum cut (as in the multi-workgroup stats)
        const double rho = gr.cst > 0.0 ? fmax(x[8], gst / gr.cst) : x[8];
        const double over = x[9] + (gr.cst > 0.0 ? fmax(0.0, gst - gr.cst) : 0.0);
        const double F = fmax(RS.flow_s, RS.flow_t) - x[10];
        RS.lower_bound = fmax(F / fmax(1.0, rho), F - over);
        st[l] = RS;
        stop_sh = a.stop_gap > 0.0 && RS.l1 - RS.lower_bound <= a.stop_gap * RS.l1;
      }
      __syncthreads();
      if (status == IRLS_ERR_CG_BREAKDOWN || stop_sh) break;
      if (!round0) eps *= a.eps_factor;
    }
  }
}

// clears the work queue and the per-round records before a batched solve
// (plain stores, so the launch can live inside a captured HIP graph)
__global__ void k_resident_reset(unsigned *next_graph, irls_round_stats *st, int64_t nrec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *next_graph = 0u;
  if (i < nrec) {
    irls_round_stats z;
    z.eps = z.rel_res = z.true_rel_res = z.s_eps = z.l1 = z.flow = z.flow_s = z.flow_t = 0.0;
    z.vmin = z.vmax = z.lower_bound = 0.0;
    z.cg_iters = 0;
    z.status = 0;
    st[i] = z;
  }
}

hipError_t launch_resident_reset(unsigned *next_graph, irls_round_stats *st, int64_t nrec, hipStream_t s) {
  const int64_t blocks = (nrec + 255) / 256;
  hipLaunchKernelGGL(k_resident_reset, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, s,
                     next_graph, st, nrec);
  return hipGetLastError();
}

int resident_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_resident, kResBlock, 0) != hipSuccess || n < 1) return 1;
  return n;
}

hipError_t launch_resident(const ResidentArgs &a, int grid, int block, hipStream_t st) {
  hipLaunchKernelGGL(k_resident, dim3(grid), dim3(block), 0, st, a);
  return hipGetLastError();
}

}  // namespace irls
