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

__device__ __forceinline__ double res_cond(double c, double d, double eps, int form, bool round0) {
  return round0 ? c : conductance<double>(c, d, eps, form);
}

__global__ __launch_bounds__(kResBlock) void k_resident(ResidentArgs a) {
  __shared__ double lds[8 * (kResBlock / 64)];
  __shared__ double bc[8];
  __shared__ int gsh;
  const int tid = threadIdx.x, bd = blockDim.x;
  for (;;) {
    if (tid == 0) gsh = (int)atomicAdd(a.next_graph, 1u);
    __syncthreads();
    const int gi = gsh;
    __syncthreads();
    if (gi >= a.G) return;
    const int g = a.order[gi];
    const BatchGraph gr = a.graphs[g];
    const int64_t nt = gr.nt;
    const int32_t *rp = a.rowptr + gr.node0 + g;
    const int32_t *col = a.col + gr.nnz0;
    const double *cc = a.ccap + gr.nnz0;
    double *w = a.w + gr.nnz0;
    const double *cs = a.cs + gr.node0, *ct = a.ct + gr.node0;
    double *D = a.D + gr.node0, *b = a.b + gr.node0, *gtv = a.gt + gr.node0;
    double *v = a.v + gr.node0, *r = a.r + gr.node0, *p = a.p + gr.node0, *q = a.q + gr.node0;
    irls_round_stats *st = a.stats + (int64_t)g * (a.rounds + 1);
    // lane groups: gr.lanes lanes per row, 64 / lanes rows per wavefront
    const int L = gr.lanes, lane = tid & 63, sub = lane / L, lid = lane % L;
    const int64_t rpw = 64 / L, wstep = (int64_t)(bd >> 6) * rpw;
    double eps = a.eps0;
    for (int l = 0; l <= a.rounds; l++) {
      const bool round0 = l == 0;
      const double eps_l = round0 ? 0.0 : eps;
      const double eps_next = round0 ? a.eps0 : eps * a.eps_factor;
      // Step 1: conductances and the reduced system of this round (a lane
      // group per row, so high-degree rows are spread over L lanes)
      for (int64_t r0 = (int64_t)(tid >> 6) * rpw; r0 < nt; r0 += wstep) {
        const int64_t i = r0 + sub;
        double diag = 0.0, vi = 0.0;
        if (i < nt) {
          vi = v[i];
          for (int32_t e = rp[i] + lid; e < rp[i + 1]; e += L) {
            double gval = res_cond(cc[e], vi - v[col[e]], eps_l, a.form, round0);
            w[e] = gval;
            diag += gval;
          }
        }
        for (int o = L >> 1; o > 0; o >>= 1) diag += __shfl_xor(diag, o, 64);
        if (i < nt && lid == 0) {
          double gs = cs[i] > 0.0 ? res_cond(cs[i], 1.0 - vi, eps_l, a.form, round0) : 0.0;
          double gt = ct[i] > 0.0 ? res_cond(ct[i], vi, eps_l, a.form, round0) : 0.0;
          D[i] = diag + gs + gt;
          b[i] = gs;
          gtv[i] = gt;
        }
      }
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
        for (int64_t r0 = (int64_t)(tid >> 6) * rpw; r0 < nt; r0 += wstep) {
          const int64_t i = r0 + sub;
          double off = 0.0;
          if (warm && i < nt)
            for (int32_t e = rp[i] + lid; e < rp[i + 1]; e += L) off += w[e] * v[col[e]];
          for (int o = L >> 1; o > 0; o >>= 1) off += __shfl_xor(off, o, 64);
          if (i < nt && lid == 0) {
            const double ri = warm ? b[i] - (D[i] * v[i] - off) : b[i];
            r[i] = ri;
            const double zi = ri / D[i];
            p[i] = zi;
            x3[0] += ri * zi;
            x3[1] += b[i] * b[i];
            x3[2] += ri * ri;
          }
        }
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
          for (int64_t r0 = (int64_t)(tid >> 6) * rpw; r0 < nt; r0 += wstep) {
            const int64_t i = r0 + sub;
            double acc = 0.0;
            if (i < nt)
              for (int32_t e = rp[i] + lid; e < rp[i + 1]; e += L) acc += w[e] * p[col[e]];
            for (int o = L >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (i < nt && lid == 0) {
              const double qi = D[i] * p[i] - acc;
              q[i] = qi;
              x1[0] += p[i] * qi;
            }
          }
          block_allreduce<1>(x1, lds, bc);
          const double pq = x1[0];
          if (!(pq > 0.0) || !isfinite(pq)) { status = IRLS_ERR_CG_BREAKDOWN; break; }
          const double alpha = rho / pq;
          double x2[2] = {0.0, 0.0};
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
          for (int64_t i = tid; i < nt; i += bd) p[i] = r[i] / D[i] + beta * p[i];
          __syncthreads();
        }
      }
      __syncthreads();
      // diagnostics of this round
      double x[8] = {0, 0, 0, 0, 0, 0, -INFINITY, -INFINITY};
      for (int64_t r0 = (int64_t)(tid >> 6) * rpw; r0 < nt; r0 += wstep) {
        const int64_t i = r0 + sub;
        const double vi = i < nt ? v[i] : 0.0;
        double off = 0.0, e0 = 0.0, e1 = 0.0, e2 = 0.0;
        if (i < nt) {
          for (int32_t e = rp[i] + lid; e < rp[i + 1]; e += L) {
            const int32_t j = col[e];
            off += w[e] * v[j];
            if (j <= i) continue;
            double c = cc[e], d = vi - v[j];
            e0 += a.form == 0 ? c * sqrt(d * d + eps_next) : sqrt((c * d) * (c * d) + eps_next);
            e1 += c * fabs(d);
            e2 += w[e] * d * d;
          }
        }
        for (int o = L >> 1; o > 0; o >>= 1) {
          off += __shfl_xor(off, o, 64);
          e0 += __shfl_xor(e0, o, 64);
          e1 += __shfl_xor(e1, o, 64);
          e2 += __shfl_xor(e2, o, 64);
        }
        if (i >= nt || lid != 0) continue;
        const double acc = D[i] * vi - off;
        x[0] += e0;
        x[1] += e1;
        x[2] += e2;
        if (cs[i] > 0.0) {
          double c = cs[i], d = 1.0 - vi;
          x[0] += a.form == 0 ? c * sqrt(d * d + eps_next) : sqrt((c * d) * (c * d) + eps_next);
          x[1] += c * fabs(d);
          x[2] += b[i] * d * d;
          x[3] += b[i] * d;
        }
        if (ct[i] > 0.0) {
          double c = ct[i], d = vi;
          x[0] += a.form == 0 ? c * sqrt(d * d + eps_next) : sqrt((c * d) * (c * d) + eps_next);
          x[1] += c * fabs(d);
          x[2] += gtv[i] * d * d;
          x[4] += gtv[i] * d;
        }
        double res = b[i] - acc;
        x[5] += res * res;
        x[6] = fmax(x[6], -vi);
        x[7] = fmax(x[7], vi);
      }
      block_reduce<8, 0xC0u>(x, lds);
      if (tid == 0) {
        double gst = 0.0, sst = 0.0;
        if (gr.cst > 0.0) {
          gst = res_cond(gr.cst, 1.0, eps_l, a.form, round0);
          sst = a.form == 0 ? gr.cst * sqrt(1.0 + eps_next) : sqrt(gr.cst * gr.cst + eps_next);
        }
        irls_round_stats R;
        R.eps = eps_l;
        R.cg_iters = iters;
        R.rel_res = bb > 0.0 ? sqrt(rr / bb) : 0.0;
        R.true_rel_res = bb > 0.0 ? sqrt(x[5] / bb) : 0.0;
        R.s_eps = x[0] + sst;
        R.l1 = x[1] + gr.cst;
        R.flow = x[2] + gst;
        R.flow_s = x[3] + gst;
        R.flow_t = x[4] + gst;
        R.vmin = nt > 0 ? -x[6] : 0.0;
        R.vmax = nt > 0 ? x[7] : 0.0;
        R.status = status;
        st[l] = R;
      }
      __syncthreads();
      if (status == IRLS_ERR_CG_BREAKDOWN) break;
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
    z.vmin = z.vmax = 0.0;
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

hipError_t launch_resident(const ResidentArgs &a, int grid, int block, hipStream_t st) {
  hipLaunchKernelGGL(k_resident, dim3(grid), dim3(block), 0, st, a);
  return hipGetLastError();
}

}  // namespace irls
