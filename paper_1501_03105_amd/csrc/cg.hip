// IRLS round kernels for gfx950: reweighting + assembly of the reduced
// Laplacian, and the Jacobi-PCG phases (Section 2.1 Steps 1-2, Section 3.1).
//
// Two storage formats of the reduced Laplacian L~ (rows = non-terminal nodes):
//   * diagonal format: the interior edges use only K distinct row offsets
//     (grids: 1, nx, nx*ny).  Each row stores the conductance of its edges to
//     row u+off[k]; the edge to u-off[k] is read from row u-off[k].  No column
//     indices are stored and every access is unit-stride.
//   * CSR: any graph; rows-per-wavefront chosen per graph.
// Vectors are FP64 (precision 0) or FP32 with FP64 potentials (precision 1).
#include "device_common.h"

namespace irls {

// ----------------------------------------------------------------------------
// neighbour visitor: f(j, capacity, index of the stored conductance)
// ----------------------------------------------------------------------------
template <bool DIA, typename T, typename Fn>
__device__ __forceinline__ void for_each_nb(const CGArgs<T> &a, int64_t u, Fn f) {
  if constexpr (DIA) {
    for (int k = 0; k < a.K; k++) {
      int64_t j = u + a.off[k];
      if (j < a.nt) {
        double c = a.dcap[k * a.nt + u];
        if (c > 0.0) f(j, c, k * a.nt + u);
      }
      j = u - a.off[k];
      if (j >= 0) {
        double c = a.dcap[k * a.nt + j];
        if (c > 0.0) f(j, c, k * a.nt + j);
      }
    }
  } else {
    for (int32_t e = a.rowptr[u]; e < a.rowptr[u + 1]; e++) f((int64_t)a.col[e], a.ccap[e], (int64_t)e);
  }
}

template <typename T>
__device__ __forceinline__ double edge_g(const CGArgs<T> &a, double c, double d) {
  if (a.round0) return c;
  if (a.weights_fp64) return conductance<double>(c, d, a.eps, a.form);
  return (double)conductance<float>((float)c, (float)d, (float)a.eps, a.form);
}

// ----------------------------------------------------------------------------
// reweight + assemble: conductances, D, b (= conductance to s), conductance to t
// ----------------------------------------------------------------------------
template <typename T, bool DIA>
__global__ __launch_bounds__(kBlock) void k_assemble(CGArgs<T> a) {
  FOR_ROWS(u, a.nt) {
    const double vu = a.v[u];
    double diag = 0.0;
    if constexpr (DIA) {
      for (int k = 0; k < a.K; k++) {
        int64_t j = u + a.off[k];
        double g = 0.0;
        if (j < a.nt) {
          double c = a.dcap[k * a.nt + u];
          if (c > 0.0) g = edge_g(a, c, vu - a.v[j]);
        }
        a.w[k * a.nt + u] = (T)g;
        if (a.w64) a.w64[k * a.nt + u] = g;
        diag += g;
        j = u - a.off[k];
        if (j >= 0) {
          double c = a.dcap[k * a.nt + j];
          if (c > 0.0) diag += edge_g(a, c, a.v[j] - vu);   // same value row j stores
        }
      }
    } else {
      for (int32_t e = a.rowptr[u]; e < a.rowptr[u + 1]; e++) {
        double g = edge_g(a, a.ccap[e], vu - a.v[a.col[e]]);
        a.w[e] = (T)g;
        if (a.w64) a.w64[e] = g;
        diag += g;
      }
    }
    double cs = a.cs[u], ct = a.ct[u];
    double gs = cs > 0.0 ? edge_g(a, cs, 1.0 - vu) : 0.0;
    double gt = ct > 0.0 ? edge_g(a, ct, vu) : 0.0;
    diag += gs + gt;
    a.D[u] = (T)diag;
    if (a.D64) a.D64[u] = diag;
    a.b[u] = gs;
    a.gt[u] = gt;
  }
}

// (L~ x)_u in FP64 with the FP64 copy of this round's conductances
template <bool DIA, typename T>
__device__ __forceinline__ double row_apply64(const CGArgs<T> &a, int64_t u, const double *x) {
  const double *w = a.w64 ? a.w64 : (const double *)a.w;
  const double *D = a.D64 ? a.D64 : (const double *)a.D;
  double acc = D[u] * x[u];
  for_each_nb<DIA>(a, u, [&](int64_t j, double, int64_t wi) { acc -= w[wi] * x[j]; });
  return acc;
}

// Snapshot of sc->done taken by thread 0, so the whole workgroup takes the
// same early exit.
__device__ __forceinline__ bool block_done(const Scalars *sc) {
  __shared__ int s_done;
  if (threadIdx.x == 0) s_done = sc->done;
  __syncthreads();
  return s_done != 0;
}

__device__ __forceinline__ bool first_thread() { return threadIdx.x == 0 && blockIdx.x == 0; }

// ----------------------------------------------------------------------------
// CG start: r = b - L~ v0 (warm) or r = b, v = 0 (cold); partial sums of
// r^T z, ||b||^2, ||r||^2 for the first direction kernel
// ----------------------------------------------------------------------------
template <typename T, bool DIA>
__global__ __launch_bounds__(kBlock) void k_cginit(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  double x[3] = {0.0, 0.0, 0.0};   // rho, bb, rr
  FOR_ROWS(u, a.nt) {
    double bu = a.b[u];
    double ru;
    if (a.warm) {
      ru = bu - row_apply64<DIA>(a, u, a.v);
    } else {
      a.v[u] = 0.0;
      ru = bu;
    }
    T rt = (T)ru;
    T zt = rt / a.D[u];
    a.z[u] = zt;                               // z = M^-1 r is what CG keeps
    double zu = (double)zt;
    x[0] += (double)rt * zu;
    x[1] += bu * bu;
    x[2] += (double)rt * (double)rt;
  }
  write_partials<3>(x, a.partials, kPInit, lds);
  if (first_thread()) {
    a.sc->iter_b = 0;
    a.sc->iter_a = 0;
    a.sc->done = 0;
    a.sc->status = IRLS_OK;
  }
}

// Start of CG iteration i = iter_b (in the kernel that forms the direction):
// totals of r^T z and ||r||^2 left by the previous kernel (the CG start, the
// vector update, or the FP64 residual replacement), the stopping test, and
// beta = rho_i / rho_{i-1}.  Workgroup 0 publishes the state.  Returns false
// when CG has stopped.
template <typename T>
__device__ bool cg_iteration_start(const CGArgs<T> &a, double *lds, double *bc, int64_t &i_out,
                                   double &beta_out) {
  Scalars *sc = a.sc;
  if (block_done(sc)) return false;
  const int nb = gridDim.x;
  const int64_t i = sc->iter_b;
  double rz, rr, bb;
  if (i == 0) {
    double t3[3];
    read_totals<3>(a.partials, kPInit, nb, t3, lds, bc);
    rz = t3[0]; bb = t3[1]; rr = t3[2];
  } else {
    double t2[2];
    read_totals<2>(a.partials, kPUpd, nb, t2, lds, bc);
    rz = t2[0]; rr = t2[1]; bb = sc->bb;
    if (sc->refine_every > 0) {
      const bool conv_rec = sqrt(rr) <= a.rtol * sqrt(bb);
      if (conv_rec || i % sc->refine_every == 0) {      // the replacement kernel ran
        read_totals<2>(a.partials, kPRep, nb, t2, lds, bc);
        rz = t2[0]; rr = t2[1];
      }
    }
  }
  bool stop = false;
  int status = IRLS_OK;
  if (!isfinite(rz) || !isfinite(rr)) { stop = true; status = IRLS_ERR_CG_BREAKDOWN; }
  else if (sqrt(rr) <= a.rtol * sqrt(bb)) stop = true;
  else if (i >= sc->maxit) { stop = true; status = IRLS_WARN_CG_MAXIT; }
  const double beta = i == 0 ? 0.0 : rz / sc->rho[(i - 1) & 1];
  if (first_thread()) {
    sc->rr = rr;
    if (i == 0) sc->bb = bb;
    if (stop) {
      sc->done = 1;
      sc->status = status;
    } else {
      sc->rho[i & 1] = rz;
      sc->iter_a = i;
      sc->beta = beta;
    }
  }
  i_out = i;
  beta_out = beta;
  return !stop;
}

// ----------------------------------------------------------------------------
// SpMV, diagonal format, with the direction update fused in:
//   p_new = z + beta p_old (z = r / D; p_new = z on the first iteration),
//   q = L~ p_new, and the partial sums of p^T q.  Each row recomputes p_new of
//   its neighbours from r, D, p_old, so p is double-buffered by iteration
//   parity.
// ----------------------------------------------------------------------------
template <typename T, int K>
__global__ __launch_bounds__(kBlock) void k_spmv_dia(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  __shared__ double bc[4];
  int64_t it;
  double beta64;
  if (!cg_iteration_start(a, lds, bc, it, beta64)) return;
  const T beta = (T)beta64;
  const bool first = it == 0;
  const T *__restrict__ pin = (it & 1) ? a.p1 : a.p0;
  T *__restrict__ pout = (it & 1) ? a.p0 : a.p1;
  const T *__restrict__ z = a.z;
  const T *__restrict__ D = a.D;
  const T *__restrict__ w = a.w;
  const int64_t nt = a.nt;
  auto dir = [&](int64_t j) -> T { return first ? z[j] : z[j] + beta * pin[j]; };
  double x[1] = {0.0};
  FOR_ROWS(u, nt) {
    const T pu = dir(u);
    T acc = D[u] * pu;
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int64_t o = a.off[k];
      if (u + o < nt) acc -= w[k * nt + u] * dir(u + o);
      if (u - o >= 0) acc -= w[k * nt + u - o] * dir(u - o);
    }
    pout[u] = pu;
    a.q[u] = acc;
    x[0] += (double)pu * (double)acc;
  }
  write_partials<1>(x, a.partials, kPSpmv, lds);
}

// Vectorised form of k_spmv_dia for grids: each thread owns R consecutive
// rows and moves them with 16-byte loads (R = 2 in FP64, 4 in FP32).  Needs
// off[0] == 1, every other offset and nt divisible by R.  The +-1 neighbours
// inside the group come from registers; the rows just outside it are scalar
// loads that hit in L1 (the neighbouring lanes loaded them).
template <typename T, int R>
using vec_t = T __attribute__((ext_vector_type(R)));

template <typename T, int R>
__device__ __forceinline__ vec_t<T, R> vload(const T *p) { return *reinterpret_cast<const vec_t<T, R> *>(p); }
template <typename T, int R>
__device__ __forceinline__ void vstore(T *p, vec_t<T, R> v) { *reinterpret_cast<vec_t<T, R> *>(p) = v; }

template <typename T, int K, int R>
__global__ __launch_bounds__(kBlock) void k_spmv_dia_vec(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  __shared__ double bc[4];
  typedef vec_t<T, R> V;
  int64_t it;
  double beta64;
  if (!cg_iteration_start(a, lds, bc, it, beta64)) return;
  const T beta = (T)beta64;
  const bool first = it == 0;
  const T *__restrict__ pin = (it & 1) ? a.p1 : a.p0;
  T *__restrict__ pout = (it & 1) ? a.p0 : a.p1;
  const T *__restrict__ z = a.z;
  const T *__restrict__ D = a.D;
  const T *__restrict__ w = a.w;
  const int64_t nt = a.nt, ng = nt / R;
  auto dirv = [&](int64_t u0) -> V {
    V zv = vload<T, R>(z + u0);
    return first ? zv : zv + beta * vload<T, R>(pin + u0);
  };
  auto dirs = [&](int64_t j) -> T { return first ? z[j] : z[j] + beta * pin[j]; };
  double x[1] = {0.0};
  FOR_ROWS(gi, ng) {
    const int64_t u0 = gi * R;
    const V pc = dirv(u0);
    V acc = vload<T, R>(D + u0) * pc;
    // offset 1: edges inside the group, and to the rows just outside it
    {
      const V w0 = vload<T, R>(w + u0);
      const T right = u0 + R < nt ? dirs(u0 + R) : (T)0;
      const T wl = u0 > 0 ? w[u0 - 1] : (T)0;
      const T left = u0 > 0 ? dirs(u0 - 1) : (T)0;
#pragma unroll
      for (int i = 0; i < R; i++) {
        acc[i] -= w0[i] * (i + 1 < R ? pc[i + 1] : right);
        acc[i] -= (i > 0 ? w0[i - 1] : wl) * (i > 0 ? pc[i - 1] : left);
      }
    }
#pragma unroll
    for (int k = 1; k < K; k++) {
      const int64_t o = a.off[k];
      if (u0 + o < nt) acc -= vload<T, R>(w + k * nt + u0) * dirv(u0 + o);
      if (u0 >= o) acc -= vload<T, R>(w + k * nt + u0 - o) * dirv(u0 - o);
    }
    vstore<T, R>(pout + u0, pc);
    vstore<T, R>(a.q + u0, acc);
#pragma unroll
    for (int i = 0; i < R; i++) x[0] += (double)pc[i] * (double)acc[i];
  }
  write_partials<1>(x, a.partials, kPSpmv, lds);
}

// direction update for CSR: p = z + beta p (p = z on the first iteration);
// the CG kernels keep z = r / D in place of r
template <typename T>
__global__ __launch_bounds__(kBlock) void k_direction(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  __shared__ double bc[4];
  int64_t it;
  double beta64;
  if (!cg_iteration_start(a, lds, bc, it, beta64)) return;
  const bool first = it == 0;
  const T beta = (T)beta64;
  FOR_ROWS(u, a.nt) {
    const T zu = a.z[u];
    a.p0[u] = first ? zu : zu + beta * a.p0[u];
  }
}

// SpMV, CSR: L lanes per row (64/L rows per wavefront), q = L~ p and p^T q
template <typename T, int L>
__global__ __launch_bounds__(kBlock) void k_spmv_csr(CGArgs<T> a) {
  __shared__ double lds[1 * (kBlock / 64)];
  if (block_done(a.sc)) return;
  const int lane = threadIdx.x & 63;
  const int sub = lane / L, lid = lane % L;
  constexpr int RPW = 64 / L;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const T *__restrict__ p = a.p0;
  const T *__restrict__ w = a.w;
  const int32_t *__restrict__ col = a.col;
  double x[1] = {0.0};
  for (int64_t r0 = wave * RPW; r0 < a.nt; r0 += nwaves * RPW) {
    const int64_t i = r0 + sub;
    T acc = 0;
    if (i < a.nt) {
      const int32_t e1 = a.rowptr[i + 1];
      for (int32_t e = a.rowptr[i] + lid; e < e1; e += L) acc += w[e] * p[col[e]];
    }
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (i < a.nt && lid == 0) {
      T pi = p[i];
      T qi = a.D[i] * pi - acc;
      a.q[i] = qi;
      x[0] += (double)pi * (double)qi;
    }
  }
  write_partials<1>(x, a.partials, kPSpmv, lds);
}

// ----------------------------------------------------------------------------
// alpha = rho / p^T q; v += alpha p; r -= alpha q; partial sums of r^T z and
// ||r||^2 for the next iteration's stopping test and beta
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  __shared__ double bc[4];
  Scalars *sc = a.sc;
  if (block_done(sc)) return;
  const int64_t it = sc->iter_a;
  double t1[1];
  read_totals<1>(a.partials, kPSpmv, gridDim.x, t1, lds, bc);
  const double pq = t1[0];
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (first_thread()) { sc->done = 1; sc->status = IRLS_ERR_CG_BREAKDOWN; }
    return;
  }
  const double alpha = sc->rho[it & 1] / pq;
  const T *__restrict__ p = (a.K > 0 && (it & 1) == 0) ? a.p1 : a.p0;   // fused diagonal kernel's output
  double x[2] = {0.0, 0.0};
  FOR_ROWS(u, a.nt) {
    const T pu = p[u];
    a.v[u] += alpha * (double)pu;
    const T Du = a.D[u];
    T ru = (T)((double)Du * (double)a.z[u] - alpha * (double)a.q[u]);   // r = D z - alpha q
    T zu = ru / Du;
    a.z[u] = zu;
    x[0] += (double)ru * (double)zu;
    x[1] += (double)ru * (double)ru;
  }
  write_partials<2>(x, a.partials, kPUpd, lds);
  if (first_thread()) {
    sc->iter_b = it + 1;
    sc->alpha = alpha;
    sc->pq = pq;
  }
}

// Vectorised k_update: R consecutive rows per thread (nt divisible by R).
template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_update_vec(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  __shared__ double bc[4];
  typedef vec_t<T, R> V;
  typedef vec_t<double, R> VD;
  Scalars *sc = a.sc;
  if (block_done(sc)) return;
  const int64_t it = sc->iter_a;
  double t1[1];
  read_totals<1>(a.partials, kPSpmv, gridDim.x, t1, lds, bc);
  const double pq = t1[0];
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (first_thread()) { sc->done = 1; sc->status = IRLS_ERR_CG_BREAKDOWN; }
    return;
  }
  const double alpha = sc->rho[it & 1] / pq;
  const T *__restrict__ p = (a.K > 0 && (it & 1) == 0) ? a.p1 : a.p0;
  const int64_t ng = a.nt / R;
  double x[2] = {0.0, 0.0};
  FOR_ROWS(gi, ng) {
    const int64_t u0 = gi * R;
    const V pv = vload<T, R>(p + u0), zv = vload<T, R>(a.z + u0), qv = vload<T, R>(a.q + u0);
    const V Dv = vload<T, R>(a.D + u0);
    VD vv = vload<double, R>(a.v + u0);
    V zn;
#pragma unroll
    for (int i = 0; i < R; i++) {
      vv[i] += alpha * (double)pv[i];
      const T ru = (T)((double)Dv[i] * (double)zv[i] - alpha * (double)qv[i]);
      zn[i] = ru / Dv[i];
      x[0] += (double)ru * (double)zn[i];
      x[1] += (double)ru * (double)ru;
    }
    vstore<double, R>(a.v + u0, vv);
    vstore<T, R>(a.z + u0, zn);
  }
  write_partials<2>(x, a.partials, kPUpd, lds);
  if (first_thread()) {
    sc->iter_b = it + 1;
    sc->alpha = alpha;
    sc->pq = pq;
  }
}

// precision 1: r = b - L~ v in FP64 replaces the recursive FP32 residual every
// refine_every iterations and whenever the recursive residual claims
// convergence (the stopping test then uses the true residual)
template <typename T, bool DIA>
__global__ __launch_bounds__(kBlock) void k_replace(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  __shared__ double bc[4];
  Scalars *sc = a.sc;
  if (block_done(sc)) return;
  const int64_t i = sc->iter_b;
  double t2[2];
  read_totals<2>(a.partials, kPUpd, gridDim.x, t2, lds, bc);
  const bool conv_rec = sqrt(t2[1]) <= a.rtol * sqrt(sc->bb);
  if (!(conv_rec || i % sc->refine_every == 0)) return;
  double x[2] = {0.0, 0.0};
  FOR_ROWS(u, a.nt) {
    double ru64 = a.b[u] - row_apply64<DIA>(a, u, a.v);
    T ru = (T)ru64;
    T zu = ru / a.D[u];
    a.z[u] = zu;
    x[0] += (double)ru * (double)zu;
    x[1] += (double)ru * (double)ru;
  }
  write_partials<2>(x, a.partials, kPRep, lds);
}

// ----------------------------------------------------------------------------
// per-round diagnostics (Section 2.1-2.2): smoothed objective, ||CBx||_1,
// flow value x^T L x and the flows at s and t (Proposition 3), the range of v
// (Proposition 2) and the true residual; k_stats_final adds the partials.
// ----------------------------------------------------------------------------
template <typename T, bool DIA>
__global__ __launch_bounds__(kBlock) void k_stats(CGArgs<T> a) {
  __shared__ double lds[8 * (kBlock / 64)];
  const double *w = a.w64 ? a.w64 : (const double *)a.w;
  // slots: s_eps, l1, flow, flow_s, flow_t, res^2, max(-v), max(v)
  double x[8] = {0, 0, 0, 0, 0, 0, -INFINITY, -INFINITY};
  FOR_ROWS(u, a.nt) {
    const double vu = a.v[u];
    for_each_nb<DIA>(a, u, [&](int64_t j, double c, int64_t wi) {
      if (j <= u) return;                       // each interior edge once
      double d = vu - a.v[j];
      x[0] += a.form == 0 ? c * sqrt(d * d + a.eps_next) : sqrt((c * d) * (c * d) + a.eps_next);
      x[1] += c * fabs(d);
      x[2] += w[wi] * d * d;
    });
    double cs = a.cs[u], ct = a.ct[u];
    if (cs > 0.0) {
      double d = 1.0 - vu;
      x[0] += a.form == 0 ? cs * sqrt(d * d + a.eps_next) : sqrt((cs * d) * (cs * d) + a.eps_next);
      x[1] += cs * fabs(d);
      x[2] += a.b[u] * d * d;
      x[3] += a.b[u] * d;
    }
    if (ct > 0.0) {
      double d = vu;
      x[0] += a.form == 0 ? ct * sqrt(d * d + a.eps_next) : sqrt((ct * d) * (ct * d) + a.eps_next);
      x[1] += ct * fabs(d);
      x[2] += a.gt[u] * d * d;
      x[4] += a.gt[u] * d;
    }
    double res = a.b[u] - row_apply64<DIA>(a, u, a.v);
    x[5] += res * res;
    x[6] = fmax(x[6], -vu);
    x[7] = fmax(x[7], vu);
  }
  write_partials<8, 0xC0u>(x, a.partials, kPStats, lds);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_stats_final(CGArgs<T> a, int nblocks) {
  __shared__ double lds[8 * (kBlock / 64)];
  __shared__ double bc[8];
  double tot[8];
  read_totals<8, 0xC0u>(a.partials, kPStats, nblocks, tot, lds, bc);
  if (threadIdx.x != 0) return;
  irls_round_stats *R = a.stat;
  const Scalars *sc = a.sc;
  double gst = 0.0, sst = 0.0;
  if (a.cst > 0.0) {
    gst = a.round0 ? a.cst : (a.weights_fp64 ? conductance<double>(a.cst, 1.0, a.eps, a.form)
                                             : (double)conductance<float>((float)a.cst, 1.0f, (float)a.eps, a.form));
    sst = a.form == 0 ? a.cst * sqrt(1.0 + a.eps_next) : sqrt(a.cst * a.cst + a.eps_next);
  }
  R->eps = a.round0 ? 0.0 : a.eps;
  R->cg_iters = sc->iter_b;
  R->rel_res = sc->bb > 0.0 ? sqrt(sc->rr / sc->bb) : 0.0;
  R->true_rel_res = sc->bb > 0.0 ? sqrt(tot[5] / sc->bb) : 0.0;
  R->s_eps = tot[0] + sst;
  R->l1 = tot[1] + a.cst;
  R->flow = tot[2] + gst;
  R->flow_s = tot[3] + gst;
  R->flow_t = tot[4] + gst;
  R->vmin = a.nt > 0 ? -tot[6] : 0.0;
  R->vmax = a.nt > 0 ? tot[7] : 0.0;
  R->status = sc->status;
}

__global__ void k_fill(double *x, int64_t n, double value) {
  for (int64_t i = row_begin(); i < n; i += row_stride()) x[i] = value;
}

__global__ void k_scalars_reset(Scalars *sc, int64_t maxit, int32_t refine_every) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc->rho[0] = sc->rho[1] = 0.0;
    sc->bb = sc->rr = sc->alpha = sc->beta = sc->pq = 0.0;
    sc->iter_a = sc->iter_b = 0;
    sc->maxit = maxit;
    sc->done = 1;
    sc->status = IRLS_OK;
    sc->refine_every = refine_every;
    sc->pad = 0;
  }
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
template <typename T>
hipError_t launch_assemble(const CGArgs<T> &a, int grid, hipStream_t st) {
  if (a.K > 0) hipLaunchKernelGGL((k_assemble<T, true>), dim3(grid), dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL((k_assemble<T, false>), dim3(grid), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cginit(const CGArgs<T> &a, int grid, hipStream_t st) {
  if (a.K > 0) hipLaunchKernelGGL((k_cginit<T, true>), dim3(grid), dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL((k_cginit<T, false>), dim3(grid), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

// rows per thread of the vectorised kernels: one 16-byte vector
template <typename T>
constexpr int kVecRows = 16 / (int)sizeof(T);

template <typename T>
bool vec_ok(const CGArgs<T> &a) {
  constexpr int R = kVecRows<T>;
  if (a.nt % R != 0) return false;
  if (a.K == 0) return true;
  if (a.K > 3 || a.off[0] != 1) return false;
  for (int k = 1; k < a.K; k++)
    if (a.off[k] % R != 0) return false;
  return true;
}

template <typename T>
hipError_t launch_spmv(const CGArgs<T> &a, int grid, int rows_per_wave, bool, hipStream_t st) {
  constexpr int R = kVecRows<T>;
  if (a.K > 0 && vec_ok(a)) {
    switch (a.K) {
      case 1: hipLaunchKernelGGL((k_spmv_dia_vec<T, 1, R>), dim3(grid), dim3(kBlock), 0, st, a); break;
      case 2: hipLaunchKernelGGL((k_spmv_dia_vec<T, 2, R>), dim3(grid), dim3(kBlock), 0, st, a); break;
      default: hipLaunchKernelGGL((k_spmv_dia_vec<T, 3, R>), dim3(grid), dim3(kBlock), 0, st, a); break;
    }
    return hipGetLastError();
  }
  if (a.K > 0) {
    switch (a.K) {
      case 1: hipLaunchKernelGGL((k_spmv_dia<T, 1>), dim3(grid), dim3(kBlock), 0, st, a); break;
      case 2: hipLaunchKernelGGL((k_spmv_dia<T, 2>), dim3(grid), dim3(kBlock), 0, st, a); break;
      case 3: hipLaunchKernelGGL((k_spmv_dia<T, 3>), dim3(grid), dim3(kBlock), 0, st, a); break;
      case 4: hipLaunchKernelGGL((k_spmv_dia<T, 4>), dim3(grid), dim3(kBlock), 0, st, a); break;
      case 5: hipLaunchKernelGGL((k_spmv_dia<T, 5>), dim3(grid), dim3(kBlock), 0, st, a); break;
      case 6: hipLaunchKernelGGL((k_spmv_dia<T, 6>), dim3(grid), dim3(kBlock), 0, st, a); break;
      case 7: hipLaunchKernelGGL((k_spmv_dia<T, 7>), dim3(grid), dim3(kBlock), 0, st, a); break;
      default: hipLaunchKernelGGL((k_spmv_dia<T, 8>), dim3(grid), dim3(kBlock), 0, st, a); break;
    }
    return hipGetLastError();
  }
  switch (rows_per_wave) {
    case 64: hipLaunchKernelGGL((k_spmv_csr<T, 1>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_spmv_csr<T, 2>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_spmv_csr<T, 4>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_spmv_csr<T, 8>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_spmv_csr<T, 16>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_spmv_csr<T, 32>), dim3(grid), dim3(kBlock), 0, st, a); break;
    default: hipLaunchKernelGGL((k_spmv_csr<T, 64>), dim3(grid), dim3(kBlock), 0, st, a); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_direction(const CGArgs<T> &a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_direction<T>), dim3(grid), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_update(const CGArgs<T> &a, int grid, hipStream_t st) {
  if (a.nt % kVecRows<T> == 0)
    hipLaunchKernelGGL((k_update_vec<T, kVecRows<T>>), dim3(grid), dim3(kBlock), 0, st, a);
  else
    hipLaunchKernelGGL((k_update<T>), dim3(grid), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_replace_residual(const CGArgs<T> &a, int grid, hipStream_t st) {
  if (a.K > 0) hipLaunchKernelGGL((k_replace<T, true>), dim3(grid), dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL((k_replace<T, false>), dim3(grid), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stats(const CGArgs<T> &a, int grid, hipStream_t st) {
  if (a.K > 0) hipLaunchKernelGGL((k_stats<T, true>), dim3(grid), dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL((k_stats<T, false>), dim3(grid), dim3(kBlock), 0, st, a);
  hipLaunchKernelGGL((k_stats_final<T>), dim3(1), dim3(kBlock), 0, st, a, grid);
  return hipGetLastError();
}

hipError_t launch_fill(double *x, int64_t n, double value, hipStream_t st) {
  int grid = (int)((n + kBlock - 1) / kBlock);
  if (grid > kMaxGrid) grid = kMaxGrid;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, st, x, n, value);
  return hipGetLastError();
}

hipError_t launch_scalars_reset(Scalars *sc, int64_t maxit, int32_t refine_every, hipStream_t st) {
  hipLaunchKernelGGL(k_scalars_reset, dim3(1), dim3(64), 0, st, sc, maxit, refine_every);
  return hipGetLastError();
}

#define IRLS_INSTANTIATE(T)                                                                  \
  template hipError_t launch_assemble<T>(const CGArgs<T> &, int, hipStream_t);             \
  template hipError_t launch_cginit<T>(const CGArgs<T> &, int, hipStream_t);               \
  template hipError_t launch_spmv<T>(const CGArgs<T> &, int, int, bool, hipStream_t);      \
  template hipError_t launch_direction<T>(const CGArgs<T> &, int, hipStream_t);            \
  template hipError_t launch_update<T>(const CGArgs<T> &, int, hipStream_t);               \
  template hipError_t launch_replace_residual<T>(const CGArgs<T> &, int, hipStream_t);     \
  template hipError_t launch_stats<T>(const CGArgs<T> &, int, hipStream_t);
IRLS_INSTANTIATE(double)
IRLS_INSTANTIATE(float)

}  // namespace irls
