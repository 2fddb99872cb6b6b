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
// Where the marching SpMV runs, Jacobi PCG is run as CG on the symmetrically
// scaled system D^-1/2 L~ D^-1/2 (the same iterates in exact arithmetic), so
// the SpMV reads no diagonal and the potentials move every second iteration.
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
// Row u's terminal edges and totals, given the sum of its interior conductances.
template <typename T>
__device__ __forceinline__ void assemble_row_tail(const CGArgs<T> &a, int64_t u, double vu, double diag) {
  const double cs = a.cs[u], ct = a.ct[u];
  const double gs = cs > 0.0 ? edge_g(a, cs, 1.0 - vu) : 0.0;
  const double gt = ct > 0.0 ? edge_g(a, ct, vu) : 0.0;
  diag += gs + gt;
  a.D[u] = (T)diag;
  if (a.D64) a.D64[u] = diag;
  a.b[u] = gs;
  a.gt[u] = gt;
}

// diagonal format: a thread per row
template <typename T>
__global__ __launch_bounds__(kBlock) void k_assemble(CGArgs<T> a) {
  FOR_ROWS(u, a.nt) {
    const double vu = a.v[u];
    double diag = 0.0;
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
    assemble_row_tail(a, u, vu, diag);
  }
}

// CSR: L lanes per row (the SpMV's), so rows with many entries (the hubs of
// power-law graphs) are not left to one thread
template <typename T, int L>
__global__ __launch_bounds__(kBlock) void k_assemble_csr(CGArgs<T> a) {
  for_row_groups<L>(a.nt, [&](int64_t u, int lid) {
    double diag = 0.0, vu = 0.0;
    if (u >= 0) {
      vu = a.v[u];
      const int32_t e1 = a.rowptr[u + 1];
      for (int32_t e = a.rowptr[u] + lid; e < e1; e += L) {
        const double g = edge_g(a, a.ccap[e], vu - a.v[a.col[e]]);
        a.w[e] = (T)g;
        if (a.w64) a.w64[e] = g;
        diag += g;
      }
    }
    diag = group_sum<L>(diag);
    if (u >= 0 && lid == 0) assemble_row_tail(a, u, vu, diag);
  });
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
template <typename T>
__device__ __forceinline__ void cginit_row(const CGArgs<T> &a, int64_t u, double bu, double ru, double (&x)[3]) {
  const T rt = (T)ru;
  if (a.bj_block > 0) {                        // block-Jacobi: z and r^T z come from k_bj_apply
    a.rbuf[u] = ru;
  } else if (a.scaled) {                       // scaled form: z = D^-1/2 r, r^T M^-1 r = z^T z
    const T zt = (T)(ru / sqrt(a.D64 ? a.D64[u] : (double)a.D[u]));
    a.z[u] = zt;
    x[0] += (double)zt * (double)zt;
  } else {
    const T zt = rt / a.D[u];
    a.z[u] = zt;                               // z = M^-1 r is what CG keeps
    x[0] += (double)rt * (double)zt;
  }
  x[1] += bu * bu;
  x[2] += (double)rt * (double)rt;
}

template <typename T>
__device__ __forceinline__ void cginit_publish(const CGArgs<T> &a) {
  if (first_thread()) {
    a.sc->iter_b = 0;
    a.sc->iter_a = 0;
    a.sc->done = 0;
    a.sc->status = IRLS_OK;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cginit(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  double x[3] = {0.0, 0.0, 0.0};   // rho, bb, rr
  FOR_ROWS(u, a.nt) {
    const double bu = a.b[u];
    double ru = bu;
    if (a.warm) ru = bu - row_apply64<true>(a, u, a.v);
    else a.v[u] = 0.0;
    cginit_row(a, u, bu, ru, x);
  }
  write_partials<3>(x, a.partials, kPInit, lds);
  cginit_publish(a);
}

template <typename T, int L>
__global__ __launch_bounds__(kBlock) void k_cginit_csr(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  double x[3] = {0.0, 0.0, 0.0};
  const double *w = a.w64 ? a.w64 : (const double *)a.w;
  const double *D = a.D64 ? a.D64 : (const double *)a.D;
  for_row_groups<L>(a.nt, [&](int64_t u, int lid) {
    double off = 0.0;                          // sum of w_uj v_j over row u's entries
    if (u >= 0 && a.warm) {
      const int32_t e1 = a.rowptr[u + 1];
      for (int32_t e = a.rowptr[u] + lid; e < e1; e += L) off += w[e] * a.v[a.col[e]];
    }
    off = group_sum<L>(off);
    if (u >= 0 && lid == 0) {
      const double bu = a.b[u];
      double ru = bu;
      if (a.warm) ru = bu - (D[u] * a.v[u] - off);
      else a.v[u] = 0.0;
      cginit_row(a, u, bu, ru, x);
    }
  });
  write_partials<3>(x, a.partials, kPInit, lds);
  cginit_publish(a);
}

// Scaled form (Jacobi as symmetric scaling, diagonal layout): the scaled
// conductances w_uj / sqrt(D_u D_j), 0 where the edge does not exist, and the
// change of variables of the potentials, v <- D^1/2 v before CG and
// v <- D^-1/2 v after it.
// In the FP32 form the scaling uses the FP64 copies of w and D; the scaled
// conductances are then rounded to FP32 once.
template <typename T>
__device__ __forceinline__ double diag64(const CGArgs<T> &a, int64_t u) {
  return a.D64 ? a.D64[u] : (double)a.D[u];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale_w(CGArgs<T> a) {
  FOR_ROWS(u, a.nt) {
    const double du = diag64(a, u);
    if constexpr (sizeof(T) == 8) a.Dn[u] = (float)du;          // the stopping norm's weights
    for (int k = 0; k < a.K; k++) {
      const int64_t j = u + a.off[k];
      const double wv = j < a.nt ? (a.w64 ? a.w64[k * a.nt + u] : (double)a.w[k * a.nt + u]) : 0.0;
      const double wh = wv != 0.0 ? wv / sqrt(du * diag64(a, j)) : 0.0;
      a.wh[k * a.nt + u] = (T)wh;
      if (a.wh64) a.wh64[k * a.nt + u] = wh;         // the FP64 residual replacement's copy
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale_v(CGArgs<T> a, int dir) {
  FOR_ROWS(u, a.nt) {
    const double sd = sqrt(diag64(a, u));
    a.v[u] = dir > 0 ? a.v[u] * sd : a.v[u] / sd;
  }
}

// Start of CG iteration i = iter_b (in the kernel that forms the direction):
// totals of r^T z and ||r||^2 left by the previous kernel (the CG start, the
// vector update, or the FP64 residual replacement), the stopping test, and
// beta = rho_i / rho_{i-1}.  Workgroup 0 publishes the state.  Returns false
// when CG has stopped.
// Start of a CG iteration, in two halves so that a kernel can issue its own
// first loads in between.  The first half loads the scalar-block fields and
// this thread's share of the vector update's partial sums (the usual
// predecessor); the second reduces them together (the done flag by max), so
// the kernel waits for one memory round trip before it knows whether and how
// to run.  Every thread reads the flag; the max makes the workgroup agree,
// and workgroups that read it at different times still agree, since each
// computes the same stopping decision from the same partial sums.
struct IterStartLoads {
  int32_t done, refine;
  int64_t i, maxit;
  double bb, rho0, rho1;
  double part[2];
};

template <typename T>
__device__ __forceinline__ IterStartLoads cg_iteration_load(const CGArgs<T> &a) {
  const Scalars *sc = a.sc;
  IterStartLoads l;
  l.done = sc->done;
  l.refine = sc->refine_every;
  l.i = sc->iter_b;
  l.maxit = sc->maxit;
  l.bb = sc->bb;
  l.rho0 = sc->rho[0];
  l.rho1 = sc->rho[1];
  partial_share<2>(a.partials, kPUpd, a.grid_main, l.part);
  return l;
}

// Second half: the stopping test and beta = rho_i / rho_{i-1}; workgroup 0
// publishes the state.  Returns false when CG has stopped.
template <typename T>
__device__ bool cg_iteration_finish(const CGArgs<T> &a, const IterStartLoads &l, double *lds, double *bc,
                                    int64_t &i_out, double &beta_out) {
  Scalars *sc = a.sc;
  const int nb = a.grid_main;
  const int64_t i = l.i;
  __shared__ double s_start[3 * (kMaxBlock / 64)];   // used once per kernel
  double t[3] = {l.part[0], l.part[1], l.done != 0 ? 1.0 : 0.0};
  block_allreduce_once<3, 0x4u>(t, s_start);
  if (t[2] != 0.0) return false;
  double rz = t[0], rr = t[1], bb = l.bb;
  if (i == 0) {                                      // after the CG start
    double t3[3];
    read_totals<3>(a.partials, kPInit, nb, t3, lds, bc);
    rz = t3[0]; bb = t3[1]; rr = t3[2];
  } else if (l.refine > 0) {
    const bool conv_rec = sqrt(rr) <= a.rtol * sqrt(bb);
    if (conv_rec || i % l.refine == 0) {             // the replacement kernel ran
      double t2[2];
      read_totals<2>(a.partials, kPRep, nb, t2, lds, bc);
      rz = t2[0]; rr = t2[1];
    }
  }
  bool stop = false;
  int status = IRLS_OK;
  if (!isfinite(rz) || !isfinite(rr)) { stop = true; status = IRLS_ERR_CG_BREAKDOWN; }
  else if (sqrt(rr) <= a.rtol * sqrt(bb)) stop = true;
  else if (i >= l.maxit) { stop = true; status = IRLS_WARN_CG_MAXIT; }
  const double beta = i == 0 ? 0.0 : rz / (((i - 1) & 1) ? l.rho1 : l.rho0);
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

template <typename T>
__device__ __forceinline__ bool cg_iteration_start(const CGArgs<T> &a, double *lds, double *bc, int64_t &i_out,
                                                   double &beta_out) {
  const IterStartLoads l = cg_iteration_load(a);
  return cg_iteration_finish(a, l, lds, bc, i_out, beta_out);
}

// Start of the vector update of iteration it = iter_a: the total of p^T q
// (the SpMV's partials) and alpha = rho_it / p^T q, in the same two halves.
// Returns false when CG has stopped or broken down (pq <= 0 marks the
// breakdown).
struct UpdateStartLoads {
  int32_t done;
  int64_t it;
  double rho0, rho1;
  double alpha_even;   // alpha of the last even iteration (the scaled form's odd updates)
  double part[1];
};

template <typename T>
__device__ __forceinline__ UpdateStartLoads cg_update_load(const CGArgs<T> &a) {
  const Scalars *sc = a.sc;
  UpdateStartLoads l;
  l.done = sc->done;
  l.it = sc->iter_a;
  l.rho0 = sc->rho[0];
  l.rho1 = sc->rho[1];
  l.alpha_even = sc->alpha_par[0];
  partial_share<1>(a.partials, kPSpmv, a.grid_spmv, l.part);
  return l;
}

template <typename T>
__device__ bool cg_update_finish(const CGArgs<T> &a, const UpdateStartLoads &l, double *lds, double *bc,
                                 int64_t &it_out, double &alpha_out, double &pq_out) {
  Scalars *sc = a.sc;
  __shared__ double s_start[2 * (kBlock / 64)];      // used once per kernel
  double t[2] = {l.part[0], l.done != 0 ? 1.0 : 0.0};
  block_allreduce_once<2, 0x2u>(t, s_start);
  if (t[1] != 0.0) return false;
  const double pq = t[0];
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (first_thread()) { sc->done = 1; sc->status = IRLS_ERR_CG_BREAKDOWN; }
    return false;
  }
  it_out = l.it;
  pq_out = pq;
  alpha_out = ((l.it & 1) ? l.rho1 : l.rho0) / pq;
  return true;
}

template <typename T>
__device__ __forceinline__ bool cg_update_start(const CGArgs<T> &a, double *lds, double *bc, int64_t &it_out,
                                                double &alpha_out, double &pq_out) {
  const UpdateStartLoads l = cg_update_load(a);
  return cg_update_finish(a, l, lds, bc, it_out, alpha_out, pq_out);
}

// Precision form: whether the FP64 residual replacement runs after the update
// of iteration i = iter_b - 1 -- every refine_every iterations, and whenever
// the recursive residual (the update's partial sums) claims convergence, so
// that the stopping test then uses the true residual.  Every thread gets the
// same answer; i_out = iter_b.
template <typename T>
__device__ __forceinline__ bool replace_due(const CGArgs<T> &a, double *lds, double *bc, int64_t &i_out) {
  const Scalars *sc = a.sc;
  const int32_t done = sc->done;
  const int64_t i = sc->iter_b;
  const int32_t refine = sc->refine_every;
  const double bb = sc->bb;
  double t[3];
  {
    double u[2];
    partial_share<2>(a.partials, kPUpd, a.grid_main, u);
    t[0] = u[0];
    t[1] = u[1];
    t[2] = done != 0 ? 1.0 : 0.0;
  }
  block_allreduce<3, 0x4u>(t, lds, bc);
  if (t[2] != 0.0) return false;
  const bool conv_rec = sqrt(t[1]) <= a.rtol * sqrt(bb);
  i_out = i;
  return conv_rec || i % refine == 0;
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
// Streaming forms (non-temporal hint) for data a kernel touches once: at sizes
// past the caches they keep such lines from pushing out the ones that are
// reused (the marching SpMV's neighbour rows).  Measured at 256^3: SpMV
// 207 -> 192 us, update 145 -> 123 us.  Where a CG iteration's data fit the
// 256 MB last-level cache they are slower (128^3: SpMV 26 -> 30 us), so the
// kernels take the choice as a template argument (vload_s / vstore_s) and the
// host sets it by size.
template <typename T, int R>
__device__ __forceinline__ vec_t<T, R> vload_nt(const T *p) {
  return __builtin_nontemporal_load(reinterpret_cast<const vec_t<T, R> *>(p));
}
template <typename T, int R>
__device__ __forceinline__ void vstore_nt(T *p, vec_t<T, R> v) {
  __builtin_nontemporal_store(v, reinterpret_cast<vec_t<T, R> *>(p));
}
template <bool NT, typename T, int R>
__device__ __forceinline__ vec_t<T, R> vload_s(const T *p) {
  if constexpr (NT) return vload_nt<T, R>(p);
  else return vload<T, R>(p);
}
template <bool NT, typename T, int R>
__device__ __forceinline__ void vstore_s(T *p, vec_t<T, R> v) {
  if constexpr (NT) vstore_nt<T, R>(p, v);
  else vstore<T, R>(p, v);
}

// Loads of one R-row group of the vectorised diagonal SpMV, taken before beta
// is known.  Neighbours outside the matrix load as zeros (their terms vanish).
template <typename T, int K, int R>
struct DiaRow {
  vec_t<T, R> zc, pc, D, w0;                // the group itself and its offset-1 edges
  T zr, pr, wl, zl, pl;                     // the rows just right and left of the group
  static constexpr int KO = K > 1 ? K - 1 : 1;
  vec_t<T, R> wf[KO], zf[KO], pf[KO];       // offset +off[k], k >= 1
  vec_t<T, R> wb[KO], zb[KO], pb[KO];       // offset -off[k], k >= 1
};

template <typename T, int K, int R>
__device__ __forceinline__ void dia_load_p(const CGArgs<T> &a, const T *pin, int64_t u0, DiaRow<T, K, R> &r) {
  const vec_t<T, R> zero = (T)0;
  r.pc = vload<T, R>(pin + u0);
  r.pr = u0 + R < a.nt ? pin[u0 + R] : (T)0;
  r.pl = u0 > 0 ? pin[u0 - 1] : (T)0;
#pragma unroll
  for (int k = 1; k < K; k++) {
    const int64_t o = a.off[k];
    r.pf[k - 1] = u0 + o < a.nt ? vload<T, R>(pin + u0 + o) : zero;
    r.pb[k - 1] = u0 >= o ? vload<T, R>(pin + u0 - o) : zero;
  }
}

template <typename T, int K, int R>
__device__ __forceinline__ void dia_load(const CGArgs<T> &a, const T *pin, int64_t u0, DiaRow<T, K, R> &r) {
  const vec_t<T, R> zero = (T)0;
  const int64_t nt = a.nt;
  r.zc = vload<T, R>(a.z + u0);
  r.D = vload<T, R>(a.D + u0);
  r.w0 = vload<T, R>(a.w + u0);
  r.zr = u0 + R < nt ? a.z[u0 + R] : (T)0;
  r.wl = u0 > 0 ? a.w[u0 - 1] : (T)0;
  r.zl = u0 > 0 ? a.z[u0 - 1] : (T)0;
#pragma unroll
  for (int k = 1; k < K; k++) {
    const int64_t o = a.off[k];
    const bool f = u0 + o < nt, b = u0 >= o;
    r.wf[k - 1] = f ? vload<T, R>(a.w + k * nt + u0) : zero;
    r.zf[k - 1] = f ? vload<T, R>(a.z + u0 + o) : zero;
    r.wb[k - 1] = b ? vload<T, R>(a.w + k * nt + u0 - o) : zero;
    r.zb[k - 1] = b ? vload<T, R>(a.z + u0 - o) : zero;
  }
  dia_load_p(a, pin, u0, r);
}

// Vectorised form of k_spmv_dia for grids: each thread owns R consecutive
// rows and moves them with 16-byte loads (R = 2 in FP64, 4 in FP32).  Needs
// off[0] == 1, every other offset and nt divisible by R.  The +-1 neighbours
// inside the group come from registers; the rows just outside it are scalar
// loads that hit in L1 (the neighbouring lanes loaded them).  The first row
// group's loads are issued before the start-of-iteration reduction (which
// reads every workgroup's partial sums and waits on barriers), so the memory
// pipes are busy while it runs.
template <typename T, int K, int R>
__global__ __launch_bounds__(kBlock) void k_spmv_dia_vec(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  __shared__ double bc[4];
  typedef vec_t<T, R> V;
  const int64_t nt = a.nt, ng = nt / R;
  int64_t gb, ge, gs;
  slab_rows(ng, gb, ge, gs);
  const IterStartLoads sl = cg_iteration_load(a);     // first: the reduction waits only for these
  const T *__restrict__ pin = (a.it_hint & 1) ? a.p1 : a.p0;
  DiaRow<T, K, R> r;
  if (gb < ge) dia_load(a, pin, gb * R, r);
  int64_t it;
  double beta64;
  if (!cg_iteration_finish(a, sl, lds, bc, it, beta64)) return;
  if (((it ^ a.it_hint) & 1) != 0) {                  // the host's guess was wrong
    pin = (it & 1) ? a.p1 : a.p0;
    if (gb < ge) dia_load_p(a, pin, gb * R, r);
  }
  T *__restrict__ pout = (it & 1) ? a.p0 : a.p1;
  const T beta = (T)beta64;
  const bool first = it == 0;
  auto dir = [&](V zv, V pv) -> V { return first ? zv : zv + beta * pv; };
  auto dirs = [&](T zv, T pv) -> T { return first ? zv : zv + beta * pv; };
  double x[1] = {0.0};
  for (int64_t gi = gb; gi < ge; gi += gs) {
    const int64_t u0 = gi * R;
    if (gi != gb) dia_load(a, pin, u0, r);
    const V pc = dir(r.zc, r.pc);
    V acc = r.D * pc;
    // offset 1: edges inside the group, and to the rows just outside it
    const T right = dirs(r.zr, r.pr), left = dirs(r.zl, r.pl);
#pragma unroll
    for (int i = 0; i < R; i++) {
      acc[i] -= r.w0[i] * (i + 1 < R ? pc[i + 1] : right);
      acc[i] -= (i > 0 ? r.w0[i - 1] : r.wl) * (i > 0 ? pc[i - 1] : left);
    }
#pragma unroll
    for (int k = 1; k < K; k++) {
      acc -= r.wf[k - 1] * dir(r.zf[k - 1], r.pf[k - 1]);
      acc -= r.wb[k - 1] * dir(r.zb[k - 1], r.pb[k - 1]);
    }
    vstore<T, R>(pout + u0, pc);
    vstore<T, R>(a.q + u0, acc);
#pragma unroll
    for (int i = 0; i < R; i++) x[0] += (double)pc[i] * (double)acc[i];
  }
  write_partials<1>(x, a.partials, kPSpmv, lds);
}

// Loads of one step of the marching SpMV (one R-row group of plane k), taken
// before beta is known: the group's next-plane values, its own conductances,
// and the neighbours at the offsets below the plane size.  Neighbours outside
// the matrix load as zeros.
template <typename T, int K, int R>
struct MarchStep {
  static constexpr int KM = K > 2 ? K - 2 : 1;
  vec_t<T, R> zp, pp, D, w0, wP;            // plane k + 1; diagonal; offsets 1 and P
  T zr, pr, wl, zl, pl;                     // the rows just right and left of the group
  vec_t<T, R> wf[KM], zf[KM], pf[KM];       // offsets off[1..K-2], forward
  vec_t<T, R> wb[KM], zb[KM], pb[KM];       // and backward
};

// A step's loads are unconditional, so the compiler can keep the next step's
// loads in flight while it waits for this one's.  A neighbour row outside the
// matrix is read at a valid index instead, chosen so that its product
// vanishes: a direction or residual value from row u0 meets a conductance
// that is zero there (the edge to a row past the end is stored as 0), and a
// conductance of an edge from before row 0 is read where one is known to be
// 0 (offset 1 at row nt - 1; offset o >= R at rows nt - R .. nt - 1).  nt and
// every offset are multiples of R, so a group lies wholly inside or outside.
template <typename T, int K, int R>
__device__ __forceinline__ void march_load_p(const CGArgs<T> &a, const T *pin, int64_t u0, MarchStep<T, K, R> &s) {
  const int64_t nt = a.nt, P = a.off[K - 1];
  s.pp = vload<T, R>(pin + (u0 + P < nt ? u0 + P : u0));     // unused past the last plane
  s.pr = pin[u0 + R < nt ? u0 + R : u0];
  s.pl = pin[u0 > 0 ? u0 - 1 : u0];
#pragma unroll
  for (int kk = 1; kk < K - 1; kk++) {
    const int64_t o = a.off[kk];
    s.pf[kk - 1] = vload<T, R>(pin + (u0 + o < nt ? u0 + o : u0));
    s.pb[kk - 1] = vload<T, R>(pin + (u0 >= o ? u0 - o : u0));
  }
}

// SC: the scaled form (scaled conductances, unit diagonal: no D load).
template <typename T, int K, int R, bool SC, bool NT>
__device__ __forceinline__ void march_load(const CGArgs<T> &a, const T *pin, int64_t u0, MarchStep<T, K, R> &s) {
  const int64_t nt = a.nt, P = a.off[K - 1];
  const T *__restrict__ w = SC ? a.wh : a.w;
  s.zp = vload<T, R>(a.z + (u0 + P < nt ? u0 + P : u0));
  if constexpr (!SC) s.D = vload<T, R>(a.D + u0);
  s.w0 = vload<T, R>(w + u0);
  s.wP = vload_s<NT, T, R>(w + (K - 1) * nt + u0);           // read by this thread only
  s.zr = a.z[u0 + R < nt ? u0 + R : u0];
  s.wl = w[u0 > 0 ? u0 - 1 : nt - 1];
  s.zl = a.z[u0 > 0 ? u0 - 1 : u0];
#pragma unroll
  for (int kk = 1; kk < K - 1; kk++) {
    const int64_t o = a.off[kk];
    const bool f = u0 + o < nt, b = u0 >= o;
    s.wf[kk - 1] = vload<T, R>(w + kk * nt + u0);
    s.zf[kk - 1] = vload<T, R>(a.z + (f ? u0 + o : u0));
    s.wb[kk - 1] = vload<T, R>(w + kk * nt + (b ? u0 - o : nt - R));
    s.zb[kk - 1] = vload<T, R>(a.z + (b ? u0 - o : u0));
  }
  march_load_p(a, pin, u0, s);
}

// Tiles of one plane of the marching SpMV, of BS row groups (R rows each).
//   ty = 0: BS consecutive row groups of the plane (any grid);
//   ty >= 1 (3-D grids, where a plane of P rows is P / N lines of N = off[1]
//   rows): ty consecutive lines by tx = BS / ty row groups of each line.
// Tiles are numbered line block by line block, so consecutive tiles, which
// run on the same XCD, are neighbours.
struct MarchTiles {
  int64_t N, lines, gx, tx, tiles_x, tiles;
  int32_t TY;
};

template <int R, int BS>
__host__ __device__ inline MarchTiles march_tiles(int64_t P, int64_t N1, int32_t ty) {
  MarchTiles m;
  m.TY = ty;
  if (ty == 0) {                                   // the plane as one line
    m.N = P;
    m.lines = 1;
    m.gx = P / R;
    m.tx = BS;
  } else {
    m.N = N1;
    m.lines = P / N1;
    m.gx = N1 / R;
    m.tx = BS / ty;
  }
  m.tiles_x = (m.gx + m.tx - 1) / m.tx;
  m.tiles = m.tiles_x * (ty == 0 ? 1 : (m.lines + ty - 1) / ty);
  return m;
}

// Diagonal SpMV marching along the largest offset P = off[K-1] (the plane
// size of a grid: rows u = c + P k).  A workgroup of BS threads owns a tile
// of one plane (see MarchTiles) and walks a chunk of consecutive planes; each
// thread keeps the direction values of planes k-1 and k and the conductance
// of its edge to plane k-1 in registers, so the +-P neighbours, which lie a
// whole plane away in memory, are never reloaded.  Offsets below P are read
// as in k_spmv_dia_vec: the +-N neighbours inside a tile are loaded by their
// own threads at the same step and hit in cache, those on the tile's two
// boundary lines come from the neighbouring tiles, so taller tiles re-read
// fewer of them from memory.  All loads of the first two steps are issued
// before the start-of-iteration reduction, so they are in flight while it
// runs.  Workgroup b runs on XCD b % 8; each XCD takes a contiguous range of
// tiles and chunks, so tile boundaries and the planes at chunk seams are
// mostly shared in its L2.  p_new and q are stored, and the conductances to
// plane k + 1 loaded, with the streaming hint: each is touched once here, and
// they should not push the neighbour rows out of the caches.  The summation
// order per row is that of k_spmv_dia_vec.
template <typename T, int K, int R, bool SC, int BS, bool NT>
__global__ __launch_bounds__(BS) void k_spmv_dia_march(CGArgs<T> a) {
  __shared__ double lds[4 * (BS / 64)];
  __shared__ double bc[4];
  typedef vec_t<T, R> V;
  const V zero = (T)0;
  const int64_t nt = a.nt, P = a.off[K - 1];
  const MarchTiles mt = march_tiles<R, BS>(P, a.off[1], a.march_ty);
  const int64_t nplanes = (nt + P - 1) / P, zc = a.march_planes;
  const int64_t L = (int64_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) + blockIdx.x / kXcds;
  const int64_t tile = L % mt.tiles, chunk = L / mt.tiles;
  const int64_t gxi = (tile % mt.tiles_x) * mt.tx + threadIdx.x % mt.tx;       // row group in its line
  const int64_t line = mt.TY == 0 ? 0 : (tile / mt.tiles_x) * mt.TY + threadIdx.x / mt.tx;
  const int64_t c = line * mt.N + gxi * R;
  const int64_t k0 = chunk * zc;
  const int64_t k1 = k0 + zc < nplanes ? k0 + zc : nplanes;
  const bool active = gxi < mt.gx && line < mt.lines && k0 < nplanes && c + P * k0 < nt;
  // planes of this chunk that hold this thread's rows (a last plane may be partial)
  const int64_t kmax = active ? (nt - c + P - 1) / P : 0;
  const int64_t kend = k1 < kmax ? k1 : kmax;
  const IterStartLoads sl = cg_iteration_load(a);     // first: the reduction waits only for these
  const T *__restrict__ pin = (a.it_hint & 1) ? a.p1 : a.p0;
  V zm = zero, pm = zero, wm = zero, zk = zero, pk = zero;
  // the first two steps are loaded before the reduction
  MarchStep<T, K, R> s0, s1;
  const bool two = kend > k0 + 1;
  if (active) {
    const int64_t u = c + P * k0;
    zk = vload<T, R>(a.z + u);
    pk = vload<T, R>(pin + u);
    if (k0 > 0) {
      zm = vload<T, R>(a.z + u - P);
      pm = vload<T, R>(pin + u - P);
      wm = vload<T, R>((SC ? a.wh : a.w) + (K - 1) * nt + u - P);
    }
    march_load<T, K, R, SC, NT>(a, pin, u, s0);
    if (two) march_load<T, K, R, SC, NT>(a, pin, u + P, s1);
  }
  int64_t it;
  double beta64;
  if (!cg_iteration_finish(a, sl, lds, bc, it, beta64)) return;
  if (((it ^ a.it_hint) & 1) != 0) {                  // the host's guess was wrong
    pin = (it & 1) ? a.p1 : a.p0;
    if (active) {
      const int64_t u = c + P * k0;
      pk = vload<T, R>(pin + u);
      if (k0 > 0) pm = vload<T, R>(pin + u - P);
      march_load_p(a, pin, u, s0);
      if (two) march_load_p(a, pin, u + P, s1);
    }
  }
  T *__restrict__ pout = (it & 1) ? a.p0 : a.p1;
  const T beta = (T)beta64;
  const bool first = it == 0;
  auto dir = [&](V zv, V pv) -> V { return first ? zv : zv + beta * pv; };
  auto dirs = [&](T zv, T pv) -> T { return first ? zv : zv + beta * pv; };
  double x[1] = {0.0};
  V dm = dir(zm, pm);                                    // plane k - 1
  auto step = [&](const MarchStep<T, K, R> &st, int64_t k) {
    const int64_t u0 = c + P * k;
    const V pc = dir(zk, pk);
    V acc;
    if constexpr (SC) acc = pc;
    else acc = st.D * pc;
    const T right = dirs(st.zr, st.pr), left = dirs(st.zl, st.pl);
#pragma unroll
    for (int i = 0; i < R; i++) {
      acc[i] -= st.w0[i] * (i + 1 < R ? pc[i + 1] : right);
      acc[i] -= (i > 0 ? st.w0[i - 1] : st.wl) * (i > 0 ? pc[i - 1] : left);
    }
#pragma unroll
    for (int kk = 1; kk < K - 1; kk++) {
      acc -= st.wf[kk - 1] * dir(st.zf[kk - 1], st.pf[kk - 1]);
      acc -= st.wb[kk - 1] * dir(st.zb[kk - 1], st.pb[kk - 1]);
    }
    const V dp = dir(st.zp, st.pp);
    if (u0 + P < nt) acc -= st.wP * dp;
    if (k > 0) acc -= wm * dm;
    vstore_s<NT, T, R>(pout + u0, pc);
    vstore_s<NT, T, R>(a.q + u0, acc);
#pragma unroll
    for (int i = 0; i < R; i++) x[0] += (double)pc[i] * (double)acc[i];
    dm = pc;
    wm = st.wP;
    zk = st.zp;
    pk = st.pp;
  };
  // Two steps in flight: s0 holds step k and s1 step k + 1; the buffer a step
  // frees is refilled with the step two planes on while the other computes.
  // The first pair runs before the loop, so the loop is entered with the same
  // loads outstanding, in the same order, as at its back edge (else the waits
  // at its top would cover both buffers).  The last two or three steps follow.
  if (active) {
    int64_t k = k0;
    auto pair = [&]() {
      step(s0, k);
      march_load<T, K, R, SC, NT>(a, pin, c + P * (k + 2), s0);
      __builtin_amdgcn_sched_barrier(0);                // keep the two steps apart
      step(s1, k + 1);
      march_load<T, K, R, SC, NT>(a, pin, c + P * (k + 3), s1);
      __builtin_amdgcn_sched_barrier(0);
      k += 2;
    };
    if (k + 3 < kend) {
      pair();
      while (k + 3 < kend) pair();
    }
    step(s0, k);
    if (k + 2 < kend) march_load<T, K, R, SC, NT>(a, pin, c + P * (k + 2), s0);
    if (k + 1 < kend) step(s1, k + 1);
    if (k + 2 < kend) step(s0, k + 2);
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
      const int32_t e0 = a.rowptr[i], e1 = a.rowptr[i + 1];
      const int32_t hf = a.csr_nheavy > 0 ? a.csr_hfirst[i] : 0;
      if (hf == 0) {
        for (int32_t e = e0 + lid; e < e1; e += L) acc += w[e] * p[col[e]];
      } else {                                   // a heavy row: its chunk sums, in order
        const int32_t c1 = hf - 1 + (e1 - e0 + kCsrChunk - 1) / kCsrChunk;
        for (int32_t c = hf - 1 + lid; c < c1; c += L) acc += (T)a.csr_cpart[c];
      }
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

// Heavy rows of the CSR SpMV (rows of more than kCsrHeavy entries, the hubs
// of power-law graphs), launched before k_spmv_csr: a wavefront sums one
// chunk of at most kCsrChunk entries, lanes over entries, then a fixed-order
// reduction across the wavefront.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_spmv_csr_chunks(CGArgs<T> a) {
  if (block_done(a.sc)) return;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const T *__restrict__ p = a.p0;
  for (int64_t c = wave; c < a.csr_nchunks; c += nwaves) {
    double acc = 0.0;
    const int32_t e1 = a.csr_cend[c];
    for (int32_t e = a.csr_cbeg[c] + lane; e < e1; e += 64) acc += (double)(a.w[e] * p[a.col[e]]);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) a.csr_cpart[c] = acc;
  }
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
  int64_t it;
  double alpha, pq;
  if (!cg_update_start(a, lds, bc, it, alpha, pq)) return;
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
// The row groups of a thread are processed in pairs from two register
// buffers, so the loads of one group are in flight while the other computes;
// the first two groups are loaded before the start-of-kernel reduction.
template <typename T, int R>
struct UpdGroup {
  vec_t<T, R> p, z, q, D;
  vec_t<double, R> v;
};

template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_update_vec(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  __shared__ double bc[4];
  typedef vec_t<T, R> V;
  const int64_t ng = a.nt / R;
  int64_t gb, ge, gs;
  slab_rows(ng, gb, ge, gs);
  const UpdateStartLoads sl = cg_update_load(a);      // first: the reduction waits only for these
  const T *__restrict__ p = (a.K > 0 && (a.it_hint & 1) == 0) ? a.p1 : a.p0;
  auto load = [&](int64_t g, UpdGroup<T, R> &b) {
    const int64_t u0 = g * R;
    b.p = vload<T, R>(p + u0); b.z = vload<T, R>(a.z + u0); b.q = vload<T, R>(a.q + u0);
    b.D = vload<T, R>(a.D + u0); b.v = vload<double, R>(a.v + u0);
  };
  UpdGroup<T, R> b0, b1;
  if (gb < ge) load(gb, b0);
  if (gb + gs < ge) load(gb + gs, b1);
  Scalars *sc = a.sc;
  int64_t it;
  double alpha, pq;
  if (!cg_update_finish(a, sl, lds, bc, it, alpha, pq)) return;
  if (((it ^ a.it_hint) & 1) != 0 && a.K > 0) {        // the host's guess was wrong
    p = (it & 1) == 0 ? a.p1 : a.p0;
    if (gb < ge) b0.p = vload<T, R>(p + gb * R);
    if (gb + gs < ge) b1.p = vload<T, R>(p + (gb + gs) * R);
  }
  double x[2] = {0.0, 0.0};
  auto work = [&](int64_t g, UpdGroup<T, R> &b) {
    V zn;
#pragma unroll
    for (int i = 0; i < R; i++) {
      b.v[i] += alpha * (double)b.p[i];
      const T ru = (T)((double)b.D[i] * (double)b.z[i] - alpha * (double)b.q[i]);
      zn[i] = ru / b.D[i];
      x[0] += (double)ru * (double)zn[i];
      x[1] += (double)ru * (double)ru;
    }
    vstore<double, R>(a.v + g * R, b.v);
    vstore<T, R>(a.z + g * R, zn);
  };
  int64_t g = gb;
  if (g + 3 * gs < ge) {                               // loop entered with both buffers' loads in flight
    auto pair = [&]() {
      work(g, b0);
      load(g + 2 * gs, b0);
      __builtin_amdgcn_sched_barrier(0);
      work(g + gs, b1);
      load(g + 3 * gs, b1);
      __builtin_amdgcn_sched_barrier(0);
      g += 2 * gs;
    };
    pair();
    while (g + 3 * gs < ge) pair();
  }
  if (g < ge) {
    work(g, b0);
    if (g + 2 * gs < ge) load(g + 2 * gs, b0);
    if (g + gs < ge) work(g + gs, b1);
    if (g + 2 * gs < ge) work(g + 2 * gs, b0);
  }
  write_partials<2>(x, a.partials, kPUpd, lds);
  if (first_thread()) {
    sc->iter_b = it + 1;
    sc->alpha = alpha;
    sc->pq = pq;
  }
}

// Vector update of the scaled form (z holds D^-1/2 r): z -= alpha q,
// r^T M^-1 r = z^T z and ||r||^2 = sum D z^2, which only decides when CG
// stops: its weights D are read in FP32 (Dn; 4 bytes a row instead of 8 in
// the FP64 form), which changes the norm by at most 2^-24 relative, so a stop
// moves only when the residual lands that close to the tolerance.  The potentials move every
// second iteration: an even iteration leaves its alpha p pending, and the odd
// one after it adds alpha_{it-1} p_{it-1} + alpha_it p_it, reading both
// direction buffers (iteration j's direction is in p0 for odd j, p1 for
// even j).  A pending step left when CG stops is added by k_flush_v.  ODD is
// the parity the host expects; the kernel checks it against the iteration it
// reads.  Rows are processed in pairs of groups as in k_update_vec.
template <typename T, int R, bool ODD>
struct ScaledGroup {
  vec_t<T, R> z, q, p, pp;
  vec_t<float, R> Dn;                       // the stopping norm's weights (D in FP32)
  vec_t<double, R> v;
};

template <typename T, int R, bool ODD, bool NT>
__global__ __launch_bounds__(kBlock) void k_update_scaled(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  __shared__ double bc[4];
  typedef vec_t<T, R> V;
  const int64_t ng = a.nt / R;
  int64_t gb, ge, gs;
  slab_rows(ng, gb, ge, gs);
  const UpdateStartLoads sl = cg_update_load(a);
  const T *__restrict__ p_it = ODD ? a.p0 : a.p1;
  const T *__restrict__ p_prev = ODD ? a.p1 : a.p0;
  auto load = [&](int64_t g, ScaledGroup<T, R, ODD> &b) {
    const int64_t u0 = g * R;
    b.z = vload_s<NT, T, R>(a.z + u0); b.q = vload_s<NT, T, R>(a.q + u0); b.Dn = vload_s<NT, float, R>(a.Dn + u0);
    if constexpr (ODD) {
      b.p = vload_s<NT, T, R>(p_it + u0); b.pp = vload_s<NT, T, R>(p_prev + u0);
      b.v = vload_s<NT, double, R>(a.v + u0);
    }
  };
  ScaledGroup<T, R, ODD> b0, b1;
  if (gb < ge) load(gb, b0);
  if (gb + gs < ge) load(gb + gs, b1);
  Scalars *sc = a.sc;
  int64_t it;
  double alpha, pq;
  if (!cg_update_finish(a, sl, lds, bc, it, alpha, pq)) return;
  if (((it & 1) != 0) != ODD) {                          // the launch sequence is out of step
    if (first_thread()) { sc->done = 1; sc->status = IRLS_ERR_DEVICE; }
    return;
  }
  const double alpha_prev = sl.alpha_even;
  double x[2] = {0.0, 0.0};
  auto work = [&](int64_t g, ScaledGroup<T, R, ODD> &b) {
    V zn;
#pragma unroll
    for (int i = 0; i < R; i++) {
      if constexpr (ODD) b.v[i] += alpha_prev * (double)b.pp[i] + alpha * (double)b.p[i];
      zn[i] = (T)((double)b.z[i] - alpha * (double)b.q[i]);
      x[0] += (double)zn[i] * (double)zn[i];
      x[1] += (double)b.Dn[i] * (double)zn[i] * (double)zn[i];
    }
    if constexpr (ODD) vstore_s<NT, double, R>(a.v + g * R, b.v);
    vstore_s<NT, T, R>(a.z + g * R, zn);
  };
  int64_t g = gb;
  if (g + 3 * gs < ge) {
    auto pair = [&]() {
      work(g, b0);
      load(g + 2 * gs, b0);
      __builtin_amdgcn_sched_barrier(0);
      work(g + gs, b1);
      load(g + 3 * gs, b1);
      __builtin_amdgcn_sched_barrier(0);
      g += 2 * gs;
    };
    pair();
    while (g + 3 * gs < ge) pair();
  }
  if (g < ge) {
    work(g, b0);
    if (g + 2 * gs < ge) load(g + 2 * gs, b0);
    if (g + gs < ge) work(g + gs, b1);
    if (g + 2 * gs < ge) work(g + 2 * gs, b0);
  }
  write_partials<2>(x, a.partials, kPUpd, lds);
  if (first_thread()) {
    sc->iter_b = it + 1;
    sc->alpha = alpha;
    sc->alpha_par[it & 1] = alpha;
    sc->pq = pq;
  }
}

// After CG in the scaled form (and with the precision form's ILU(0) tiles):
// if the last completed update was an even iteration, its alpha p is still
// pending; add it (its direction is in p1).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_flush_v(CGArgs<T> a) {
  const int64_t done_updates = a.sc->iter_b;
  if ((done_updates & 1) == 0) return;
  const double alpha = a.sc->alpha_par[0];
  FOR_ROWS(u, a.nt) a.v[u] += alpha * (double)a.p1[u];
}

// ----------------------------------------------------------------------------
// Block-Jacobi (Section 3.1).  Blocks are bj_block consecutive rows inside one
// line of offset-1 edges, so each block of L~ is tridiagonal:
//   diagonal D_i, sub- and super-diagonal -w0 (w0[i] couples rows i and i+1).
// Its LU factors are formed once per round (Thomas): pivot m_i = D_i - a_i c'_{i-1}
// with a_i = c_{i-1} = -w0[i-1], c'_i = c_i / m_i.  Applying M^-1 is the forward
// recurrence y_i = f_i y_{i-1} + r_i / m_i (f_i = -a_i / m_i) and the backward one
// z_i = y_i + g_i z_{i+1} (g_i = -c'_i); both are affine maps composed by a
// wavefront scan, one block (up to 128 rows, 2 per lane) per wavefront.
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bj_factor(CGArgs<T> a) {
  const int64_t B = a.bj_block, nb = (a.nt + B - 1) / B;
  const T *w0 = a.w;
  for (int64_t k = row_begin(); k < nb; k += row_stride()) {
    const int64_t lo = k * B, hi = lo + B < a.nt ? lo + B : a.nt;
    double cprev = 0.0;                        // c'_{i-1}
    for (int64_t i = lo; i < hi; i++) {
      const double ai = i > lo ? -(double)w0[i - 1] : 0.0;
      const double ci = i + 1 < hi ? -(double)w0[i] : 0.0;
      const double m = (double)a.D[i] - ai * cprev;
      const double im = 1.0 / m;
      const double cp = ci * im;
      a.bj_f[i] = -ai * im;
      a.bj_im[i] = im;
      a.bj_g[i] = -cp;
      cprev = cp;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bj_apply(CGArgs<T> a, int slot) {
  __shared__ double lds[4 * (kBlock / 64)];
  if (block_done(a.sc)) return;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t B = a.bj_block, nb = (a.nt + B - 1) / B;
  double x[1] = {0.0};
  for (int64_t k = wave; k < nb; k += nwaves) {
    const int64_t lo = k * B, hi = lo + B < a.nt ? lo + B : a.nt;
    const int64_t u0 = lo + 2 * lane;
    const bool v0 = u0 < hi, v1 = u0 + 1 < hi;
    const double r0 = v0 ? a.rbuf[u0] : 0.0, r1 = v1 ? a.rbuf[u0 + 1] : 0.0;
    const double f0 = v0 ? a.bj_f[u0] : 0.0, f1 = v1 ? a.bj_f[u0 + 1] : 0.0;
    const double i0 = v0 ? a.bj_im[u0] : 0.0, i1 = v1 ? a.bj_im[u0 + 1] : 0.0;
    const double g0 = v0 ? a.bj_g[u0] : 0.0, g1 = v1 ? a.bj_g[u0 + 1] : 0.0;
    // forward: this lane's pair maps y before it to y at its second row
    double A = f1 * f0, Bv = f1 * (i0 * r0) + i1 * r1;
    for (int d = 1; d < 64; d <<= 1) {
      const double Ap = __shfl_up(A, d, 64), Bp = __shfl_up(Bv, d, 64);
      if (lane >= d) {
        Bv = A * Bp + Bv;
        A = A * Ap;
      }
    }
    double yprev = __shfl_up(Bv, 1, 64);
    if (lane == 0) yprev = 0.0;
    const double y0 = f0 * yprev + i0 * r0, y1 = Bv;
    // backward: this lane's pair maps z after it to z at its first row
    double Cm = g0 * g1, Cb = y0 + g0 * y1;
    for (int d = 1; d < 64; d <<= 1) {
      const double Cn = __shfl_down(Cm, d, 64), Cbn = __shfl_down(Cb, d, 64);
      if (lane + d < 64) {
        Cb = Cm * Cbn + Cb;
        Cm = Cm * Cn;
      }
    }
    double znext = __shfl_down(Cb, 1, 64);
    if (lane == 63) znext = 0.0;
    const double z0 = Cb, z1 = y1 + g1 * znext;
    if (v0) a.z[u0] = (T)z0;
    if (v1) a.z[u0 + 1] = (T)z1;
    x[0] += r0 * z0 + r1 * z1;
  }
  write_partials<1>(x, a.partials, slot, lds);
}

// ----------------------------------------------------------------------------
// Block-Jacobi with ILU(0) blocks (Section 3.1, the second block strategy): the
// blocks are cubic tiles of B x B x B rows of a 3-D grid in its natural order
// (x fastest, then y, then z).  A grid graph has no triangles, so ILU(0) of a
// tile leaves every off-diagonal entry as it is (U_ij = A_ij, L_ik = A_ik / d_k)
// and changes only the pivots:
//   d_i = D_i - sum over the tile's lower neighbours k (z-1, y-1, x-1 in that
//         order) of (A_ik / d_k) A_ki,       A_ik = -w_ik.
// z = (LU)^-1 r by forward substitution y_i = r_i - sum_k (A_ik / d_k) y_k and
// backward substitution z_i = (y_i - sum_j A_ij z_j) / d_i over the upper
// neighbours j (x+1, y+1, z+1).  One thread per tile; it moves the tile's x
// segments (B consecutive rows) as vectors and keeps y in registers.  Tiles
// are numbered x fastest, so a wavefront's segments are contiguous.  Since
// U = D L^T here, r^T z = y^T D^-1 y comes out of the forward pass.
// ----------------------------------------------------------------------------
struct IluTiles {
  int64_t N, P, nz, tx, ty, tiles;
};

template <typename T>
__device__ __forceinline__ IluTiles ilu_tiles(const CGArgs<T> &a, int B) {
  IluTiles t;
  t.N = a.off[1];
  t.P = a.off[2];
  t.nz = a.nt / t.P;
  t.tx = t.N / B;
  t.ty = t.P / t.N / B;
  t.tiles = t.tx * t.ty * ((t.nz + B - 1) / B);
  return t;
}

// first row of tile k's segment (dy, dz), and whether that plane exists
__device__ __forceinline__ int64_t ilu_seg(const IluTiles &t, int B, int64_t k, int dy, int dz, bool &ok) {
  const int64_t x = (k % t.tx) * B, y = ((k / t.tx) % t.ty) * B + dy, z = (k / (t.tx * t.ty)) * B + dz;
  ok = z < t.nz;
  return z * t.P + y * t.N + x;
}

// The pivots are formed in FP64 from the working-precision D and w and stored
// in the working precision (FP32 only in the precision form, 4x4x4 tiles).
template <typename T, int B>
__device__ __forceinline__ vec_t<double, B> vload_f64(const T *p) {
  return __builtin_convertvector(vload<T, B>(p), vec_t<double, B>);
}

template <typename T, int B>
__global__ __launch_bounds__(kBlock) void k_ilu_factor(CGArgs<T> a) {
  typedef vec_t<double, B> V;
  const IluTiles tl = ilu_tiles(a, B);
  const int64_t nt = a.nt;
  const T *w0 = a.w, *w1 = a.w + nt, *w2 = a.w + 2 * nt;
  for (int64_t k = row_begin(); k < tl.tiles; k += row_stride()) {
    V d[B][B];                                     // pivots by (dz, dy), x in the vector
#pragma unroll
    for (int dz = 0; dz < B; dz++) {
#pragma unroll
      for (int dy = 0; dy < B; dy++) {
        bool ok;
        const int64_t u = ilu_seg(tl, B, k, dy, dz, ok);
        if (!ok) continue;
        const V D = vload_f64<T, B>(a.D + u);
        const V wx = vload_f64<T, B>(w0 + u);      // wx[i] couples rows i and i + 1
        const V wy = dy > 0 ? vload_f64<T, B>(w1 + u - tl.N) : V(0.0);
        const V wz = dz > 0 ? vload_f64<T, B>(w2 + u - tl.P) : V(0.0);
        V piv;
#pragma unroll
        for (int i = 0; i < B; i++) {
          double p = D[i];
          if (dz > 0) p -= (-wz[i] / d[dz - 1][dy][i]) * (-wz[i]);
          if (dy > 0) p -= (-wy[i] / d[dz][dy - 1][i]) * (-wy[i]);
          if (i > 0) p -= (-wx[i - 1] / piv[i - 1]) * (-wx[i - 1]);
          piv[i] = p;
        }
        d[dz][dy] = piv;
        vstore<T, B>(a.bj_im + u, __builtin_convertvector(piv, vec_t<T, B>));
      }
    }
  }
}

template <int B>
__global__ __launch_bounds__(kBlock) void k_ilu_apply(CGArgs<double> a, int slot) {
  __shared__ double lds[4 * (kBlock / 64)];
  if (block_done(a.sc)) return;
  typedef vec_t<double, B> V;
  const IluTiles tl = ilu_tiles(a, B);
  const int64_t nt = a.nt;
  const double *w0 = a.w, *w1 = a.w + nt, *w2 = a.w + 2 * nt;
  double x[1] = {0.0};
  for (int64_t k = row_begin(); k < tl.tiles; k += row_stride()) {
    V y[B][B];
    // forward: y_i = r_i - sum_k (A_ik / d_k) y_k over the lower neighbours
#pragma unroll
    for (int dz = 0; dz < B; dz++) {
#pragma unroll
      for (int dy = 0; dy < B; dy++) {
        bool ok;
        const int64_t u = ilu_seg(tl, B, k, dy, dz, ok);
        if (!ok) continue;
        const V r = vload<double, B>(a.rbuf + u);
        const V d = vload<double, B>(a.bj_im + u);
        const V wx = vload<double, B>(w0 + u);
        const V wy = dy > 0 ? vload<double, B>(w1 + u - tl.N) : V(0.0);
        const V wz = dz > 0 ? vload<double, B>(w2 + u - tl.P) : V(0.0);
        const V dyp = dy > 0 ? vload<double, B>(a.bj_im + u - tl.N) : V(1.0);
        const V dzp = dz > 0 ? vload<double, B>(a.bj_im + u - tl.P) : V(1.0);
        V yv;
#pragma unroll
        for (int i = 0; i < B; i++) {
          double v = r[i];
          if (dz > 0) v -= (-wz[i] / dzp[i]) * y[dz - 1][dy][i];
          if (dy > 0) v -= (-wy[i] / dyp[i]) * y[dz][dy - 1][i];
          if (i > 0) v -= (-wx[i - 1] / d[i - 1]) * yv[i - 1];
          yv[i] = v;
          x[0] += v * v / d[i];
        }
        y[dz][dy] = yv;
      }
    }
    // backward: z_i = (y_i - sum_j A_ij z_j) / d_i over the upper neighbours
#pragma unroll
    for (int dz = B - 1; dz >= 0; dz--) {
#pragma unroll
      for (int dy = B - 1; dy >= 0; dy--) {
        bool ok;
        const int64_t u = ilu_seg(tl, B, k, dy, dz, ok);
        if (!ok) continue;
        bool okz;
        (void)ilu_seg(tl, B, k, dy, dz + 1 < B ? dz + 1 : dz, okz);
        const bool up_z = dz + 1 < B && okz;
        const V d = vload<double, B>(a.bj_im + u);
        const V wx = vload<double, B>(w0 + u);
        const V wy = dy + 1 < B ? vload<double, B>(w1 + u) : V(0.0);
        const V wz = up_z ? vload<double, B>(w2 + u) : V(0.0);
        V zv;
#pragma unroll
        for (int i = B - 1; i >= 0; i--) {
          double v = y[dz][dy][i];
          if (i + 1 < B) v -= (-wx[i]) * zv[i + 1];
          if (dy + 1 < B) v -= (-wy[i]) * y[dz][dy + 1][i];
          if (up_z) v -= (-wz[i]) * y[dz + 1][dy][i];
          zv[i] = v / d[i];
        }
        y[dz][dy] = zv;                              // z overwrites y, which is no longer needed
        vstore<double, B>(a.z + u, zv);
      }
    }
  }
  write_partials<1>(x, a.partials, slot, lds);
}

// The same ILU(0) application for 4x4x4 tiles, a wavefront per four tiles
// that are neighbours in x: lane (q, y, z) = 16 q + 4 z + y owns the x
// segment (4 rows, one 32-byte vector per array) at (y, z) of tile q.  Each
// lane loads its own segment once: r, the pivots, and its edges to x + 1,
// y + 1 and z + 1; the edges from below and the neighbours' values come from
// the lanes one and four below (or above), which lie in the same row of 16
// lanes, by DPP row shifts.  The substitutions run as wavefronts over the
// anti-diagonals y + z (seven steps each way); within a segment the x
// recurrence runs in the lane.  Every lane forms 1/d and the forward
// multipliers A_ik / d_k once, before the steps, so the steps (where at most
// four lanes in sixteen are active) hold only fused multiply-adds.  The sums
// are the thread-per-tile kernel's, in its order, except that it divides by
// d where this kernel multiplies by 1/d.
//
// DPP row shifts: with row_shr:S lane i reads lane i - S, with row_shl:S lane
// i + S, both within lane i's row of 16; a lane whose source lies outside its
// row reads 0.
constexpr int kDppRowShl1 = 0x101, kDppRowShl4 = 0x104, kDppRowShr1 = 0x111, kDppRowShr4 = 0x114;

template <int CTRL>
__device__ __forceinline__ int dpp_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)dpp_int<CTRL>((int)(unsigned)b);
  const unsigned hi = (unsigned)dpp_int<CTRL>((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int CTRL, typename T, int W>
__device__ __forceinline__ vec_t<T, W> dppv(vec_t<T, W> v) {
  vec_t<T, W> o;
#pragma unroll
  for (int i = 0; i < W; i++) {
    if constexpr (sizeof(T) == 8) o[i] = dpp_double<CTRL>(v[i]);
    else o[i] = __int_as_float(dpp_int<CTRL>(__float_as_int(v[i])));
  }
  return o;
}

// MODE 0: z = M^-1 r of the residual in rbuf, r^T z into partial slot `slot`.
// MODE 1: the CG vector update of the iteration is fused in (v += alpha p,
// r -= alpha q on each lane's own segment, then the application to the new
// r), so r is not read back, and the kernel writes the partial sums
// [r^T z, ||r||^2] that k_update_bj and the application write separately.
// MODE 2 (precision form): the FP64 residual replacement of these tiles.  When
// it is due (replace_due), r = b - L~ v is formed in FP64 from the FP64
// conductances and potentials, rounded into rbuf, and the application follows;
// the partial sums are [r^T z, ||r||^2 of the FP64 residual].
// T is the working precision: the residual, pivots, conductances, direction
// and z, and the substitutions' arithmetic; the potentials and every sum are
// FP64.  With T = double the sums are the FP64 kernel's.
// TPL tiles per lane: with TPL = 2 (FP32, an even number of tiles along x)
// lane (q, y, z) owns the (y, z) segments of tiles 2q and 2q + 1 of its
// wavefront's eight, which are adjacent in x: 8 rows, one 32-byte vector per
// array as in FP64, and two independent recurrences in each step.
// VU (MODE 1): how the potentials move.  0: v += alpha p every iteration.
// In the CG iterations they move every second iteration, as in the scaled
// form: 1 (even iterations) leaves v alone and reads no direction;
// 2 (odd iterations) adds alpha_{i-1} p_{i-1} + alpha_i p_i (p_{i-1} is in p1,
// p_i in p0).  A step left pending when CG stops is added by k_flush_v, and
// the replacement includes it.  The kernel checks the parity the host chose.
template <typename T, int MODE, int TPL, bool PF, int VU>
__global__ __launch_bounds__(kBlock) void k_ilu_apply4w(CGArgs<T> a, int slot) {
  constexpr int S = 4 * TPL;                                     // rows per lane
  __shared__ double lds[4 * (kBlock / 64)];
  __shared__ double bc[4];
  int64_t it = 0;
  double alpha = 0.0, pq = 0.0, alpha_prev = 0.0;
  if constexpr (MODE == 1) {
    if constexpr (VU == 2) alpha_prev = a.sc->alpha_par[0];
    if (!cg_update_start(a, lds, bc, it, alpha, pq)) return;
    if constexpr (VU != 0) {
      if (((it & 1) != 0) != (VU == 2)) {                        // the launch sequence is out of step
        if (first_thread()) { a.sc->done = 1; a.sc->status = IRLS_ERR_DEVICE; }
        return;
      }
    }
  } else if constexpr (MODE == 2) {
    if (!replace_due(a, lds, bc, it)) return;
  } else {
    if (block_done(a.sc)) return;
  }
  typedef vec_t<T, S> V;
  const IluTiles tl = ilu_tiles(a, 4);
  const int64_t nt = a.nt;
  const T *w0 = a.w, *w1 = a.w + nt, *w2 = a.w + 2 * nt;
  const T *__restrict__ pdir = (a.K > 0 && (it & 1) == 0) ? a.p1 : a.p0;   // the SpMV's direction
  const int lane = threadIdx.x & 63, q = lane >> 4, y = lane & 3, z = (lane >> 2) & 3;
  const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwv = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const V zero = (T)0;
  double x[2] = {0.0, 0.0};
  // one trip's loads; with PF (prefetch) the next trip's are issued before
  // this trip's substitutions, so they are in flight while those run
  struct TripLoads {
    V r0, qv, pv, pp, d, wx, wy, wz;
    vec_t<double, S> vv;
    int64_t u;
    bool ok;
  };
  auto fetch = [&](int64_t tb_, TripLoads &L) {
    const int64_t k = tb_ + q * TPL;
    L.ok = false;
    L.u = 0;
    if (k < tl.tiles) L.u = ilu_seg(tl, 4, k, y, z, L.ok);
    const bool ok = L.ok;
    const int64_t u = L.u;
    if constexpr (MODE != 2) L.r0 = ok ? vload<T, S>(a.rbuf + u) : zero;
    if constexpr (MODE == 1) {
      L.qv = ok ? vload<T, S>(a.q + u) : zero;
      if constexpr (VU != 1) {
        L.pv = ok ? vload<T, S>(pdir + u) : zero;
        L.vv = ok ? vload<double, S>(a.v + u) : vec_t<double, S>(0.0);
      }
      if constexpr (VU == 2) L.pp = ok ? vload<T, S>(a.p1 + u) : zero;
    }
    L.d = ok ? vload<T, S>(a.bj_im + u) : V((T)1);
    L.wx = ok ? vload<T, S>(w0 + u) : zero;                    // wx[i] couples rows i and i + 1
    L.wy = ok ? vload<T, S>(w1 + u) : zero;                    // edges to y + 1
    L.wz = ok ? vload<T, S>(w2 + u) : zero;                    // edges to z + 1
  };
  const int64_t step = nwv * 4 * TPL;
  TripLoads cur;
  fetch(wv * 4 * TPL, cur);
  for (int64_t tb = wv * 4 * TPL; tb < tl.tiles; tb += step) {   // the same trip count on every lane
    TripLoads nxt;
    if constexpr (PF) fetch(tb + step, nxt);
    const bool ok = cur.ok;
    const int64_t u = cur.u;
    V r;
    if constexpr (MODE == 1) {
      if (ok) {
        vec_t<double, S> vv = cur.vv;
#pragma unroll
        for (int i = 0; i < S; i++) {
          if constexpr (VU == 0) vv[i] += alpha * (double)cur.pv[i];
          if constexpr (VU == 2) vv[i] += alpha_prev * (double)cur.pp[i] + alpha * (double)cur.pv[i];
          r[i] = (T)((double)cur.r0[i] - alpha * (double)cur.qv[i]);
          x[1] += (double)r[i] * (double)r[i];
        }
        if constexpr (VU != 1) vstore<double, S>(a.v + u, vv);
        vstore<T, S>(a.rbuf + u, r);
      } else {
        r = zero;
      }
    } else if constexpr (MODE == 2) {
      if (ok) {
        // L~ v on the lane's segment from vector loads: the FP64 conductances
        // of edges that do not exist are stored as zeros, so every neighbour
        // term is formed (a neighbour outside the grid reads as 0) and the
        // sums are row_apply64's, in its order (offsets 1, N, P; the edge
        // to the higher row, then to the lower one)
        typedef vec_t<double, S> V64;
        const double *W = a.w64 ? a.w64 : (const double *)a.w;
        const double *Dv = a.D64 ? a.D64 : (const double *)a.D;
        const V64 z64 = 0.0;
        // the true potentials: v plus the step an even iteration left pending
        // (iter_b odd; its direction is in p1)
        const bool pend = (it & 1) != 0;
        const double ap = pend ? a.sc->alpha_par[0] : 0.0;
        auto vseg = [&](int64_t at) -> V64 {
          V64 w = vload<double, S>(a.v + at);
          if (pend) {
            const V pp = vload<T, S>(a.p1 + at);
#pragma unroll
            for (int i = 0; i < S; i++) w[i] += ap * (double)pp[i];
          }
          return w;
        };
        auto vone = [&](int64_t at) { return a.v[at] + (pend ? ap * (double)a.p1[at] : 0.0); };
        const V64 vc = vseg(u);
        const double vxm = u >= 1 ? vone(u - 1) : 0.0, vxp = u + S < nt ? vone(u + S) : 0.0;
        const V64 vym = u >= tl.N ? vseg(u - tl.N) : z64;
        const V64 vyp = u + tl.N < nt ? vseg(u + tl.N) : z64;
        const V64 vzm = u >= tl.P ? vseg(u - tl.P) : z64;
        const V64 vzp = u + tl.P < nt ? vseg(u + tl.P) : z64;
        const V64 gx = vload<double, S>(W + u), gy = vload<double, S>(W + nt + u);
        const V64 gz = vload<double, S>(W + 2 * nt + u);
        const double gxm = u >= 1 ? W[u - 1] : 0.0;
        const V64 gym = u >= tl.N ? vload<double, S>(W + nt + u - tl.N) : z64;
        const V64 gzm = u >= tl.P ? vload<double, S>(W + 2 * nt + u - tl.P) : z64;
        const V64 dd = vload<double, S>(Dv + u), bv = vload<double, S>(a.b + u);
#pragma unroll
        for (int i = 0; i < S; i++) {
          double acc = dd[i] * vc[i];
          acc -= gx[i] * (i < S - 1 ? vc[i + 1] : vxp);
          acc -= (i > 0 ? gx[i - 1] : gxm) * (i > 0 ? vc[i - 1] : vxm);
          acc -= gy[i] * vyp[i];
          acc -= gym[i] * vym[i];
          acc -= gz[i] * vzp[i];
          acc -= gzm[i] * vzm[i];
          const double r64 = bv[i] - acc;
          r[i] = (T)r64;
          x[1] += r64 * r64;
        }
        vstore<T, S>(a.rbuf + u, r);
      } else {
        r = zero;
      }
    } else {
      r = cur.r0;
    }
    const V d = cur.d, wx = cur.wx, wy = cur.wy, wz = cur.wz;
    V di;
#pragma unroll
    for (int i = 0; i < S; i++) di[i] = (T)1 / d[i];
    // every lane takes part in the row shifts (a shift inside a condition
    // would read lanes that skipped it)
    const V wy_lo = dppv<kDppRowShr1>(wy), wz_lo = dppv<kDppRowShr4>(wz);   // edges from y - 1, z - 1
    const V di_ylo = dppv<kDppRowShr1>(di), di_zlo = dppv<kDppRowShr4>(di);
    V ly, lz, lx;                                                // -L_ik = w_ik / d_k
#pragma unroll
    for (int i = 0; i < S; i++) {
      ly[i] = wy_lo[i] * di_ylo[i];
      lz[i] = wz_lo[i] * di_zlo[i];
      lx[i] = (i & 3) > 0 ? wx[i - 1] * di[i - 1] : (T)0;        // within the row's own tile
    }
    const int ok_up_y = dpp_int<kDppRowShl1>((int)ok), ok_up_z = dpp_int<kDppRowShl4>((int)ok);
    const bool ok_yup = y < 3 && ok_up_y != 0;
    const bool ok_zup = z < 3 && ok_up_z != 0;
    // forward: y_i = r_i - sum_k (A_ik / d_k) y_k over z - 1, y - 1, x - 1
    V yv = zero;
    for (int st = 0; st <= 6; st++) {
      const V yy = dppv<kDppRowShr1>(yv), yz = dppv<kDppRowShr4>(yv);
      if (ok && y + z == st) {
        V t;
#pragma unroll
        for (int i = 0; i < S; i++) {
          T v = r[i];
          if (z > 0) v += lz[i] * yz[i];
          if (y > 0) v += ly[i] * yy[i];
          if ((i & 3) > 0) v += lx[i] * t[i - 1];
          t[i] = v;
        }
        yv = t;
      }
    }
    if (ok) {
#pragma unroll
      for (int i = 0; i < S; i++) x[0] += (double)yv[i] * (double)yv[i] * (double)di[i];   // r^T z = y^T D^-1 y
    }
    // backward: z_i = (y_i - sum_j A_ij z_j) / d_i over x + 1, y + 1, z + 1
    V zv = zero;
    for (int st = 6; st >= 0; st--) {
      const V zy = dppv<kDppRowShl1>(zv), zz = dppv<kDppRowShl4>(zv);
      if (ok && y + z == st) {
        V t;
#pragma unroll
        for (int i = S - 1; i >= 0; i--) {
          T v = yv[i];
          if ((i & 3) < 3) v += wx[i] * t[i + 1];
          if (ok_yup) v += wy[i] * zy[i];
          if (ok_zup) v += wz[i] * zz[i];
          t[i] = v * di[i];
        }
        zv = t;
      }
    }
    if (ok) vstore<T, S>(a.z + u, zv);
    if constexpr (PF) cur = nxt;
    else fetch(tb + step, cur);
  }
  if constexpr (MODE == 1) {
    write_partials<2>(x, a.partials, kPUpd, lds);
    if (first_thread()) {
      a.sc->iter_b = it + 1;
      a.sc->alpha = alpha;
      if constexpr (VU != 0) a.sc->alpha_par[it & 1] = alpha;
      a.sc->pq = pq;
    }
  } else if constexpr (MODE == 2) {
    write_partials<2>(x, a.partials, kPRep, lds);
  } else {
    double x1[1] = {x[0]};
    write_partials<1>(x1, a.partials, slot, lds);
  }
}

// Tiles per lane of k_ilu_apply4w: two in FP32 where the tiles along x come
// in pairs (lines a multiple of 8 rows), else one; one for the replacement.
template <typename T>
inline int ilu_tpl(const CGArgs<T> &a) {
  return (sizeof(T) == 4 && (a.off[1] / 4) % 2 == 0) ? 2 : 1;
}

template <typename T, int MODE, int VU>
void launch_ilu_apply4w_vu(const CGArgs<T> &a, int grid, int slot, hipStream_t st) {
  // the replacement (MODE 2) moves mostly FP64 data, already 32 bytes a lane
  // with one tile per lane, and two would double its live vectors
  if constexpr (sizeof(T) == 4 && MODE != 2) {
    if (ilu_tpl(a) == 2) {
      hipLaunchKernelGGL((k_ilu_apply4w<T, MODE, 2, MODE == 1, VU>), dim3(grid), dim3(kBlock), 0, st, a, slot);
      return;
    }
  }
  hipLaunchKernelGGL((k_ilu_apply4w<T, MODE, 1, false, VU>), dim3(grid), dim3(kBlock), 0, st, a, slot);
}

template <typename T, int MODE>
void launch_ilu_apply4w(const CGArgs<T> &a, int grid, int slot, hipStream_t st) {
  if constexpr (MODE == 1) {                                     // paired potential updates
    if (a.it_hint & 1) launch_ilu_apply4w_vu<T, 1, 2>(a, grid, slot, st);
    else launch_ilu_apply4w_vu<T, 1, 1>(a, grid, slot, st);
  } else {
    launch_ilu_apply4w_vu<T, MODE, 0>(a, grid, slot, st);
  }
}

// ILU(0) of 8x8x8 tiles, a wavefront per tile: lane y + 8 z owns the x
// segment (8 rows) at (y, z).  Its y neighbours are the lanes one below and
// one above, in the same row of 16 lanes (DPP row shifts); its z neighbours
// are eight lanes away, in the next row of 16 for half of the lanes, and come
// by __shfl.  The wavefront steps run over the anti-diagonals y + z (fifteen
// each way).  The factorisation has the same wavefront form as the forward
// substitution: a pivot needs the pivots of its lower neighbours.  The sums
// are those of the thread-per-tile kernels, in their order (the application
// multiplies by 1/d where they divide by d).
__device__ __forceinline__ void load8(const double *p, double (&v)[8]) {
  const vec_t<double, 4> lo = vload<double, 4>(p), hi = vload<double, 4>(p + 4);
#pragma unroll
  for (int i = 0; i < 4; i++) {
    v[i] = lo[i];
    v[i + 4] = hi[i];
  }
}

__device__ __forceinline__ void store8(double *p, const double (&v)[8]) {
  vec_t<double, 4> lo, hi;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    lo[i] = v[i];
    hi[i] = v[i + 4];
  }
  vstore<double, 4>(p, lo);
  vstore<double, 4>(p + 4, hi);
}

template <int CTRL>
__device__ __forceinline__ void dpp8(const double (&v)[8], double (&o)[8]) {
#pragma unroll
  for (int i = 0; i < 8; i++) o[i] = dpp_double<CTRL>(v[i]);
}

__device__ __forceinline__ void shfl8(const double (&v)[8], int src, double (&o)[8]) {
#pragma unroll
  for (int i = 0; i < 8; i++) o[i] = __shfl(v[i], src, 64);
}

__global__ __launch_bounds__(kBlock) void k_ilu_factor8w(CGArgs<double> a) {
  const IluTiles tl = ilu_tiles(a, 8);
  const int64_t nt = a.nt;
  const double *w0 = a.w, *w1 = a.w + nt, *w2 = a.w + 2 * nt;
  const int lane = threadIdx.x & 63, y = lane & 7, z = lane >> 3;
  const int lo_z = lane >= 8 ? lane - 8 : lane;
  const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwv = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t k = wv; k < tl.tiles; k += nwv) {                // uniform across the wavefront
    bool ok;
    const int64_t u = ilu_seg(tl, 8, k, y, z, ok);
    double D[8], wx[8], wy[8], wz[8];
    if (ok) {
      load8(a.D + u, D);
      load8(w0 + u, wx);                                        // wx[i] couples rows i and i + 1
      load8(w1 + u, wy);                                        // edges to y + 1
      load8(w2 + u, wz);                                        // edges to z + 1
    } else {
#pragma unroll
      for (int i = 0; i < 8; i++) {
        D[i] = 1.0;
        wx[i] = wy[i] = wz[i] = 0.0;
      }
    }
    double wy_lo[8], wz_lo[8];                                  // edges from y - 1, z - 1
    dpp8<kDppRowShr1>(wy, wy_lo);
    shfl8(wz, lo_z, wz_lo);
    double piv[8];
#pragma unroll
    for (int i = 0; i < 8; i++) piv[i] = 1.0;
    for (int st = 0; st <= 14; st++) {
      double dy[8], dz[8];
      dpp8<kDppRowShr1>(piv, dy);
      shfl8(piv, lo_z, dz);
      if (ok && y + z == st) {
#pragma unroll
        for (int i = 0; i < 8; i++) {
          double p = D[i];
          if (z > 0) p -= (-wz_lo[i] / dz[i]) * (-wz_lo[i]);
          if (y > 0) p -= (-wy_lo[i] / dy[i]) * (-wy_lo[i]);
          if (i > 0) p -= (-wx[i - 1] / piv[i - 1]) * (-wx[i - 1]);
          piv[i] = p;
        }
      }
    }
    if (ok) store8(a.bj_im + u, piv);
  }
}

__global__ __launch_bounds__(kBlock) void k_ilu_apply8w(CGArgs<double> a, int slot) {
  __shared__ double lds[4 * (kBlock / 64)];
  if (block_done(a.sc)) return;
  const IluTiles tl = ilu_tiles(a, 8);
  const int64_t nt = a.nt;
  const double *w0 = a.w, *w1 = a.w + nt, *w2 = a.w + 2 * nt;
  const int lane = threadIdx.x & 63, y = lane & 7, z = lane >> 3;
  const int lo_z = lane >= 8 ? lane - 8 : lane, up_z = lane < 56 ? lane + 8 : lane;
  const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwv = ((int64_t)gridDim.x * blockDim.x) >> 6;
  double x[1] = {0.0};
  for (int64_t k = wv; k < tl.tiles; k += nwv) {                // uniform across the wavefront
    bool ok;
    const int64_t u = ilu_seg(tl, 8, k, y, z, ok);
    double r[8], di[8], wx[8], wy[8], wz[8];
    if (ok) {
      load8(a.rbuf + u, r);
      load8(a.bj_im + u, di);
      load8(w0 + u, wx);
      load8(w1 + u, wy);
      load8(w2 + u, wz);
    } else {
#pragma unroll
      for (int i = 0; i < 8; i++) {
        r[i] = wx[i] = wy[i] = wz[i] = 0.0;
        di[i] = 1.0;
      }
    }
#pragma unroll
    for (int i = 0; i < 8; i++) di[i] = 1.0 / di[i];
    // every lane takes part in the shifts and shuffles (one inside a
    // condition would read lanes that skipped it)
    double wy_lo[8], wz_lo[8], di_ylo[8], di_zlo[8];
    dpp8<kDppRowShr1>(wy, wy_lo);
    shfl8(wz, lo_z, wz_lo);
    dpp8<kDppRowShr1>(di, di_ylo);
    shfl8(di, lo_z, di_zlo);
    double ly[8], lz[8], lx[8];                                 // -L_ik = w_ik / d_k
#pragma unroll
    for (int i = 0; i < 8; i++) {
      ly[i] = wy_lo[i] * di_ylo[i];
      lz[i] = wz_lo[i] * di_zlo[i];
      lx[i] = i > 0 ? wx[i - 1] * di[i - 1] : 0.0;
    }
    const int ok_up_y = dpp_int<kDppRowShl1>((int)ok), ok_up_z = __shfl((int)ok, up_z, 64);
    const bool ok_yup = y < 7 && ok_up_y != 0;
    const bool ok_zup = z < 7 && ok_up_z != 0;
    // forward: y_i = r_i - sum_k (A_ik / d_k) y_k over z - 1, y - 1, x - 1
    double yv[8];
#pragma unroll
    for (int i = 0; i < 8; i++) yv[i] = 0.0;
    for (int st = 0; st <= 14; st++) {
      double yy[8], yz[8];
      dpp8<kDppRowShr1>(yv, yy);
      shfl8(yv, lo_z, yz);
      if (ok && y + z == st) {
#pragma unroll
        for (int i = 0; i < 8; i++) {
          double v = r[i];
          if (z > 0) v += lz[i] * yz[i];
          if (y > 0) v += ly[i] * yy[i];
          if (i > 0) v += lx[i] * yv[i - 1];
          yv[i] = v;
        }
      }
    }
    if (ok) {
#pragma unroll
      for (int i = 0; i < 8; i++) x[0] += yv[i] * yv[i] * di[i];       // r^T z = y^T D^-1 y
    }
    // backward: z_i = (y_i - sum_j A_ij z_j) / d_i over x + 1, y + 1, z + 1
    double zv[8];
#pragma unroll
    for (int i = 0; i < 8; i++) zv[i] = 0.0;
    for (int st = 14; st >= 0; st--) {
      double zy[8], zz[8];
      dpp8<kDppRowShl1>(zv, zy);
      shfl8(zv, up_z, zz);
      if (ok && y + z == st) {
#pragma unroll
        for (int i = 7; i >= 0; i--) {
          double v = yv[i];
          if (i < 7) v += wx[i] * zv[i + 1];
          if (ok_yup) v += wy[i] * zy[i];
          if (ok_zup) v += wz[i] * zz[i];
          zv[i] = v * di[i];
        }
      }
    }
    if (ok) store8(a.z + u, zv);
  }
  write_partials<1>(x, a.partials, slot, lds);
}

// ----------------------------------------------------------------------------
// ILU(0) of general blocks of a CSR graph (bj_kind 3): block k is the rows
// blk_rows[blk_ptr[k] .. blk_ptr[k+1]) in ascending order (a piece of a
// breadth-first ordering, chosen on the host).  Saad's row-wise ILU(0) on the
// block's pattern: for each row i, for each lower entry k of row i in the
// block (ascending), l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for every
// entry j > k of row i that row k also holds (the diagonal included: the
// pivot).  One thread per block; ilu_f holds l_ik (k < i) and u_ij (j > i) per
// CSR entry, 0 for entries to other blocks, and bj_im the pivots u_ii.
// ----------------------------------------------------------------------------
// u_kj of row k (k's entry for column j), or the pivot when j == k; 0 if row k
// has no entry j
__device__ __forceinline__ double ilu_u(const CGArgs<double> &a, int64_t k, int64_t j) {
  if (j == k) return a.bj_im[k];
  int32_t lo = a.rowptr[k], hi = a.rowptr[k + 1];
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (a.col[mid] < j) lo = mid + 1;
    else hi = mid;
  }
  return lo < a.rowptr[k + 1] && a.col[lo] == j ? a.ilu_f[lo] : 0.0;
}

__global__ __launch_bounds__(kBlock) void k_ilu_csr_factor(CGArgs<double> a) {
  for (int64_t b = row_begin(); b < a.nblk; b += row_stride()) {
    const int32_t r0 = a.blk_ptr[b], r1 = a.blk_ptr[b + 1];
    for (int32_t q = r0; q < r1; q++) {
      const int64_t i = a.blk_rows[q];
      const int32_t e0 = a.rowptr[i], e1 = a.rowptr[i + 1];
      for (int32_t e = e0; e < e1; e++)                     // the block's part of row i of L~
        a.ilu_f[e] = a.row_blk[a.col[e]] == b ? -(double)a.w[e] : 0.0;
      double piv = a.D[i];
      for (int32_t e = e0; e < e1; e++) {
        const int64_t k = a.col[e];
        if (k >= i) break;
        if (a.row_blk[k] != b) continue;                    // another block
        const double l = a.ilu_f[e] / a.bj_im[k];
        a.ilu_f[e] = l;
        for (int32_t e2 = e + 1; e2 < e1; e2++) {           // entries j > k of row i
          const int64_t j = a.col[e2];
          if (a.row_blk[j] != b) continue;
          a.ilu_f[e2] -= l * ilu_u(a, k, j);
        }
        piv -= l * ilu_u(a, k, i);                          // j = i: the pivot
      }
      a.bj_im[i] = piv;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_ilu_csr_apply(CGArgs<double> a, int slot) {
  __shared__ double lds[4 * (kBlock / 64)];
  if (block_done(a.sc)) return;
  double x[1] = {0.0};
  for (int64_t b = row_begin(); b < a.nblk; b += row_stride()) {
    const int32_t r0 = a.blk_ptr[b], r1 = a.blk_ptr[b + 1];
    for (int32_t q = r0; q < r1; q++) {                     // y = L^-1 r, L unit lower
      const int64_t i = a.blk_rows[q];
      double v = a.rbuf[i];
      for (int32_t e = a.rowptr[i]; e < a.rowptr[i + 1]; e++) {
        const int64_t k = a.col[e];
        if (k >= i) break;
        const double f = a.ilu_f[e];
        if (f != 0.0) v -= f * a.z[k];
      }
      a.z[i] = v;
      x[0] += v * v / a.bj_im[i];                           // r^T z = y^T D^-1 y (U = D L^T)
    }
    for (int32_t q = r1 - 1; q >= r0; q--) {                // z = U^-1 y
      const int64_t i = a.blk_rows[q];
      double v = a.z[i];
      for (int32_t e = a.rowptr[i + 1] - 1; e >= a.rowptr[i]; e--) {
        const int64_t j = a.col[e];
        if (j <= i) break;
        const double f = a.ilu_f[e];
        if (f != 0.0) v -= f * a.z[j];
      }
      a.z[i] = v / a.bj_im[i];
    }
  }
  write_partials<1>(x, a.partials, slot, lds);
}

// vector update with the residual kept explicitly (block-Jacobi):
// v += alpha p, r -= alpha q; partial sums [0, ||r||^2] (k_bj_apply fills r^T z)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_bj(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  __shared__ double bc[4];
  Scalars *sc = a.sc;
  int64_t it;
  double alpha, pq;
  if (!cg_update_start(a, lds, bc, it, alpha, pq)) return;
  const T *__restrict__ p = (a.K > 0 && (it & 1) == 0) ? a.p1 : a.p0;
  double x[2] = {0.0, 0.0};
  FOR_ROWS(u, a.nt) {
    a.v[u] += alpha * (double)p[u];
    const double ru = a.rbuf[u] - alpha * (double)a.q[u];
    a.rbuf[u] = ru;
    x[1] += ru * ru;
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
  int64_t i = 0;
  if (!replace_due(a, lds, bc, i)) return;
  double x[2] = {0.0, 0.0};
  if (a.scaled) {
    // v holds D^1/2 v, and when the last update was an even iteration its
    // step alpha p (in p1) is still pending: both enter the true potentials.
    const bool pending = (i & 1) != 0;
    const double ap = pending ? sc->alpha_par[0] : 0.0;
    auto vtrue = [&](int64_t j) {
      const double vh = a.v[j] + (pending ? ap * (double)a.p1[j] : 0.0);
      return vh / sqrt(diag64(a, j));
    };
    const double *w = a.w64 ? a.w64 : (const double *)a.w;
    FOR_ROWS(u, a.nt) {
      double acc = diag64(a, u) * vtrue(u);
      for_each_nb<DIA>(a, u, [&](int64_t j, double, int64_t wi) { acc -= w[wi] * vtrue(j); });
      const double ru64 = a.b[u] - acc;
      const T zu = (T)(ru64 / sqrt(diag64(a, u)));
      a.z[u] = zu;
      x[0] += (double)zu * (double)zu;
      x[1] += ru64 * ru64;
    }
  } else {
    FOR_ROWS(u, a.nt) {
      double ru64 = a.b[u] - row_apply64<DIA>(a, u, a.v);
      T ru = (T)ru64;
      T zu = ru / a.D[u];
      a.z[u] = zu;
      x[0] += (double)ru * (double)zu;
      x[1] += (double)ru * (double)ru;
    }
  }
  write_partials<2>(x, a.partials, kPRep, lds);
}

// precision 1 on the symmetrically scaled system (diagonal layout, 16-byte
// row vectors): the same replacement, formed in the scaled variables with the
// round's FP64 scaled conductances wh64 = w / sqrt(D_u D_j):
//   r^ = D^-1/2 b - (v^ - W^ v^),   v^ = D^1/2 v (the CG variable, plus the
//   step alpha p an even iteration left pending),
// which equals D^-1/2 (b - L~ v) without a square root per neighbour.  Each
// thread takes R consecutive rows with unconditional vector loads; a
// neighbour outside the matrix is read at a valid index whose conductance is
// zero (as in the marching SpMV).  ||r||^2 = sum D_u r^_u^2 for the stopping
// test, r^T z = ||z||^2 with z = r^ rounded to T.
template <typename T, int K, int R>
__global__ __launch_bounds__(kBlock) void k_replace_scaled(CGArgs<T> a) {
  __shared__ double lds[4 * (kBlock / 64)];
  __shared__ double bc[4];
  typedef vec_t<double, R> VD;
  typedef vec_t<T, R> VT;
  Scalars *sc = a.sc;
  const int32_t done = sc->done;
  const int64_t i = sc->iter_b;
  const int32_t refine = sc->refine_every;
  const double bb = sc->bb;
  double t[3];
  {
    double u[2];
    partial_share<2>(a.partials, kPUpd, a.grid_main, u);
    t[0] = u[0];
    t[1] = u[1];
    t[2] = done != 0 ? 1.0 : 0.0;
  }
  block_allreduce<3, 0x4u>(t, lds, bc);
  if (t[2] != 0.0) return;
  const bool conv_rec = sqrt(t[1]) <= a.rtol * sqrt(bb);
  if (!(conv_rec || i % refine == 0)) return;
  const bool pending = (i & 1) != 0;
  const double ap = pending ? sc->alpha_par[0] : 0.0;
  const int64_t nt = a.nt;
  const double *__restrict__ wh = a.wh64;
  auto vhat = [&](int64_t j) -> VD {                     // R consecutive true scaled potentials
    const VD v = vload<double, R>(a.v + j);
    const VT p = vload<T, R>(a.p1 + j);
    VD o;
#pragma unroll
    for (int q = 0; q < R; q++) o[q] = v[q] + ap * (double)p[q];
    return o;
  };
  auto vhat1 = [&](int64_t j) -> double { return a.v[j] + ap * (double)a.p1[j]; };
  double x[2] = {0.0, 0.0};
  const int64_t ng = nt / R;
  FOR_ROWS(g, ng) {
    const int64_t u0 = g * R;
    const VD vc = vhat(u0);
    const VD w0 = vload<double, R>(wh + u0);
    const double vr = vhat1(u0 + R < nt ? u0 + R : u0);   // w0 of row nt - 1 is 0
    const double vl = vhat1(u0 > 0 ? u0 - 1 : u0);
    const double wl = wh[u0 > 0 ? u0 - 1 : nt - 1];       // row nt - 1 has no +1 edge
    VD acc = vc;
#pragma unroll
    for (int q = 0; q < R; q++) {
      acc[q] -= w0[q] * (q + 1 < R ? vc[q + 1] : vr);
      acc[q] -= (q > 0 ? w0[q - 1] : wl) * (q > 0 ? vc[q - 1] : vl);
    }
#pragma unroll
    for (int k = 1; k < K; k++) {
      const int64_t o = a.off[k];
      const bool f = u0 + o < nt, b = u0 >= o;
      const VD wf = vload<double, R>(wh + k * nt + u0);   // 0 where u + o is past the end
      const VD vf = vhat(f ? u0 + o : u0);
      const VD wb = vload<double, R>(wh + k * nt + (b ? u0 - o : nt - R));   // the last R rows have no +o edge
      const VD vb = vhat(b ? u0 - o : u0);
      acc -= wf * vf;
      acc -= wb * vb;
    }
    const VD bv = vload<double, R>(a.b + u0);
    const VD Dv = vload<double, R>(a.D64 + u0);
    VT zv;
#pragma unroll
    for (int q = 0; q < R; q++) {
      const double rh = bv[q] / sqrt(Dv[q]) - acc[q];
      zv[q] = (T)rh;
      x[0] += (double)zv[q] * (double)zv[q];
      x[1] += Dv[q] * rh * rh;
    }
    vstore<T, R>(a.z + u0, zv);
  }
  write_partials<2>(x, a.partials, kPRep, lds);
}

// ----------------------------------------------------------------------------
// Streaming probe: NR input and NW output streams of n doubles (input stream r
// at in + r n), two rows per thread with 16-byte loads and stores, rows in XCD
// slabs as the row-slab kernels take them.  Each output row gets the sum of
// the inputs (plus its stream index), so no load can be dropped.  It measures
// the bandwidth the GPU sustains for a given mix of streams, the ceiling the
// CG kernels' rooflines are read against.  NT: every access with the
// streaming (non-temporal) hint, which is faster for large streams (at 16.8M
// rows, five reads and two writes: 6.1 against 5.4 TB/s) and slower for ones
// the last-level cache can hold.
// ----------------------------------------------------------------------------
template <int NR, int NW, bool NT>
__global__ __launch_bounds__(kBlock) void k_stream(const double *__restrict__ in, double *__restrict__ out,
                                                  int64_t n) {
  typedef vec_t<double, 2> V;
  const int64_t ng = n / 2;
  auto ld = [](const double *q) { return NT ? vload_nt<double, 2>(q) : vload<double, 2>(q); };
  FOR_ROWS(g, ng) {
    V acc = ld(in + 2 * g);
#pragma unroll
    for (int r = 1; r < NR; r++) acc += ld(in + r * n + 2 * g);
#pragma unroll
    for (int w = 0; w < NW; w++) {
      if constexpr (NT) vstore_nt<double, 2>(out + w * n + 2 * g, acc + (double)w);
      else vstore<double, 2>(out + w * n + 2 * g, acc + (double)w);
    }
  }
}

template <int NR, bool NT>
hipError_t launch_stream_nr(const double *in, double *out, int64_t n, int nw, int grid, hipStream_t st) {
  if (nw == 1) hipLaunchKernelGGL((k_stream<NR, 1, NT>), dim3(grid), dim3(kBlock), 0, st, in, out, n);
  else hipLaunchKernelGGL((k_stream<NR, 2, NT>), dim3(grid), dim3(kBlock), 0, st, in, out, n);
  return hipGetLastError();
}

template <bool NT>
hipError_t launch_stream_form(const double *in, double *out, int64_t n, int nr, int nw, int grid, hipStream_t st) {
  switch (nr) {
    case 1: return launch_stream_nr<1, NT>(in, out, n, nw, grid, st);
    case 2: return launch_stream_nr<2, NT>(in, out, n, nw, grid, st);
    case 3: return launch_stream_nr<3, NT>(in, out, n, nw, grid, st);
    case 4: return launch_stream_nr<4, NT>(in, out, n, nw, grid, st);
    case 5: return launch_stream_nr<5, NT>(in, out, n, nw, grid, st);
    default: return launch_stream_nr<6, NT>(in, out, n, nw, grid, st);
  }
}

hipError_t launch_stream_probe(const double *in, double *out, int64_t n, int nr, int nw, int grid, bool nt,
                               hipStream_t st) {
  return nt ? launch_stream_form<true>(in, out, n, nr, nw, grid, st)
            : launch_stream_form<false>(in, out, n, nr, nw, grid, st);
}

// ----------------------------------------------------------------------------
// per-round diagnostics (Section 2.1-2.2): smoothed objective, ||CBx||_1,
// flow value x^T L x and the flows at s and t (Proposition 3), the range of v
// (Proposition 2), the true residual, and for the lower bound on the minimum
// cut rho = max g|d|/c, the overload sum max(0, g|d| - c) and ||r||_1;
// k_stats_final adds the partials.
// ----------------------------------------------------------------------------
// Diagnostics of one row: its interior edges' terms are added by the caller
// (each edge once, from its lower endpoint); this adds the terminal edges'
// terms, the squared true residual b_u - (L~ v)_u and the range of v.
// slots: s_eps, l1, flow, flow_s, flow_t, res^2, max(-v), max(v), max g|d|/c,
// overload, |res|
constexpr int kStatQ = 11;
constexpr unsigned kStatMax = 0x1C0u;                 // slots 6..8 are maxima
template <typename T>
__device__ __forceinline__ void stats_edge(const CGArgs<T> &a, double c, double g, double d,
                                           double (&x)[kStatQ]) {
  x[0] += a.form == 0 ? c * sqrt(d * d + a.eps_next) : sqrt((c * d) * (c * d) + a.eps_next);
  x[1] += c * fabs(d);
  x[2] += g * d * d;
  if (c > 0.0) {
    x[8] = fmax(x[8], g * fabs(d) / c);
    x[9] += fmax(0.0, g * fabs(d) - c);
  }
}

template <typename T>
__device__ __forceinline__ void stats_row_tail(const CGArgs<T> &a, int64_t u, double vu, double lv,
                                               double (&x)[kStatQ]) {
  const double cs = a.cs[u], ct = a.ct[u];
  if (cs > 0.0) {
    stats_edge(a, cs, a.b[u], 1.0 - vu, x);
    x[3] += a.b[u] * (1.0 - vu);
  }
  if (ct > 0.0) {
    stats_edge(a, ct, a.gt[u], vu, x);
    x[4] += a.gt[u] * vu;
  }
  const double res = a.b[u] - lv;
  x[5] += res * res;
  x[10] += fabs(res);
  x[6] = fmax(x[6], -vu);
  x[7] = fmax(x[7], vu);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_stats(CGArgs<T> a) {
  __shared__ double lds[kStatQ * (kBlock / 64)];
  const double *w = a.w64 ? a.w64 : (const double *)a.w;
  double x[kStatQ] = {0, 0, 0, 0, 0, 0, -INFINITY, -INFINITY, 0, 0, 0};
  FOR_ROWS(u, a.nt) {
    const double vu = a.v[u];
    for_each_nb<true>(a, u, [&](int64_t j, double c, int64_t wi) {
      if (j > u) stats_edge(a, c, w[wi], vu - a.v[j], x);    // each interior edge once
    });
    stats_row_tail(a, u, vu, row_apply64<true>(a, u, a.v), x);
  }
  write_partials<kStatQ, kStatMax>(x, a.partials, kPStats, lds);
}

template <typename T, int L>
__global__ __launch_bounds__(kBlock) void k_stats_csr(CGArgs<T> a) {
  __shared__ double lds[kStatQ * (kBlock / 64)];
  const double *w = a.w64 ? a.w64 : (const double *)a.w;
  const double *D = a.D64 ? a.D64 : (const double *)a.D;
  double x[kStatQ] = {0, 0, 0, 0, 0, 0, -INFINITY, -INFINITY, 0, 0, 0};
  for_row_groups<L>(a.nt, [&](int64_t u, int lid) {
    double off = 0.0, vu = 0.0;                // off: sum of w_uj v_j over row u's entries
    if (u >= 0) {
      vu = a.v[u];
      const int32_t e1 = a.rowptr[u + 1];
      for (int32_t e = a.rowptr[u] + lid; e < e1; e += L) {
        const int64_t j = a.col[e];
        const double vj = a.v[j];
        off += w[e] * vj;
        if (j > u) stats_edge(a, a.ccap[e], w[e], vu - vj, x);
      }
    }
    off = group_sum<L>(off);
    if (u >= 0 && lid == 0) stats_row_tail(a, u, vu, D[u] * vu - off, x);
  });
  write_partials<kStatQ, kStatMax>(x, a.partials, kPStats, lds);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_stats_final(CGArgs<T> a, int nblocks) {
  __shared__ double lds[kStatQ * (kBlock / 64)];
  __shared__ double bc[kStatQ];
  double tot[kStatQ];
  read_totals<kStatQ, kStatMax>(a.partials, kPStats, nblocks, tot, lds, bc);
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
  // Lower bound on the minimum cut from the electrical flow f = g d: its net
  // flow across any cut is at least F (the residual is each node's
  // imbalance); scaled by 1 / max(1, rho) it respects every capacity, and
  // across any cut it exceeds the capacity by at most the total overload.
  // The s-t edge carries g_st at d = 1.
  const double rho = a.cst > 0.0 ? fmax(tot[8], gst / a.cst) : tot[8];
  const double over = tot[9] + (a.cst > 0.0 ? fmax(0.0, gst - a.cst) : 0.0);
  const double F = fmax(R->flow_s, R->flow_t) - tot[10];
  R->lower_bound = fmax(F / fmax(1.0, rho), F - over);
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
// launch KERNEL<T, lanes> for a CSR kernel with `lanes` lanes per row
#define CSR_LANES(lanes, KERNEL, grid, st, a)                                                 \
  switch (lanes) {                                                                            \
    case 1: hipLaunchKernelGGL((KERNEL<T, 1>), dim3(grid), dim3(kBlock), 0, st, a); break;    \
    case 2: hipLaunchKernelGGL((KERNEL<T, 2>), dim3(grid), dim3(kBlock), 0, st, a); break;    \
    case 4: hipLaunchKernelGGL((KERNEL<T, 4>), dim3(grid), dim3(kBlock), 0, st, a); break;    \
    case 8: hipLaunchKernelGGL((KERNEL<T, 8>), dim3(grid), dim3(kBlock), 0, st, a); break;    \
    case 16: hipLaunchKernelGGL((KERNEL<T, 16>), dim3(grid), dim3(kBlock), 0, st, a); break;  \
    case 32: hipLaunchKernelGGL((KERNEL<T, 32>), dim3(grid), dim3(kBlock), 0, st, a); break;  \
    default: hipLaunchKernelGGL((KERNEL<T, 64>), dim3(grid), dim3(kBlock), 0, st, a); break;  \
  }

template <typename T>
hipError_t launch_assemble(const CGArgs<T> &a, int grid, hipStream_t st) {
  if (a.K > 0) hipLaunchKernelGGL((k_assemble<T>), dim3(grid), dim3(kBlock), 0, st, a);
  else CSR_LANES(a.csr_lanes, k_assemble_csr, grid, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cginit(const CGArgs<T> &a, int grid, hipStream_t st) {
  if (a.K > 0) hipLaunchKernelGGL((k_cginit<T>), dim3(grid), dim3(kBlock), 0, st, a);
  else CSR_LANES(a.csr_lanes, k_cginit_csr, grid, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_w(const CGArgs<T> &a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_scale_w<T>), dim3(grid), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_flush_v(const CGArgs<T> &a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_flush_v<T>), dim3(grid), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_v(const CGArgs<T> &a, int dir, int grid, hipStream_t st) {
  if (dir < 0) hipLaunchKernelGGL((k_flush_v<T>), dim3(grid), dim3(kBlock), 0, st, a);
  hipLaunchKernelGGL((k_scale_v<T>), dim3(grid), dim3(kBlock), 0, st, a, dir);
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

// Marching needs the vector layout, at least two planes, and planes of at
// least one full tile; the chunk length keeps the grid near kMarchGrid
// workgroups: one per CU, each keeping two steps of loads in flight per
// thread (measured faster than two or four per CU on 256^3 grids, and no
// slower on 128^3, where the longer chunks halve the re-read seams).
constexpr int kMarchGrid = 256;
constexpr double kLastLevelCacheBytes = 256.0 * 1024 * 1024;

// Whether a marching launch can take a tile shape: bs threads (256 or 512);
// ty = 0 (planes of at least one tile), or on 3-D grids ty >= 1 dividing bs,
// with planes made of whole lines of whole row groups and a tile no wider or
// taller than a plane.
template <typename T>
bool march_shape_ok(const CGArgs<T> &a, int bs, int ty) {
  constexpr int R = kVecRows<T>;
  if (bs != 256 && bs != 512) return false;
  const int64_t P = a.off[a.K - 1];
  if (ty == 0) return P / R >= bs;
  if (a.K != 3) return false;
  const int64_t N = a.off[1];
  if (ty < 1 || bs % ty != 0 || N <= 0 || P % N != 0 || N % R != 0) return false;
  return ty <= P / N && bs / ty <= N / R;
}

template <typename T>
int64_t march_tile_count(const CGArgs<T> &a, int bs, int ty) {
  constexpr int R = kVecRows<T>;
  const int64_t P = a.off[a.K - 1], N = a.K == 3 ? a.off[1] : P;
  return (bs == 256 ? march_tiles<R, 256>(P, N, ty) : march_tiles<R, 512>(P, N, ty)).tiles;
}

// The tile shape is the caller's (a.march_bs, a.march_ty) when a launch can
// take it, else 256 consecutive row groups.
template <typename T>
void spmv_layout(CGArgs<T> &a, int grid_main) {
  constexpr int R = kVecRows<T>;
  a.grid_spmv = grid_main;
  int bs = a.march_bs, ty = a.march_ty;
  a.march_planes = 0;
  a.march_bs = 0;
  a.march_ty = 0;
  // streaming accesses once a CG iteration's vectors and conductances (about
  // 104 B a row in FP64, 56 B in FP32) exceed the 256 MB last-level cache
  a.stream_nt = (double)a.nt * (sizeof(T) == 8 ? 104.0 : 56.0) > kLastLevelCacheBytes;
  if (a.K < 2 || !vec_ok(a)) return;
  if (!march_shape_ok(a, bs, ty)) {
    bs = 256;
    ty = 0;
  }
  if (!march_shape_ok(a, bs, ty)) return;
  const int64_t P = a.off[a.K - 1];
  const int64_t nplanes = (a.nt + P - 1) / P;
  const int64_t tiles = march_tile_count(a, bs, ty);
  if (nplanes < 2 || tiles > kMaxGrid) return;
  a.march_bs = bs;
  a.march_ty = ty;
  int64_t zc = (tiles * nplanes + kMarchGrid - 1) / kMarchGrid;
  if (zc < 4) zc = 4;
  int64_t grid = tiles * ((nplanes + zc - 1) / zc);
  while ((grid + kXcds - 1) / kXcds * kXcds > kMaxGrid) {       // never more partials than slots
    zc *= 2;
    grid = tiles * ((nplanes + zc - 1) / zc);
  }
  a.march_planes = (int32_t)zc;
  a.grid_spmv = (int)((grid + kXcds - 1) / kXcds * kXcds);
}

template <typename T>
int spmv_variant(const CGArgs<T> &a) {
  if (a.K == 0) return 0;
  if (a.march_planes > 0) return a.scaled ? 4 : 3;
  return vec_ok(a) ? 2 : 1;
}

template <typename T, int K, bool SC, int BS>
void launch_march(const CGArgs<T> &a, dim3 g, hipStream_t st) {
  constexpr int R = kVecRows<T>;
  if (a.stream_nt) hipLaunchKernelGGL((k_spmv_dia_march<T, K, R, SC, BS, true>), g, dim3(BS), 0, st, a);
  else hipLaunchKernelGGL((k_spmv_dia_march<T, K, R, SC, BS, false>), g, dim3(BS), 0, st, a);
}

template <typename T>
hipError_t launch_spmv(const CGArgs<T> &a, int grid, int rows_per_wave, bool, hipStream_t st) {
  constexpr int R = kVecRows<T>;
  if (a.march_planes > 0) {
    const dim3 g(a.grid_spmv);
    if (a.march_bs == 512) {
      if (a.scaled) {
        if (a.K == 2) launch_march<T, 2, true, 512>(a, g, st);
        else launch_march<T, 3, true, 512>(a, g, st);
      } else {
        if (a.K == 2) launch_march<T, 2, false, 512>(a, g, st);
        else launch_march<T, 3, false, 512>(a, g, st);
      }
    } else {
      if (a.scaled) {
        if (a.K == 2) launch_march<T, 2, true, 256>(a, g, st);
        else launch_march<T, 3, true, 256>(a, g, st);
      } else {
        if (a.K == 2) launch_march<T, 2, false, 256>(a, g, st);
        else launch_march<T, 3, false, 256>(a, g, st);
      }
    }
    return hipGetLastError();
  }
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
  if (a.csr_nheavy > 0) {
    const int64_t cg = (a.csr_nchunks * 64 + kBlock - 1) / kBlock;
    hipLaunchKernelGGL((k_spmv_csr_chunks<T>), dim3((unsigned)std::min<int64_t>(cg, kMaxGrid)), dim3(kBlock), 0, st, a);
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
hipError_t launch_bj_factor(const CGArgs<T> &a, int grid, hipStream_t st) {
  if constexpr (sizeof(T) == 8) {
    if (a.bj_kind == 3) {
      hipLaunchKernelGGL(k_ilu_csr_factor, dim3(grid), dim3(kBlock), 0, st, a);
      return hipGetLastError();
    }
    if (a.bj_kind == 2) {
      if (a.bj_tile == 2) hipLaunchKernelGGL((k_ilu_factor<double, 2>), dim3(grid), dim3(kBlock), 0, st, a);
      else if (a.bj_tile == 8) hipLaunchKernelGGL(k_ilu_factor8w, dim3(grid), dim3(kBlock), 0, st, a);
      else hipLaunchKernelGGL((k_ilu_factor<double, 4>), dim3(grid), dim3(kBlock), 0, st, a);
      return hipGetLastError();
    }
  } else if (bj_update_fused(a)) {             // the precision form's 4x4x4 tiles
    hipLaunchKernelGGL((k_ilu_factor<T, 4>), dim3(grid), dim3(kBlock), 0, st, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_bj_factor<T>), dim3(grid), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bj_apply(const CGArgs<T> &a, int grid, int slot, hipStream_t st) {
  if constexpr (sizeof(T) == 8) {
    if (a.bj_kind == 3) {
      hipLaunchKernelGGL(k_ilu_csr_apply, dim3(grid), dim3(kBlock), 0, st, a, slot);
      return hipGetLastError();
    }
    if (a.bj_kind == 2) {
      if (a.bj_tile == 2) hipLaunchKernelGGL((k_ilu_apply<2>), dim3(grid), dim3(kBlock), 0, st, a, slot);
      else if (a.bj_tile == 8) hipLaunchKernelGGL(k_ilu_apply8w, dim3(grid), dim3(kBlock), 0, st, a, slot);
      else launch_ilu_apply4w<double, 0>(a, grid, slot, st);
      return hipGetLastError();
    }
  } else if (bj_update_fused(a)) {
    launch_ilu_apply4w<T, 0>(a, grid, slot, st);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_bj_apply<T>), dim3(grid), dim3(kBlock), 0, st, a, slot);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_update(const CGArgs<T> &a, int grid, hipStream_t st) {
  if (bj_update_fused(a)) {                      // the update and the ILU(0) application in one kernel
    launch_ilu_apply4w<T, 1>(a, grid, (int)kPUpd, st);
    return hipGetLastError();
  }
  if (a.bj_block > 0)
    hipLaunchKernelGGL((k_update_bj<T>), dim3(grid), dim3(kBlock), 0, st, a);
  else if (a.scaled && (a.it_hint & 1))
    if (a.stream_nt) hipLaunchKernelGGL((k_update_scaled<T, kVecRows<T>, true, true>), dim3(grid), dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL((k_update_scaled<T, kVecRows<T>, true, false>), dim3(grid), dim3(kBlock), 0, st, a);
  else if (a.scaled)
    if (a.stream_nt) hipLaunchKernelGGL((k_update_scaled<T, kVecRows<T>, false, true>), dim3(grid), dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL((k_update_scaled<T, kVecRows<T>, false, false>), dim3(grid), dim3(kBlock), 0, st, a);
  else if (a.nt % kVecRows<T> == 0)
    hipLaunchKernelGGL((k_update_vec<T, kVecRows<T>>), dim3(grid), dim3(kBlock), 0, st, a);
  else
    hipLaunchKernelGGL((k_update<T>), dim3(grid), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_replace_residual(const CGArgs<T> &a, int grid, hipStream_t st) {
  constexpr int R = kVecRows<T>;
  if (bj_update_fused(a)) {                      // the replacement, then the ILU(0) application
    launch_ilu_apply4w<T, 2>(a, grid, (int)kPRep, st);
    return hipGetLastError();
  }
  if (a.scaled && a.wh64 && a.D64 && (a.K == 2 || a.K == 3) && vec_ok(a)) {
    if (a.K == 2) hipLaunchKernelGGL((k_replace_scaled<T, 2, R>), dim3(grid), dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL((k_replace_scaled<T, 3, R>), dim3(grid), dim3(kBlock), 0, st, a);
  } else if (a.K > 0) hipLaunchKernelGGL((k_replace<T, true>), dim3(grid), dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL((k_replace<T, false>), dim3(grid), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stats(const CGArgs<T> &a, int grid, hipStream_t st) {
  if (a.K > 0) hipLaunchKernelGGL((k_stats<T>), dim3(grid), dim3(kBlock), 0, st, a);
  else CSR_LANES(a.csr_lanes, k_stats_csr, grid, st, a);
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
  template hipError_t launch_scale_w<T>(const CGArgs<T> &, int, hipStream_t);              \
  template hipError_t launch_scale_v<T>(const CGArgs<T> &, int, int, hipStream_t);         \
  template hipError_t launch_flush_v<T>(const CGArgs<T> &, int, hipStream_t);              \
  template hipError_t launch_spmv<T>(const CGArgs<T> &, int, int, bool, hipStream_t);      \
  template void spmv_layout<T>(CGArgs<T> &, int);                                          \
  template int spmv_variant<T>(const CGArgs<T> &);                                         \
  template hipError_t launch_direction<T>(const CGArgs<T> &, int, hipStream_t);            \
  template hipError_t launch_update<T>(const CGArgs<T> &, int, hipStream_t);               \
  template hipError_t launch_bj_factor<T>(const CGArgs<T> &, int, hipStream_t);            \
  template hipError_t launch_bj_apply<T>(const CGArgs<T> &, int, int, hipStream_t);        \
  template hipError_t launch_replace_residual<T>(const CGArgs<T> &, int, hipStream_t);     \
  template hipError_t launch_stats<T>(const CGArgs<T> &, int, hipStream_t);
IRLS_INSTANTIATE(double)
IRLS_INSTANTIATE(float)

}  // namespace irls
