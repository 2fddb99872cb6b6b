// Two-level rounding of the final potentials (the paper's two-level rounding
// procedure): the GPU side.  K-means sums for the two centres, the split of
// the non-terminal nodes into S0 (x <= gamma0), S1 (x >= gamma1) and the
// middle set Sc, Sc's compaction to coarse ids in ascending node order, and
// the coarse graph's capacities as exact 128-bit fixed-point sums (the scale
// of the sweep), so that they do not depend on the order of summation.  The
// host finds the coarse minimum cut.  Rows are the CSR of the handle (each
// interior edge stored in both rows); s always lies in S1 and t in S0.
#include "device_common.h"

namespace irls {

typedef __int128 i128;

// round-half-even(c * 2^k) for c >= 0 (the sweep's fixed point)
__device__ __forceinline__ i128 tl_fx(double c, int k) {
  if (!(c > 0.0)) return 0;
  uint64_t bits = (uint64_t)__double_as_longlong(c);
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

// Per workgroup: count of potentials above m, their sum, and the sum of the
// rest (the workgroup partials are added by the host in order).
__global__ __launch_bounds__(kBlock) void k_tl_kmeans(const double *v, int64_t nt, double m, double *part) {
  __shared__ double lds[3 * (kBlock / 64)];
  double x[3] = {0.0, 0.0, 0.0};
  for (int64_t u = row_begin(); u < nt; u += row_stride()) {
    const double xu = v[u];
    if (xu > m) { x[0] += 1.0; x[1] += xu; }
    else x[2] += xu;
  }
  block_reduce<3>(x, lds);
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; q++) part[3 * (int64_t)blockIdx.x + q] = x[q];
}

// 0: S0, 1: S1, 2: Sc
__global__ __launch_bounds__(kBlock) void k_tl_classify(const double *v, int64_t nt, double g0, double g1,
                                                        int8_t *cls) {
  for (int64_t u = row_begin(); u < nt; u += row_stride()) {
    const double xu = v[u];
    cls[u] = xu <= g0 ? 0 : (xu >= g1 ? 1 : 2);
  }
}

// Workgroup b owns rows [b chunk, (b+1) chunk); thread i of it the
// consecutive sub-range [lo + i per, lo + (i+1) per).
struct TlRange {
  int64_t lo, hi;
};
__device__ __forceinline__ TlRange tl_rows(int64_t nt, int64_t chunk) {
  const int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = b0 + chunk < nt ? b0 + chunk : nt;
  const int64_t per = (chunk + blockDim.x - 1) / blockDim.x;
  int64_t lo = b0 + (int64_t)threadIdx.x * per, hi = lo + per;
  if (lo > b1) lo = b1;
  if (hi > b1) hi = b1;
  return {lo, hi};
}

// Exclusive prefix over the workgroup's threads (in thread order) and the total.
__device__ int64_t tl_block_scan(int64_t val, int64_t &total) {
  __shared__ int64_t s[kBlock];
  const int tid = threadIdx.x;
  s[tid] = val;
  __syncthreads();
  for (int o = 1; o < (int)blockDim.x; o <<= 1) {
    const int64_t add = tid >= o ? s[tid - o] : 0;
    __syncthreads();
    s[tid] += add;
    __syncthreads();
  }
  total = s[blockDim.x - 1];
  const int64_t excl = s[tid] - val;
  __syncthreads();
  return excl;
}

// Count of Sc rows and of Sc-Sc edges (j > u) in thread's rows.
__device__ __forceinline__ void tl_counts(const int8_t *cls, const int32_t *rowptr, const int32_t *col,
                                          TlRange r, int64_t &nodes, int64_t &edges) {
  nodes = 0;
  edges = 0;
  for (int64_t u = r.lo; u < r.hi; u++) {
    if (cls[u] != 2) continue;
    nodes++;
    for (int32_t e = rowptr[u]; e < rowptr[u + 1]; e++) {
      const int32_t j = col[e];
      if (j > u && cls[j] == 2) edges++;
    }
  }
}

// Per workgroup: Sc rows and Sc-Sc edges (for the host's prefix over workgroups).
__global__ __launch_bounds__(kBlock) void k_tl_count(const int8_t *cls, const int32_t *rowptr, const int32_t *col,
                                                     int64_t nt, int64_t chunk, int64_t *bnodes, int64_t *bedges) {
  int64_t nn, ne, tn, te;
  tl_counts(cls, rowptr, col, tl_rows(nt, chunk), nn, ne);
  tl_block_scan(nn, tn);
  tl_block_scan(ne, te);
  if (threadIdx.x == 0) {
    bnodes[blockIdx.x] = tn;
    bedges[blockIdx.x] = te;
  }
}

// Coarse id of every row: Sc rows 0..nc-1 in ascending order, S1 -> nc (s_c),
// S0 -> nc + 1 (t_c).
__global__ __launch_bounds__(kBlock) void k_tl_ids(const int8_t *cls, int64_t nt, int64_t chunk,
                                                   const int64_t *boff, int64_t nc, int32_t *cid) {
  const TlRange r = tl_rows(nt, chunk);
  int64_t cnt = 0;
  for (int64_t u = r.lo; u < r.hi; u++) cnt += cls[u] == 2;
  int64_t tot;
  int64_t next = boff[blockIdx.x] + tl_block_scan(cnt, tot);
  for (int64_t u = r.lo; u < r.hi; u++) {
    const int8_t c = cls[u];
    cid[u] = (int32_t)(c == 2 ? next++ : (c == 1 ? nc : nc + 1));
  }
}

// The coarse capacities: Sc-Sc edges (cu < cv) at the workgroup's offset in
// row order, each Sc node's capacity to s_c (to S1 and s) and to t_c (to S0
// and t), and per workgroup the capacity between S1 and S0 (s-S0 and S1-t
// edges included; the s-t edge is added by the host).
__global__ __launch_bounds__(kBlock) void k_tl_edges(const int8_t *cls, const int32_t *cid, const int32_t *rowptr,
                                                     const int32_t *col, const double *ccap, const double *cs,
                                                     const double *ct, int64_t nt, int64_t chunk, int fx_k,
                                                     const int64_t *eoff, int32_t *eu, int32_t *ev, i128 *ecap,
                                                     i128 *ws, i128 *wt, i128 *bst) {
  const TlRange r = tl_rows(nt, chunk);
  int64_t nn, ne, tot;
  tl_counts(cls, rowptr, col, r, nn, ne);
  int64_t next = eoff[blockIdx.x] + tl_block_scan(ne, tot);
  i128 st = 0;
  for (int64_t u = r.lo; u < r.hi; u++) {
    const int8_t c = cls[u];
    if (c == 2) {
      i128 a = tl_fx(cs[u], fx_k), b = tl_fx(ct[u], fx_k);
      for (int32_t e = rowptr[u]; e < rowptr[u + 1]; e++) {
        const int32_t j = col[e];
        const int8_t cj = cls[j];
        if (cj == 1) a += tl_fx(ccap[e], fx_k);
        else if (cj == 0) b += tl_fx(ccap[e], fx_k);
        else if (j > u) {
          eu[next] = cid[u];
          ev[next] = cid[j];
          ecap[next] = tl_fx(ccap[e], fx_k);
          next++;
        }
      }
      ws[cid[u]] = a;
      wt[cid[u]] = b;
    } else if (c == 1) {                               // S1 row: its edges to S0 and to t
      st += tl_fx(ct[u], fx_k);
      for (int32_t e = rowptr[u]; e < rowptr[u + 1]; e++)
        if (cls[col[e]] == 0) st += tl_fx(ccap[e], fx_k);
    } else {                                           // S0 row: its edge from s
      st += tl_fx(cs[u], fx_k);
    }
  }
  // workgroup sum of st in a fixed order (integer sums are exact anyway)
  __shared__ i128 s_st[kBlock];
  s_st[threadIdx.x] = st;
  __syncthreads();
  if (threadIdx.x == 0) {
    i128 t = 0;
    for (int i = 0; i < (int)blockDim.x; i++) t += s_st[i];
    bst[blockIdx.x] = t;
  }
}

// The lifted cut in original node ids: S1, and the Sc rows whose coarse node
// lies on the source side (side[cid] = 1).
__global__ __launch_bounds__(kBlock) void k_tl_lift(const int8_t *cls, const int32_t *cid, const uint8_t *side,
                                                    int64_t nt, int64_t lo, int64_t hi, uint8_t *mask) {
  for (int64_t u = row_begin(); u < nt; u += row_stride()) {
    int64_t o = u;                                     // non-terminal index -> node id
    if (o >= lo) o++;
    if (o >= hi) o++;
    const int8_t c = cls[u];
    mask[o] = c == 1 ? 1 : (c == 2 ? side[cid[u]] : 0);
  }
}

hipError_t launch_tl_kmeans(const double *v, int64_t nt, double m, double *part, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_tl_kmeans, dim3(grid), dim3(kBlock), 0, st, v, nt, m, part);
  return hipGetLastError();
}

hipError_t launch_tl_classify(const double *v, int64_t nt, double g0, double g1, int8_t *cls, int grid,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_tl_classify, dim3(grid), dim3(kBlock), 0, st, v, nt, g0, g1, cls);
  return hipGetLastError();
}

hipError_t launch_tl_count(const int8_t *cls, const int32_t *rowptr, const int32_t *col, int64_t nt, int64_t chunk,
                           int64_t *bnodes, int64_t *bedges, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_tl_count, dim3(grid), dim3(kBlock), 0, st, cls, rowptr, col, nt, chunk, bnodes, bedges);
  return hipGetLastError();
}

hipError_t launch_tl_ids(const int8_t *cls, int64_t nt, int64_t chunk, const int64_t *boff, int64_t nc,
                         int32_t *cid, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_tl_ids, dim3(grid), dim3(kBlock), 0, st, cls, nt, chunk, boff, nc, cid);
  return hipGetLastError();
}

hipError_t launch_tl_edges(const int8_t *cls, const int32_t *cid, const int32_t *rowptr, const int32_t *col,
                           const double *ccap, const double *cs, const double *ct, int64_t nt, int64_t chunk,
                           int fx_k, const int64_t *eoff, int32_t *eu, int32_t *ev, i128 *ecap, i128 *ws,
                           i128 *wt, i128 *bst, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_tl_edges, dim3(grid), dim3(kBlock), 0, st, cls, cid, rowptr, col, ccap, cs, ct, nt, chunk,
                     fx_k, eoff, eu, ev, ecap, ws, wt, bst);
  return hipGetLastError();
}

hipError_t launch_tl_lift(const int8_t *cls, const int32_t *cid, const uint8_t *side, int64_t nt, int64_t lo,
                          int64_t hi, uint8_t *mask, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_tl_lift, dim3(grid), dim3(kBlock), 0, st, cls, cid, side, nt, lo, hi, mask);
  return hipGetLastError();
}

}  // namespace irls
