// Device helpers shared by the gfx950 kernels of libirls_mincut.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace irls {

// Conductance of an edge of capacity c whose end potentials differ by d.
// Step 1 of the IRLS round (eq. define-reweight-vector) combined with the
// reweighted Laplacian (eq. reweighted-laplacian): the Laplacian weight of an
// edge is c^2 / w with w = sqrt((c d)^2 + eps^2) (form 1, eps standing for the
// squared smoothing); form 0 divides out one factor of c inside the root.
template <typename F>
__device__ __forceinline__ F conductance(F c, F d, F eps, int form) {
  if (form == 0) return c / sqrt(d * d + eps);
  F cd = c * d;
  return (c * c) / sqrt(cd * cd + eps);
}

// Sum (or max, for the slots set in MAXMASK) of NQ values over the whole
// workgroup.  Fixed butterfly inside each wavefront, then the per-wave
// results in wave order: the result does not depend on timing.  On return
// thread 0 holds the totals.  lds must hold NQ * (blockDim.x / 64) doubles.
template <int NQ, unsigned MAXMASK = 0u>
__device__ __forceinline__ void block_reduce(double (&x)[NQ], double *lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    double v = x[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      double u = __shfl_xor(v, o, 64);
      v = ((MAXMASK >> q) & 1u) ? fmax(v, u) : v + u;
    }
    x[q] = v;
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NQ; q++) lds[q * nw + wid] = x[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; q++) {
      double acc = lds[q * nw];
      for (int w = 1; w < nw; w++)
        acc = ((MAXMASK >> q) & 1u) ? fmax(acc, lds[q * nw + w]) : acc + lds[q * nw + w];
      x[q] = acc;
    }
  }
  __syncthreads();
}

// All-reduce with a single barrier: every thread adds the wavefront totals
// in the order thread 0 of block_reduce does, so the bits are the same.  The
// LDS array (NQ * waves doubles) must not be reused by the workgroup
// afterwards, since there is no barrier after the reads.
template <int NQ, unsigned MAXMASK = 0u>
__device__ __forceinline__ void block_allreduce_once(double (&x)[NQ], double *lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    double v = x[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      double u = __shfl_xor(v, o, 64);
      v = ((MAXMASK >> q) & 1u) ? fmax(v, u) : v + u;
    }
    if (lane == 0) lds[q * nw + wid] = v;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    double acc = lds[q * nw];
    for (int w = 1; w < nw; w++) acc = ((MAXMASK >> q) & 1u) ? fmax(acc, lds[q * nw + w]) : acc + lds[q * nw + w];
    x[q] = acc;
  }
}

template <int NQ, unsigned MAXMASK = 0u>
__device__ __forceinline__ void block_allreduce(double (&x)[NQ], double *lds, double *bc) {
  block_reduce<NQ, MAXMASK>(x, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; q++) bc[q] = x[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; q++) x[q] = bc[q];
}

__device__ __forceinline__ double *pslot(double *partials, int slot, int q) {
  return partials + ((size_t)slot * kNumPartial + q) * kMaxGrid;
}

// This workgroup's share of NQ grid-wide sums: stored at [slot][q][blockIdx].
template <int NQ, unsigned MAXMASK = 0u>
__device__ __forceinline__ void write_partials(double (&x)[NQ], double *partials, int slot, double *lds) {
  block_reduce<NQ, MAXMASK>(x, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; q++) pslot(partials, slot, q)[blockIdx.x] = x[q];
  }
}

// This thread's share of the totals of NQ partial-sum arrays (the sums over
// partials threadIdx.x, threadIdx.x + kBlock, ...); block_allreduce then
// finishes them.  Threads kBlock and up (in larger workgroups) hold zeros, so
// every workgroup size adds the partials in the same order and gets the same
// bits.  The loads are unrolled so they are all in flight at once; the sum
// order is the loop order.  Split from read_totals so a kernel can issue
// other loads in the same memory round trip and reduce them together.
template <int NQ>
__device__ __forceinline__ void partial_share(const double *partials, int slot, int nblocks, double (&acc)[NQ]) {
  constexpr int kPer = kMaxGrid / kBlock;
  double v[NQ][kPer];
  const bool mine = threadIdx.x < kBlock;
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    const double *P = partials + ((size_t)slot * kNumPartial + q) * kMaxGrid;
#pragma unroll
    for (int j = 0; j < kPer; j++) {
      const int b = threadIdx.x + j * kBlock;
      v[q][j] = mine && b < nblocks ? P[b] : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kPer; j++) s += v[q][j];
    acc[q] = s;
  }
}

// Totals of the partial sums a previous kernel of `nblocks` workgroups left in
// `slot`.  Every workgroup adds them in the same fixed order, so all get the
// same bits; no atomics and no fences are needed (kernel boundaries order the
// memory traffic).  As in partial_share, threads kBlock and up contribute the
// neutral element; MAXMASK marks the components reduced by max instead of sum.
template <int NQ, unsigned MAXMASK = 0u>
__device__ __forceinline__ void read_totals(const double *partials, int slot, int nblocks,
                                            double (&tot)[NQ], double *lds, double *bc) {
  constexpr int kPer = kMaxGrid / kBlock;
  double v[NQ][kPer];
  const bool mine = threadIdx.x < kBlock;
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    const double *P = partials + ((size_t)slot * kNumPartial + q) * kMaxGrid;
#pragma unroll
    for (int j = 0; j < kPer; j++) {
      const int b = threadIdx.x + j * kBlock;
      v[q][j] = mine && b < nblocks ? P[b] : (((MAXMASK >> q) & 1u) ? -INFINITY : 0.0);
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    double acc = ((MAXMASK >> q) & 1u) ? -INFINITY : 0.0;
#pragma unroll
    for (int j = 0; j < kPer; j++) acc = ((MAXMASK >> q) & 1u) ? fmax(acc, v[q][j]) : acc + v[q][j];
    tot[q] = acc;
  }
  block_allreduce<NQ, MAXMASK>(tot, lds, bc);
}

// Grid-stride row loop helper: first row and stride of this thread.
__device__ __forceinline__ int64_t row_begin() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t row_stride() { return (int64_t)gridDim.x * blockDim.x; }

// XCD-aware row ranges.  Workgroups are dispatched round-robin over the 8
// XCDs, each with its own L2; workgroup b runs on XCD b % 8.  Giving each XCD
// one contiguous slab of rows keeps the stencil neighbours of a row (offsets
// 1, nx, nx*ny) in the same L2 except at slab boundaries.
constexpr int kXcds = 8;
__device__ __forceinline__ void slab_rows(int64_t n, int64_t &begin, int64_t &end, int64_t &step) {
  if (gridDim.x < kXcds || gridDim.x % kXcds != 0) {
    begin = row_begin();
    end = n;
    step = row_stride();
    return;
  }
  const int64_t x = blockIdx.x % kXcds, lb = blockIdx.x / kXcds, nb = gridDim.x / kXcds;
  const int64_t slab = (n + kXcds - 1) / kXcds;
  const int64_t lo = x * slab;
  end = lo + slab < n ? lo + slab : n;
  begin = lo + lb * blockDim.x + threadIdx.x;
  step = nb * blockDim.x;
}

// CSR rows with L lanes each (L a power of two <= 64): every wavefront takes
// 64 / L consecutive rows at a time, in XCD slabs of row groups as slab_rows
// forms them for single rows.  f(u, lid) runs on every lane, with u = -1 on
// lanes past the last row, so that shuffles inside f see the whole
// wavefront; lid is the lane's index within its row's group.
template <int L, typename F>
__device__ __forceinline__ void for_row_groups(int64_t n, F f) {
  constexpr int RPW = 64 / L;
  const int lane = threadIdx.x & 63, sub = lane / L, lid = lane % L;
  const int64_t ng = (n + RPW - 1) / RPW, wpb = blockDim.x >> 6, w = threadIdx.x >> 6;
  int64_t gb, ge, gs;
  if (gridDim.x < kXcds || gridDim.x % kXcds != 0) {
    gb = (int64_t)blockIdx.x * wpb + w;
    ge = ng;
    gs = (int64_t)gridDim.x * wpb;
  } else {
    const int64_t x = blockIdx.x % kXcds, lb = blockIdx.x / kXcds, nb = gridDim.x / kXcds;
    const int64_t slab = (ng + kXcds - 1) / kXcds, lo = x * slab;
    ge = lo + slab < ng ? lo + slab : ng;
    gb = lo + lb * wpb + w;
    gs = nb * wpb;
  }
  for (int64_t g = gb; g < ge; g += gs) {            // the same trip count on every lane
    const int64_t u = g * RPW + sub;
    f(u < n ? u : (int64_t)-1, lid);
  }
}

// Sum over the L lanes of a row group (L a power of two).
template <int L>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

#define FOR_ROWS(u, n)                                   \
  int64_t u##_b_, u##_e_, u##_s_;                        \
  slab_rows((n), u##_b_, u##_e_, u##_s_);                \
  for (int64_t u = u##_b_; u < u##_e_; u += u##_s_)

}  // namespace irls
