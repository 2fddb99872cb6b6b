// Sweep cut on the GPU (Section 3.4): order the non-terminal nodes by their
// final potential (descending, ties by ascending id), evaluate every prefix
// set S_k = {s} + first k nodes exactly, take the smallest k of least cut.
//
//   1. keys:    potential -> 64-bit key whose ascending order is descending x
//   2. sort:    stable LSD radix sort, 8 passes of 8-bit digits; per pass a
//               per-workgroup digit histogram, one exclusive scan over
//               (digit, workgroup) (a workgroup per digit: digit totals,
//               then each digit's counts from its offset), and a stable
//               scatter ranked with wavefront ballots
//   3. rank:    rank[id] = position + 1
//   4. delta:   cut(S_k) - cut(S_{k-1}) for the node entering at step k, in
//               128-bit fixed point round(c 2^k): edges to nodes already in S
//               leave the cut, edges to later nodes and to t enter it
//   5. scan:    prefix sums of the deltas per workgroup, exclusive scan of the
//               workgroup sums, then per-workgroup minimum and its first index
//   6. mask:    source-side flag of every node
#include <mutex>

#include "device_common.h"

namespace irls {

typedef __int128 i128;

constexpr int kSortItems = 16;                       // keys per thread per sort tile
constexpr int kSortTile = kBlock * kSortItems;       // 4096
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

size_t sweep_sort_blocks(int64_t nt) { return (size_t)((nt + kSortTile - 1) / kSortTile); }
size_t sweep_scan_blocks(int64_t nt) { return (size_t)((nt + kScanTile - 1) / kScanTile); }

// round-half-even(c * 2^k) for c >= 0, exact for every c >= 2^(52-k)
__device__ __forceinline__ i128 fx_round(double c, int k) {
  if (!(c > 0.0)) return 0;
  uint64_t bits = (uint64_t)__double_as_longlong(c);
  int ef = (int)((bits >> 52) & 0x7FF);
  uint64_t mant = bits & ((1ull << 52) - 1);
  int e2;
  if (ef == 0) { e2 = -1074; } else { mant |= 1ull << 52; e2 = ef - 1075; }   // c = mant 2^e2
  int sh = e2 + k;
  if (sh >= 0) return ((i128)mant) << sh;
  int r = -sh;
  if (r >= 64) return 0;
  uint64_t q = mant >> r, rem = mant & ((1ull << r) - 1), half = 1ull << (r - 1);
  if (rem > half || (rem == half && (q & 1ull))) q++;
  return (i128)q;
}

__device__ __forceinline__ int64_t orig_id(int64_t i, int64_t lo, int64_t hi) {
  // non-terminal index -> node id (ids in ascending order skipping s and t)
  if (i >= lo) i++;
  if (i >= hi) i++;
  return i;
}

__global__ __launch_bounds__(kBlock) void k_keys(const double *v, int64_t nt, uint64_t *key, uint32_t *id) {
  for (int64_t i = row_begin(); i < nt; i += row_stride()) {
    double x = v[i];
    uint64_t b = x == 0.0 ? 0ull : (uint64_t)__double_as_longlong(x);   // -0 -> +0
    uint64_t asc = (b >> 63) ? ~b : (b | (1ull << 63));
    key[i] = ~asc;
    id[i] = (uint32_t)i;
  }
}

__global__ __launch_bounds__(kBlock) void k_hist(const uint64_t *key, int64_t nt, int shift, uint32_t *hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int it = 0; it < kSortItems; it++) {
    int64_t i = base + (int64_t)it * kBlock + threadIdx.x;
    if (i < nt) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of hist[256 * nb] (digit-major: digit d's count in block b
// at hist[d * nb + b]) in place, by two kernels of one workgroup per digit.
// The first writes each digit's total to dsum[d] (the 256 entries after the
// histogram); the second starts digit d at the sum of dsum over the digits
// below it and scans the digit's nb counts in tiles of kScanThreads.  Integer
// sums: the result is the sequential scan's exactly.
constexpr int kScanThreads = 1024;

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

__global__ __launch_bounds__(kScanThreads) void k_hist_digit_sum(const uint32_t *hist, int64_t nb, uint32_t *dsum) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t *h = hist + (size_t)blockIdx.x * nb;
  uint32_t s = 0;
  for (int64_t i = threadIdx.x; i < nb; i += kScanThreads) s += h[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) wsum[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kScanThreads / 64; w++) t += wsum[w];
    dsum[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_hist_digit_scan(uint32_t *hist, int64_t nb, const uint32_t *dsum) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  __shared__ uint32_t s_off;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int nw = kScanThreads / 64;
  // digit offset: the totals of the digits below this one (fewer than 256 < kScanThreads)
  uint32_t o = threadIdx.x < blockIdx.x ? dsum[threadIdx.x] : 0u;
#pragma unroll
  for (int k = 32; k > 0; k >>= 1) o += __shfl_xor(o, k, 64);
  if (lane == 0) wsum[wid] = o;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < nw; w++) t += wsum[w];
    s_off = t;
  }
  __syncthreads();
  uint32_t carry = s_off;
  uint32_t *h = hist + (size_t)blockIdx.x * nb;
  for (int64_t base = 0; base < nb; base += kScanThreads) {
    const int64_t i = base + threadIdx.x;
    const uint32_t v = i < nb ? h[i] : 0u;
    const uint32_t inc = wave_inclusive_scan(v, lane);
    __syncthreads();                                   // wsum is free again
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    uint32_t before = 0, tile = 0;
    for (int w = 0; w < nw; w++) {
      const uint32_t t = wsum[w];
      if (w < wid) before += t;
      tile += t;
    }
    if (i < nb) h[i] = carry + before + inc - v;
    carry += tile;
  }
}

// The exclusive scan of one radix pass's histogram (its 256 * nb counts,
// then 256 digit totals, in hist).
static void scan_hist(uint32_t *hist, int64_t nb, hipStream_t st) {
  hipLaunchKernelGGL(k_hist_digit_sum, dim3(256), dim3(kScanThreads), 0, st, (const uint32_t *)hist, nb,
                     hist + 256 * nb);
  hipLaunchKernelGGL(k_hist_digit_scan, dim3(256), dim3(kScanThreads), 0, st, hist, nb,
                     (const uint32_t *)(hist + 256 * nb));
}

// stable scatter: sub-tiles of kBlock keys in order; within a sub-tile the
// rank of a key among equal digits follows lane order inside a wavefront and
// wavefront order inside the workgroup
__global__ __launch_bounds__(kBlock) void k_scatter(const uint64_t *kin, const uint32_t *iin,
                                                     uint64_t *kout, uint32_t *iout, int64_t nt,
                                                     int shift, const uint32_t *hist) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t cnt[kBlock / 64][256];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  base[threadIdx.x] = hist[(size_t)threadIdx.x * gridDim.x + blockIdx.x];
  const uint64_t lt = (1ull << lane) - 1ull;
  const int64_t tile = (int64_t)blockIdx.x * kSortTile;
  for (int it = 0; it < kSortItems; it++) {
    for (int w = 0; w < kBlock / 64; w++) cnt[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = tile + (int64_t)it * kBlock + threadIdx.x;
    const bool valid = i < nt;
    uint64_t k = valid ? kin[i] : 0ull;
    uint32_t idv = valid ? iin[i] : 0u;
    uint32_t d = (uint32_t)((k >> shift) & 255u);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; bit++) {
      uint64_t bset = __ballot((d >> bit) & 1u);
      peers &= ((d >> bit) & 1u) ? bset : ~bset;
    }
    const uint32_t before = (uint32_t)__popcll(peers & lt);
    if (valid && before == 0) cnt[wid][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[d] + before;
      for (int w = 0; w < wid; w++) pos += cnt[w][d];
      kout[pos] = k;
      iout[pos] = idv;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kBlock / 64; w++) add += cnt[w][threadIdx.x];
    base[threadIdx.x] += add;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_rank(const uint32_t *id, int64_t nt, uint32_t *rank) {
  for (int64_t i = row_begin(); i < nt; i += row_stride()) rank[id[i]] = (uint32_t)(i + 1);
}

__global__ __launch_bounds__(kBlock) void k_delta(SweepArgs a, const uint32_t *rank, i128 *delta) {
  for (int64_t u = row_begin(); u < a.nt; u += row_stride()) {
    const uint32_t ru = rank[u];
    i128 d = fx_round(a.ct[u], a.fx_k) - fx_round(a.cs[u], a.fx_k);
    for (int32_t e = a.rowptr[u]; e < a.rowptr[u + 1]; e++) {
      i128 q = fx_round(a.ccap[e], a.fx_k);
      d += rank[a.col[e]] > ru ? q : -q;
    }
    delta[ru - 1] = d;
  }
}

// block sums of the deltas
__global__ __launch_bounds__(kBlock) void k_bsum(const i128 *delta, int64_t nt, i128 *bsum) {
  __shared__ i128 sh[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  i128 s = 0;
  for (int j = 0; j < kScanItems; j++)
    if (base + j < nt) s += delta[base + j];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = sh[0];
}

// exclusive scan of the nb block sums in place (one workgroup)
__global__ __launch_bounds__(kBlock) void k_bscan(i128 *bsum, int64_t nb) {
  __shared__ i128 part[kBlock];
  const int64_t per = (nb + kBlock - 1) / kBlock;
  const int64_t lo = (int64_t)threadIdx.x * per;
  const int64_t hi = lo + per < nb ? lo + per : nb;
  i128 s = 0;
  for (int64_t i = lo; i < hi; i++) s += bsum[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    i128 add = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : (i128)0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  i128 run = threadIdx.x ? part[threadIdx.x - 1] : (i128)0;
  for (int64_t i = lo; i < hi; i++) {
    i128 c = bsum[i];
    bsum[i] = run;
    run += c;
  }
}

// per block: inclusive prefix values P_k (k = global position + 1), minimum
// and the smallest k attaining it
__global__ __launch_bounds__(kBlock) void k_bmin(const i128 *delta, int64_t nt, const i128 *boff,
                                                 i128 *bmin, int64_t *barg) {
  __shared__ i128 part[kBlock];
  __shared__ i128 mv[kBlock];
  __shared__ int64_t mk[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  i128 s = 0;
  for (int j = 0; j < kScanItems; j++)
    if (base + j < nt) s += delta[base + j];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    i128 add = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : (i128)0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  i128 run = boff[blockIdx.x] + (threadIdx.x ? part[threadIdx.x - 1] : (i128)0);
  i128 best = 0;
  int64_t bk = -1;
  for (int j = 0; j < kScanItems; j++) {
    if (base + j >= nt) break;
    run += delta[base + j];
    if (bk < 0 || run < best) { best = run; bk = base + j + 1; }
  }
  mv[threadIdx.x] = best;
  mk[threadIdx.x] = bk;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      int64_t k2 = mk[threadIdx.x + o];
      if (k2 >= 0) {
        int64_t k1 = mk[threadIdx.x];
        i128 v2 = mv[threadIdx.x + o], v1 = mv[threadIdx.x];
        if (k1 < 0 || v2 < v1 || (v2 == v1 && k2 < k1)) { mv[threadIdx.x] = v2; mk[threadIdx.x] = k2; }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { bmin[blockIdx.x] = mv[0]; barg[blockIdx.x] = mk[0]; }
}

// global minimum over blocks, including the empty prefix (k = 0, P_0 = 0)
__global__ __launch_bounds__(kBlock) void k_final(const i128 *bmin, const int64_t *barg, int64_t nb,
                                                  i128 *best, int64_t *kstar) {
  __shared__ i128 mv[kBlock];
  __shared__ int64_t mk[kBlock];
  i128 b = 0;
  int64_t k = 0;                                  // S_0 = {s}
  for (int64_t i = threadIdx.x; i < nb; i += kBlock) {
    int64_t k2 = barg[i];
    if (k2 < 0) continue;
    i128 v2 = bmin[i];
    if (v2 < b || (v2 == b && k2 < k)) { b = v2; k = k2; }
  }
  mv[threadIdx.x] = b;
  mk[threadIdx.x] = k;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      i128 v2 = mv[threadIdx.x + o], v1 = mv[threadIdx.x];
      int64_t k2 = mk[threadIdx.x + o], k1 = mk[threadIdx.x];
      if (v2 < v1 || (v2 == v1 && k2 < k1)) { mv[threadIdx.x] = v2; mk[threadIdx.x] = k2; }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { best[0] = mv[0]; kstar[0] = mk[0]; }
}

__global__ __launch_bounds__(kBlock) void k_mask(SweepArgs a, const uint32_t *rank, const int64_t *kstar,
                                                 uint8_t *mask) {
  const int64_t ks = *kstar;
  const int64_t lo = a.s < a.t ? a.s : a.t, hi = a.s < a.t ? a.t : a.s;
  for (int64_t u = row_begin(); u < a.nt; u += row_stride())
    mask[orig_id(u, lo, hi)] = (int64_t)rank[u] <= ks ? 1 : 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) { mask[a.s] = 1; mask[a.t] = 0; }
}

// ----------------------------------------------------------------------------
// batched sweep
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_gidkey(const uint32_t *id, const uint32_t *gid, int64_t n,
                                                   uint64_t *key) {
  for (int64_t i = row_begin(); i < n; i += row_stride()) key[i] = gid[id[i]];
}

// sorted by (graph, potential desc, id): rank inside the graph
__global__ __launch_bounds__(kBlock) void k_rank_batch(const uint32_t *id, const uint32_t *gid,
                                                       const BatchGraph *gs, int64_t n, uint32_t *rank) {
  for (int64_t i = row_begin(); i < n; i += row_stride()) {
    const uint32_t u = id[i];
    rank[u] = (uint32_t)(i - gs[gid[u]].node0 + 1);
  }
}

__global__ __launch_bounds__(kBlock) void k_delta_batch(SweepBatchArgs a, const uint32_t *rank, i128 *delta) {
  for (int64_t u = row_begin(); u < a.rows; u += row_stride()) {
    const BatchGraph G = a.graphs[a.gid[u]];
    const int64_t lu = u - G.node0;
    const int32_t *rp = a.rowptr + G.node0 + a.gid[u];
    const uint32_t ru = rank[u];
    i128 d = fx_round(a.ct[u], G.fx_k) - fx_round(a.cs[u], G.fx_k);
    for (int32_t e = rp[lu]; e < rp[lu + 1]; e++) {
      const int64_t j = G.node0 + a.col[G.nnz0 + e];
      const i128 q = fx_round(a.ccap[G.nnz0 + e], G.fx_k);
      d += rank[j] > ru ? q : -q;
    }
    delta[G.node0 + ru - 1] = d;
  }
}

// in-place inclusive prefix sums of the deltas (tile offsets from k_bscan)
__global__ __launch_bounds__(kBlock) void k_prefix(i128 *delta, int64_t nt, const i128 *boff) {
  __shared__ i128 part[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  i128 s = 0;
  for (int j = 0; j < kScanItems; j++)
    if (base + j < nt) s += delta[base + j];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    i128 add = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : (i128)0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  i128 run = boff[blockIdx.x] + (threadIdx.x ? part[threadIdx.x - 1] : (i128)0);
  for (int j = 0; j < kScanItems; j++) {
    if (base + j >= nt) break;
    run += delta[base + j];
    delta[base + j] = run;
  }
}

// one workgroup per graph: least prefix (k = 0 included) and its smallest k
__global__ __launch_bounds__(kBlock) void k_segmin(const i128 *P, const BatchGraph *gs, i128 *best,
                                                   int64_t *kstar, uint8_t *mask) {
  __shared__ i128 mv[kBlock];
  __shared__ int64_t mk[kBlock];
  const BatchGraph G = gs[blockIdx.x];
  const i128 base = G.node0 > 0 ? P[G.node0 - 1] : (i128)0;
  i128 b = 0;
  int64_t k = 0;
  for (int64_t i = threadIdx.x; i < G.nt; i += kBlock) {
    const i128 v = P[G.node0 + i] - base;
    if (v < b) { b = v; k = i + 1; }               // ascending i: first minimum kept
  }
  mv[threadIdx.x] = b;
  mk[threadIdx.x] = k;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      i128 v2 = mv[threadIdx.x + o], v1 = mv[threadIdx.x];
      int64_t k2 = mk[threadIdx.x + o], k1 = mk[threadIdx.x];
      if (v2 < v1 || (v2 == v1 && k2 < k1)) { mv[threadIdx.x] = v2; mk[threadIdx.x] = k2; }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    best[blockIdx.x] = mv[0];
    kstar[blockIdx.x] = mk[0];
    mask[G.node_off + G.s] = 1;
    mask[G.node_off + G.t] = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_mask_batch(SweepBatchArgs a, const uint32_t *rank,
                                                       const int64_t *kstar, uint8_t *mask) {
  for (int64_t u = row_begin(); u < a.rows; u += row_stride()) {
    const uint32_t g = a.gid[u];
    const BatchGraph G = a.graphs[g];
    const int64_t lo = G.s < G.t ? G.s : G.t, hi = G.s < G.t ? G.t : G.s;
    mask[G.node_off + orig_id(u - G.node0, lo, hi)] = (int64_t)rank[u] <= kstar[g] ? 1 : 0;
  }
}

static int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > kMaxGrid) g = kMaxGrid;
  return g < 1 ? 1 : (int)g;
}

hipError_t sweep_run(const SweepArgs &a, SweepBufs &b, hipStream_t st) {
  const int64_t nt = a.nt;
  if (nt > 0) {
    const int gs = grid_for(nt);
    const int nb = (int)sweep_sort_blocks(nt);
    hipLaunchKernelGGL(k_keys, dim3(gs), dim3(kBlock), 0, st, a.v, nt, b.keyA, b.idA);
    uint64_t *kin = b.keyA, *kout = b.keyB;
    uint32_t *iin = b.idA, *iout = b.idB;
    for (int pass = 0; pass < 8; pass++) {
      const int shift = 8 * pass;
      hipLaunchKernelGGL(k_hist, dim3(nb), dim3(kBlock), 0, st, kin, nt, shift, b.hist);
      scan_hist(b.hist, nb, st);
      hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kBlock), 0, st, kin, iin, kout, iout, nt, shift,
                         (const uint32_t *)b.hist);
      uint64_t *tk = kin; kin = kout; kout = tk;
      uint32_t *ti = iin; iin = iout; iout = ti;
    }
    // eight passes: the sorted ids are back in idA
    hipLaunchKernelGGL(k_rank, dim3(gs), dim3(kBlock), 0, st, (const uint32_t *)iin, nt, b.rank);
    hipLaunchKernelGGL(k_delta, dim3(gs), dim3(kBlock), 0, st, a, (const uint32_t *)b.rank, b.delta);
    const int sb = (int)sweep_scan_blocks(nt);
    hipLaunchKernelGGL(k_bsum, dim3(sb), dim3(kBlock), 0, st, (const i128 *)b.delta, nt, b.bsum);
    hipLaunchKernelGGL(k_bscan, dim3(1), dim3(kBlock), 0, st, b.bsum, (int64_t)sb);
    hipLaunchKernelGGL(k_bmin, dim3(sb), dim3(kBlock), 0, st, (const i128 *)b.delta, nt,
                       (const i128 *)b.bsum, b.bmin, b.barg);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, st, (const i128 *)b.bmin,
                       (const int64_t *)b.barg, (int64_t)sb, b.best, b.kstar);
    hipLaunchKernelGGL(k_mask, dim3(gs), dim3(kBlock), 0, st, a, (const uint32_t *)b.rank,
                       (const int64_t *)b.kstar, b.mask);
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Static scratch of irls_mincut_cut_noalloc: the work buffers of sweep_run for
// up to kNoallocRows non-terminal nodes, carved from one file-scope device
// array (each GPU holds its own copy until the process ends).  Host code uses
// the array only through the address hipGetSymbolAddress gives on each device.
// ----------------------------------------------------------------------------
struct SweepLayout {
  size_t keyA, keyB, idA, idB, rank, delta, hist, bsum, bmin, barg, best, kstar, mask, total;
};

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr SweepLayout sweep_layout(int64_t nt, int64_t n) {
  SweepLayout L{};
  const size_t nb = (size_t)((nt + kSortTile - 1) / kSortTile), sb = (size_t)((nt + kScanTile - 1) / kScanTile);
  size_t at = 0;
  auto place = [&at](size_t bytes) {
    const size_t off = at;
    at = align256(at + bytes);
    return off;
  };
  L.keyA = place(8 * (size_t)nt);
  L.keyB = place(8 * (size_t)nt);
  L.idA = place(4 * (size_t)nt);
  L.idB = place(4 * (size_t)nt);
  L.rank = place(4 * (size_t)nt);
  L.delta = place(16 * (size_t)nt);
  L.hist = place(4 * (256 * nb + 256));                  // the counts, then the digit totals
  L.bsum = place(16 * sb);
  L.bmin = place(16 * sb);
  L.barg = place(8 * sb);
  L.best = place(16 * 2);
  L.kstar = place(8);
  L.mask = place((size_t)n);
  L.total = at;
  return L;
}

constexpr int64_t kNoallocRows = IRLS_NOALLOC_MAX_NONTERMINAL;
constexpr size_t kNoallocBytes = sweep_layout(kNoallocRows, kNoallocRows + 2).total;

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

// The scratch array's address on the current device, looked up once per
// device (each GPU holds the array at its own address).
static hipError_t scratch_address(unsigned char **out) {
  constexpr int kDevs = 64;
  static std::mutex mu;
  static unsigned char *addr[kDevs] = {nullptr};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kDevs) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = (unsigned char *)p;
  }
  *out = addr[dev];
  return hipSuccess;
}

hipError_t sweep_noalloc_buffers(int64_t nt, int64_t n, SweepBufs &b) {
  if (nt > kNoallocRows || n > kNoallocRows + 2) return hipErrorInvalidValue;
  unsigned char *base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return e;
  const SweepLayout L = sweep_layout(nt, n);
  b.keyA = (uint64_t *)(base + L.keyA);
  b.keyB = (uint64_t *)(base + L.keyB);
  b.idA = (uint32_t *)(base + L.idA);
  b.idB = (uint32_t *)(base + L.idB);
  b.rank = (uint32_t *)(base + L.rank);
  b.delta = (__int128 *)(base + L.delta);
  b.hist = (uint32_t *)(base + L.hist);
  b.bsum = (__int128 *)(base + L.bsum);
  b.bmin = (__int128 *)(base + L.bmin);
  b.barg = (int64_t *)(base + L.barg);
  b.best = (__int128 *)(base + L.best);
  b.kstar = (int64_t *)(base + L.kstar);
  b.mask = base + L.mask;
  b.sort_blocks = (int)sweep_sort_blocks(nt);
  b.scan_blocks = (int)sweep_scan_blocks(nt);
  return hipSuccess;
}

hipError_t sweep_batch_run(const SweepBatchArgs &a, SweepBufs &b, SweepBatchBufs &bb, hipStream_t st) {
  const int64_t n = a.rows;
  if (n > 0) {
    const int gs = grid_for(n);
    const int nb = (int)sweep_sort_blocks(n);
    hipLaunchKernelGGL(k_keys, dim3(gs), dim3(kBlock), 0, st, a.v, n, b.keyA, b.idA);
    uint64_t *kin = b.keyA, *kout = b.keyB;
    uint32_t *iin = b.idA, *iout = b.idB;
    for (int pass = 0; pass < 10; pass++) {
      if (pass == 8)       // then by graph: stable, so potential order survives inside a graph
        hipLaunchKernelGGL(k_gidkey, dim3(gs), dim3(kBlock), 0, st, (const uint32_t *)iin, a.gid, n, kin);
      const int shift = pass < 8 ? 8 * pass : 8 * (pass - 8);
      hipLaunchKernelGGL(k_hist, dim3(nb), dim3(kBlock), 0, st, kin, n, shift, b.hist);
      scan_hist(b.hist, nb, st);
      hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kBlock), 0, st, kin, iin, kout, iout, n, shift,
                         (const uint32_t *)b.hist);
      uint64_t *tk = kin; kin = kout; kout = tk;
      uint32_t *ti = iin; iin = iout; iout = ti;
    }
    hipLaunchKernelGGL(k_rank_batch, dim3(gs), dim3(kBlock), 0, st, (const uint32_t *)iin, a.gid,
                       a.graphs, n, b.rank);
    hipLaunchKernelGGL(k_delta_batch, dim3(gs), dim3(kBlock), 0, st, a, (const uint32_t *)b.rank, b.delta);
    const int sb = (int)sweep_scan_blocks(n);
    hipLaunchKernelGGL(k_bsum, dim3(sb), dim3(kBlock), 0, st, (const i128 *)b.delta, n, b.bsum);
    hipLaunchKernelGGL(k_bscan, dim3(1), dim3(kBlock), 0, st, b.bsum, (int64_t)sb);
    hipLaunchKernelGGL(k_prefix, dim3(sb), dim3(kBlock), 0, st, b.delta, n, (const i128 *)b.bsum);
  }
  hipLaunchKernelGGL(k_segmin, dim3(a.G), dim3(kBlock), 0, st, (const i128 *)b.delta, a.graphs, bb.best,
                     bb.kstar, bb.mask);
  if (n > 0)
    hipLaunchKernelGGL(k_mask_batch, dim3(grid_for(n)), dim3(kBlock), 0, st, a, (const uint32_t *)b.rank,
                       (const int64_t *)bb.kstar, bb.mask);
  return hipGetLastError();
}

}  // namespace irls
