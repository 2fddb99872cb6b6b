// Internal declarations of libirls_mincut (host driver <-> HIP kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/irls_mincut.h"
#include "host_graph.h"

namespace irls {

constexpr int kBlock = 256;          // threads per workgroup of the streaming kernels
constexpr int kMaxBlock = 512;       // largest workgroup (the marching SpMV's wide tiles)
constexpr int kMaxGrid = 1024;       // workgroups of the streaming kernels (grid-stride)
using irls_host::kMaxDiag;            // most index offsets the diagonal format stores
constexpr int kNumPartial = 11;      // reduction slots per workgroup

// CG state shared between consecutive kernels of one solve, in device memory.
// Only workgroup 0 of a kernel writes it, and never a field that the same
// kernel reads: every kernel first reduces the per-workgroup partial sums of
// its predecessor itself (fixed order, so every workgroup gets the same bits)
// and derives alpha, beta and the stopping test from them.
struct Scalars {
  double rho[2];     // r^T z, by iteration parity
  double bb;         // ||b||^2
  double rr;         // ||r||^2 of the last stopping test
  double alpha, beta, pq;
  double alpha_par[2]; // alpha by iteration parity (the scaled form's paired potential update)
  int64_t iter_a;    // index of the last SpMV started (written by the SpMV)
  int64_t iter_b;    // CG iterations completed (written by the update)
  int64_t maxit;
  int32_t done;      // 1 once converged, at maxit, or broken down
  int32_t status;    // IRLS_OK, IRLS_WARN_CG_MAXIT or IRLS_ERR_CG_BREAKDOWN
  int32_t refine_every;  // precision 1: FP64 residual replacement period
  int32_t pad;
};

// partial-sum slots (each kNumPartial x kMaxGrid doubles)
enum { kPInit = 0, kPSpmv = 1, kPUpd = 2, kPRep = 3, kPStats = 4, kNumPSlots = 5 };

// Everything a CG-phase kernel needs; passed by value.
template <typename T>
struct CGArgs {
  int64_t nt;                     // non-terminal rows
  // pattern (one of the two)
  const int32_t *rowptr;          // CSR: [nt+1]
  const int32_t *col;             // CSR: [nnz] neighbour rows, ascending
  const double *ccap;             // CSR: [nnz] capacity of each entry's edge
  int32_t K;                      // diagonal format: number of offsets
  int32_t off[kMaxDiag];          // diagonal format: positive row offsets
  const double *dcap;             // diagonal format: [K*nt] capacity of edge (u, u+off[k])
  const double *cs, *ct;          // [nt] capacity to s / to t (0 = no edge)
  // this round's system
  T *w;                           // conductances: CSR [nnz] or diagonal [K*nt]
  T *D;                           // diagonal of L~
  double *w64, *D64;              // precision 1: FP64 copies for residual replacement
  double *b;                      // [nt] b = conductance to s (FP64)
  double *gt;                     // [nt] conductance to t (FP64)
  // CG vectors
  double *v;                      // potentials (FP64 always)
  T *z, *q;                       // z = M^-1 r (Jacobi), q = L~ p
  T *p0, *p1;                     // direction, double-buffered for the fused diagonal kernel
  // Jacobi as symmetric scaling (scaled = 1): CG runs on D^-1/2 L~ D^-1/2,
  // whose unit diagonal needs no storage.  Then z holds D^-1/2 r, p and q the
  // scaled direction and product, v holds D^1/2 v during CG, and wh the
  // scaled conductances w_uj / sqrt(D_u D_j) in the diagonal layout.
  T *wh;
  double *wh64;                   // precision 1, scaled: FP64 scaled conductances (replacement)
  float *Dn;                      // scaled form: D rounded to FP32, the weights of the stopping
                                  // norm ||r||^2 = sum D r^2 (the FP32 form: its D)
  int32_t scaled;
  // reductions
  double *partials;               // [kNumPSlots][kNumPartial][kMaxGrid]
  Scalars *sc;
  irls_round_stats *stat;         // this round's record
  double eps, eps_next;
  int32_t form;
  int32_t round0;                 // conductance = capacity
  int32_t warm;
  int32_t weights_fp64;           // precision 1: compute conductances in FP64
  double cst;                     // s-t capacity
  double rtol;                    // CG stopping tolerance relative to ||b||
  // block-Jacobi: the residual kept explicitly (rbuf) and, for exact line
  // blocks (precond 1), per row the forward multiplier, 1/pivot and backward
  // multiplier of its block's tridiagonal LU factors; bj_block rows per block
  // (0: Jacobi).  rbuf and bj_im are in the working precision: FP32 only for
  // ILU(0) of 4x4x4 tiles in the precision form, FP64 for every other kind.
  T *rbuf;
  double *bj_f;
  T *bj_im;
  double *bj_g;
  int32_t bj_block;
  // bj_kind 2: ILU(0) of cubic tiles of a 3-D grid (bj_tile rows on a side,
  // bj_block = bj_tile^3); bj_im then holds the ILU(0) pivot of each row.
  // bj_kind 3: ILU(0) of CSR blocks (nblk of them; rows blk_rows[blk_ptr[k] ..
  // blk_ptr[k+1]) ascending), factor values per CSR entry in ilu_f (0 for
  // entries leaving the block), pivots in bj_im
  int32_t bj_kind, bj_tile;
  int64_t nblk;
  const int32_t *blk_ptr, *blk_rows, *row_blk;
  double *ilu_f;
  // CSR SpMV of the multi-workgroup path: rows of more than kCsrHeavy entries
  // (hubs) are cut into chunks of at most kCsrChunk entries, summed a
  // wavefront each by k_spmv_csr_chunks; the row's lanes in k_spmv_csr then
  // add its chunk sums instead of its entries
  int32_t csr_nheavy, csr_nchunks;
  const int32_t *csr_hfirst;      // [nt] 1 + the first chunk of a heavy row, 0 for the others
  const int32_t *csr_cbeg, *csr_cend;   // [csr_nchunks] entry range of each chunk
  double *csr_cpart;              // [csr_nchunks] chunk sums
  int32_t grid_main;              // workgroups of the init / update / replacement kernels
  int32_t grid_spmv;              // workgroups of the SpMV kernel (its partial-sum count)
  int32_t csr_lanes;              // CSR per-round kernels: lanes per row (the SpMV's)
  int32_t march_planes;           // diagonal SpMV marching along off[K-1]: planes per
                                  // workgroup (0: the row-slab kernels)
  int32_t march_bs;               // marching SpMV: threads per workgroup (256 or 512)
  int32_t march_ty;               // marching SpMV on 3-D grids: grid lines (offset off[1])
                                  // per tile; a tile is march_bs / march_ty row groups wide
  int32_t stream_nt;              // 1: the marching SpMV and the scaled update use streaming
                                  // (non-temporal) accesses for data touched once (set when a
                                  // CG iteration's data exceed the last-level cache)
  int64_t it_hint;                // CG iteration the host expects this launch to run: picks
                                  // the p buffer for loads issued before the kernel has read
                                  // the scalar block (checked there; a mismatch reloads)
};

// Device arrays of one graph.
struct GraphDev {
  int64_t n = 0, s = 0, t = 0, nt = 0;
  int64_t nnz = 0;                // stored off-diagonal CSR entries (2 per interior edge)
  int32_t *rowptr = nullptr, *col = nullptr;
  double *ccap = nullptr, *cs = nullptr, *ct = nullptr;
  double cst = 0.0;
  int32_t format = 1, K = 0;
  int32_t off[kMaxDiag] = {0};
  double *dcap = nullptr;
  int32_t fx_k = 0;               // fixed-point scale of cut values
  double cmax = 0.0;
  bool no_source_edges = false;
};

struct SweepBufs {
  uint64_t *keyA = nullptr, *keyB = nullptr;
  uint32_t *idA = nullptr, *idB = nullptr;
  uint32_t *rank = nullptr;
  __int128 *delta = nullptr;      // per rank position
  uint32_t *hist = nullptr;       // [256 * blocks + 256]: digit counts per block, digit totals
  __int128 *bsum = nullptr;       // per scan block
  __int128 *bmin = nullptr;
  int64_t *barg = nullptr;
  __int128 *best = nullptr;       // [2]: best prefix, D0
  int64_t *kstar = nullptr;
  uint8_t *mask = nullptr;        // [n]
  int sort_blocks = 0, scan_blocks = 0;
};

// ----------------------------------------------------------------------------
// launchers (defined in the .hip files)
// ----------------------------------------------------------------------------
template <typename T> hipError_t launch_assemble(const CGArgs<T> &a, int grid, hipStream_t st);
template <typename T> hipError_t launch_cginit(const CGArgs<T> &a, int grid, hipStream_t st);
// scaled form: wh from w and D (after the assembly), and v <- D^(dir/2) v
// (dir < 0, after CG: first adds the potential step an even iteration left
// pending)
template <typename T> hipError_t launch_scale_w(const CGArgs<T> &a, int grid, hipStream_t st);
template <typename T> hipError_t launch_scale_v(const CGArgs<T> &a, int dir, int grid, hipStream_t st);
// SpMV grid and kernel choice for a system: sets a.grid_spmv and a.march_planes
template <typename T> void spmv_layout(CGArgs<T> &a, int grid_main);
// 0 CSR, 1 diagonal (a row per thread), 2 diagonal (R-row vectors), 3 diagonal marching
template <typename T> int spmv_variant(const CGArgs<T> &a);
template <typename T> hipError_t launch_spmv(const CGArgs<T> &a, int grid, int rows_per_wave,
                                             bool fused_dia, hipStream_t st);
template <typename T> hipError_t launch_direction(const CGArgs<T> &a, int grid, hipStream_t st);
template <typename T> hipError_t launch_update(const CGArgs<T> &a, int grid, hipStream_t st);
// With ILU(0) of 4x4x4 tiles the CG update and the application z = M^-1 r of
// an iteration are one kernel, launched by launch_update; the iteration then
// makes no launch_bj_apply call.  In the precision form the FP64 residual
// replacement of these tiles also applies the preconditioner to the new
// residual, in the same kernel (launch_replace_residual).  That kernel moves
// the potentials every second iteration (as the scaled form does); a step
// left pending when CG stops is added by launch_flush_v.
template <typename T> inline bool bj_update_fused(const CGArgs<T> &a) { return a.bj_kind == 2 && a.bj_tile == 4; }
template <typename T> hipError_t launch_flush_v(const CGArgs<T> &a, int grid, hipStream_t st);
// block-Jacobi: factors once per round, and z = M^-1 r with r^T z into partial slot `slot`
template <typename T> hipError_t launch_bj_factor(const CGArgs<T> &a, int grid, hipStream_t st);
template <typename T> hipError_t launch_bj_apply(const CGArgs<T> &a, int grid, int slot, hipStream_t st);
template <typename T> hipError_t launch_replace_residual(const CGArgs<T> &a, int grid,
                                                         hipStream_t st);
template <typename T> hipError_t launch_stats(const CGArgs<T> &a, int grid, hipStream_t st);
hipError_t launch_fill(double *x, int64_t n, double value, hipStream_t st);
// streaming probe: nr (1..6) input and nw (1..2) output streams of n doubles (n even)
hipError_t launch_stream_probe(const double *in, double *out, int64_t n, int nr, int nw, int grid, bool nt,
                               hipStream_t st);

// two-level rounding (twolevel.hip)
struct TwoLevelBufs {
  int grid = 0;
  int64_t chunk = 0;
  int8_t *cls = nullptr;          // [nt] 0: S0, 1: S1, 2: Sc
  int32_t *cid = nullptr;         // [nt] coarse id
  double *part = nullptr;         // [3 grid] K-means partial sums
  int64_t *bnodes = nullptr, *bedges = nullptr, *boff = nullptr, *eoff = nullptr;   // [grid]
  __int128 *bst = nullptr;        // [grid] S1-S0 capacity per workgroup
  int32_t *eu = nullptr, *ev = nullptr;   // [interior edges] coarse Sc-Sc edges
  __int128 *ecap = nullptr;
  __int128 *ws = nullptr, *wt = nullptr;  // [nt] capacity of each coarse node to s_c / t_c
  uint8_t *side = nullptr;        // [nt + 2] source side of the coarse cut
  uint8_t *mask = nullptr;        // [n] lifted cut
};
hipError_t launch_tl_kmeans(const double *v, int64_t nt, double m, double *part, int grid, hipStream_t st);
hipError_t launch_tl_classify(const double *v, int64_t nt, double g0, double g1, int8_t *cls, int grid,
                              hipStream_t st);
hipError_t launch_tl_count(const int8_t *cls, const int32_t *rowptr, const int32_t *col, int64_t nt, int64_t chunk,
                           int64_t *bnodes, int64_t *bedges, int grid, hipStream_t st);
hipError_t launch_tl_ids(const int8_t *cls, int64_t nt, int64_t chunk, const int64_t *boff, int64_t nc,
                         int32_t *cid, int grid, hipStream_t st);
hipError_t launch_tl_edges(const int8_t *cls, const int32_t *cid, const int32_t *rowptr, const int32_t *col,
                           const double *ccap, const double *cs, const double *ct, int64_t nt, int64_t chunk,
                           int fx_k, const int64_t *eoff, int32_t *eu, int32_t *ev, __int128 *ecap, __int128 *ws,
                           __int128 *wt, __int128 *bst, int grid, hipStream_t st);
hipError_t launch_tl_lift(const int8_t *cls, const int32_t *cid, const uint8_t *side, int64_t nt, int64_t lo,
                          int64_t hi, uint8_t *mask, int grid, hipStream_t st);
hipError_t launch_scalars_reset(Scalars *sc, int64_t maxit, int32_t refine_every,
                                hipStream_t st);

// One graph of a batch (the single-graph resident solver uses one of these).
// Rows of all graphs are concatenated; each graph keeps local CSR indices.
// Rows with more than kHeavyRow entries (the hubs of power-law graphs) are
// not walked by one lane group in the resident solver: their entries are cut
// into chunks of kChunk (one wavefront each) whose partial sums are then
// added per row in a fixed order.
constexpr int32_t kHeavyRow = 128;
constexpr int32_t kCsrHeavy = 256;       // multi-workgroup CSR SpMV: rows longer than this are chunked
constexpr int32_t kCsrChunk = 256;
constexpr int32_t kChunk = 64;
constexpr int kChunkQ = 4;        // partial sums kept per chunk (the most any pass needs)
// Light rows are binned by length: bin b holds rows of at most 2^(b+1)
// entries (bin 5: at most 128).  By default a group of min(2^(b+1), 64)
// lanes walks each row of bin b, so the lanes of a wavefront finish their
// rows together; the lane code (3 bits per bin: log2 of the lanes) may set
// fewer lanes per row, each then taking several entries.
constexpr int kBins = 6;
constexpr int bin_default_lg(int b) { return b + 1 < 6 ? b + 1 : 6; }
constexpr uint32_t kDefaultLaneCode = (1u << 0) | (2u << 3) | (3u << 6) | (4u << 9) | (5u << 12) | (6u << 15);
static_assert(kBins == 6, "the default lane code lists six bins");

struct BatchGraph {
  int64_t node0;                  // first row in the concatenated non-terminal arrays
  int64_t nt;                     // rows of this graph
  int64_t nnz0;                   // first CSR entry of this graph
  int64_t node_off;               // first node id of this graph in the caller's arrays
  int64_t s, t;                   // local source and sink
  double cst;                     // s-t capacity
  int64_t chunk0;                 // first chunk of this graph's heavy rows
  int64_t heavy0;                 // first heavy-row record of this graph
  int32_t nchunks, nheavy;        // its chunks and heavy rows
  int32_t bin[kBins + 1];         // light rows of bin b: [bin[b], bin[b+1]) of its binned list
  int32_t nnz;                    // its CSR entries
  int32_t fx_k;                   // fixed-point scale of its cut values
  int32_t lanes;                  // lanes per light row (64 / rows per wavefront)
  int32_t no_source_edges;
  int32_t pad;
};
struct ResidentArgs {
  int32_t G;
  const BatchGraph *graphs;
  const int32_t *rowptr;          // per graph local row pointers, concatenated ([nt_g+1] each,
                                  // at node0 + g)
  const int32_t *col;             // local neighbour rows
  const double *ccap;
  const double *cs, *ct;
  double *w, *D, *b, *gt, *v, *r, *p, *q;
  irls_round_stats *stats;        // [G * (T+1)]
  unsigned *next_graph;           // work-queue counter
  const int32_t *order;           // graph processing order (largest first)
  // heavy rows, per graph at chunk0 / heavy0: chunk c covers local entries
  // [chunk_beg[c], chunk_end[c]) of local row chunk_row[c]; heavy row h is
  // local row heavy_row[h] with chunks [heavy_c0[h], heavy_c1[h]) of its graph
  const int32_t *chunk_row, *chunk_beg, *chunk_end;
  const int32_t *heavy_row, *heavy_c0, *heavy_c1;
  double *chunk_part;             // [total chunks * kChunkQ] partial sums
  // light rows by bin, per graph at node0: local row and its entry range
  const int32_t *bin_row, *bin_beg, *bin_end;
  int32_t rounds;
  double eps0, eps_factor;
  int32_t form, init, warm;
  double rtol;
  int64_t maxit;
  uint32_t lane_code;             // lanes per light row by bin (see kBins)
  double stop_gap;                // > 0: a graph stops after the first round with
                                  // l1 - lower_bound <= stop_gap * l1
};
hipError_t launch_resident(const ResidentArgs &a, int grid, int block, hipStream_t st);
// workgroups of k_resident (1024 threads) that fit on one CU at once (at least 1)
int resident_blocks_per_cu();
hipError_t launch_resident_reset(unsigned *next_graph, irls_round_stats *st, int64_t nrec, hipStream_t s);

// sweep
struct SweepArgs {
  int64_t nt, n, s, t;
  const double *v;
  const int32_t *rowptr, *col;
  const double *ccap, *cs, *ct;
  double cst;
  int32_t fx_k;
};
hipError_t sweep_run(const SweepArgs &a, SweepBufs &b, hipStream_t st);

// batched sweep: all graphs sorted at once by (graph, potential, id)
struct SweepBatchArgs {
  int32_t G;
  int64_t rows;                   // total non-terminal rows
  const BatchGraph *graphs;
  const uint32_t *gid;            // [rows] graph of each row
  const double *v;
  const int32_t *rowptr, *col;
  const double *ccap, *cs, *ct;
};
struct SweepBatchBufs {
  int64_t *kstar = nullptr;       // [G]
  __int128 *best = nullptr;       // [G] least prefix value of each graph
  uint8_t *mask = nullptr;        // [total nodes]
};
hipError_t sweep_batch_run(const SweepBatchArgs &a, SweepBufs &b, SweepBatchBufs &bb, hipStream_t st);
size_t sweep_scan_blocks(int64_t nt);
size_t sweep_sort_blocks(int64_t nt);
// sweep_run's buffers in the library's static scratch array on the current
// device (nt <= IRLS_NOALLOC_MAX_NONTERMINAL); allocates nothing
hipError_t sweep_noalloc_buffers(int64_t nt, int64_t n, SweepBufs &b);

}  // namespace irls
