// Learned warm start for the IRLS rounds (gfx950 kernels).
//
// Not part of the paper: it extends the paper's warm start (Section 3.1,
// each solve starts from the previous round) across instances.  A
// message-passing network predicts a starting potential vector and a starting
// smoothing eps from per-node inputs:
//   f_u  = [log1p(c_us), log1p(c_ut), log1p(w_u), I_u, x0_u]   (w_u: all capacity at u,
//                                                              x0: round-0 potentials)
//   h0   = bf16(relu(f W_in + b_in))
//   a_l  = A h_{l-1},  A_uv = c_uv / sum_v' c_uv'               (capacity-weighted mean)
//   h_l  = bf16(relu(bf16([h_{l-1} | a_l]) W_l + b_l))          (W_l: 128 x 64, bf16)
//   z_u  = h_L,u . w_x + b_x;  xhat = sigmoid(z);  s = mean(h_L) . w_e + b_e = log eps
// Each layer is one kernel: the capacity-weighted SpMM of a 16-row tile into
// LDS, then the dense product on the matrix cores (v_mfma_f32_16x16x16_bf16,
// FP32 accumulation), bias, ReLU and the bf16 store.  The backward pass uses
// the same MFMA for dZ W^T and X^T dZ, and a transposed SpMM (gather form, the
// CSR pattern is symmetric) for the aggregation.  Every grid-wide sum is a
// per-workgroup (or per-wavefront) partial reduced later in fixed order.
#include <algorithm>

#include "device_common.h"
#include "gnn.h"

namespace irls {

constexpr int kGB = 256;             // threads per workgroup (4 wavefronts)
constexpr int kTile = 16;            // rows per wavefront tile (MFMA M)

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16_t f2bf(float f) {        // round to nearest even
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)(u >> 16 | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ----------------------------------------------------------------------------
// inputs
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kGB) void k_gnn_feats(GnnArgs a) {
  for (int64_t u = row_begin(); u < a.nt; u += row_stride()) {
    double csum = 0.0;
    for (int32_t e = a.rowptr[u]; e < a.rowptr[u + 1]; e++) csum += a.ccap[e];
    const double w = csum + a.cs[u] + a.ct[u];
    a.feats[kF * u + 0] = (float)log1p(a.cs[u]);
    a.feats[kF * u + 1] = (float)log1p(a.ct[u]);
    a.feats[kF * u + 2] = (float)log1p(w);
    a.feats[kF * u + 3] = a.intensity ? (float)a.intensity[u] : 0.0f;
    a.feats[kF * u + 4] = (float)a.xstart[u];
    a.invsum[u] = csum > 0.0 ? (float)(1.0 / csum) : 0.0f;
  }
}

// h0 = bf16(relu(f W_in + b_in)); one thread per (row, hidden unit)
__global__ __launch_bounds__(kGB) void k_gnn_in(GnnArgs a) {
  const int64_t n = a.nt * kH;
  for (int64_t i = row_begin(); i < n; i += row_stride()) {
    const int64_t u = i / kH;
    const int j = (int)(i % kH);
    float acc = a.P[a.off_bin + j];
#pragma unroll
    for (int f = 0; f < kF; f++) acc += a.feats[kF * u + f] * a.P[a.off_Win + f * kH + j];
    a.h[i] = f2bf(fmaxf(acc, 0.0f));
  }
}

// ----------------------------------------------------------------------------
// forward layer: a = A h_prev (16-row tiles), Z = [h_prev | a] W + b, relu
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kGB) void k_gnn_layer_fwd(GnnArgs a, int l) {
  __shared__ bf16_t sW[2 * kH * kH];                 // W_l, 128 x 64
  __shared__ bf16_t sX[kGB / 64][kTile][2 * kH];      // per wavefront: [h | a] tile
  const bf16_t *Wl = a.Wbf + (int64_t)l * 2 * kH * kH;
  for (int i = threadIdx.x; i < 2 * kH * kH; i += kGB) sW[i] = Wl[i];
  __syncthreads();
  const bf16_t *hp = a.h + (int64_t)l * a.nt * kH;
  bf16_t *hn = a.h + (int64_t)(l + 1) * a.nt * kH;
  bf16_t *ag = a.agg + (int64_t)l * a.nt * kH;
  const float *bias = a.P + gnn_off_W(a, l) + 2 * kH * kH;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t ntiles = (a.nt + kTile - 1) / kTile;
  for (int64_t tile = (int64_t)blockIdx.x * (kGB / 64) + wid; tile < ntiles; tile += (int64_t)gridDim.x * (kGB / 64)) {
    const int64_t r0 = tile * kTile;
    // the tile's LDS rows are written and read by lanes of this wavefront
    // only; the wave barriers keep the compiler from moving LDS accesses
    // across the hand-over
    __builtin_amdgcn_wave_barrier();
    // aggregation, lane = hidden unit
    for (int m = 0; m < kTile; m++) {
      const int64_t u = r0 + m;
      float acc = 0.0f;
      bf16_t hu = 0;
      if (u < a.nt) {
        const float is = a.invsum[u];
        for (int32_t e = a.rowptr[u]; e < a.rowptr[u + 1]; e++)
          acc += (float)a.ccap[e] * is * bf2f(hp[(int64_t)a.col[e] * kH + lane]);
        hu = hp[u * kH + lane];
      }
      const bf16_t ab = f2bf(acc);
      sX[wid][m][lane] = hu;
      sX[wid][m][kH + lane] = ab;
      if (u < a.nt) ag[u * kH + lane] = ab;
    }
    __builtin_amdgcn_wave_barrier();
    // MFMA: 4 column tiles of 16, 8 k-steps of 16
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; t++) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const int mr = lane % 16, kq = 4 * (lane / 16);
#pragma unroll
    for (int s = 0; s < 8; s++) {
      bf16x4 A;
#pragma unroll
      for (int i = 0; i < 4; i++) A[i] = (short)sX[wid][mr][16 * s + kq + i];
#pragma unroll
      for (int t = 0; t < 4; t++) {
        bf16x4 B;
#pragma unroll
        for (int i = 0; i < 4; i++) B[i] = (short)sW[(16 * s + kq + i) * kH + 16 * t + mr];
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[t], 0, 0, 0);
      }
    }
    // epilogue: lane holds rows kq+i, column 16t + mr
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int n = 16 * t + mr;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int64_t u = r0 + kq + i;
        if (u < a.nt) hn[u * kH + n] = f2bf(fmaxf(acc[t][i] + bias[n], 0.0f));
      }
    }
  }
}

// ----------------------------------------------------------------------------
// heads: z = h_L w_x + b_x per row; per-workgroup partial sums of h_L (pooling)
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kGB) void k_gnn_heads(GnnArgs a) {
  __shared__ float sp[kGB / 64][kH];
  const bf16_t *hL = a.h + (int64_t)a.layers * a.nt * kH;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const float wx = a.P[a.off_x + lane], bx = a.P[a.off_x + kH];
  float pool = 0.0f;
  const int64_t wave = (int64_t)blockIdx.x * (kGB / 64) + wid, nwaves = (int64_t)gridDim.x * (kGB / 64);
  for (int64_t u = wave; u < a.nt; u += nwaves) {           // one row per wavefront, lane = unit
    const float hv = bf2f(hL[u * kH + lane]);
    pool += hv;
    float d = hv * wx;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
    if (lane == 0) a.z[u] = d + bx;
  }
  sp[wid][lane] = pool;
  __syncthreads();
  if (threadIdx.x < kH) {
    float s = 0.0f;
    for (int w = 0; w < kGB / 64; w++) s += sp[w][threadIdx.x];
    a.part[(int64_t)blockIdx.x * kH + threadIdx.x] = s;
  }
}

// s = mean(h_L) . w_e + b_e, from the pooling partials of nb workgroups
__global__ __launch_bounds__(kH) void k_gnn_pool(GnnArgs a, int nb) {
  __shared__ float sp[kH];
  float s = 0.0f;
  for (int b = 0; b < nb; b++) s += a.part[(int64_t)b * kH + threadIdx.x];
  const float pooled = s / (float)a.nt;
  sp[threadIdx.x] = pooled * a.P[a.off_e + threadIdx.x];
  a.scal[8 + threadIdx.x] = pooled;
  __syncthreads();
  if (threadIdx.x == 0) {
    float d = 0.0f;
    for (int j = 0; j < kH; j++) d += sp[j];
    a.scal[0] = d + a.P[a.off_e + kH];
  }
}

// ----------------------------------------------------------------------------
// loss: mean BCE(sigmoid(z), y) + lam (s - t)^2 and its gradient at h_L
// partials per workgroup: [loss, dbx, dwx[64]]
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kGB) void k_gnn_loss(GnnArgs a) {
  __shared__ float sp[kGB / 64][kH + 2];
  const bf16_t *hL = a.h + (int64_t)a.layers * a.nt * kH;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const float s = a.scal[0];
  const float ds = (float)(2.0 * a.lam * ((double)s - a.t));
  const float inv = 1.0f / (float)a.nt;
  const float wx = a.P[a.off_x + lane], we = a.P[a.off_e + lane];
  float dwx = 0.0f, dbx = 0.0f, loss = 0.0f;
  const int64_t wave = (int64_t)blockIdx.x * (kGB / 64) + wid, nwaves = (int64_t)gridDim.x * (kGB / 64);
  for (int64_t u = wave; u < a.nt; u += nwaves) {
    const float z = a.z[u], y = (float)a.y[u];
    const float sg = 1.0f / (1.0f + expf(-z));
    const float dz = (sg - y) * inv;
    const float hv = bf2f(hL[u * kH + lane]);
    dwx += dz * hv;
    if (lane == 0) {
      dbx += dz;
      // BCE with logits: max(z,0) - z y + log(1 + exp(-|z|))
      loss += (fmaxf(z, 0.0f) - z * y + log1pf(expf(-fabsf(z)))) * inv;
    }
    a.dh0[u * kH + lane] = dz * wx + ds * inv * we;
  }
  sp[wid][lane] = dwx;
  if (lane == 0) { sp[wid][kH] = dbx; sp[wid][kH + 1] = loss; }
  __syncthreads();
  if (threadIdx.x < kH + 2) {
    float t = 0.0f;
    for (int w = 0; w < kGB / 64; w++) t += sp[w][threadIdx.x];
    a.part[(int64_t)blockIdx.x * (kH + 2) + threadIdx.x] = t;
  }
}

// ----------------------------------------------------------------------------
// backward of layer l: dZ = bf16(dh ⊙ [h_l > 0]); dX = dZ W^T -> (dh_prev, da);
// per-wavefront partials of dW = X^T dZ (128 x 64) and db (64)
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kGB) void k_gnn_layer_bwd(GnnArgs a, int l, const float *dh, float *dhp) {
  __shared__ bf16_t sW[2 * kH * kH];
  __shared__ bf16_t sX[kGB / 64][kTile][2 * kH];
  __shared__ bf16_t sD[kGB / 64][kTile][kH];
  const bf16_t *Wl = a.Wbf + (int64_t)l * 2 * kH * kH;
  for (int i = threadIdx.x; i < 2 * kH * kH; i += kGB) sW[i] = Wl[i];
  __syncthreads();
  const bf16_t *hp = a.h + (int64_t)l * a.nt * kH;
  const bf16_t *hl = a.h + (int64_t)(l + 1) * a.nt * kH;
  const bf16_t *ag = a.agg + (int64_t)l * a.nt * kH;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int mr = lane % 16, kq = 4 * (lane / 16);
  f32x4 gW[8][4];                                     // dW partial: 8 x 4 tiles of 16 x 16
#pragma unroll
  for (int i = 0; i < 8; i++)
#pragma unroll
    for (int t = 0; t < 4; t++) gW[i][t] = (f32x4){0.f, 0.f, 0.f, 0.f};
  float gb = 0.0f;
  const int64_t ntiles = (a.nt + kTile - 1) / kTile;
  const int64_t wave = (int64_t)blockIdx.x * (kGB / 64) + wid, nwaves = (int64_t)gridDim.x * (kGB / 64);
  for (int64_t tile = wave; tile < ntiles; tile += nwaves) {
    const int64_t r0 = tile * kTile;
    __builtin_amdgcn_wave_barrier();
    for (int m = 0; m < kTile; m++) {
      const int64_t u = r0 + m;
      bf16_t d = 0, xh = 0, xa = 0;
      if (u < a.nt) {
        const float g = dh[u * kH + lane];
        d = bf2f(hl[u * kH + lane]) > 0.0f ? f2bf(g) : (bf16_t)0;
        xh = hp[u * kH + lane];
        xa = ag[u * kH + lane];
      }
      sD[wid][m][lane] = d;
      sX[wid][m][lane] = xh;
      sX[wid][m][kH + lane] = xa;
      gb += bf2f(d);
    }
    __builtin_amdgcn_wave_barrier();
    // dX = dZ W^T: 8 column tiles (inputs) x 4 k-steps (hidden)
    f32x4 dx[8];
#pragma unroll
    for (int t = 0; t < 8; t++) dx[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; s++) {
      bf16x4 A;
#pragma unroll
      for (int i = 0; i < 4; i++) A[i] = (short)sD[wid][mr][16 * s + kq + i];
#pragma unroll
      for (int t = 0; t < 8; t++) {
        bf16x4 B;                                    // B[k][n] = W[n][k]
#pragma unroll
        for (int i = 0; i < 4; i++) B[i] = (short)sW[(16 * t + mr) * kH + 16 * s + kq + i];
        dx[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, dx[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < 8; t++) {
      const int n = 16 * t + mr;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int64_t u = r0 + kq + i;
        if (u >= a.nt) continue;
        if (n < kH) dhp[u * kH + n] = dx[t][i];
        else a.da[u * kH + n - kH] = dx[t][i];
      }
    }
    // dW += X^T dZ: 8 row tiles (inputs) x 4 column tiles (hidden), K = the 16 rows
#pragma unroll
    for (int i8 = 0; i8 < 8; i8++) {
      bf16x4 A;                                      // A[m][k] = X[k][16 i8 + m]
#pragma unroll
      for (int i = 0; i < 4; i++) A[i] = (short)sX[wid][kq + i][16 * i8 + mr];
#pragma unroll
      for (int t = 0; t < 4; t++) {
        bf16x4 B;                                    // B[k][n] = dZ[k][16 t + n]
#pragma unroll
        for (int i = 0; i < 4; i++) B[i] = (short)sD[wid][kq + i][16 * t + mr];
        gW[i8][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, gW[i8][t], 0, 0, 0);
      }
    }
  }
  // per-wavefront partials: 8192 dW entries then 64 db entries
  float *pw = a.part + wave * (2 * kH * kH + kH);
#pragma unroll
  for (int i8 = 0; i8 < 8; i8++)
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
      for (int i = 0; i < 4; i++) pw[(16 * i8 + kq + i) * kH + 16 * t + mr] = gW[i8][t][i];
  pw[2 * kH * kH + lane] = gb;
}

// dh_prev[j] += sum over neighbours u of A_uj da[u], A_uj = c_uj / sum_v c_uv
__global__ __launch_bounds__(kGB) void k_gnn_aggT(GnnArgs a, float *dhp) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t j = wave; j < a.nt; j += nwaves) {
    float acc = dhp[j * kH + lane];
    for (int32_t e = a.rowptr[j]; e < a.rowptr[j + 1]; e++) {
      const int64_t u = a.col[e];
      acc += (float)a.ccap[e] * a.invsum[u] * a.da[u * kH + lane];
    }
    dhp[j * kH + lane] = acc;
  }
}

// input layer: dZ0 = dh0 ⊙ [h0 > 0]; per-workgroup partials of dW_in (kF x 64), db_in
constexpr int kInG = kF + 1;                 // gradient rows of the input layer: W_in, b_in
__global__ __launch_bounds__(kGB) void k_gnn_in_bwd(GnnArgs a, const float *dh) {
  __shared__ float sp[kGB / 64][kInG * kH];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  float g[kInG] = {};
  const int64_t wave = (int64_t)blockIdx.x * (kGB / 64) + wid, nwaves = (int64_t)gridDim.x * (kGB / 64);
  for (int64_t u = wave; u < a.nt; u += nwaves) {
    const float d = bf2f(a.h[u * kH + lane]) > 0.0f ? dh[u * kH + lane] : 0.0f;
#pragma unroll
    for (int f = 0; f < kF; f++) g[f] += a.feats[kF * u + f] * d;
    g[kF] += d;
  }
#pragma unroll
  for (int f = 0; f < kInG; f++) sp[wid][f * kH + lane] = g[f];
  __syncthreads();
  for (int i = threadIdx.x; i < kInG * kH; i += kGB) {
    float s = 0.0f;
    for (int w = 0; w < kGB / 64; w++) s += sp[w][i];
    a.part[(int64_t)blockIdx.x * kInG * kH + i] = s;
  }
}

// fixed-order sum of nparts partial vectors of length len into out (+ offset)
__global__ __launch_bounds__(kGB) void k_gnn_sum_parts(const float *part, int64_t nparts, int64_t stride,
                                                       int64_t len, float *out) {
  for (int64_t i = row_begin(); i < len; i += row_stride()) {
    float s = 0.0f;
    for (int64_t p = 0; p < nparts; p++) s += part[p * stride + i];
    out[i] = s;
  }
}

// heads: dw_x, db_x from the summed partials (scal[80..145] = dwx[64], dbx,
// BCE); the eps head dw_e = ds pooled, db_e = ds; total loss into scal[2]
__global__ void k_gnn_head_grads(GnnArgs a) {
  const double sd = (double)a.scal[0] - a.t;
  const float ds = (float)(2.0 * a.lam * sd);
  const int j = threadIdx.x;
  if (j < kH) {
    a.grad[a.off_x + j] = a.scal[80 + j];
    a.grad[a.off_e + j] = ds * a.scal[8 + j];
  }
  if (j == 0) {
    a.grad[a.off_x + kH] = a.scal[80 + kH];
    a.grad[a.off_e + kH] = ds;
    a.scal[2] = a.scal[80 + kH + 1] + (float)(a.lam * sd * sd);
  }
}

// Adam on the FP32 master parameters, then the bf16 copies of W_l
__global__ __launch_bounds__(kGB) void k_gnn_adam(float *P, const float *g, float *m, float *v, int64_t n,
                                                  float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = row_begin(); i < n; i += row_stride()) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ __launch_bounds__(kGB) void k_gnn_wbf(const float *P, int64_t off_W0, int layers, bf16_t *Wbf) {
  const int64_t per = 2 * kH * kH;
  for (int64_t i = row_begin(); i < (int64_t)layers * per; i += row_stride()) {
    const int64_t l = i / per, k = i % per;
    Wbf[i] = f2bf(P[off_W0 + l * (per + kH) + k]);
  }
}

// predictions: xhat = sigmoid(z) scattered to node ids (s = 1, t = 0 set by host)
__global__ __launch_bounds__(kGB) void k_gnn_xhat(const float *z, int64_t nt, int64_t s, int64_t t, double *x) {
  const int64_t lo = s < t ? s : t, hi = s < t ? t : s;
  for (int64_t i = row_begin(); i < nt; i += row_stride()) {
    int64_t u = i;
    if (u >= lo) u++;
    if (u >= hi) u++;
    x[u] = 1.0 / (1.0 + exp(-(double)z[i]));
  }
}

// warm start in place: v <- v + gamma (sigmoid(z) - v) on the non-terminal rows
__global__ __launch_bounds__(kGB) void k_gnn_blend(const float *z, int64_t nt, double gamma, double *v) {
  for (int64_t i = row_begin(); i < nt; i += row_stride()) {
    const double xh = 1.0 / (1.0 + exp(-(double)z[i]));
    v[i] += gamma * (xh - v[i]);
  }
}

// ----------------------------------------------------------------------------
// drivers
// ----------------------------------------------------------------------------
static int ggrid(int64_t n, int per) {
  int64_t g = (n + per - 1) / per;
  if (g > 1024) g = 1024;
  return g < 1 ? 1 : (int)g;
}

hipError_t gnn_forward(const GnnArgs &a, hipStream_t st) {
  const int gr = ggrid(a.nt, kGB);
  hipLaunchKernelGGL(k_gnn_feats, dim3(gr), dim3(kGB), 0, st, a);
  hipLaunchKernelGGL(k_gnn_in, dim3(ggrid(a.nt * kH, kGB)), dim3(kGB), 0, st, a);
  const int tiles = (int)std::min<int64_t>((a.nt + kTile * 4 - 1) / (kTile * 4), 1024);
  for (int l = 0; l < a.layers; l++)
    hipLaunchKernelGGL(k_gnn_layer_fwd, dim3(tiles > 0 ? tiles : 1), dim3(kGB), 0, st, a, l);
  const int hb = ggrid(a.nt, kGB / 64);
  hipLaunchKernelGGL(k_gnn_heads, dim3(hb), dim3(kGB), 0, st, a);
  hipLaunchKernelGGL(k_gnn_pool, dim3(1), dim3(kH), 0, st, a, hb);
  return hipGetLastError();
}

// loss and the full gradient (into a.grad); a.part must hold
// max(waves * (128*64+64), blocks * 5*64) floats
hipError_t gnn_backward(const GnnArgs &a, int64_t nparams, hipStream_t st) {
  const int hb = ggrid(a.nt, kGB / 64);
  hipLaunchKernelGGL(k_gnn_loss, dim3(hb), dim3(kGB), 0, st, a);
  // head partials per workgroup: dwx[64], dbx, BCE -> scal[80..145]
  hipLaunchKernelGGL(k_gnn_sum_parts, dim3(1), dim3(kGB), 0, st, (const float *)a.part, (int64_t)hb,
                     (int64_t)(kH + 2), (int64_t)(kH + 2), a.scal + 80);
  hipLaunchKernelGGL(k_gnn_head_grads, dim3(1), dim3(kH), 0, st, a);
  const int lb = (int)std::min<int64_t>((a.nt + kTile * 4 - 1) / (kTile * 4), 256);
  const int nw = (lb > 0 ? lb : 1) * (kGB / 64);
  float *dh = a.dh0, *dhp = a.dh1;
  for (int l = a.layers - 1; l >= 0; l--) {
    hipLaunchKernelGGL(k_gnn_layer_bwd, dim3(lb > 0 ? lb : 1), dim3(kGB), 0, st, a, l, (const float *)dh, dhp);
    hipLaunchKernelGGL(k_gnn_sum_parts, dim3(ggrid(2 * kH * kH + kH, kGB)), dim3(kGB), 0, st,
                       (const float *)a.part, (int64_t)nw, (int64_t)(2 * kH * kH + kH),
                       (int64_t)(2 * kH * kH + kH), a.grad + gnn_off_W(a, l));
    hipLaunchKernelGGL(k_gnn_aggT, dim3(ggrid(a.nt * 64, kGB)), dim3(kGB), 0, st, a, dhp);
    float *tmp = dh; dh = dhp; dhp = tmp;
  }
  const int ib = ggrid(a.nt, kGB / 64);
  hipLaunchKernelGGL(k_gnn_in_bwd, dim3(ib), dim3(kGB), 0, st, a, (const float *)dh);
  hipLaunchKernelGGL(k_gnn_sum_parts, dim3(2), dim3(kGB), 0, st, (const float *)a.part, (int64_t)ib,
                     (int64_t)(kInG * kH), (int64_t)(kInG * kH), a.grad + a.off_Win);
  (void)nparams;
  return hipGetLastError();
}

hipError_t gnn_adam(float *P, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                    float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_gnn_adam, dim3(ggrid(n, kGB)), dim3(kGB), 0, st, P, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t gnn_refresh_bf16(const float *P, int64_t off_W0, int layers, uint16_t *Wbf, hipStream_t st) {
  hipLaunchKernelGGL(k_gnn_wbf, dim3(ggrid((int64_t)layers * 2 * kH * kH, kGB)), dim3(kGB), 0, st, P, off_W0,
                     layers, Wbf);
  return hipGetLastError();
}

hipError_t gnn_xhat(const float *z, int64_t nt, int64_t s, int64_t t, double *x, hipStream_t st) {
  hipLaunchKernelGGL(k_gnn_xhat, dim3(ggrid(nt, kGB)), dim3(kGB), 0, st, z, nt, s, t, x);
  return hipGetLastError();
}

hipError_t gnn_blend(const float *z, int64_t nt, double gamma, double *v, hipStream_t st) {
  hipLaunchKernelGGL(k_gnn_blend, dim3(ggrid(nt, kGB)), dim3(kGB), 0, st, z, nt, gamma, v);
  return hipGetLastError();
}

}  // namespace irls
