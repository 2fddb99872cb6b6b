// Internal declarations of the learned warm start (host <-> HIP kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace irls {

constexpr int kH = 64;               // hidden width
constexpr int kF = 5;                // input features per node
typedef uint16_t bf16_t;

struct GnnArgs {
  int64_t nt;
  int32_t layers;
  const int32_t *rowptr, *col;    // the graph's CSR over non-terminal rows
  const double *ccap, *cs, *ct;
  const double *intensity;        // [nt] or null
  const double *xstart;           // [nt] potentials the solve starts from (round 0)
  const float *P;                 // FP32 parameters (flat, oracle order)
  const bf16_t *Wbf;              // [layers][128*64] bf16 copies of W_l
  int64_t off_Win, off_bin, off_W0, off_x, off_e;
  float *feats;                   // [nt*kF]
  float *invsum;                  // [nt]
  bf16_t *h;                      // [(layers+1)*nt*64] activations (bf16)
  bf16_t *agg;                    // [layers*nt*64] aggregated inputs (bf16)
  float *z;                       // [nt] logits
  float *dh0, *dh1;               // [nt*64] activation gradients (ping-pong)
  float *da;                      // [nt*64]
  float *part;                    // partial sums
  float *scal;                    // [256]: s, lam term, total loss, pooled[8..71], head sums[80..145]
  const double *y;                // [nt] targets
  double t, lam;
  float *grad;                    // [nparams]
};

__host__ __device__ inline int64_t gnn_off_W(const GnnArgs &a, int l) {
  return a.off_W0 + (int64_t)l * (2 * kH * kH + kH);
}

hipError_t gnn_forward(const GnnArgs &a, hipStream_t st);
hipError_t gnn_backward(const GnnArgs &a, int64_t nparams, hipStream_t st);
hipError_t gnn_adam(float *P, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                    float eps, float c1, float c2, hipStream_t st);
hipError_t gnn_refresh_bf16(const float *P, int64_t off_W0, int layers, uint16_t *Wbf, hipStream_t st);
hipError_t gnn_xhat(const float *z, int64_t nt, int64_t s, int64_t t, double *x, hipStream_t st);
hipError_t gnn_blend(const float *z, int64_t nt, double gamma, double *v, hipStream_t st);

}  // namespace irls
