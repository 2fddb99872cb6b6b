// Host side of the learned warm start: parameters, workspaces, the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/irls_gnn.h"
#include "gnn.h"
#include "internal.h"

using namespace irls;

namespace irls {
const GraphDev *handle_graph(irls_mincut_t h);       // defined in host.cpp
bool handle_is_batch(irls_mincut_t h);
double *handle_potentials(irls_mincut_t h);         // device rows, NULL before a solve
hipStream_t handle_stream(irls_mincut_t h);
}

struct irls_gnn_s {
  hipStream_t stream = nullptr;
  int32_t layers = 3;
  int64_t nparams = 0;
  int64_t off_Win = 0, off_bin = 0, off_W0 = 0, off_x = 0, off_e = 0;
  float *P = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *scal = nullptr;
  uint16_t *Wbf = nullptr;
  int64_t adam_t = 0;
  // workspace, grown to the largest graph seen
  int64_t cap = -1;
  float *feats = nullptr, *invsum = nullptr, *z = nullptr, *dh0 = nullptr, *dh1 = nullptr, *da = nullptr,
        *part = nullptr;
  uint16_t *h = nullptr, *agg = nullptr;
  double *y = nullptr, *inten = nullptr, *xs = nullptr, *xout = nullptr;
  std::string err;
  std::vector<void *> ws;       // workspace allocations
  std::vector<void *> fixed;    // parameter allocations

  void free_ws() {
    for (void *p : ws) (void)hipFree(p);
    ws.clear();
    cap = -1;
  }
  void free_all() {
    free_ws();
    for (void *p : fixed) (void)hipFree(p);
    fixed.clear();
  }
};

namespace {

thread_local std::string g_gnn_error;

irls_status gfail(irls_gnn_t g, hipError_t e, const char *what) {
  g->err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? IRLS_ERR_OOM : IRLS_ERR_DEVICE;
}

#define GCHK(g, expr, what)                          \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return gfail(g, e_, what); \
  } while (0)

template <typename T>
hipError_t galloc(std::vector<void *> &list, T **p, size_t count) {
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipSuccess) { list.push_back(q); *p = (T *)q; }
  return e;
}

// partial-sum floats the kernels need for nt rows
int64_t part_floats(int64_t nt) {
  const int64_t lb = std::min<int64_t>((nt + 63) / 64, 256);
  const int64_t waves = std::max<int64_t>(lb, 1) * 4;
  const int64_t hb = std::min<int64_t>((nt + 3) / 4, 1024);
  return std::max({waves * (2 * kH * kH + kH), hb * (kH + 2), hb * kH, hb * (kF + 1) * kH,
                   (int64_t)1024 * (kF + 1) * kH});
}

irls_status ensure_ws(irls_gnn_t g, int64_t nt) {
  if (nt <= g->cap) return IRLS_OK;
  g->free_ws();
  const int64_t n = std::max<int64_t>(nt, 1);
  GCHK(g, galloc(g->ws, &g->feats, n * kF), "alloc");
  GCHK(g, galloc(g->ws, &g->invsum, n), "alloc");
  GCHK(g, galloc(g->ws, &g->z, n), "alloc");
  GCHK(g, galloc(g->ws, &g->dh0, n * kH), "alloc");
  GCHK(g, galloc(g->ws, &g->dh1, n * kH), "alloc");
  GCHK(g, galloc(g->ws, &g->da, n * kH), "alloc");
  GCHK(g, galloc(g->ws, &g->part, part_floats(n)), "alloc");
  GCHK(g, galloc(g->ws, &g->h, (size_t)(g->layers + 1) * n * kH), "alloc");
  GCHK(g, galloc(g->ws, &g->agg, (size_t)g->layers * n * kH), "alloc");
  GCHK(g, galloc(g->ws, &g->y, n), "alloc");
  GCHK(g, galloc(g->ws, &g->inten, n), "alloc");
  GCHK(g, galloc(g->ws, &g->xs, n), "alloc");
  GCHK(g, galloc(g->ws, &g->xout, n + 2), "alloc");
  g->cap = nt;
  return IRLS_OK;
}

int64_t nid(int64_t u, int64_t s, int64_t t) { return u - (u > s) - (u > t); }

// host n-vector (by node id) -> device non-terminal rows
irls_status upload_rows(irls_gnn_t g, const GraphDev *gd, const double *src, double *dst) {
  std::vector<double> rows(gd->nt);
  for (int64_t u = 0; u < gd->n; u++)
    if (u != gd->s && u != gd->t) rows[nid(u, gd->s, gd->t)] = src[u];
  if (gd->nt > 0)
    GCHK(g, hipMemcpyAsync(dst, rows.data(), gd->nt * sizeof(double), hipMemcpyHostToDevice, g->stream), "upload");
  GCHK(g, hipStreamSynchronize(g->stream), "sync");
  return IRLS_OK;
}

GnnArgs make_args(irls_gnn_t g, const GraphDev *gd, bool with_intensity, const double *xstart) {
  GnnArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nt = gd->nt;
  a.xstart = xstart;
  a.layers = g->layers;
  a.rowptr = gd->rowptr;
  a.col = gd->col;
  a.ccap = gd->ccap;
  a.cs = gd->cs;
  a.ct = gd->ct;
  a.intensity = with_intensity ? g->inten : nullptr;
  a.P = g->P;
  a.Wbf = g->Wbf;
  a.off_Win = g->off_Win;
  a.off_bin = g->off_bin;
  a.off_W0 = g->off_W0;
  a.off_x = g->off_x;
  a.off_e = g->off_e;
  a.feats = g->feats;
  a.invsum = g->invsum;
  a.h = g->h;
  a.agg = g->agg;
  a.z = g->z;
  a.dh0 = g->dh0;
  a.dh1 = g->dh1;
  a.da = g->da;
  a.part = g->part;
  a.scal = g->scal;
  a.y = g->y;
  a.grad = g->grad;
  return a;
}

// SplitMix64 of (seed, index) -> uniform in [-1, 1)
double unit(uint64_t seed, uint64_t i) {
  uint64_t z = seed * 0x9E3779B97F4A7C15ull + i + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

const GraphDev *checked_graph(irls_gnn_t g, irls_mincut_t h) {
  if (!h) { g->err = "graph handle must not be NULL"; return nullptr; }
  if (handle_is_batch(h)) { g->err = "the network reads single-graph handles"; return nullptr; }
  return handle_graph(h);
}

// per-row inputs of one call: intensity (optional) and the start potentials,
// from the caller's host arrays or, for x_start == NULL, the handle's device
// potentials (after the handle's own stream has finished with them)
irls_status stage_inputs(irls_gnn_t g, irls_mincut_t h, const GraphDev *gd, const double *intensity,
                         const double *x_start, const double **xdev) {
  irls_status rc;
  if (intensity && (rc = upload_rows(g, gd, intensity, g->inten)) != IRLS_OK) return rc;
  if (x_start) {
    if ((rc = upload_rows(g, gd, x_start, g->xs)) != IRLS_OK) return rc;
    *xdev = g->xs;
    return IRLS_OK;
  }
  *xdev = handle_potentials(h);
  if (!*xdev) { g->err = "x_start is NULL and the graph handle holds no potentials"; return IRLS_ERR_NOT_SOLVED; }
  GCHK(g, hipStreamSynchronize(handle_stream(h)), "sync");
  return IRLS_OK;
}

}  // namespace

extern "C" {

irls_status irls_gnn_create(irls_gnn_t *out, int32_t hidden, int32_t layers, uint64_t seed, void *hip_stream) {
  if (!out) { g_gnn_error = "out must not be NULL"; return IRLS_ERR_NULL; }
  *out = nullptr;
  if (hidden != kH || layers < 1 || layers > 8) { g_gnn_error = "hidden must be 64 and 1 <= layers <= 8"; return IRLS_ERR_OPTIONS; }
  irls_gnn_t g = new irls_gnn_s();
  g->stream = (hipStream_t)hip_stream;
  g->layers = layers;
  g->off_Win = 0;
  g->off_bin = kF * kH;
  g->off_W0 = g->off_bin + kH;
  g->off_x = g->off_W0 + (int64_t)layers * (2 * kH * kH + kH);
  g->off_e = g->off_x + kH + 1;
  g->nparams = g->off_e + kH + 1;
  std::vector<float> P(g->nparams, 0.0f);
  auto glorot = [&](int64_t off, int64_t fan_in, int64_t fan_out, uint64_t stream) {
    const double lim = std::sqrt(6.0 / (double)(fan_in + fan_out));
    for (int64_t i = 0; i < fan_in * fan_out; i++) P[off + i] = (float)(lim * unit(seed * 131 + stream, i));
  };
  glorot(g->off_Win, kF, kH, 1);
  for (int l = 0; l < layers; l++) glorot(g->off_W0 + (int64_t)l * (2 * kH * kH + kH), 2 * kH, kH, 10 + l);
  glorot(g->off_x, kH, 1, 30);
  glorot(g->off_e, kH, 1, 31);
  P[g->off_e + kH] = (float)std::log(1e-4);
  hipError_t e = galloc(g->fixed, &g->P, g->nparams);
  if (e == hipSuccess) e = galloc(g->fixed, &g->m, g->nparams);
  if (e == hipSuccess) e = galloc(g->fixed, &g->v, g->nparams);
  if (e == hipSuccess) e = galloc(g->fixed, &g->grad, g->nparams);
  if (e == hipSuccess) e = galloc(g->fixed, &g->scal, 256);
  if (e == hipSuccess) e = galloc(g->fixed, &g->Wbf, (size_t)layers * 2 * kH * kH);
  if (e == hipSuccess) e = hipMemcpy(g->P, P.data(), g->nparams * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(g->m, 0, g->nparams * sizeof(float));
  if (e == hipSuccess) e = hipMemset(g->v, 0, g->nparams * sizeof(float));
  if (e == hipSuccess) e = hipMemset(g->grad, 0, g->nparams * sizeof(float));
  if (e == hipSuccess) e = hipMemset(g->scal, 0, 256 * sizeof(float));
  if (e == hipSuccess) e = gnn_refresh_bf16(g->P, g->off_W0, layers, g->Wbf, g->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
  if (e != hipSuccess) {
    g_gnn_error = std::string("network set-up: ") + hipGetErrorString(e);
    g->free_all();
    delete g;
    return e == hipErrorOutOfMemory ? IRLS_ERR_OOM : IRLS_ERR_DEVICE;
  }
  *out = g;
  return IRLS_OK;
}

irls_status irls_gnn_num_params(irls_gnn_t g, int64_t *count) {
  if (!g || !count) { g_gnn_error = "NULL argument"; return IRLS_ERR_NULL; }
  *count = g->nparams;
  return IRLS_OK;
}

irls_status irls_gnn_get_params(irls_gnn_t g, float *params) {
  if (!g || !params) { g_gnn_error = "NULL argument"; return IRLS_ERR_NULL; }
  GCHK(g, hipMemcpyAsync(params, g->P, g->nparams * sizeof(float), hipMemcpyDeviceToHost, g->stream), "download");
  GCHK(g, hipStreamSynchronize(g->stream), "sync");
  return IRLS_OK;
}

irls_status irls_gnn_set_params(irls_gnn_t g, const float *params) {
  if (!g || !params) { g_gnn_error = "NULL argument"; return IRLS_ERR_NULL; }
  GCHK(g, hipMemcpyAsync(g->P, params, g->nparams * sizeof(float), hipMemcpyHostToDevice, g->stream), "upload");
  GCHK(g, gnn_refresh_bf16(g->P, g->off_W0, g->layers, g->Wbf, g->stream), "bf16 weights");
  GCHK(g, hipStreamSynchronize(g->stream), "sync");
  return IRLS_OK;
}

irls_status irls_gnn_predict(irls_gnn_t g, irls_mincut_t h, const double *intensity, const double *x_start,
                             double *x_out, double *log_eps) {
  if (!g) { g_gnn_error = "network must not be NULL"; return IRLS_ERR_NULL; }
  const GraphDev *gd = checked_graph(g, h);
  if (!gd) return IRLS_ERR_OPTIONS;
  irls_status rc = ensure_ws(g, gd->nt);
  if (rc != IRLS_OK) return rc;
  const double *xdev = nullptr;
  if ((rc = stage_inputs(g, h, gd, intensity, x_start, &xdev)) != IRLS_OK) return rc;
  GnnArgs a = make_args(g, gd, intensity != nullptr, xdev);
  if (gd->nt > 0) GCHK(g, gnn_forward(a, g->stream), "forward");
  float s = (float)std::log(1e-4);
  if (gd->nt > 0) GCHK(g, hipMemcpyAsync(&s, g->scal, sizeof(float), hipMemcpyDeviceToHost, g->stream), "download");
  if (x_out) {
    if (gd->nt > 0) {
      GCHK(g, gnn_xhat(g->z, gd->nt, gd->s, gd->t, g->xout, g->stream), "xhat");
      GCHK(g, hipMemcpyAsync(x_out, g->xout, gd->n * sizeof(double), hipMemcpyDeviceToHost, g->stream), "download");
    }
  }
  GCHK(g, hipStreamSynchronize(g->stream), "sync");
  if (x_out) { x_out[gd->s] = 1.0; x_out[gd->t] = 0.0; }
  if (log_eps) *log_eps = s;
  return IRLS_OK;
}

irls_status irls_gnn_warm_start(irls_gnn_t g, irls_mincut_t h, const double *intensity, double gamma,
                                double *log_eps) {
  if (!g) { g_gnn_error = "network must not be NULL"; return IRLS_ERR_NULL; }
  if (!(gamma >= 0.0 && gamma <= 1.0)) { g->err = "gamma must lie in [0, 1]"; return IRLS_ERR_OPTIONS; }
  const GraphDev *gd = checked_graph(g, h);
  if (!gd) return IRLS_ERR_OPTIONS;
  irls_status rc = ensure_ws(g, gd->nt);
  if (rc != IRLS_OK) return rc;
  const double *xdev = nullptr;
  if ((rc = stage_inputs(g, h, gd, intensity, nullptr, &xdev)) != IRLS_OK) return rc;
  float s = (float)std::log(1e-4);
  if (gd->nt > 0) {
    GnnArgs a = make_args(g, gd, intensity != nullptr, xdev);
    GCHK(g, gnn_forward(a, g->stream), "forward");
    GCHK(g, hipMemcpyAsync(&s, g->scal, sizeof(float), hipMemcpyDeviceToHost, g->stream), "download");
    GCHK(g, gnn_blend(g->z, gd->nt, gamma, handle_potentials(h), g->stream), "blend");
  }
  GCHK(g, hipStreamSynchronize(g->stream), "sync");
  if (log_eps) *log_eps = s;
  return IRLS_OK;
}

irls_status irls_gnn_loss_grad(irls_gnn_t g, irls_mincut_t h, const double *intensity, const double *x_start,
                               const double *y, double log_eps_target, double lambda, double *loss,
                               float *grad_out) {
  if (!g) { g_gnn_error = "network must not be NULL"; return IRLS_ERR_NULL; }
  if (!y) { g->err = "targets must not be NULL"; return IRLS_ERR_NULL; }
  const GraphDev *gd = checked_graph(g, h);
  if (!gd) return IRLS_ERR_OPTIONS;
  if (gd->nt < 1) { g->err = "the graph has no non-terminal nodes"; return IRLS_ERR_RANGE; }
  irls_status rc = ensure_ws(g, gd->nt);
  if (rc != IRLS_OK) return rc;
  const double *xdev = nullptr;
  if ((rc = stage_inputs(g, h, gd, intensity, x_start, &xdev)) != IRLS_OK) return rc;
  if ((rc = upload_rows(g, gd, y, g->y)) != IRLS_OK) return rc;
  GnnArgs a = make_args(g, gd, intensity != nullptr, xdev);
  a.t = log_eps_target;
  a.lam = lambda;
  GCHK(g, gnn_forward(a, g->stream), "forward");
  GCHK(g, gnn_backward(a, g->nparams, g->stream), "backward");
  float L = 0.0f;
  GCHK(g, hipMemcpyAsync(&L, g->scal + 2, sizeof(float), hipMemcpyDeviceToHost, g->stream), "download");
  if (grad_out)
    GCHK(g, hipMemcpyAsync(grad_out, g->grad, g->nparams * sizeof(float), hipMemcpyDeviceToHost, g->stream), "download");
  GCHK(g, hipStreamSynchronize(g->stream), "sync");
  if (loss) *loss = L;
  return IRLS_OK;
}

irls_status irls_gnn_adam_step(irls_gnn_t g, double lr, double beta1, double beta2, double eps) {
  if (!g) { g_gnn_error = "network must not be NULL"; return IRLS_ERR_NULL; }
  if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0)) {
    g->err = "Adam hyper-parameters out of range";
    return IRLS_ERR_OPTIONS;
  }
  g->adam_t++;
  const float c1 = (float)(1.0 - std::pow(beta1, (double)g->adam_t));
  const float c2 = (float)(1.0 - std::pow(beta2, (double)g->adam_t));
  GCHK(g, gnn_adam(g->P, g->grad, g->m, g->v, g->nparams, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2,
                   g->stream), "adam");
  GCHK(g, gnn_refresh_bf16(g->P, g->off_W0, g->layers, g->Wbf, g->stream), "bf16 weights");
  return IRLS_OK;
}

void irls_gnn_destroy(irls_gnn_t g) {
  if (!g) return;
  (void)hipStreamSynchronize(g->stream);
  g->free_all();
  delete g;
}

const char *irls_gnn_last_error(irls_gnn_t g) { return g ? g->err.c_str() : g_gnn_error.c_str(); }

}  // extern "C"
