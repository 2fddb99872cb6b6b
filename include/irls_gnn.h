/*
 * irls_gnn.h -- learned warm start for the IRLS min-cut (libirls_mincut.so).
 *
 * Not part of the paper.  The paper warm-starts every CG solve from the
 * previous IRLS round (Section 3.1); this network carries a warm start across
 * instances: from per-node inputs it predicts the potentials the IRLS rounds
 * converge to and a starting smoothing eps.  A caller starts the reweighted
 * rounds from a blend of the round-0 potentials and the prediction, at the
 * predicted eps (irls_mincut_solve_range with start 2).
 *
 * Model (hidden width 64, `layers` message-passing layers):
 *   f_u  = [log1p(c_us), log1p(c_ut), log1p(w_u), I_u, x0_u]
 *          w_u: all capacity at u, I_u: optional intensity (0 if absent),
 *          x0_u: the potentials the rounds start from (normally round 0's,
 *          the solution with W = C)
 *   h0   = bf16(relu(f W_in + b_in))
 *   h_l  = bf16(relu(bf16([h_{l-1} | A h_{l-1}]) bf16(W_l) + b_l)),
 *          A_uv = c_uv / sum_v' c_uv' over interior neighbours
 *   xhat = sigmoid(h_L w_x + b_x);  log eps = mean_u(h_L) w_e + b_e
 * loss = mean_u BCE(xhat_u, y_u) + lambda (log eps - t)^2.
 * Parameters are FP32 masters (flat, in the order W_in, b_in, then W_l, b_l
 * per layer, then w_x, b_x, w_e, b_e; matrices row-major input x output);
 * the dense layers run on bf16 copies with FP32 accumulation.
 *
 * All functions return irls_status (see irls_mincut.h).  A network is tied to
 * the HIP stream given at creation; it reads graphs from single-graph
 * irls_mincut handles (their device CSR, and their potentials when x_start is
 * NULL: the call first waits for the handle's stream).  Host arrays are
 * indexed by node id.  A network keeps a workspace sized for the largest graph
 * it has seen (about 1.7 KB per non-terminal node with 3 layers).
 */
#ifndef IRLS_GNN_H
#define IRLS_GNN_H
#include <stdint.h>

#include "irls_mincut.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct irls_gnn_s *irls_gnn_t;

/* hidden must be 64; 1 <= layers <= 8; weights drawn from `seed` (Glorot
 * uniform, biases 0, b_e = log 1e-4). */
irls_status irls_gnn_create(irls_gnn_t *out, int32_t hidden, int32_t layers, uint64_t seed,
                            void *hip_stream);
irls_status irls_gnn_num_params(irls_gnn_t g, int64_t *count);
irls_status irls_gnn_get_params(irls_gnn_t g, float *params);          /* host, count floats */
irls_status irls_gnn_set_params(irls_gnn_t g, const float *params);    /* host, count floats */

/* Prediction for the graph of h.  intensity: n doubles or NULL (treated as 0).
 * x_start: n doubles, or NULL = the potentials h holds (IRLS_ERR_NOT_SOLVED if
 * it holds none).  x_out: n doubles (host), NULL allowed; x_s = 1, x_t = 0.
 * log_eps: NULL allowed. */
irls_status irls_gnn_predict(irls_gnn_t g, irls_mincut_t h, const double *intensity,
                             const double *x_start, double *x_out, double *log_eps);

/* Warm start in place: h must hold potentials x0 (normally round 0's, from
 * irls_mincut_solve_range(h, 0, NULL, 0, 0, NULL)).  Runs the network with
 * x_start = x0 and replaces the potentials on the device by
 * x0 + gamma (xhat - x0), 0 <= gamma <= 1; log_eps (NULL allowed) receives the
 * predicted log eps.  Continue with irls_mincut_solve_range(h, 1, ...) from
 * that eps.  Nothing crosses PCIe but the eps. */
irls_status irls_gnn_warm_start(irls_gnn_t g, irls_mincut_t h, const double *intensity, double gamma,
                                double *log_eps);

/* Loss and gradient for one graph: inputs as for irls_gnn_predict, targets y
 * (n doubles, entries of s and t ignored) and t = log_eps_target; lambda
 * weights the eps term.  The gradient stays on the device for
 * irls_gnn_adam_step; grad_out (count floats, host) may be NULL.
 * IRLS_ERR_RANGE if the graph has no non-terminal node. */
irls_status irls_gnn_loss_grad(irls_gnn_t g, irls_mincut_t h, const double *intensity,
                               const double *x_start, const double *y, double log_eps_target,
                               double lambda, double *loss, float *grad_out);

/* One Adam step with the last gradient (FP32 moments, bias-corrected). */
irls_status irls_gnn_adam_step(irls_gnn_t g, double lr, double beta1, double beta2, double eps);

/* Free the network and its device memory (NULL is a no-op). */
void irls_gnn_destroy(irls_gnn_t g);

/* Text of the last error of g, or of the calling thread's last failed
 * irls_gnn_create when g == NULL.  Valid until the next call on the same
 * network / thread. */
const char *irls_gnn_last_error(irls_gnn_t g);

#ifdef __cplusplus
}
#endif
#endif
