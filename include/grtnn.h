/*
 * grtnn.h -- C ABI of the learned warm start of the constraint solver.
 *
 * The paper starts the constraint solve from psi = 1 (u = 0), W = 0.  This
 * library adds a small 3D convolutional network that maps the sources
 * (rho5 + rho1, S_x, S_y, S_z) of a periodic problem to a starting state
 * (u, W_x, W_y, W_z); the multigrid solve (grtmg.h) always finishes the job
 * and judges the result, and a prediction that is not better than the zero
 * start is discarded.  The network is trained on solves that the method
 * itself produces, with the forward and backward kernels of this library.
 *
 * Network (a U-Net; every convolution is 3x3x3 with circular padding):
 *   encoder level l = 0..levels-1: [pool 2x2x2 average if l > 0], conv, SiLU,
 *     conv, SiLU -> e_l  (widths ch[l]);
 *   decoder level l = levels-2..0: trilinear x2 upsampling of the level below
 *     (cell-centred, weights 3/4 and 1/4 per axis), concatenation
 *     [e_l, upsampled], conv, SiLU, conv, SiLU -> d_l (d_{levels-1} = e_{levels-1});
 *   head: conv (no activation) to c_out channels.
 * SiLU(z) = z / (1 + exp(-z)).  A convolution computes
 *   y[co](p) = b[co] + sum_ci sum_{d in {-1,0,1}^3} W[co][ci][d+1] x[ci](p+d),
 * indices taken modulo n.
 *
 * Parameters: one FP32 array; for every convolution in the order enc0a,
 * enc0b, enc1a, enc1b, ..., dec(levels-2)a, dec(levels-2)b, ..., dec0a, dec0b,
 * head: W[co][ci][kx][ky][kz] (kx = dx+1) followed by b[co].
 *
 * Arithmetic: BF16 weights and activations (round to nearest even), FP32
 * accumulation on the matrix cores, FP32 master weights, gradients and Adam
 * moments.  Activations are stored channels-last: element c of cell
 * (i,j,k) of a C-channel tensor is at ((i*n + j)*n + k)*C + c.  BF16 values
 * cross the ABI as uint16_t bit patterns.
 *
 * Conventions: d_ pointers are device pointers, h_ host pointers; the caller
 * owns every array and the workspace (the library only carves it); all work
 * is enqueued on the stream given at setup (void* hipStream_t, NULL = default)
 * and calls returning host values wait for it.  Statuses are those of
 * grtmg.h; arguments are checked before any HIP call.
 */
#ifndef GRTNN_H
#define GRTNN_H

#include <stddef.h>
#include <stdint.h>

#include "grtmg.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Network shape.
 *  n       cells per axis of the (periodic, cubic) grid; n divisible by
 *          2^(levels-1), n >> (levels-1) >= 2.
 *  levels  1..4.
 *  ch      channel widths per level, each a multiple of 16 in 16..128.
 *  c_in    input channels, 1..8 (stored padded to 8).
 *  c_out   output channels, 1..16.
 */
typedef struct nn_config {
    int32_t n;
    int32_t levels;
    int32_t ch[4];
    int32_t c_in;
    int32_t c_out;
} nn_config;

typedef struct nn_ctx nn_ctx;

/* Standardisation of the fields (mean and standard deviation per channel):
 * input channels (rho5 + rho1, S_x, S_y, S_z), output channels (u, W_x, W_y, W_z). */
typedef struct nn_norm {
    double in_mean[4], in_std[4];
    double out_mean[4], out_std[4];
} nn_norm;

/* Number of FP32 parameters of the network. */
mg_status nn_param_count(const nn_config *cfg, int64_t *count);

/* Workspace bytes for inference (training = 0) or training (training = 1). */
mg_status nn_workspace_size(const nn_config *cfg, int32_t training, size_t *bytes);

/* Create a context on a 256-byte aligned workspace of at least
 * nn_workspace_size bytes.  The weights are undefined until nn_load_params. */
mg_status nn_setup(const nn_config *cfg, int32_t training, void *d_workspace, size_t bytes,
                   void *stream, nn_ctx **out);

/* Round the FP32 parameters (layout above) to the BF16 working copies used
 * by the forward and backward kernels. */
mg_status nn_load_params(nn_ctx *ctx, const float *d_params);

/* Forward pass.  d_in: BF16 [n^3][8] standardised input (channels >= c_in
 * zero); d_out: FP32 [n^3][c_out].  The pre-activations stay in the
 * workspace for nn_backward, which also reads d_in again: keep it unchanged
 * until then. */
mg_status nn_forward(nn_ctx *ctx, const uint16_t *d_in, float *d_out);

/* Mean squared error of d_out (FP32 [n^3][c_out]) against d_target (BF16
 * [n^3][c_out]) over all values; writes the loss gradient for nn_backward
 * into the context and the loss to *h_loss (host; waits for the stream). */
mg_status nn_mse(nn_ctx *ctx, const float *d_out, const uint16_t *d_target, double *h_loss);

/* Backward pass of the last nn_forward (training contexts) for the loss
 * gradient left by nn_mse: adds dLoss/dparams to d_grad (FP32, parameter
 * layout above). */
mg_status nn_backward(nn_ctx *ctx, float *d_grad);

/* Adam step on the FP32 master parameters (bias-corrected, step >= 1):
 *   g = grad_scale * d_grad; m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 *   p -= lr * (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps)
 * then refreshes the BF16 working copies (as nn_load_params). */
mg_status nn_adam_step(nn_ctx *ctx, float *d_params, const float *d_grad, float *d_m, float *d_v,
                       int32_t step, double lr, double beta1, double beta2, double eps,
                       double grad_scale);

/* Standardised BF16 input [n^3][8] from the FP64 sources of grtmg.h
 * (rho5, rho1: n^3; S: 3 n^3, SoA). */
mg_status nn_pack_input(nn_ctx *ctx, const double *d_rho5, const double *d_rho1, const double *d_S,
                        const nn_norm *norm, uint16_t *d_in);

/* Standardised BF16 target [n^3][4] from an FP64 state (u: n^3, W: 3 n^3). */
mg_status nn_pack_target(nn_ctx *ctx, const double *d_u, const double *d_W, const nn_norm *norm,
                         uint16_t *d_target);

/* FP64 state (u, W; SoA) from the FP32 network output [n^3][4]. */
mg_status nn_unpack_output(nn_ctx *ctx, const float *d_out, const nn_norm *norm, double *d_u,
                           double *d_W);

/* Sum and sum of squares of v = x + y over count FP64 values (d_y may be
 * null: v = x), for the standardisation statistics; h_out[0] = sum of v,
 * h_out[1] = sum of v^2; waits. */
mg_status nn_moments(nn_ctx *ctx, const double *d_x, const double *d_y, int64_t count, double h_out[2]);

/* Warm start of a constraint solve: predicts (u, W) from the sources into
 * d_u, d_W, applies one outer iteration of the solver to it (as one outer
 * iteration of mg_solve_constraints: the smoother removes the BF16-level
 * roughness of the prediction at once), and
 * keeps the result (*h_used = 1) only if its RMS constraint residuals are
 * finite and their maximum is below that of the zero state u = 0, W = 0;
 * otherwise d_u and d_W are set to zero (*h_used = 0).  The solver context
 * must have the network's grid (n cells per axis), periodic boundaries and
 * the coupled momentum solve, and must have been set up on the network's
 * stream; otherwise MG_ERR_INVALID is returned before any work is queued.
 * h_norms (may be NULL): RMS H, M after the iteration; RMS H, M of the zero state. */
mg_status nn_warm_start(nn_ctx *ctx, mg_ctx *solver, const double *d_rho5, const double *d_rho1,
                        const double *d_S, const nn_norm *norm, double *d_u, double *d_W,
                        int32_t *h_used, double h_norms[4]);

/*
 * The same with the fallback comparing like with like: the prediction is kept only
 * if, after its check iteration, max(rms H, rms M) is below keep_ratio (0 < keep_ratio
 * <= 1) times that of the zero state, where the caller passes for keep_ratio the
 * contraction of one outer iteration from the zero start on this workload (measured
 * once, e.g. with mg_solve_constraints at max_outer = 1).  A kept prediction then
 * leaves a state at least as good as one zero-start iteration would.  keep_ratio = 1
 * is nn_warm_start.  MG_ERR_INVALID for keep_ratio outside (0, 1]; otherwise as
 * nn_warm_start.
 */
mg_status nn_warm_start_ratio(nn_ctx *ctx, mg_ctx *solver, const double *d_rho5, const double *d_rho1,
                              const double *d_S, const nn_norm *norm, double *d_u, double *d_W,
                              double keep_ratio, int32_t *h_used, double h_norms[4]);

void nn_destroy(nn_ctx *ctx);

/*
 * Single-operation entry points (parity tests of the kernels).  Weights in
 * the parameter layout (FP32 W[co][ci][27], b[co]); activations channels-last
 * BF16 with the channel counts given (multiples of 8); d_scratch: device
 * scratch of at least nn_op_scratch_bytes(cin, cout, n) bytes.
 *  nn_conv3_forward:  y = conv(act ? SiLU(x) : x) + b, FP32 out [n^3][cout].
 *  nn_conv3_backward_data: dx[ci] = sum_co sum_d W[co][ci][d] dy[co](p - d),
 *                     FP32 out [n^3][cin] (dy BF16 [n^3][cout8], cout8 = cout
 *                     rounded up to 8).
 *  nn_conv3_backward_weight: dW[co][ci][d] = sum_p dy[co](p) a[ci](p + d),
 *                     db[co] = sum_p dy[co](p), a = act ? SiLU(x) : x; FP32
 *                     outputs overwritten.
 */
size_t nn_op_scratch_bytes(int32_t cin, int32_t cout, int32_t n);
mg_status nn_conv3_forward(int32_t n, int32_t cin, int32_t cout, const uint16_t *d_x, int32_t act,
                           const float *d_w, const float *d_b, float *d_y, void *d_scratch,
                           size_t scratch_bytes, void *stream);
mg_status nn_conv3_backward_data(int32_t n, int32_t cin, int32_t cout, const uint16_t *d_dy,
                                 const float *d_w, float *d_dx, void *d_scratch, size_t scratch_bytes,
                                 void *stream);
mg_status nn_conv3_backward_weight(int32_t n, int32_t cin, int32_t cout, const uint16_t *d_x,
                                   int32_t act, const uint16_t *d_dy, float *d_dw, float *d_db,
                                   void *d_scratch, size_t scratch_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GRTNN_H */
