/*
 * bec_mlp.h -- C ABI of the learned initial guess: a dense network that maps the physical
 * parameters of a problem to a coarse complex field, trained on ground states computed by the
 * PCG-ATKM solver (Algorithm 1) of the same library.
 *
 * The paper starts Algorithm 1 from analytic guesses (Sec. 3, initial data (a)-(f)) or from a
 * coarser-grid ground state interpolated to the fine grid (Algorithm 2, cascadic multigrid).
 * The network is a third source of initial data for Algorithm 1: its coarse output goes
 * through the same spectral interpolation (bec_interp_spectral in bec.h) to the target grid,
 * and the solver, not the network, decides the final ground state.
 *
 * Network (all matrices row-major [out][in]):
 *   h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  y = W3 h2 + b3.
 * Precision: weights are used as BF16 copies (round-to-nearest-even of the FP32 master
 * weights); the inputs of the two large layers (h1, h2) and, in the backward pass, the output
 * and hidden-layer gradients are rounded to BF16 as matrix-core operands; every product is
 * accumulated in FP32; biases, x, y and the first layer (d_in inputs) stay FP32; Adam updates
 * the FP32 master weights. Loss: mean squared error over all batch x d_out outputs.
 *
 * Ownership: the caller owns every buffer (device memory) named in bec_mlp and the scratch
 * buffer; the library allocates nothing. Streams: every call enqueues on `stream`
 * (hipStream_t, NULL = default stream) and returns without synchronising.
 * Errors: BEC_EINVAL for a NULL pointer, a dimension that is not a positive multiple of 8
 * (d_h, d_out; d_in only needs to be positive), batch < 1 or a scratch buffer that is too
 * small (BEC_ENOMEM); BEC_EHIP for a failed launch. Status codes are those of bec.h.
 */
#ifndef BEC_MLP_H
#define BEC_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t d_in, d_h, d_out;
    /* FP32 master parameters, packed: W1[d_h][d_in] b1[d_h] W2[d_h][d_h] b2[d_h]
     * W3[d_out][d_h] b3[d_out]; bec_mlp_param_count elements. */
    float* params;
    uint16_t* params_bf16;  /* BF16 bit patterns of params, same packing (written by sync / Adam) */
    uint16_t* w2t_bf16;     /* BF16 W2 transposed, [d_h][d_h] (in-major) */
    uint16_t* w3t_bf16;     /* BF16 W3 transposed, [d_h][d_out] */
    float* grads;           /* gradient of the loss, same packing as params */
    float* adam_m;          /* Adam first and second moments, same packing */
    float* adam_v;
} bec_mlp;

/* Thread-local message of the last failing bec_mlp_* / bec_gemm_* call. */
const char* bec_mlp_last_error(void);

/* Number of parameters of the packed vector (0 for a non-positive dimension). */
size_t bec_mlp_param_count(int d_in, int d_h, int d_out);

/* Scratch bytes needed by bec_mlp_forward / bec_mlp_loss_grad for `batch` samples. */
int bec_mlp_scratch_bytes(const bec_mlp* net, int batch, size_t* bytes);

/* Refresh params_bf16, w2t_bf16 and w3t_bf16 from params (after the caller wrote params). */
int bec_mlp_sync(const bec_mlp* net, void* stream);

/* y[b][:] = network(x[idx[b]][:]) for b < batch; x is FP32 [*][d_in], y FP32 [batch][d_out].
 * d_idx (int32, nullable) selects the input rows; NULL means rows 0..batch-1. */
int bec_mlp_forward(const bec_mlp* net, int batch, const float* d_x, const int32_t* d_idx, float* d_y,
                    void* d_scratch, size_t scratch_bytes, void* stream);

/* Forward pass, loss = mean over batch x d_out of (y - target[idx[b]])^2, and its gradient
 * with respect to every parameter, written (not accumulated) to net->grads. d_loss: one
 * double on the device. d_y (nullable) receives the network output. */
int bec_mlp_loss_grad(const bec_mlp* net, int batch, const float* d_x, const float* d_target,
                      const int32_t* d_idx, float* d_y, double* d_loss, void* d_scratch,
                      size_t scratch_bytes, void* stream);

/* One Adam step (Kingma and Ba, Algorithm 1 of "Adam: a method for stochastic optimization"):
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 * on every parameter, t >= 1 the step number; then refreshes the BF16 copies. */
int bec_mlp_adam_step(const bec_mlp* net, double lr, double beta1, double beta2, double eps, int32_t t,
                      void* stream);

/* Matrix-core GEMM used by the network, exposed for testing and reuse:
 *   C[m][n] = sum_k A[m][k] B[n][k] (+ bias[n])   for m < M, n < N
 * A: BF16 [M][lda], B: BF16 [N][ldb] (both K-contiguous), C: FP32 [M][ldc]. K, lda, ldb must
 * be multiples of 8 and the pointers 16-byte aligned. With splits > 1 the K range is cut into
 * at most `splits` parts, each a multiple of 64 long (the kernel's K step); their partial
 * products go to d_part (FP32, splits*M*N) and are summed in a fixed order. d_part may be NULL
 * when that leaves a single part (always when splits == 1). bias may be NULL. */
int bec_gemm_bf16_nt(int M, int N, int K, const uint16_t* d_A, int lda, const uint16_t* d_B, int ldb,
                     float* d_C, int ldc, const float* d_bias, int splits, float* d_part, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* BEC_MLP_H */
