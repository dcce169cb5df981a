/*
 * ssn.h -- C ABI of the learned initialiser's network (BF16 MFMA, gfx950).
 *
 * A U-Net (Ronneberger, Fischer and Brox 2015) with `levels` resolution
 * levels and `base` channels at the top (doubling per level): per encoder
 * level two 3x3 convolutions with SiLU, kept as the skip, then 2x2 average
 * pooling; a bottleneck of two 3x3 convolutions; per decoder level a nearest
 * 2x upsampling, concatenation [upsampled, skip], two 3x3 convolutions with
 * SiLU; a 1x1 head to `cout` channels. Convolutions are zero-padded with bias.
 * It maps the vortex image of ss_learned_input (cin = 2) to the corrections
 * of ss_init_learned (cout = 4); it is not part of the paper's method but the
 * learned start of this project's minimisation workloads.
 *
 * Arithmetic: activations and weights BF16, products on v_mfma_f32_32x32x16_bf16
 * with FP32 accumulation; master weights, gradients and Adam moments FP32;
 * reductions in fixed order (a run is bitwise repeatable).
 *
 * Launch shape: a convolution runs as an LDS-tiled GEMM (input patch and
 * weights staged per 32 input channels) where image rows are at least 32
 * pixels wide and that gives at least 256 workgroups; otherwise its MFMA
 * operands are read directly, in workgroups of 4 waves (64 pixels per wave)
 * when that gives at least 1024 workgroups, else of one wave (32 pixels). The
 * environment variable SSN_CONV_SHAPE, read by ssn_create, forces one
 * (1: direct large, 2: direct small, 3: tiled where rows allow it).
 *
 * Memory: images are fp32 device arrays (n, H, W, channels) row-major. The
 * caller owns the workspace (ssn_workspace_bytes, 256-byte aligned) and all
 * device buffers; the library owns the host object. Work is queued on the
 * stream given to ssn_create; calls returning host data synchronise it.
 * Parameters are exchanged as one flat fp32 host array in the order: for
 * each 3x3 layer (encoder levels top-down, bottleneck, decoder levels
 * bottom-up, each level "a" then "b") weight [co][ky][kx][ci] then bias [co];
 * then the head weight [cout][base] and bias [cout].
 * Errors: 0 OK, negative codes of ss.h; ssn_last_error() gives the message.
 */
#ifndef SSN_H
#define SSN_H

#include <stddef.h>
#include <stdint.h>

#include "ss.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ssn_net ssn_net;

/* Number of parameters in the flat exchange order. */
long ssn_param_count(int levels, int base, int cin, int cout);
/* Workspace for batches of up to N images of H x W (H, W multiples of
 * 16 * 2^(levels-1); base a multiple of 16; cin <= 16; cout * base <= 256). */
int ssn_workspace_bytes(int levels, int base, int cin, int cout, int N, int H, int W, size_t* bytes);
int ssn_create(int levels, int base, int cin, int cout, int N, int H, int W, void* workspace, size_t ws_bytes,
               void* stream, ssn_net** out);
void ssn_destroy(ssn_net* net);
long ssn_num_params(ssn_net* net);
/* Set all parameters from a host array (also resets the Adam state); read them back. */
int ssn_set_weights(ssn_net* net, const float* host, long count);
int ssn_get_weights(ssn_net* net, float* host, long count);
/* Gradients of the last ssn_backward, same order. */
int ssn_get_grads(ssn_net* net, float* host, long count);
/* Forward pass of n <= N images x (n, H, W, cin); the output (n, H, W, cout)
 * is kept for ssn_backward and copied to out if out != NULL. */
int ssn_forward(ssn_net* net, const float* x, int n, float* out);
/* As ssn_forward (out required), but the forward pass is captured as a HIP
 * graph on the first call for a given (x, n, out) and replayed afterwards (one
 * launch instead of one per kernel); a call with other pointers or n captures
 * anew. The graph reads the weights at replay, so training between calls is
 * seen. For callers that repeat small forwards on fixed buffers. */
int ssn_forward_graph(ssn_net* net, const float* x, int n, float* out);
/* Gradients of the mean squared error between the last output and target
 * (n, H, W, cout); *loss (may be NULL) receives the loss (synchronises). */
int ssn_backward(ssn_net* net, const float* target, int n, double* loss);
/* One Adam step (Kingma and Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr. */
int ssn_adam_step(ssn_net* net, float lr);
/* Clip the gradient by its global L2 norm in every later ssn_adam_step: the
 * step uses g * min(1, max_norm / |g|), |g| summed in FP64 in a fixed order on
 * the device (no host synchronisation). max_norm = 0 (the default) turns it
 * off; negative or non-finite values return SS_EINVAL. */
int ssn_set_grad_clip(ssn_net* net, float max_norm);
/* forward + backward + Adam. */
int ssn_train_step(ssn_net* net, const float* x, const float* target, int n, float lr, double* loss);
/* Learned start in one call, for a network made with cin = 2, cout = 4 and
 * H = Ny, W = Nx of the Abelian Higgs context ctx: the input image of
 * ss_learned_input (nv centres xy, kappa) is written to work, the network's
 * forward pass maps it to corrections, and ss_init_learned (windings w, sigma,
 * pin, seed, noise_amp as documented there) sets the field from them; the flow
 * then starts from rest. The result equals those three calls made in turn.
 * work: device memory of at least ssn_init_field_workspace_bytes(net) bytes,
 * 256-byte aligned, owned by the caller. The network's last output is replaced.
 * SS_EINVAL for NULL pointers, a network of other channel counts, another
 * theory or a small or misaligned work; SS_ESHAPE if the network's image size
 * is not the lattice's. Synchronises the network's and the context's streams. */
size_t ssn_init_field_workspace_bytes(ssn_net* net);
int ssn_init_field(ssn_net* net, ss_ctx* ctx, int nv, const double* xy, const double* w, double kappa, double sigma,
                   double pin, uint64_t seed, double noise_amp, void* work, size_t work_bytes);
/* Read-back of the network's internal BF16 tensors (as floats, host array of
 * (n, H, W, C)) for inspection and per-layer checks: for 3x3 layer `layer` (the
 * order of the parameter exchange; 0 .. 4 levels - 1),
 *   SSN_T_INPUT        its input (for a decoder "a" layer the concatenation
 *                      [upsampled, skip]; for layer 0 the BF16 image, its
 *                      channels padded with zeros to 16),
 *   SSN_T_PREACT       its pre-activation z = conv + bias (rounded to BF16),
 *   SSN_T_OUTPUT       its output SiLU(z) (rounded from the FP32 z),
 *   SSN_T_GRAD_PREACT  the loss gradient at z, and
 *   SSN_T_GRAD_DATA    what its backward-data pass wrote: for an "a" layer the
 *                      gradient at its input (none for layer 0), for a "b" layer
 *                      the gradient at the "a" layer's z (the product with
 *                      SiLU'(z_a) is fused),
 * as the last ssn_forward / ssn_backward left them. ssn_tensor_shape gives
 * H, W, C of a tensor. count must be n * H * W * C. Synchronises. */
#define SSN_T_INPUT 0
#define SSN_T_PREACT 1
#define SSN_T_OUTPUT 2
#define SSN_T_GRAD_PREACT 3
#define SSN_T_GRAD_DATA 4
int ssn_tensor_shape(ssn_net* net, int kind, int layer, int* H, int* W, int* C);
int ssn_read_tensor(ssn_net* net, int kind, int layer, int n, float* host, long count);

/* Multiply-add flops (2 per MAC) of one image's forward and backward passes. */
int ssn_flops(ssn_net* net, double* fwd, double* bwd);
const char* ssn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SSN_H */
