/*
 * ptyr_cnn.h - C ABI of the learned initial guess in libptyr: a small
 * convolutional net, trained and run on the gfx950 matrix cores in BF16 with
 * FP32 accumulation, that maps the diffraction patterns of a 3 x 3
 * neighbourhood of scan positions to the projected object phase of the
 * 32 x 32 pixel patch centred on the middle position.  Stitched patches give
 * an initial phase for the gradient reconstruction of ptyr.h, whose plain
 * initial object (unit amplitude, near-zero random phase; paper, Sec.
 * "Preprocessing and initialization") stays the fallback.  The paper has no
 * such network: its introduction names machine-learned direct solvers only as
 * related work.
 *
 * Network (cross-correlation, zero padding 1, ReLU after layers 0-3):
 *   a_0 = log(1 + max(I, 0))              9 x 64 x 64 (neighbourhood row-major)
 *   layer 0: 3x3,  9 -> 32, stride 1      32 x 64 x 64
 *   layer 1: 3x3, 32 -> 32, stride 2      32 x 32 x 32
 *   layer 2: 3x3, 32 -> 32, stride 1
 *   layer 3: 3x3, 32 -> 32, stride 1
 *   layer 4: 3x3, 32 ->  1, stride 1      out: 32 x 32 (no ReLU)
 *   loss = mean over the batch and the 32 x 32 pixels of (out - target)^2
 * Operands are rounded to BF16 where they are stored: the input a_0, the
 * weights, every hidden activation and every back-propagated gradient; sums
 * run in FP32; the output and the parameter gradients are FP32.
 *
 * Parameter vector (FP32, ptyr_cnn_param_count() floats): for each layer l in
 * order, W_l as Cout_p x K_p row-major with K_p = 32 * ceil(9 Cin_p / 32) and
 * reduction index k = (3 u + v) Cin_p + c for tap (u, v) (u along y) and input
 * channel c, then bias_l (Cout_p floats).  Cin_p = 16 for layer 0 (9 used),
 * else 32; Cout_p = 16 for layer 4 (1 used), else 32.  Padding entries must
 * be zero; their gradient is exactly zero, so Adam keeps them zero.
 *
 * Conventions follow ptyr.h: device pointers unless marked host, caller-owned
 * memory, the context's workspace as the only scratch, asynchronous calls on
 * the context's stream, gradients ACCUMULATED (+=) into caller-zeroed buffers,
 * argument errors returned before any launch, and index errors found by the
 * kernels reported by ptyr_cnn_sync() as PTYR_E_ARG.  Calls on one context
 * must not overlap (they share its workspace).
 */
#ifndef PTYR_CNN_H
#define PTYR_CNN_H

#include "ptyr.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PTYR_CNN_NB 9          /* patterns per neighbourhood */
#define PTYR_CNN_IN 64         /* pattern side (pixels) */
#define PTYR_CNN_OUT 32        /* phase patch side (pixels) */

typedef struct ptyr_cnn ptyr_cnn;

/* Pure host: floats in the packed parameter vector. */
size_t ptyr_cnn_param_count(void);

/* Pure host: bytes of device workspace for batches of up to B_max
 * neighbourhoods (B_max >= 1). */
size_t ptyr_cnn_workspace_bytes(int B_max);

/* Bind a context to a workspace (>= ptyr_cnn_workspace_bytes(B_max) bytes)
 * and a stream (hipStream_t as void*; NULL = default stream).  PTYR_E_ARG for
 * B_max < 1 or a null pointer, PTYR_E_NOMEM for a small workspace. */
ptyr_status ptyr_cnn_create(int B_max, void* workspace, size_t ws_bytes, void* stream, ptyr_cnn** out);
void ptyr_cnn_destroy(ptyr_cnn* ctx);

/* Wait for the stream; PTYR_E_ARG if a neighbourhood index was out of range
 * since the last sync (that pattern read as zeros), PTYR_E_DEVICE on a HIP
 * error.  Clears the flag. */
ptyr_status ptyr_cnn_sync(ptyr_cnn* ctx);

/* Network output.  patterns: n_pat x 64 x 64 fftshifted intensities (the
 * layout ptyr_forward writes and measured data use); nbr: B x 9 ints, the
 * patterns of each neighbourhood in row-major (dy, dx) order; out: B x 32 x 32
 * (overwritten).  1 <= B <= B_max. */
ptyr_status ptyr_cnn_forward(ptyr_cnn* ctx, const float* params, const float* patterns, int n_pat,
                             const int* nbr, int B, float* out);

/* Mean-squared-error loss against target (B x 32 x 32) and its gradient with
 * respect to the parameter vector: grad (param_count floats) += dL/dparams,
 * loss_dev (1 double) = loss (overwritten; may be NULL). */
ptyr_status ptyr_cnn_gradient(ptyr_cnn* ctx, const float* params, const float* patterns, int n_pat,
                              const int* nbr, const float* target, int B, float* grad, double* loss_dev);

/* One Adam step on the parameter vector (PyTorch's form): m, v are the
 * moment buffers (param_count floats each, zero before step 1); step is the
 * 1-based step number. */
ptyr_status ptyr_cnn_adam(ptyr_cnn* ctx, float* params, const float* grad, float* m, float* v, int64_t step,
                          float lr, float beta1, float beta2, float eps);

/* Stitch P network outputs (P x 32 x 32) into img (H x W, updated in place):
 * each pixel covered by at least one patch becomes the mean of the covering
 * patch values, a patch spanning rows round(cy) - 16 .. round(cy) + 15 and
 * columns likewise (round half to even); other pixels keep their value.
 * centres: P x 2 (y, x) floats in image pixels. */
ptyr_status ptyr_cnn_stitch(ptyr_cnn* ctx, const float* patches, const float* centres, int P, int H, int W,
                            float* img);

#ifdef __cplusplus
}
#endif

#endif /* PTYR_CNN_H */
