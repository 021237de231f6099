/*
 * ptyr.h - C ABI of libptyr, a gfx950 (MI355X) library for the hot path of
 * gradient-based multislice electron ptychography as described in the PtyRAD
 * paper (arXiv 2505.07814): the batched mixed-state multislice forward model,
 * its loss, its gradient with respect to all six optimisable parameters, and
 * an Adam step.
 *
 * What is computed (paper, Sec. "Physical model", Eq. 1-4; Sec. "Optimizers
 * and loss functions", Eq. 5-6; Sec. "AD-optimizable parameters"):
 *
 *   for every scan position j of a batch and every probe mode m
 *     r_j  = round_half_even(rho_j),  dr_j = rho_j - r_j,  t_j = r_j - N/2
 *     phi_0 = F^-1[ F[P_m] * exp(-2 pi i (q_y dr_y + q_x dr_x)) ]
 *     for s = 0 .. S-1:
 *        chi_s = O_s[t_j + (0..N-1)] * phi_s,        O_s = a_s exp(i phase_s)
 *        phi_{s+1} = F^-1[ H_j * F[chi_s] ]           (s < S-1)
 *     H_j(k) = exp(-i pi lambda |k|^2 dz + 2 pi i dz (k_x tan th_x + k_y tan th_y))
 *   I_j = fftshift( sum_m |F[chi_{S-1}]|^2 )
 *
 *   F is the orthonormal 2-D DFT (sign -1); q = fftfreq(N); k = q / dx.
 *   Axis 0 of every 2-D array is y; positions and tilts are (y, x) pairs;
 *   positions are in object pixels.  S slices use S-1 propagations.
 *
 * Memory conventions (all entry points):
 *  - Every array argument is a caller-owned, contiguous, row-major DEVICE
 *    pointer unless marked "host".  Complex values are interleaved (re, im)
 *    float32.  The library never allocates or frees caller memory: its scratch
 *    is the caller-provided workspace of ptyr_workspace_bytes() bytes.
 *  - All calls enqueue work on the context's HIP stream (a hipStream_t passed
 *    as void*) and return without synchronising.  Scalars computed on the
 *    device (loss) are written to device memory.
 *  - Gradient outputs ACCUMULATE (+=); the caller zeroes them.  Repeated calls
 *    on sub-batches therefore sum their gradients (gradient accumulation).
 *    Complex gradients follow dL/dRe + i dL/dIm.
 *
 * Errors: argument validation runs on the host before any launch and returns
 * a status without launching.  Positions live on the device, so a patch that
 * leaves the object is detected by the kernels, which then skip that position
 * (no out-of-bounds access) and raise PTYR_E_BOUNDS in a device flag that
 * ptyr_sync() reports.  Nothing aborts.
 */
#ifndef PTYR_H
#define PTYR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PTYR_OK = 0,
    PTYR_E_ARG = 1,          /* bad size, null pointer, unsupported N, B > B_max, zero data mean */
    PTYR_E_BOUNDS = 2,       /* a patch leaves the object */
    PTYR_E_NOMEM = 3,        /* workspace smaller than ptyr_workspace_bytes() */
    PTYR_E_DEVICE = 4,       /* a HIP call failed */
    PTYR_E_NONFINITE = 5     /* NaN/Inf met with PTYR_CHECK_FINITE set */
} ptyr_status;

enum { PTYR_LOSS_GAUSSIAN = 0, PTYR_LOSS_POISSON = 1 };

/* geometry flags */
#define PTYR_GLOBAL_TILT   0x1u  /* one (th_y, th_x) pair for all positions; its gradient is summed */
#define PTYR_CHECK_FINITE  0x2u  /* flag NaN/Inf in the loss sums as PTYR_E_NONFINITE */

/* adjoint flags */
#define PTYR_REUSE_FORWARD 0x1u  /* reuse the waves and intensities stored by the
                                    last ptyr_forward on this context (same inputs) */

typedef struct {
    int N;                    /* probe window / detector size: 64, 128 or 256 */
    int M;                    /* probe modes, >= 1 */
    int S;                    /* object slices, >= 1 */
    int H, W;                 /* object size in pixels, >= N */
    int B_max;                /* largest batch the context serves */
    double dx;                /* real-space pixel size, angstrom */
    double lambda;            /* electron wavelength, angstrom */
    int loss_kind;            /* PTYR_LOSS_GAUSSIAN (Eq. 5) or PTYR_LOSS_POISSON (Eq. 6) */
    double loss_p;            /* power p on both intensities (paper defaults 0.5 / 1) */
    size_t wave_budget_bytes; /* bytes of workspace the forward may keep per batch for
                                 the gradient; less than all S waves -> per-slice
                                 recomputation from checkpoints */
    unsigned flags;           /* PTYR_GLOBAL_TILT | PTYR_CHECK_FINITE */
    int n_scan;               /* scan positions ptyr_step may address (sizes its dense
                                 position / tilt gradients); 0 if ptyr_step is unused */
    double sparse_w;          /* weight of the sparsity term added to the loss of
                                 ptyr_adjoint / ptyr_step (Sec. "Optimizers and loss
                                 functions", L^p of the object phase with p = 1: the
                                 mean |phase| over the batch's N x N object patches,
                                 every slice); 0 = off (the paper's default when on: 0.1) */
    double pacbed_w;          /* weight of the PACBED term added to the loss of ptyr_loss,
                                 ptyr_adjoint and ptyr_step (Sec. "Optimizers and loss
                                 functions": RMS over the detector of <I_model>_B^p -
                                 <I_meas>_B^p over <I_meas^p>_{D,B}, the same p as the
                                 data term); 0 = off.  It couples the rows of a batch, so
                                 with it a batch runs on one stream */
    int n_obj;                /* object modes (Sec. "Physical model", mixed-state formalism,
                                 Eq. 2): amplitude and
                                 phase hold n_obj stacks of S x H x W, object mode o is
                                 transmitted with every probe mode and the model
                                 intensity sums over all M x n_obj pairs; 0 or 1 = one
                                 object, at most 64 */
    double w_gaussian;        /* weighted total loss (Sec. "Optimizers and loss functions",
                                 Eq. 9): w_1 of the Gaussian term (Eq. 5) ... */
    double w_poisson;         /* ... and w_2 of the Poisson term (Eq. 6), each with its own
                                 batch normaliser <I_meas^p>; both 0 = the loss_kind
                                 term alone at weight 1 (loss_kind is then ignored when
                                 either is set).  With both set the batch runs on one
                                 stream (the weights of each pixel need both terms'
                                 batch factors) */
    double p_gaussian, p_poisson; /* powers of the two terms when w_gaussian or w_poisson
                                 is set; 0 = the paper's defaults 0.5 and 1.  The PACBED
                                 term then takes the power of the first weighted term
                                 (Gaussian if w_gaussian > 0), else loss_p */
} ptyr_geom;

/* Parameters of one reconstruction and their Adam moments (all device). */
typedef struct {
    float *amp, *phase;       /* n_obj x S x H x W */
    float *probe;             /* M x N x N complex */
    float *pos;               /* n_pos x 2 (y, x) */
    float *tilt;              /* n_pos x 2, or 2 with PTYR_GLOBAL_TILT */
    float *dz;                /* 1 */
    float *m_amp, *v_amp, *m_phase, *v_phase, *m_probe, *v_probe;
    float *m_pos, *v_pos, *m_tilt, *v_tilt, *m_dz, *v_dz;
    int n_pos;                /* scan positions of the whole data set */
    int64_t step;             /* Adam updates taken so far; ptyr_step increments it */
} ptyr_params;

/* Per-parameter learning rates (0 freezes a parameter: its values and its
 * moments are left untouched, which realises an onset iteration on the host)
 * and the Adam constants. */
typedef struct {
    float amp, phase, probe, pos, tilt, dz;
    float beta1, beta2, eps;  /* 0.9, 0.999, 1e-8 reproduce PyTorch's defaults */
} ptyr_lr;

typedef struct ptyr_ctx ptyr_ctx;

/* Human-readable text for a status. */
const char* ptyr_status_str(ptyr_status s);

/* Pure host: validate a geometry (N in {64,128,256}, M,S,B_max >= 1,
 * H,W >= N, dx, lambda > 0, loss kind and p, non-negative finite weights,
 * B_max * M * n_obj <= 2^30, at most 2^40 object elements). */
ptyr_status ptyr_check_geom(const ptyr_geom* g);

/* Pure host: validate a batch size and, when pos_host is not NULL, that every
 * patch of the B host positions (B x 2, (y, x)) lies inside the object.
 * Rounding follows the kernels: round half to even, corner = round - N/2. */
ptyr_status ptyr_check_args(const ptyr_geom* g, int B, const float* pos_host);

/* Pure host: bytes of device workspace a context for g needs. */
size_t ptyr_workspace_bytes(const ptyr_geom* g);

/* Pure host: how the forward keeps waves for the gradient under
 * g->wave_budget_bytes, counted in N x N complex64 waves per (row, mode)
 * chain of a B_max batch.  *stride = 1: all 2S waves of a chain are kept
 * (incident wave and its spectrum per slice, far field; at N = 256 S + 1:
 * the wave entering each slice's row pass, far field).  Otherwise three
 * waves per chain are scratch for recomputation and the incident wave is
 * kept every *stride >= 2 slices; *stride = S+1: none is kept and the
 * gradient recomputes from the probe (O(S^2) slice steps). */
ptyr_status ptyr_checkpoint_plan(const ptyr_geom* g, int* stride);

/* Bind a context to a workspace (device, caller-owned, >= ptyr_workspace_bytes,
 * 256-byte aligned) and a stream (hipStream_t as void*; NULL = the default
 * stream), on the current device.  Besides pointers the context owns one
 * extra stream of default priority and seven events: a batch with more
 * (row, mode) chains than the device has compute units runs part of its
 * chains on that stream, joined back to the caller's stream before
 * ptyr_adjoint / ptyr_step return, so callers only ever order work against
 * their own stream.  PTYR_E_DEVICE if the stream or events cannot be made. */
ptyr_status ptyr_create(const ptyr_geom* g, void* workspace, size_t ws_bytes,
                        void* stream, ptyr_ctx** out);
/* Release the context, its stream and events (waits for the side stream's
 * work).  The context is freed in any case; PTYR_E_DEVICE reports that one of
 * the HIP releases failed. */
ptyr_status ptyr_destroy(ptyr_ctx* ctx);

/* Wait for the context's stream and report the first asynchronous error:
 * PTYR_E_BOUNDS / PTYR_E_NONFINITE raised by kernels since the last call, or
 * PTYR_E_DEVICE.  Clears the device flags. */
ptyr_status ptyr_sync(ptyr_ctx* ctx);

/* Forward model, Eq. 1-4 (a_s, phase_s: n_obj x S x H x W; probe: M x N x N complex;
 * pos: rows x 2; tilt: rows x 2 or 2 (global); dz: 1 float).  Writes the
 * fftshifted intensities I_out (B x N x N).  idx (nullable, B device ints)
 * selects rows idx[b] (0 <= idx[b] < n_rows) of pos/tilt for batch row b;
 * with idx NULL, row b is used and n_rows is ignored.  A row index outside
 * [0, n_rows) is skipped by the kernels and reported by ptyr_sync as
 * PTYR_E_ARG.  Keeps waves for a following ptyr_adjoint(PTYR_REUSE_FORWARD)
 * within wave_budget_bytes. */
ptyr_status ptyr_forward(ptyr_ctx* ctx, const float* amp, const float* phase,
                         const float* probe, const float* pos, const float* tilt,
                         const float* dz, const int* idx, int n_rows, int B,
                         float* I_out);

/* Loss of Eq. 5 (Gaussian) or Eq. 6 (Poisson, eps = 1e-6), or their weighted
 * sum of Eq. 9 (w_gaussian, w_poisson), between fftshifted model and measured
 * intensities (B x N x N each), averaged over detector and batch.  Writes the loss to loss_dev (1 double, overwritten) and, if dLdI is
 * not NULL, dL/dI_model (B x N x N, overwritten).  meas_idx (nullable, B
 * device ints) selects measured pattern meas_idx[b] of the n_meas patterns in
 * I_meas for batch row b. */
ptyr_status ptyr_loss(ptyr_ctx* ctx, const float* I_model, const float* I_meas,
                      const int* meas_idx, int n_meas, int B, double* loss_dev,
                      float* dLdI);

/* Allocation-free ptyr_loss, for callers that cannot allocate device memory
 * while they run (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same kernels and results as ptyr_loss
 * (bit for bit, same launch shapes), but no context: the loss geometry comes
 * from g (N, loss_kind / loss_p or the Eq. 9 weights, pacbed_w,
 * PTYR_CHECK_FINITE; the whole struct must pass ptyr_check_geom), the work
 * is enqueued on `stream` (hipStream_t as void*, NULL = default) of the
 * current device, and the loss passes' scratch (partial sums, batch scalars,
 * PACBED buffers: PTYR_NOALLOC_SCRATCH_BYTES) lives in a static device array
 * of the library, one per GPU, held until the process ends.  The call makes
 * no hipMalloc / hipFree and no allocating library call; the first call on a
 * device looks the array's address up (hipGetSymbolAddress).
 *  err_dev: one device int (required) that the kernels OR their error bits
 *    into (PTYR_ERRBIT_*: a measured-row index outside [0, n_meas), a zero
 *    data mean, NaN/Inf with PTYR_CHECK_FINITE); the caller clears it and
 *    reads it after synchronising the stream.
 *  Calls on one GPU share that GPU's scratch: calls that overlap in time
 *    (several streams or host threads) race and must be serialised by the
 *    caller.  The scratch is never read before the call writes it, so
 *    nothing needs clearing between calls.
 * Returns PTYR_E_ARG as ptyr_loss (and for err_dev NULL), PTYR_E_NOMEM if
 * the geometry needs more scratch than the array holds (not reachable with
 * N <= 256), PTYR_E_DEVICE if the array's address cannot be found. */
#define PTYR_NOALLOC_SCRATCH_BYTES ((5 * 512 + 8 + 2 * 256 * 256 + 64) * 8)
#define PTYR_ERRBIT_BOUNDS    0x1
#define PTYR_ERRBIT_NONFINITE 0x2
#define PTYR_ERRBIT_ZERO_MEAN 0x4
#define PTYR_ERRBIT_INDEX     0x8
ptyr_status ptyr_loss_noalloc(const ptyr_geom* g, const float* I_model, const float* I_meas,
                              const int* meas_idx, int n_meas, int B, double* loss_dev,
                              float* dLdI, int* err_dev, void* stream);

/* Loss and its gradient with respect to object amplitude and phase, probe,
 * positions, tilts and dz (chain rule through Eq. 1-6).  Runs the forward
 * itself unless flags has PTYR_REUSE_FORWARD.  idx (nullable, B device ints in
 * [0, n_rows)) selects rows of pos/tilt/I_meas and the rows of g_pos/g_tilt
 * that receive the gradient; the rows of one batch must be distinct (a row
 * met again later in the batch is skipped and reported by ptyr_sync as
 * PTYR_E_ARG: its gradient would otherwise race with the first one's).
 * Gradients accumulate (+=): g_amp, g_phase n_obj x S x H x W; g_probe M x N x N
 * complex; g_pos, g_tilt like pos, tilt; g_dz 1.  Any gradient pointer may be
 * NULL to skip it.  loss_dev (nullable) receives the batch loss. */
ptyr_status ptyr_adjoint(ptyr_ctx* ctx, const float* amp, const float* phase,
                         const float* probe, const float* pos, const float* tilt,
                         const float* dz, const int* idx, int n_rows, int B,
                         const float* I_meas, float* g_amp, float* g_phase,
                         float* g_probe, float* g_pos, float* g_tilt, float* g_dz,
                         double* loss_dev, unsigned flags);

/* One mini-batch update (Sec. "Optimizers and loss functions": Adam by
 * default, per-parameter learning rates): gradient of the batch idx (B
 * distinct device ints into the p->n_pos <= g->n_scan positions / patterns of
 * I_meas_all, n_pos x N x N), then a dense Adam update of every parameter
 * whose rate is non-zero (entries outside the batch see a zero gradient, as
 * in PyTorch), and p->step += 1.  loss_dev (nullable) receives the batch
 * loss.  Row indices outside [0, n_pos) and repeats of an earlier row of the
 * batch are skipped and reported by ptyr_sync as PTYR_E_ARG. */
ptyr_status ptyr_step(ptyr_ctx* ctx, ptyr_params* p, const int* idx, int B,
                      const float* I_meas_all, const ptyr_lr* lr, double* loss_dev);

/* Per-iteration constraints on the object and probe (Sec. "Physical
 * constraints"), applied by ptyr_constrain after a gradient step, in this
 * order:
 *  kz_beta > 0 or kz_alpha > 0: the k_z filter (Sec. "Fourier-space depth
 *    regularization"): the amplitude and the phase are each multiplied in
 *    3-D Fourier space by W_a(k) = (1 - (2/pi) atan(beta^2 k_z^2 /
 *    (k_x^2 + k_y^2 + 1e-3))) exp(-alpha (k_x^2 + k_y^2)), k in 1/angstrom
 *    from the geometry's dx and kz_dz (periodic in all three directions).
 *    S, H and W must have no prime factor other than 2, 3 and 5 and be at
 *    most 4096.
 *  rz_sigma > 0: the r_z filter (Sec. "Real-space depth regularization"): the
 *    amplitude and the phase are each convolved along the slice axis with a
 *    Gaussian of standard deviation rz_sigma slices, truncated at
 *    |k| <= ceil(4 rz_sigma) and normalised to sum 1; the stack is mirrored
 *    about its outer slice faces, so the first and last slices never mix.
 *    0 < rz_sigma <= 16, S <= 256.
 *  phase_positive: negative phase is set to 0 (Sec. "Positivity and
 *    sparsity").
 *  probe_orthogonal: the M probe modes are replaced by the eigenvectors of
 *    their overlap matrix A[m][n] = sum_r conj(P_m(r)) P_n(r), in order of
 *    decreasing power (after Thibault & Menzel 2013); each new mode's phase
 *    factor makes its largest mixing coefficient real and positive.  The
 *    incoherent sum of |P_m|^2, and so every model intensity, is unchanged.
 *    M <= 24. */
typedef struct {
    float rz_sigma;           /* r_z filter width in slices; 0 = off */
    int phase_positive;       /* clip negative object phase to 0 */
    int probe_orthogonal;     /* orthogonalise the probe modes */
    float kz_beta, kz_alpha;  /* k_z filter strength beta and lateral blur alpha
                                 (angstrom^2); both 0 = off */
    float kz_dz;              /* slice spacing for the k_z filter, angstrom */
} ptyr_constraints;

/* Apply the constraints in place on the context's stream: amp, phase
 * (n_obj x S x H x W; the filters act on each object mode's stack on its
 * own), probe (M x N x N complex); the pointer of a constraint that is
 * off may be NULL.  PTYR_E_ARG for rz_sigma outside [0, 16], S > 256 with the
 * r_z filter, M > 24 with probe_orthogonal, negative k_z parameters, kz_dz <= 0
 * or a side with another prime factor or longer than 4096 with the k_z filter,
 * or a needed NULL pointer. */
ptyr_status ptyr_constrain(ptyr_ctx* ctx, float* amp, float* phase, float* probe,
                           const ptyr_constraints* cfg);

/* Instrumentation (not part of the method): when enabled, the context brackets
 * each launch of its fused wave kernels with HIP events on its stream.
 * kernel ids: PTYR_K_FORWARD (the multislice forward kernel),
 * PTYR_K_GRADIENT (the gradient kernel) and PTYR_K_RZ (the r_z depth filter
 * in ptyr_constrain: one launch for amplitude and phase while S <= 32, one
 * per field beyond).  Enabling creates the events (no
 * device memory is allocated); at most 4096 launches are recorded between
 * reads, later ones are not timed. */
enum { PTYR_K_FORWARD = 0, PTYR_K_GRADIENT = 1, PTYR_K_RZ = 2 };
ptyr_status ptyr_timing_enable(ptyr_ctx* ctx, int on);
/* Synchronise the stream and write the summed kernel time in milliseconds and
 * the number of timed launches of kernel `which` since timing was last
 * enabled (ptyr_timing_enable clears the record).  PTYR_E_DEVICE if an event
 * could not be recorded since then (those launches are left out). */
ptyr_status ptyr_timing_read(ptyr_ctx* ctx, int which, double* total_ms, int* launches);

#ifdef __cplusplus
}
#endif
#endif /* PTYR_H */
