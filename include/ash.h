/*
 * ash.h -- C ABI of the aberration-space holography hot path on MI355X.
 *
 * The library computes, for N target spots with per-spot kernel
 * coefficients w[n][d] over a basis {Z_d} of D pupil functions,
 *
 *   kernel phase  theta_n(x) = sum_d w[n][d] Z_d(xh, yh)           (radians)
 *   forward       E_n  = sum_x f(x) exp(-i theta_n(x))
 *   adjoint       g(x) = sum_n y_n exp(+i theta_n(x))
 *
 * over every SLM pixel x = (i, j) (i = column, the fastest index), which is
 * the compressed spot-holography transform pair with generalised "Zernike
 * kernels" (paper: "Aberration-Space Holography", compressed-sum equations
 * and modal-expansion paragraph), with kernels generated on the fly from a
 * monomial expansion of the basis and the N x D coefficient matrix
 * (paper: Methods, "Computational Scaling").  A weighted Gerchberg-Saxton
 * loop runs both transforms on the device ("A Full-Field 2D Tweezer Array",
 * WGS paragraph).
 *
 * Conventions
 *   - Normalised pupil coordinates xh = (i - cx)/R, yh = (j - cy)/R.
 *   - Transforms are unnormalised; the adjoint is the exact conjugate
 *     transpose of the forward.  With the orthonormal Zernike tilts
 *     Z_2 = 2 xh and Z_1 = 2 yh, integer-bin tilts w = pi u R / nx reproduce
 *     numpy's fft2 bins up to the factor exp(2 pi i (u cx/nx + v cy/ny)).
 *   - Complex arrays are interleaved (re, im) float pairs (torch complex64).
 *   - Pixel arrays are row-major [ny][nx] float32 (phase, amplitude) or
 *     [ny][nx][2] (complex field).
 *   - Arithmetic: phases in turns, range-reduced before the hardware
 *     sine/cosine.  Per-spot constant and tilt terms are wrapped per pixel
 *     tile in FP64 when spots are set, and the basis is evaluated in FP64
 *     as a small remainder about each tile anchor.  The in-tile phase is a
 *     dot product evaluated on the matrix cores from exact bf16 pieces of
 *     these FP64/FP32 values with FP32 accumulation (see
 *     ash_set_precision); magnitudes and sums are FP32, with compensated
 *     reductions across the SLM.  Results are bitwise deterministic for
 *     fixed inputs.
 *
 * Ownership and threading
 *   - Every *_dev pointer is a device pointer owned by the caller, on the
 *     context's device, contiguous, and must stay valid until the enqueued
 *     work that uses it has finished.  *_host arrays are read before the
 *     call returns.
 *   - The library owns the context and all scratch memory.  Scratch is
 *     allocated only by ash_set_basis / ash_set_spots (and the batch's
 *     create / tune / load_tuning calls), never by a single-context compute
 *     call (transforms, WGS, gradients, Adam, moments, window quality).
 *   - Compute calls are asynchronous on the context's stream.  A context is
 *     not thread-safe: use one context per host thread / stream.
 *   - The single-context compute calls (transforms, WGS iterations, the
 *     gradients and the Adam descent) neither synchronise, nor record
 *     memsets, nor allocate, so a caller can capture them in a HIP graph
 *     and replay it.
 *     The batched calls synchronise once per call and cannot be captured.
 *
 * Errors
 *   Every call returns ASH_OK (0) or a negative ASH_E* code.  Argument
 *   errors are detected before any work is enqueued and leave the context
 *   unchanged.  HIP runtime errors return ASH_EHIP with the runtime's
 *   message in ash_last_error().  The library never aborts or prints.
 */
#ifndef ASH_H
#define ASH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASH_OK 0
#define ASH_EINVAL (-1)       /* null / negative / non-finite argument     */
#define ASH_ESHAPE (-2)       /* sizes inconsistent with the context       */
#define ASH_ENOTREADY (-3)    /* basis or spots not set yet                */
#define ASH_EUNSUPPORTED (-4) /* outside the supported limits below        */
#define ASH_ENOMEM (-5)       /* device or host allocation failed          */
#define ASH_EHIP (-6)         /* HIP runtime error (see ash_last_error)    */

#define ASH_MAX_MODES 32       /* D                                          */
#define ASH_MAX_NONLINEAR 28   /* modes with a term of total degree >= 2     */
#define ASH_MAX_MONOMIALS 128  /* n_mono                                     */
#define ASH_MAX_DEGREE 12      /* p + q of any monomial x^p y^q              */
#define ASH_MAX_SIDE 65536     /* nx, ny                                     */
#define ASH_MAX_SPOTS 1048576  /* N                                          */
#define ASH_MAX_PRINCIPAL_MODES 66 /* D of ash_principal_modes' input          */

typedef struct ash_ctx ash_ctx;

/* Weighted-GS parameters (the paper cites weighted GS, with its
 * phase-fixed variant, without a formula; the reading implemented is, per
 * iteration:
 *   a_k = |E_k|,  r_k = (a_k/||a||) / (t_k/||t||),
 *   W_k <- W_k r_k^(-power) where a_k > 0, then W <- W / mean(W),
 *   y_k = W_k t_k exp(i psi_k),  psi_k = arg E_k (0 where E_k = 0),
 *   phi <- arg(F_c^{-1} y)   with arg(0) = 0.
 * Phase fixing freezes psi_k at the phases of one iteration; experimental
 * feedback (ash_wgs_feedback) takes a_k from measurements.)                */
typedef struct ash_wgs_params {
  float power; /* weight exponent p; 1 = classic WGS, 0 = plain GS         */
  /* 0: psi = arg E every iteration.  n > 0: iterations 0 .. n-1 of the
   * call are free and the psi of iteration n-1 are stored in the context;
   * iterations n .. use the stored psi.  n < 0: every iteration uses the
   * psi stored by an earlier call (ASH_ENOTREADY if none since the last
   * ash_set_spots).                                                        */
  int32_t fix_phase_after;
} ash_wgs_params;

/* Library version (major*10000 + minor*100 + patch). */
int ash_version(void);

/* Human-readable text for a status code (static storage). */
const char* ash_strerror(int code);

/* Detail of the last error on ctx (static per context; "" if none). */
const char* ash_last_error(const ash_ctx* ctx);

/* Failure injection, for tests of the error paths (process-wide):
 *   ASH_INJECT_ALLOC    the next `count` device allocations made by any
 *                       context or batch fail as if the device were out of
 *                       memory: the call returns ASH_ENOMEM and leaves the
 *                       object valid (what it was setting up is unset, and
 *                       repeating the call succeeds);
 *   ASH_INJECT_BARRIER  the next `count` one-launch batch calls start with
 *                       their barrier error flag set: every barrier gives
 *                       up at once, nothing waits, and the call returns
 *                       ASH_EHIP as for a barrier past its time limit.
 * count 0 disarms.  Returns ASH_OK or ASH_EINVAL (unknown `what`, count
 * < 0). */
#define ASH_INJECT_ALLOC 1
#define ASH_INJECT_BARRIER 2
int ash_inject_failure(int what, int count);

/* Create a context on HIP device `device`, enqueueing on `stream` (a
 * hipStream_t, NULL = the device's null stream).  *out receives the handle. */
int ash_create(ash_ctx** out, int device, void* stream);

/* Release the context and its device memory (synchronises its stream). */
int ash_destroy(ash_ctx* ctx);

/* Change the stream later calls enqueue on. */
int ash_set_stream(ash_ctx* ctx, void* stream);

/* Block until all work enqueued by ctx has finished. */
int ash_sync(ash_ctx* ctx);

/* Expand the orthonormal Zernike polynomial with ANSI index `ansi` into
 * monomials: Z(xh, yh) = sum_k coef_out[k] xh^pow_out[2k] yh^pow_out[2k+1].
 * Host-only, no device needed.  Writes at most `cap` terms; returns the
 * number of terms (>= 0) or a negative code (ASH_EINVAL for ansi < 0 or
 * null outputs, ASH_EUNSUPPORTED if the radial order exceeds
 * ASH_MAX_DEGREE or the expansion needs more than cap terms).
 * Paper: the modal-expansion paragraph (ANSI indexing) and Methods,
 * "Computational Scaling" (basis given by monomial coefficients). */
int ash_zernike_monomials(int ansi, int cap, int32_t* pow_out,
                          double* coef_out);

/* Principal isoplanatic modes (paper: Methods, "Anisoplanatic Singular
 * Value Decomposition"; the modal-expansion paragraph of "Computational
 * Scaling" notes that such a basis lowers D).  Host-only: touches no
 * context or device memory.
 *   N, D, n_mono, mono_pow, mono_coef  a basis as for ash_set_basis and
 *              w (host [N][D] float64) the spots' coefficients on it.
 *   K          principal modes to keep, 0 .. n_rot, where the n_rot rotated
 *              modes are those with a non-zero term of total degree >= 2;
 *              the others (piston, tilts: constant and position of each
 *              spot) are kept unchanged and come first, in their order.
 * With W_R = U S V^T the SVD of the rotated modes' coefficients (singular
 * values descending; each singular vector's largest entry positive), the
 * new basis is [kept modes, B_1 .. B_K], B_j = sum_i V[i][j] Z_rot[i], and
 * the new coefficients are [w_kept, W_R V_K]: the kernel phases change by
 * replacing W_R with its best rank-K approximation W_R V_K V_K^T.
 * Outputs (host, caller-allocated):
 *   D_out      number of output modes, n_keep + K.
 *   sigma      [n_rot] singular values of W_R, descending (n_rot <= D).
 *   mono_out   [D_out][n_mono] monomial coefficients of the new basis
 *              (same mono_pow), contiguous with row stride n_mono.
 *   w_out      [N][D_out] new coefficients, contiguous with row stride
 *              D_out (a [N][D] buffer is large enough).
 * Pass mono_out / w_out to ash_set_basis / ash_set_spots.  The input may
 * hold up to ASH_MAX_PRINCIPAL_MODES modes (the paper's 44-mode
 * calibration, say): only the output, n_keep + K modes, has to fit the
 * transforms' ASH_MAX_MODES / ASH_MAX_NONLINEAR.  Errors: ASH_EINVAL (sizes
 * < 1, null pointers, non-finite values, negative exponents, K outside
 * 0 .. n_rot), ASH_EUNSUPPORTED (D above ASH_MAX_PRINCIPAL_MODES, n_mono
 * above ASH_MAX_MONOMIALS, N above ASH_MAX_SPOTS). */
int ash_principal_modes(int N, int D, int n_mono, const int32_t* mono_pow,
                        const double* mono_coef, const double* w, int K,
                        int* D_out, double* sigma, double* mono_out,
                        double* w_out);

/* Checks of the ash_set_basis / ash_set_spots arguments without a context
 * or device (host-only code, also built without HIP): the code, and in
 * *detail (static storage, may be NULL) the message, that those calls
 * return for the same arguments before they touch the device (the source
 * amplitude, read from the device, and the spots' phase bound, computed
 * there, are checked by the calls themselves).  ASH_OK, ASH_EINVAL or
 * ASH_EUNSUPPORTED. */
int ash_check_basis(int nx, int ny, double cx, double cy, double R, int D,
                    int n_mono, const int32_t* mono_pow,
                    const double* mono_coef, const char** detail);
int ash_check_spots(int N, int D, const double* w, const float* target,
                    const char** detail);

/* Define the SLM and the basis.
 *   nx, ny     SLM size in pixels (1 .. ASH_MAX_SIDE).
 *   cx, cy, R  pupil centre (pixels) and unit radius (pixels, > 0).
 *   D          number of basis modes (1 .. ASH_MAX_MODES).
 *   n_mono     number of distinct monomials (1 .. ASH_MAX_MONOMIALS).
 *   mono_pow   host [n_mono][2] int32 exponents (p, q) of xh^p yh^q,
 *              p, q >= 0, p + q <= ASH_MAX_DEGREE.
 *   mono_coef  host [D][n_mono] float64: Z_d = sum_k mono_coef[d][k] mono_k.
 *   amp_dev    device [ny][nx] float32 source amplitude A(x) >= 0 (copied
 *              into the context), or NULL for A = 1.
 * Replaces any previous basis; clears the spots (call ash_set_spots again).
 * Paper: Methods, "Computational Scaling" (Z_d as a monomial sum evaluated
 * per pixel) and the source amplitude measured in "A Full-Field 2D
 * Tweezer Array".  Errors: ASH_EINVAL, ASH_EUNSUPPORTED, ASH_ENOMEM,
 * ASH_EHIP. */
int ash_set_basis(ash_ctx* ctx, int nx, int ny, double cx, double cy,
                  double R, int D, int n_mono, const int32_t* mono_pow,
                  const double* mono_coef, const float* amp_dev);

/* Set the N spots.
 *   w_host       host [N][D] float64 kernel coefficients in radians (the
 *                aberration-space coordinates w_d^(n) of each spot).
 *   target_host  host [N] float32 target amplitudes t_n > 0, or NULL for 1.
 * May be called between iterations without touching pixel data (paper:
 * Methods, "Computational Scaling", agile spot updates).  Runs an FP64
 * device kernel that wraps each spot's constant and tilt terms per pixel
 * tile and bounds the phase each kernel spans inside a 32 x 16 pixel tile
 * (ash_info.theta_bound, turns).  Spots whose bound exceeds 256 turns are
 * refused with ASH_EUNSUPPORTED: such kernels change by several turns
 * between neighbouring pixels (aliased many times over), and the FP32
 * accumulation of the in-tile phase would miss 1e-4 relative on the fields.
 * After that refusal the context has no spots, and ash_get_info reports the
 * refused spots' bounds.  Errors: ASH_ENOTREADY (no basis), ASH_EINVAL
 * (N < 1, null w, non-finite values, t <= 0), ASH_EUNSUPPORTED (N above
 * ASH_MAX_SPOTS, phase bound above 256 turns, record too long),
 * ASH_ENOMEM, ASH_EHIP. */
int ash_set_spots(ash_ctx* ctx, int N, const double* w_host,
                  const float* target_host);

/* Forward transform E_n = sum_x f(x) exp(-i theta_n(x)).
 * Exactly one input is non-NULL:
 *   phase_dev  device [ny][nx] float32 phase; f = A exp(i phase), or
 *   field_dev  device [ny][nx][2] float32 complex nearfield f (A unused).
 *   E_dev      device [N][2] float32 output (unnormalised).
 * Paper: "Aberration-Space Holography", compressed forward sum.
 * Errors: ASH_EINVAL, ASH_ENOTREADY, ASH_EHIP. */
int ash_forward(ash_ctx* ctx, const float* phase_dev, const float* field_dev,
                float* E_dev);

/* ash_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same transform, arguments and result as ash_forward, computed by the
 * same kernels, with the forward's partial sums and their reduction held in
 * a device-resident array inside the library (16 MiB per GPU, held until
 * the process ends) instead of the context's buffers.  The call allocates
 * nothing, neither records a memset nor synchronises.  Every call on one
 * GPU shares that array: calls that overlap in time on one GPU (two streams,
 * two contexts) race and their results are undefined; calls ordered on one
 * stream are safe.  Nothing in the array has to start at zero (every entry
 * read is written first by the same call).  Errors: as ash_forward, plus
 * ASH_EUNSUPPORTED when the set-up's partial sums (forward ranges x N x 8
 * bytes, plus N x 8) exceed 16 MiB (ash_get_info gives the ranges). */
int ash_forward_noalloc(ash_ctx* ctx, const float* phase_dev,
                        const float* field_dev, float* E_dev);

/* Adjoint transform g(x) = sum_n y_n exp(+i theta_n(x)).
 *   y_dev          device [N][2] float32 spot fields.
 *   g_dev          device [ny][nx][2] float32 output, or NULL.
 *   phase_out_dev  device [ny][nx] float32 output arg g in (-pi, pi]
 *                  (arg 0 = 0), or NULL.  At least one output non-NULL.
 * Paper: "Aberration-Space Holography", compressed adjoint sum; the
 * phase output is the GS nearfield projection.
 * Errors: ASH_EINVAL, ASH_ENOTREADY, ASH_EHIP. */
int ash_adjoint(ash_ctx* ctx, const float* y_dev, float* g_dev,
                float* phase_out_dev);

/* n_iter weighted-GS iterations, all on the device without host sync.
 *   phase_dev    device [ny][nx] float32, in: start phase, out: final.
 *   weights_dev  device [N] float32 spot weights W, in/out (start with 1).
 *   params       see ash_wgs_params (NULL = power 1).
 *   E_dev        device [N][2] float32: fields of the last iteration's
 *                forward transform (before its phase update), or NULL.
 *   stats_dev    device [n_iter][4] float32 per-iteration figures of the
 *                forward fields: efficiency sum|E|^2/(P sum A^2),
 *                uniformity 1-(max-min)/(max+min) of |E|^2/t^2, its
 *                std/mean, and sum|E|^2; or NULL.
 * Paper: "A Full-Field 2D Tweezer Array" (weighted GS) and the GS
 * description in "Aberration-Space Holography".
 * Errors: ASH_EINVAL (n_iter < 0, null phase/weights, power not finite),
 * ASH_ENOTREADY, ASH_EHIP. */
int ash_wgs_iterate(ash_ctx* ctx, float* phase_dev, float* weights_dev,
                    int n_iter, const ash_wgs_params* params, float* E_dev,
                    float* stats_dev);

/* One weighted-GS iteration driven by measured spot amplitudes
 * (experimental feedback: the paper's software closes the loop on camera
 * measurements, "A Full-Field 2D Tweezer Array" and Discussion):
 *   measured_dev  device [N] float32 amplitudes a_k of the spots produced by
 *                 phase_dev on the system (values <= 0 or NaN count as dark:
 *                 their weights are kept).
 * The weights are updated from these a_k instead of |E_k|; the projection
 * uses psi_k = arg E_k of the model, or the stored phases
 * (params->fix_phase_after as for ash_wgs_iterate with n_iter = 1).
 * phase_dev and weights_dev are updated in place; E_dev [N] complex64 and
 * stats_dev [4] (of the model fields E) are optional.  Errors: ASH_EINVAL,
 * ASH_ENOTREADY, ASH_EHIP. */
int ash_wgs_feedback(ash_ctx* ctx, float* phase_dev, float* weights_dev,
                     const float* measured_dev, const ash_wgs_params* params,
                     float* E_dev, float* stats_dev);

/* The farfield phases stored by phase fixing, in turns (arg E / 2 pi, in
 * [-1/2, 1/2]), copied verbatim so that a phase-fixed run can be
 * checkpointed and resumed bitwise in a context with the same spots:
 *   ash_get_fixed_phases copies them to psi_dev (device [N] float32);
 *   ASH_ENOTREADY if none are stored.
 *   ash_set_fixed_phases stores psi_dev (device [N] float32) as if an
 *   iteration had stored them.
 * Errors: ASH_EINVAL, ASH_ENOTREADY, ASH_EHIP. */
int ash_get_fixed_phases(ash_ctx* ctx, float* psi_dev);
int ash_set_fixed_phases(ash_ctx* ctx, const float* psi_dev);

/* Phase gradient of a real loss of the spot fields (the backward of
 * ash_forward with respect to the phase):
 *   grad(x) = Im( conj(f(x)) * sum_n G_n exp(+i theta_n(x)) ),
 *   f = A exp(i phase), G_n = dL/dRe E_n + i dL/dIm E_n.
 *   phase_dev  device [ny][nx] float32 phase at which E was taken.
 *   G_dev      device [N][2] float32 field gradient (torch's gradient of a
 *              real loss with respect to a complex tensor has this form).
 *   grad_dev   device [ny][nx] float32 output.
 * Paper: Methods, "Computational Scaling" (gradient descent through the
 * transforms for precision targets); the derivative of the compressed
 * forward sum by the phase, evaluated with the adjoint kernels.
 * Errors: ASH_EINVAL, ASH_ENOTREADY, ASH_EHIP. */
int ash_phase_grad(ash_ctx* ctx, const float* phase_dev, const float* G_dev,
                   float* grad_dev);

/* Adam descent of the spot-amplitude loss with a phase-gradient TV term
 *   L = sum_n (|E_n/s|^2 - t_n)^2 + tv_weight * TV(phase),
 *   s = sqrt(P sum_x A^2 / N),  t the targets of ash_set_spots,
 *   TV = (1/P) sum_x sqrt(dx^2 + dy^2 + tv_eps^2), dx, dy the forward
 *   differences of the phase wrapped into (-pi, pi], 0 at the last
 *   column / row.
 * Adam (Kingma and Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
 * phase -= lr (m/(1-b1^k)) / (sqrt(v/(1-b2^k)) + eps) at update k. */
/* Basis moments of the forward transform,
 *   M[k][d] = sum_x Z_d(x) f(x) exp(-i theta_k(x)),   f = A exp(i phase),
 * so that dE_k/dw[k][d] = -i M[k][d]: the derivative of every spot field
 * along its own kernel coefficients (paper: Methods, "Computational
 * Scaling": spots move in aberration space through w; the same sums give
 * the gradients for fitting w).
 *   phase_dev  device [ny][nx] float32 phase (A is the context's amplitude).
 *   M_dev      device [N][D] complex64 output (row k: spot k).
 * Evaluated like the forward (same phases and precision; the products with
 * A Z_d are matrix-core sums of bf16 pieces, relative error ~2^-16 per
 * term).  Errors: ASH_EINVAL, ASH_ENOTREADY, ASH_EHIP. */
int ash_forward_moments(ash_ctx* ctx, const float* phase_dev, float* M_dev);

/* Gradient of a real loss L(E) with respect to the kernel coefficients:
 *   dL/dw[k][d] = Im(conj(G_k) M[k][d]),   G_k = dL/dRe E_k + i dL/dIm E_k.
 *   phase_dev  device [ny][nx] float32 phase (A is the context's amplitude).
 *   G_dev      device [N] complex64 field gradient.
 *   grad_dev   device [N][D] float32 output.
 * Errors: ASH_EINVAL, ASH_ENOTREADY, ASH_EHIP. */
int ash_coef_grad(ash_ctx* ctx, const float* phase_dev, const float* G_dev,
                  float* grad_dev);

/* In-silico spot quality (paper: Methods, "Relative Strehl Metrology":
 * S' = max I / sum I over a 21 x 21 camera box around each spot).  The
 * "image" near a spot is sampled as the spot fields of kernels whose tilt
 * coefficients are moved by the window offsets.
 *
 * ash_window_coefficients (host-only): expand w (host [N][D] float64) into
 * w_out (host [N*win*win][D]), spot-major with the window's x offset
 * fastest: row (k*win + b)*win + a is w[k] with the spot moved by
 * ((a - win/2) step, (b - win/2) step) DFT bins of an nx x ny SLM:
 * w[k][ix] += (a - win/2) dwx, w[k][iy] += (b - win/2) dwy, with
 * dwx = pi step R / nx and dwy = pi step R / ny (radians), the coefficient
 * change that moves the orthonormal tilts Z = 2 xh (mode ix) and Z = 2 yh
 * (mode iy) of a pupil of radius R pixels by `step` bins.  win odd;
 * ix != iy.  Errors: ASH_EINVAL (sizes < 1, even win, bad mode indices,
 * R <= 0 or non-finite R / step), ASH_EUNSUPPORTED (N*win*win >
 * ASH_MAX_SPOTS).
 *
 * ash_window_strehl: with the context's spots set to such an expansion
 * (N = n_windows * win * win), the forward transform of A exp(i phase)
 * and, per window, S_dev[w] = max |E|^2 / sum |E|^2 over its win*win
 * fields (0 for a dark window).  phase_dev device [ny][nx] float32; S_dev
 * device [n_windows] float32.  Errors: ASH_EINVAL, ASH_ENOTREADY,
 * ASH_ESHAPE (spot count not n_windows*win*win), ASH_EHIP. */
int ash_window_coefficients(int N, int D, const double* w, int ix, int iy,
                            int nx, int ny, double R, double step, int win,
                            double* w_out);
int ash_window_strehl(ash_ctx* ctx, const float* phase_dev, int n_windows,
                      int win, float* S_dev);

typedef struct ash_adam_params {
  float lr;         /* 0.05 */
  float beta1;      /* 0.9 */
  float beta2;      /* 0.999 */
  float eps;        /* 1e-8 */
  float tv_weight;  /* 1e-3 */
  float tv_eps;     /* 1e-3 rad */
} ash_adam_params;

/* n_steps Adam updates on the device, each a forward transform, the loss
 * and its field gradient, the adjoint with the phase gradient and TV term
 * in its epilogue, and the update.
 *   phase_dev   device [ny][nx] float32, in: start, out: after n_steps.
 *   m_dev, v_dev device [ny][nx] float32 Adam moments, in/out (zero at
 *               the start of a descent).
 *   step0       updates already made with these moments (0 at the start).
 *   params      NULL for the defaults above.
 *   loss_dev    device [n_steps] float32: L at the phase before each
 *               update, or NULL.
 *   E_dev       device [N][2] float32: fields of the last forward, or NULL.
 * Paper: Methods, "Computational Scaling"; the loss, TV term and Adam are
 * stated readings (the paper names gradient descent only).
 * Errors: ASH_EINVAL (null arrays, n_steps or step0 < 0, parameters out of
 * range, zero source amplitude), ASH_ENOTREADY, ASH_EHIP. */
int ash_adam_iterate(ash_ctx* ctx, float* phase_dev, float* m_dev,
                     float* v_dev, int step0, int n_steps,
                     const ash_adam_params* params, float* loss_dev,
                     float* E_dev);

/* Precision of the in-tile remainder terms.  The phase is a sum of
 * products of bf16 pieces.  ASH_PRECISION_AUTO (default) carries the basis
 * remainders and their coefficients in 2 pieces (relative error below
 * 2^-16 of the remainder phase) when, for every tile and spot,
 * sum_s |c_s| max|Rm_s| <= 1/2 turn, and in 3 pieces (~2^-24) otherwise;
 * ASH_PRECISION_FULL always uses 3 pieces.  Takes effect at the next
 * ash_set_spots.  Errors: ASH_EINVAL. */
#define ASH_PRECISION_AUTO 0
#define ASH_PRECISION_FULL 1
int ash_set_precision(ash_ctx* ctx, int mode);

/* Shape of the current set-up, for measurement and tests. */
typedef struct ash_info {
  int32_t n_tiles;       /* 32 x 16 pixel tiles                           */
  int32_t nonlinear;     /* modes with a monomial of degree >= 2          */
  int32_t pieces;        /* bf16 pieces of remainders / coefficients      */
  int32_t groups;        /* 16-slot groups = matrix-core ops per 32x32    */
  int32_t fwd_ranges;    /* pixel-block ranges of the forward transform   */
  float rm_bound;        /* max over tiles/spots of sum |c_s| max|Rm_s|   */
  float theta_bound;     /* bound on |phase| (turns) of any spot-pixel pair
                            inside a tile; at most 256 (ash_set_spots)    */
  int32_t range_reduce;  /* 1: phases reduced to one turn before sin/cos,
                            0: bound <= 64 turns, the hardware reduces    */
} ash_info;
int ash_get_info(const ash_ctx* ctx, ash_info* out);

/* ---- Batched form ----------------------------------------------------
 * Many holograms' weighted-GS loops run together, in one of two forms.
 *
 * One launch (members of at most 512 spots, on a device with cooperative
 * launches): one cooperative launch per record shape runs every iteration
 * of its holograms.  Each resident block owns a contiguous range of one
 * hologram's 32-pixel blocks (the blocks shared out over the holograms in
 * proportion to their work, in pairs) and, per iteration, runs fused rows
 * over its range (the adjoint of the last spot fields and the forward of
 * the new phases, its four waves taking pairs of pixel blocks), meets the
 * hologram's other blocks at a barrier (a counter per hologram), and
 * computes the whole hologram's weight update from all blocks' sums; a
 * last pass of adjoint rows writes the phase.  Its resident blocks per CU
 * are tuned.
 *
 * Launches per phase (any members): each phase of an iteration is one
 * persistent launch over the work items of all holograms of a record
 * shape: the forward over (hologram, pixel range, 32-spot block) items, a
 * fixed-order reduction and the weight updates of all holograms, and the
 * adjoint over (hologram, tile row) items.  Forward items sit in eight
 * per-XCD queues (longest first, balanced by work); resident waves take
 * them with an atomic counter and move to the other queues when theirs runs
 * dry.  The forward range length (pixel blocks per item) is tuned.  When
 * every member has at most 512 spots, the transforms are fused launches
 * over (hologram, pixel range) items instead: per 32-pixel block the
 * adjoint of this iteration over all spots, the phase it projects to, and
 * the block's terms of the next iteration's forward, so the pixel records
 * are read once per iteration and no nearfield records are built (the
 * first launch of a call runs only the forward of the start phases, the
 * last only the adjoint, which writes the phases).  A hologram of B 32-spot
 * blocks takes ranges of about 1/B of the tuned length, so that items hold
 * about equal work.  Results differ from the separate kernels' in FP32
 * summation order only.
 *
 * A batch starts in the one-launch form when its members allow it;
 * ash_batch_tune keeps the faster form for the batch at hand and
 * ash_batch_set_form chooses one.
 * Paper: Methods, "Computational Scaling" (many holograms); the batched
 * forms are this library's. */
typedef struct ash_batch ash_batch;

/* A batch of H holograms, each a context with its basis and spots set, all
 * on one device.  The members stay owned by the caller and must outlive the
 * batch; the batch computes in their buffers, so a member must not be used
 * on another stream while a batch call runs.  Changing a member's basis or
 * spots invalidates the batch: its calls then fail with ASH_ENOTREADY.
 *   stream  HIP stream of the batch's launches (NULL: the default stream).
 * Errors: ASH_EINVAL (H < 1, null or unready members, members on different
 * devices), ASH_ENOMEM, ASH_EUNSUPPORTED (more than 2^31 work items),
 * ASH_EHIP. */
int ash_batch_create(ash_batch** out, int H, ash_ctx* const* members,
                     void* stream);
int ash_batch_destroy(ash_batch* batch);
const char* ash_batch_last_error(const ash_batch* batch);
int ash_batch_set_stream(ash_batch* batch, void* stream);

/* n_iter weighted-GS iterations of every hologram.
 *   phase_dev    host array of H device pointers, hologram h's
 *                [ny_h][nx_h] float32 phase, in: start, out: final.
 *   weights_dev  host array of H device pointers, [N_h] float32 weights,
 *                in/out (start with 1).
 *   params       as for ash_wgs_iterate (NULL = power 1; phase fixing is
 *                not supported in a batch).
 * Each hologram's results equal its own ash_wgs_iterate up to the FP32
 * summation order of the forward sums.  The call synchronises the stream
 * at its start (descriptor upload); the one-launch form also at its end
 * (to read the barriers' error flag: a barrier that waits more than 10 s
 * ends the launch and the call returns ASH_EHIP).  The per-phase form keeps
 * 2 KB of queue counters per iteration (and one more) and record shape on
 * the device, grown on demand.  Errors: ASH_EINVAL, ASH_ENOTREADY, ASH_EUNSUPPORTED,
 * ASH_ENOMEM, ASH_EHIP. */
int ash_batch_wgs(ash_batch* batch, float* const* phase_dev,
                  float* const* weights_dev, int n_iter,
                  const ash_wgs_params* params);

/* Autotuner.  For each record shape, times the per-phase form's forward
 * plus its reduction for range lengths of 16, 32, 64, 128, 256 and 512
 * pixel blocks (fused: an adjoint-and-forward launch for 4, 8, 16, 32, 64
 * and 128) and keeps the fastest; when the one-launch form is possible,
 * costs it for 1 up to the most resident blocks per CU that fit, keeps the
 * cheapest, costs the per-phase form, and selects the cheaper form.  A
 * form's cost is the time of one more iteration (runs of 2 and 22
 * iterations, their time difference over 20), so that the first forward
 * and last adjoint of a call do not weigh.  The timed iterations run on
 * copies of the phases (the caller's are left untouched).  The table written to table_out (if not NULL) holds lines
 * "groups range_reduce range_blocks ms", "one_launch groups range_reduce
 * blocks_per_cu ms_per_iteration" and "form one_launch ms_per_iteration".
 * Errors: ASH_EINVAL (null phases, unwritable file), ASH_ENOTREADY,
 * ASH_ENOMEM, ASH_EHIP. */
int ash_batch_tune(ash_batch* batch, float* const* phase_dev,
                   const char* table_out);
/* Apply a table written by ash_batch_tune (lines for absent record shapes
 * are ignored).  Errors: ASH_EINVAL (unreadable file), ASH_ENOMEM. */
int ash_batch_load_tuning(ash_batch* batch, const char* table_in);

/* Choose the form: one_launch = 1 the one-launch form, 0 the launches per
 * phase.  Errors: ASH_EINVAL, ASH_EUNSUPPORTED (one launch requested for
 * members of more than 512 spots or on a device without cooperative
 * launches). */
int ash_batch_set_form(ash_batch* batch, int one_launch);

typedef struct ash_batch_info {
  int32_t holograms;
  int32_t shapes;           /* record shapes (one launch each per phase)   */
  int32_t groups[4];        /* matrix-core groups of the first 4 shapes    */
  int32_t range_blocks[4];  /* their forward range lengths (fused: for a
                               hologram of one 32-spot block)             */
  int64_t items;            /* work items of the per-phase launches:
                               forward + adjoint, or fused units          */
  double evals_per_transform;  /* sum over holograms of N * P              */
  int32_t one_launch;       /* 1: the one-launch form (see ash_batch_wgs)  */
  int32_t blocks_per_cu[4]; /* its resident blocks per CU (grid / CUs)     */
  int32_t grid[4];          /* its blocks per launch                       */
  int32_t fused;            /* 1: per-phase iterations fuse the adjoint
                               with the next forward (members <= 512 spots)*/
} ash_batch_info;
int ash_batch_get_info(const ash_batch* batch, ash_batch_info* out);

/* Event timing of the batch's launches, as ash_profile_enable/read.  With
 * fused launches (ash_batch_info.fused), ASH_PROF_ADJOINT times all of
 * them (n_iter + 1 per record shape and ash_batch_wgs call: both
 * transforms of every hologram in all but the first and the last, which
 * hold the first forward and the last adjoint). */
int ash_batch_profile_enable(ash_batch* batch, int mask);
int ash_batch_profile_read(ash_batch* batch, double* ms_out,
                           int64_t* launches_out);

/* Kernel timing, for measurement.  Kernels of the categories selected by
 * `mask` (bit 1 << category) are bracketed by HIP events on the context's
 * stream.  Categories:
 *   ASH_PROF_FORWARD   forward transform kernel (and the moment kernel)
 *   ASH_PROF_ADJOINT   adjoint transform kernel (with its epilogue)
 *   ASH_PROF_REDUCE    partial-sum reductions, weighted-GS update, loss
 *   ASH_PROF_FIELD     nearfield preparation A exp(i phase), Adam update
 * ASH_PROF_ALL selects all; 0 (the default) records nothing.  Each event
 * pair costs a few microseconds of stream time, so select only what is
 * measured.  ash_profile_read synchronises the stream, writes the summed
 * milliseconds and the launch count of each category into ms_out[4] /
 * launches_out[4] (either may be NULL) and clears the record. */
#define ASH_PROF_FORWARD 0
#define ASH_PROF_ADJOINT 1
#define ASH_PROF_REDUCE 2
#define ASH_PROF_FIELD 3
#define ASH_PROF_ALL 0xF
int ash_profile_enable(ash_ctx* ctx, int mask);
int ash_profile_read(ash_ctx* ctx, double* ms_out, int64_t* launches_out);

/* Time one launch in every `stride` (>= 1, default 1) of each selected
 * category, counted from the last ash_profile_enable: each event pair
 * costs stream time, and for short kernels a sample measures their
 * average duration with little of that cost.  launches_out then counts
 * the timed launches.  Errors: ASH_EINVAL (stride < 1). */
int ash_profile_stride(ash_ctx* ctx, int stride);

#ifdef __cplusplus
}
#endif

#endif /* ASH_H */
