/*
 * fpm.h - C ABI of libfpm, the MI355X (gfx950) hot path of Batch-FPM
 * (random batch-update Fourier ptychography, arXiv 2408.13782).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Sizes.  N = n_lr is the low-resolution (LR) image side, s = upsample,
 *   M = s*N the high-resolution (HR) side. Supported N: 64, 128, 192, 256,
 *   384, 512.
 *
 * Spectrum O.  complex [M][M] row-major (row = k_y, column = k_x), centred
 *   (zero frequency at [M/2][M/2]) and orthonormally scaled:
 *   O = fftshift(fft2(o)) / M for the HR object o (Sec. 2.1, Eq. 1).
 *
 * Pupil P.  complex [N][N], centred like O. Its support is the disk
 *   |u| <= NA/lambda (in spectral pixels); entries off the support are
 *   ignored on input and never written by gradients.
 *
 * LED windows.  The plan owns the LED table: int32 [n_led][2] spectral
 *   offsets (row, col) s_b = round(k_b / dk). LED b reads the N x N window
 *   of O whose top-left corner is (M/2 - N/2) + s_b (this is O(k - k_m) of
 *   Eq. 2 with k_m the illumination propagation direction).
 *
 * Images.  Measured amplitudes A = sqrt(I), float [n_led][N][N] natural
 *   order, indexed by LED id. Batches are int32 HOST arrays of LED ids (the
 *   random schedule is host data; each launch receives its batch's ids and
 *   window offsets by value). Every id must lie in [0, n_led): a call with
 *   an id outside fails with FPM_EINVAL and enqueues nothing.
 *
 * Loss (Eq. 5, amplitude form, summed over the batch as in Eq. 13):
 *   L = sum_b sum_r (sqrt(gamma_b) |psi_b(r)| - A_b(r))^2,
 *   psi_b = (N^2/M) ifft2(ifftshift(C_b * P)), C_b = window of O.
 * Gradients are real gradients written as complex numbers,
 *   g = dL/dRe + i dL/dIm, accumulated (+=) into caller buffers.
 *
 * Memory.  Every pointer argument except `desc`, `shifts_host`, `leds`,
 *   `batch_sizes`, the fpm_led_shifts outputs, the timing outputs and the
 *   output `plan` handle is DEVICE memory on the current HIP device, owned by
 *   the caller. The plan owns only its scratch (sized at creation from N, M
 *   and max_batch). No entry point allocates after plan creation.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = default
 *   stream). Calls enqueue kernels and return without synchronising;
 *   results are ready when the stream reaches them. Calls on one plan must
 *   not overlap on different streams (they share the plan's scratch).
 *
 * Errors.  Every call returns FPM_OK (0) or a negative code; arguments are
 *   validated on the host before any launch, so a failed call has enqueued
 *   nothing. fpm_strerror() names the code; fpm_last_error() gives a
 *   human-readable message for the last failure on the calling thread. No
 *   C++ exception leaves a call (a failed host allocation is FPM_ENOMEM).
 */
#ifndef FPM_H
#define FPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FPM_OK = 0,
  FPM_EINVAL = -1,        /* bad size, null required pointer, B > max_batch ... */
  FPM_ENOMEM = -2,        /* device allocation failed at plan creation */
  FPM_EHIP = -3,          /* a HIP runtime call failed */
  FPM_EUNSUPPORTED = -4,  /* N or M outside the compiled set */
  FPM_ENONFINITE = -5     /* a served solve ended with a non-finite loss (fpm_serve.h) */
};

typedef struct fpm_plan fpm_plan;

/* Interleaved complex float (8 bytes, same layout as float2 / std::complex<float>). */
typedef struct { float re, im; } fpm_c32;

/* Optics and sizes of one reconstruction problem (Sec. 2.1, Sec. 3). */
typedef struct {
  int32_t n_lr;          /* N */
  int32_t upsample;      /* s, M = s N (M <= 4096) */
  int32_t n_led;         /* rows of the LED table */
  int32_t max_batch;     /* largest B any call on this plan will pass (<= 1024;
                            the multi-parameter calls take at most 64 per batch) */
  double wavelength_um;  /* lambda */
  double na;             /* objective numerical aperture */
  double mag;            /* objective magnification */
  double pixel_um;       /* camera pixel pitch; object-plane pitch = pixel/mag */
} fpm_desc;

/* Read-only facts about a plan, filled by fpm_plan_info(). */
typedef struct {
  int32_t n_lr, m_hr, n_led, max_batch;
  int32_t support_px;      /* |S|: pixels of the pupil disk */
  int32_t support_rows;    /* rows of the pupil grid that meet the disk */
  int32_t adam_tiles;      /* 32 x 32 HR tiles of the rectangle bounding the union of windows */
  double pupil_radius_px;  /* NA / lambda / dk */
  double dk;               /* spectral pitch, 1/um */
  int64_t device_bytes;    /* device memory the plan holds (its scratch and tables) */
  int32_t fused_chain;     /* 1: a step runs the loss and its adjoint as one launch
                              (N = 64: the image stays in one CU's LDS), then the
                              update; 0: three passes (rows, columns, rows), then the update */
} fpm_info;

/*
 * Create a plan. `shifts_host` is HOST memory, int32 [n_led][2] (row, col)
 * spectral offsets; it is copied. Every window must lie inside the HR grid
 * (FPM_EINVAL otherwise). The plan records the current HIP device.
 */
int fpm_plan_create(const fpm_desc* desc, const int32_t* shifts_host, fpm_plan** plan);
int fpm_plan_destroy(fpm_plan* plan);

/*
 * Replace the plan's LED table (same n_led; HOST int32 [n_led][2], copied),
 * e.g. for another tile of the field of view, whose illumination angles
 * differ (Sec. 2.1 k_m with the tile centre as the sample point). Windows are
 * validated as in fpm_plan_create (FPM_EINVAL, nothing changed). Nothing is
 * uploaded (the table and the Adam tile rectangle travel in the launch
 * arguments), so launches already enqueued keep the old table and calls on the
 * plan after this one use the new one; `stream` is not used and may be NULL.
 */
int fpm_plan_set_shifts(fpm_plan* plan, const int32_t* shifts_host, void* stream);

/*
 * Loss of every later call on the plan (Eqs. 4-5; default amplitude):
 *   FPM_LOSS_AMPLITUDE: L = sum (sqrt(gamma)|psi| - A)^2, as stated below;
 *   FPM_LOSS_INTENSITY: L = sum (gamma |psi|^2 - A^2)^2 (Eq. 4 with I = A^2),
 *     g_psi = 4 gamma e psi with e = gamma |psi|^2 - A^2, dL/dgamma = 2 sum e |psi|^2.
 * The measured input stays the amplitude A = sqrt(I) either way.
 */
enum { FPM_LOSS_AMPLITUDE = 0, FPM_LOSS_INTENSITY = 1 };
int fpm_plan_set_loss(fpm_plan* plan, int32_t kind);
int fpm_plan_info(const fpm_plan* plan, fpm_info* info);
const char* fpm_strerror(int code);
const char* fpm_last_error(void);
/* Identification of the build: a digest of the library's sources (its HIP,
 * C++ and C header files), fixed at compile time. Measurements taken on one
 * build (hardware counters of its kernels) apply to another only if the tags
 * agree. Static string, never NULL. */
const char* fpm_build_tag(void);

/* Square LED grid below the sample and its errors (Sec. 2.1; Sec. 2.2). */
typedef struct {
  int32_t n_side;       /* LEDs per side; ids run row-major */
  double pitch_mm;      /* LED spacing */
  double height_mm;     /* LED plane to sample distance */
  double shift_x_mm, shift_y_mm;   /* lateral offset of the whole array */
  double rot_rad;       /* in-plane rotation of the array */
  double dh_mm;         /* height error */
  double roi_x_mm, roi_y_mm;       /* sample point (field-of-view position) */
} fpm_led_grid;

/*
 * LED geometry -> spectral offsets (Sec. 2.1, k_m = sin(theta)/lambda), in
 * FP64 on the host. LED (column i, row j) offsets from the grid centre sits
 * at x = p(i cos r - j sin r) + dx, y = p(i sin r + j cos r) + dy, height
 * H = h + dh; with d the LED-to-sample distance, k = ((x - x_s), (y - y_s)) / (lambda d)
 * and the offset in spectral pixels is s = k / dk, dk = 1 / (N pixel/mag).
 * All outputs are HOST arrays [n_side^2][2] in (row, col) order, each nullable:
 * k_out in 1/um, s_out fractional pixels, nearest_out = floor(s + 1/2).
 */
int fpm_led_shifts(const fpm_desc* desc, const fpm_led_grid* grid, double* k_out,
                   double* s_out, int32_t* nearest_out);

/*
 * Pupil with aberrations and defocus (Eq. 3 with H folded into P):
 *   P(u) = mask(u) exp(i (sum_{j<n_zern} c_j Z_j(u) + z kappa(u))),
 *   kappa(u) = 2 pi (sqrt(1/lambda^2 - |k|^2) - 1/lambda), k = u dk,
 * Z_j the OSA/ANSI Zernike terms (unit RMS on the disk, rho = |u| / R).
 * coeffs: float [n_zern] (n_zern <= 15) or NULL (all zero);
 * z_um: float [1] or NULL (zero). P_out: complex [N][N], zero off the disk.
 */
int fpm_pupil(fpm_plan* plan, const float* coeffs, int32_t n_zern, const float* z_um,
              fpm_c32* P_out, void* stream);

/*
 * Forward model (Eq. 3): for each LED id leds[b], b < B,
 *   amp_out[b]   = sqrt(gamma[led]) |psi_b|      float [B][N][N]
 *   field_out[b] = psi_b                          complex [B][N][N] (nullable)
 * gamma: float [n_led] or NULL (all ones).
 */
int fpm_forward(fpm_plan* plan, const fpm_c32* O, const fpm_c32* P, const int32_t* leds,
                int32_t B, const float* gamma, float* amp_out, fpm_c32* field_out,
                void* stream);

/*
 * Loss and adjoint of one random batch (Eqs. 5 and 13):
 *   gO[w_b + u] += conj(P(u)) g_Phi_b(u)     (atomic scatter-add, complex [M][M])
 *   gP[u]       += conj(C_b(u)) g_Phi_b(u)   (nullable, complex [N][N], disk only)
 *   loss[0]     += L                         (nullable, double, device)
 * with g_Phi_b = (1/M) fftshift(fft2(2 sqrt(gamma) e psi/|psi|)),
 * e = sqrt(gamma)|psi| - A (psi/|psi| taken as 0 where psi = 0).
 * meas_amp: float [n_led][N][N]. The summation order of the atomics is not
 * fixed, so results agree with a sequential sum to rounding only.
 */
int fpm_backward(fpm_plan* plan, const fpm_c32* O, const fpm_c32* P, const int32_t* leds,
                 int32_t B, const float* gamma, const float* meas_amp, fpm_c32* gO,
                 fpm_c32* gP, double* loss, void* stream);

/*
 * fpm_backward without any device memory of its own: for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation). Same arguments, operation and results as fpm_backward;
 * the row/column intermediate and the loss partial sums live in a static
 * device array of the library (16 MiB + 256 KiB on each device the library
 * runs on, held until the process ends) instead of the plan's scratch.
 * Limit: min(B, 64) * N * N * 8 bytes <= 16 MiB (e.g. B <= 32 at N = 256,
 * B <= 8 at N = 512) and the column pass's partial sums within 256 KiB;
 * a larger batch fails with FPM_EINVAL before anything is enqueued. The call
 * allocates nothing (its first call on a device looks up the array's device
 * address once) and is not recorded by fpm_timing, whose events are created
 * on demand. Every call on one device shares that array and leaves its
 * contents behind: calls that overlap on one device (several streams or
 * threads) race and must be ordered by the caller.
 */
int fpm_backward_noalloc(fpm_plan* plan, const fpm_c32* O, const fpm_c32* P,
                         const int32_t* leds, int32_t B, const float* gamma,
                         const float* meas_amp, fpm_c32* gO, fpm_c32* gP, double* loss,
                         void* stream);

/*
 * Projection of a pupil gradient onto its phase parameters:
 *   g_theta(u) = Im(gP(u) conj(P(u))),
 *   g_par[j] += sum_u g_theta(u) Z_j(u)  (j < 15),  g_par[15] += sum_u g_theta(u) kappa(u)
 * in FP64. g_par: double [16]. gP is read only.
 */
int fpm_pupil_grad(fpm_plan* plan, const fpm_c32* gP, const fpm_c32* P, double* g_par,
                   void* stream);

/* Adam hyper-parameters and learning rates (torch.optim.Adam semantics). */
typedef struct {
  float lr_object, lr_zernike, lr_z;
  float beta1, beta2, eps;
  int32_t learn_zernike;   /* update coeffs[1..14]; the piston coeffs[0] is a global
                              phase with zero gradient and is held fixed */
  int32_t learn_z;         /* update z_um */
} fpm_hparams;

/*
 * Device-resident optimiser state of one reconstruction (all caller-owned):
 * O, m_O, v_O: complex [M][M] (m, v per real component); g_O is not used by
 * fpm_step / fpm_run (the object gradient is gathered from per-LED patches in
 * the plan's scratch, in batch order) and may be NULL;
 * P: complex [N][N] pupil (input if the pupil is fixed, rebuilt otherwise);
 * coeffs/m_c/v_c: float [15]; z_um/m_z/v_z: float [1] (may be NULL when not
 * learned); g_par: double [16] or NULL: when the pupil is learned, += the
 * gradients with respect to coeffs[0..14] and z of each step (diagnostics);
 * loss: double [1] or NULL (+= the batch loss).
 * `t` is the number of Adam steps already taken; fpm_step increments it.
 */
typedef struct {
  fpm_c32* O; fpm_c32* m_O; fpm_c32* v_O; fpm_c32* g_O;
  fpm_c32* P;
  float* coeffs; float* m_c; float* v_c;
  float* z_um; float* m_z; float* v_z;
  double* g_par;
  double* loss;
  int32_t t;
} fpm_state;

/*
 * One random-batch update (Eq. 13): rebuild P from (coeffs, z) when either
 * is learned (written to state->P), loss and gradients of the batch,
 * pupil-parameter projection, Adam on the learned pupil parameters, then
 * Adam on the object (over the union of LED windows; elsewhere the gradient
 * is identically zero and Adam leaves O unchanged). The loss and the
 * pupil-parameter gradients and the object gradient are all summed in a
 * fixed order: a step is deterministic.
 * The pupil state->P must hold P(coeffs, z) on entry (fpm_pupil builds it);
 * each step leaves it rebuilt from the updated parameters.
 */
int fpm_step(fpm_plan* plan, fpm_state* state, const fpm_hparams* hp, const int32_t* leds,
             int32_t B, const float* gamma, const float* meas_amp, void* stream);

/*
 * n_steps consecutive updates (a whole solve or a slice of one) in one call:
 * step i uses the batch_sizes[i] LED ids that follow those of step i-1 in
 * `leds` (HOST, int32, concatenated); batch_sizes is HOST memory [n_steps],
 * each in [1, max_batch]. Same effect as n_steps fpm_step calls; all ids
 * are validated before anything is enqueued.
 *
 * Batches of more than 64 LEDs (up to the full set, the full-gradient
 * descent of Eq. 6) run in groups of 64: the passes of each group store its
 * LEDs' patches, the update of every group but the last adds them into a
 * gradient accumulator of the plan, the last one applies Adam. The additions
 * keep the batch order, so the step equals a single pass over the batch.
 */
int fpm_run(fpm_plan* plan, fpm_state* state, const fpm_hparams* hp, const int32_t* leds,
            const int32_t* batch_sizes, int32_t n_steps, const float* gamma,
            const float* meas_amp, void* stream);

/* Learned parameters of the multi-parameter model (device memory). */
typedef struct {
  const fpm_c32* O;        /* [M][M] spectrum (required) */
  const float* coeffs;     /* [15] Zernike coefficients, or NULL (zero) */
  const float* z_um;       /* [1] defocus, or NULL (zero) */
  const double* geom;      /* [4] LED-array errors added to grid's: shift_x_mm,
                              shift_y_mm, rot_rad, dh_mm; NULL: the plan's integer
                              LED table (no geometry gradient) */
  const float* gamma;      /* [n_led] LED intensity factors, or NULL (ones) */
} fpm_params;

/* Gradient accumulators (device memory, +=); each may be NULL. */
typedef struct {
  fpm_c32* g_O;            /* [M][M] */
  double* g_par;           /* [16]: coeffs[0..14], z */
  double* g_geom;          /* [4] */
  double* g_gamma;         /* [n_led] */
  double* loss;            /* [1] */
  int32_t* oob;            /* [1] += number of windows that left the HR grid */
} fpm_grads;

/*
 * Loss and gradients of one batch for every parameter group (Sec. 2.1
 * Eq. 3, Sec. 2.2): spectrum, pupil Zernike coefficients and defocus, the
 * LED-array geometry and the LED intensities. LED offsets are fractional,
 * s_b = k_b(geometry)/dk computed in FP64 on the device from `grid` (HOST
 * struct: the nominal array) plus params->geom; the crop samples the spectrum
 * bilinearly at the fractional window (the loss is piecewise smooth in s_b;
 * the offset gradient is the one-sided derivative where s_b crosses an
 * integer). A window that would leave the HR grid is clamped and counted in
 * grads->oob. All sums are in a fixed order (deterministic). Requires
 * grid->n_side^2 == n_led and B <= 64.
 */
int fpm_loss_grad(fpm_plan* plan, const fpm_led_grid* grid, const fpm_params* params,
                  const int32_t* leds, int32_t B, const float* meas_amp, fpm_grads* grads,
                  void* stream);

/* Learned LED-array geometry of fpm_run_multi (device memory unless stated). */
typedef struct {
  double* geom;            /* [4] errors added to the grid's: shift_x_mm, shift_y_mm,
                              rot_rad, dh_mm */
  double* m_geom;          /* [4] Adam moments */
  double* v_geom;          /* [4] */
  double* g_geom;          /* [4] += each step's gradient, or NULL (diagnostics) */
  double lr_shift_mm, lr_rot_rad, lr_height_mm;   /* host values */
  int32_t learn;           /* update geom (else held; the offsets still follow it) */
} fpm_geometry;

/*
 * n_steps fused multi-parameter updates (Sec. 2.2): per step the loss and the
 * gradients of the spectrum, the Zernike coefficients, the defocus and the
 * LED-array geometry (sub-pixel offsets and bilinear crop as in
 * fpm_loss_grad), then Adam on all of them (torch semantics, FP64 for the
 * scalars; the spectrum's Adam runs over the whole HR grid because the union
 * of windows moves with the geometry). state: as fpm_run, with coeffs, z_um
 * and their moments required (learned or not, per hp->learn_zernike,
 * hp->learn_z); state->P must hold P(coeffs, z) on entry and is rebuilt each
 * step. No LED intensities. Deterministic; one call is the same as n_steps
 * calls of one step. Same batch layout as fpm_run, at most 64 LEDs per batch.
 */
int fpm_run_multi(fpm_plan* plan, const fpm_led_grid* grid, fpm_state* state,
                  fpm_geometry* geometry, const fpm_hparams* hp, const int32_t* leds,
                  const int32_t* batch_sizes, int32_t n_steps, const float* meas_amp,
                  void* stream);

/*
 * HR object <-> spectrum (Sec. 2.1, Eq. 1) with the orthonormal scaling:
 *   direction +1: O = fftshift(fft2(o)) / M;   direction -1: o = ifft2(ifftshift(O)) * M.
 * in, out: complex [M][M]; in == out is allowed.
 */
int fpm_hr_transform(fpm_plan* plan, const fpm_c32* in, fpm_c32* out, int32_t direction,
                     void* stream);

/*
 * Initial value (Sec. 2.3): spectrum of the bilinearly upsampled amplitude
 * image `centre_amp` (float [N][N], pixel-centre aligned, clamped borders),
 * zero phase. O_out: complex [M][M].
 */
int fpm_init_spectrum(fpm_plan* plan, const float* centre_amp, fpm_c32* O_out, void* stream);

/*
 * Digital refocusing (Abstract; Sec. 3.3): for each of nz distances z_um[i]
 * (device float [nz]), out[i] = ifft2(ifftshift(O H(z_i))) * M with
 * H = exp(i z kappa(k)) over the HR spectrum, 0 where |k| > 1/lambda.
 * out: complex [nz][M][M].
 */
int fpm_refocus(fpm_plan* plan, const fpm_c32* O, const float* z_um, int32_t nz, fpm_c32* out,
                void* stream);

/*
 * Per-kernel timing (diagnostics for profiling and roofline reports).
 * While enabled, every kernel the plan launches is bracketed by a pair of
 * HIP events recorded on the launch's stream (at most 65536 pairs are kept).
 * fpm_timing_collect() waits for the recorded events, writes for each kernel
 * kind k < *n_kinds (at most max_kinds): names[k] (static string), total_ms[k]
 * and counts[k], then clears the record. All arrays are HOST memory.
 */
int fpm_timing_enable(fpm_plan* plan, int32_t enable);
/*
 * While timing is enabled, issue every launch of kernel kind `kind` (the
 * index of its name in fpm_timing_collect's list; -1: none) `reps` times back
 * to back inside one event bracket, so that the bracket divided by reps is
 * the kernel's own duration on the step's real operands (the count reported
 * for the bracket is reps). Only fpm_step / fpm_run honour it. The repeated
 * launches recompute or re-apply their step: the state they leave is not a
 * valid optimisation state, so use a state whose results are discarded.
 */
int fpm_timing_repeat(fpm_plan* plan, int32_t kind, int32_t reps);
int fpm_timing_collect(fpm_plan* plan, int32_t max_kinds, const char** names, double* total_ms,
                       int32_t* counts, int32_t* n_kinds);

#ifdef __cplusplus
}
#endif

#endif /* FPM_H */
