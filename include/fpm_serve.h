/*
 * fpm_serve.h - C ABI of the tile-reconstruction server in libfpm.
 *
 * Whole-slide FPM splits the field of view into tiles that are reconstructed
 * independently (Sec. 3.3 of arXiv 2408.13782: per-ROI reconstruction with
 * its own aberrations and defocus). The server runs such reconstructions as
 * requests arrive, several at once on one GPU:
 *
 *  - A request is one complete solve: the initial value from one LED's
 *    amplitude (Sec. 2.3), then n_steps random-batch updates (Eq. 13) with the
 *    caller's schedule and loss (amplitude or intensity, Eqs. 4-5), exactly as
 *    fpm_init_spectrum + fpm_pupil + fpm_plan_set_loss + fpm_run on a fresh
 *    plan and state.
 *  - Continuous batching: up to n_lanes requests run at the same time, each on
 *    a lane with its own HIP stream, so their kernels overlap on the device.
 *    A request waiting in the queue is admitted as soon as a lane is idle and
 *    its memory footprint fits the budget together with the requests running;
 *    admission is first-in first-out.
 *  - Per-request device state (spectrum, pupil, pupil parameters, Adam
 *    moments) and plan scratch live in slots kept in HBM between requests;
 *    slots are reused by later requests of the same shape (sizes and optics).
 *    A slot holding another LED table (another tile of the field of view) is
 *    rebound to the request's table (fpm_plan_set_shifts) on the lane's
 *    stream. fpm_server_reserve() creates slots ahead of time, otherwise a
 *    lane creates a slot when no free one of the request's shape exists.
 *    Idle slots are not counted in the budget; when a new slot does not fit
 *    in device memory, the lane frees every idle slot and tries once more
 *    (the request fails with FPM_ENOMEM only if it still does not fit).
 *  - A request's result depends only on the request: every reduction in the
 *    update is in a fixed order and a slot is used by one request at a time,
 *    so the same request gives bitwise the same result alone or in a mix.
 *  - A solve whose summed loss is not finite (NaN or infinite measured data,
 *    a diverging learning rate) completes with status FPM_ENONFINITE; its
 *    outputs are still written. Other requests are not affected.
 *
 * Footprint of a request (bytes, what admission counts):
 *   state 3 M^2 * 8 (spectrum and the two Adam moments) + N^2 * 8 (pupil)
 *   + the plan's scratch (fpm_info.device_bytes) + measured data n_led N^2 4.
 *
 * Threads.  fpm_server_* calls may come from any host thread; the server's
 * lanes are host threads of its own. All calls return FPM_OK or a negative
 * code from fpm.h (fpm_last_error() has the message on the calling thread);
 * no C++ exception leaves them (a failed host allocation is FPM_ENOMEM).
 * The server uses the HIP device that is current when it is created.
 */
#ifndef FPM_SERVE_H
#define FPM_SERVE_H

#include <stdint.h>

#include "fpm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fpm_server fpm_server;

typedef struct {
  int32_t n_lanes;            /* requests on the GPU at once, 1..64 */
  int64_t hbm_budget_bytes;   /* limit on the summed footprints of running requests */
} fpm_server_desc;

/* One tile reconstruction. HOST arrays are copied by fpm_server_submit. */
typedef struct {
  fpm_desc desc;              /* sizes and optics; max_batch >= every batch size */
  const int32_t* shifts_host; /* HOST int32 [n_led][2] LED table (as fpm_plan_create) */
  const float* meas_amp;      /* DEVICE float [n_led][N][N]; caller-owned, valid until done */
  int32_t centre_led;         /* the initial value is the upsampled amplitude of this LED */
  fpm_hparams hp;             /* Adam settings and learned pupil groups */
  const int32_t* leds;        /* HOST int32, the batches concatenated (as fpm_run) */
  const int32_t* batch_sizes; /* HOST int32 [n_steps] */
  int32_t n_steps;
  fpm_c32* O_out;             /* DEVICE [M][M]: the final spectrum */
  float* coeffs_out;          /* DEVICE [15] or NULL: final Zernike coefficients */
  double* loss_out;           /* DEVICE [1] or NULL: loss summed over all steps */
  int64_t tag;                /* caller's id, returned in the completion record */
  int32_t loss_kind;          /* FPM_LOSS_AMPLITUDE (0, the zero default) or FPM_LOSS_INTENSITY */
  /* Multi-parameter solve (NULL grid: the nearest-pixel solve above). With a
     HOST grid (copied; n_side^2 == n_led, every batch <= 64 LEDs) the request
     runs fpm_run_multi instead of fpm_run: sub-pixel offsets from the grid
     plus the learned LED-array errors (starting from zero), learned with Adam
     at these rates when learn_geometry, besides the spectrum and the pupil
     parameters hp asks for. */
  const fpm_led_grid* grid;
  double lr_shift_mm, lr_rot_rad, lr_height_mm;
  int32_t learn_geometry;
  double* geom_out;           /* DEVICE [4] or NULL: final shift_x, shift_y, rot, dh errors */
} fpm_request;

/* What happened to one request. Times are ms on the server's clock
   (steady clock, zero at creation; fpm_server_clock_ms reads it). */
typedef struct {
  int64_t tag;
  int32_t status;             /* FPM_OK, FPM_ENONFINITE, or the code of the call that failed */
  int32_t lane;               /* lane that ran it */
  double t_submit_ms;         /* fpm_server_submit returned */
  double t_admit_ms;          /* a lane took it */
  double t_done_ms;           /* its last kernel and the result copies finished */
  int64_t footprint_bytes;
} fpm_completion;

/* Create a server on the current HIP device with n_lanes lane threads. */
int fpm_server_create(const fpm_server_desc* desc, fpm_server** server);

/* Wait for every submitted request, stop the lanes, free all slots. */
int fpm_server_destroy(fpm_server* server);

/* Footprint of a request of this shape (see above); creates and frees a
   plan to read its scratch size. */
int fpm_request_footprint(const fpm_desc* desc, const int32_t* shifts_host, int64_t* bytes);

/* Create `count` free slots of a shape ahead of time (device allocations
   happen here, not while serving). */
int fpm_server_reserve(fpm_server* server, const fpm_desc* desc, const int32_t* shifts_host,
                       int32_t count);

/* Queue a request. Fails with FPM_EINVAL (nothing queued) if its arguments
   are invalid or its footprint alone exceeds the budget. */
int fpm_server_submit(fpm_server* server, const fpm_request* request);

/* Move up to max_out completion records (in completion order) to out;
   *n_out receives the count. wait_ms > 0 waits up to that long for at least
   one record when none is ready; 0 returns at once. */
int fpm_server_poll(fpm_server* server, fpm_completion* out, int32_t max_out, int32_t* n_out,
                    int32_t wait_ms);

/* Block until every submitted request has completed. */
int fpm_server_drain(fpm_server* server);

/* The server clock, ms since creation. */
double fpm_server_clock_ms(const fpm_server* server);

/* Counters: requests queued, running, completed; footprint bytes in use;
   the largest number of requests that ran at once; slots held. Each
   output pointer may be NULL. */
int fpm_server_stats(fpm_server* server, int32_t* queued, int32_t* running, int64_t* completed,
                     int64_t* bytes_in_use, int32_t* max_running, int32_t* slots);

#ifdef __cplusplus
}
#endif

#endif /* FPM_SERVE_H */
