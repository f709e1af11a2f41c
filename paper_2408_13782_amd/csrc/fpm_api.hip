// fpm_api.hip - host side of libfpm: plans, argument validation, launches.
// The C ABI is declared in include/fpm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "fpm.h"
#include "fpm_aux.hpp"
#include "fpm_fused.hpp"
#include "fpm_kernels.hpp"
#include "fpm_subpixel.hpp"

using namespace fpm;

namespace fpm {

thread_local std::string g_last_error;

// Record the message of a failure for fpm_last_error() on this thread.
int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

}  // namespace fpm

namespace {

int fail(int code, const std::string& msg) { return fpm::set_error(code, msg); }

// Runs the body of an entry point; a C++ exception (a failed host allocation,
// a thread that cannot start) becomes an error code: none crosses the C ABI.
template <class F>
int guarded(F&& body) {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail(FPM_ENOMEM, "host memory allocation failed");
  } catch (const std::exception& e) {
    return fail(FPM_EHIP, std::string("host runtime error: ") + e.what());
  }
}

#define FPM_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(FPM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

#define FPM_REQUIRE(cond, msg) \
  do {                         \
    if (!(cond)) return fail(FPM_EINVAL, msg); \
  } while (0)

bool lr_supported(int n) {
  return n == 64 || n == 128 || n == 192 || n == 256 || n == 384 || n == 512;
}
bool hr_supported(int m) {
  return m == 256 || m == 512 || m == 768 || m == 1024 || m == 1536 || m == 2048;
}

const char* const kHrSizes = "HR transforms support M in {256, 512, 768, 1024, 1536, 2048}";

// A launch serves at most kMaxSlots LEDs (their windows travel in the kernel
// arguments); larger batches of the nearest-pixel path run as consecutive
// groups of kMaxSlots, up to kMaxBatch LEDs per batch.
constexpr int kMaxBatch = 1024;

template <int V> using Size = std::integral_constant<int, V>;

// f(Size<N>{}) for the supported LR image sizes N (the kernels are templates on N).
template <class F>
int with_lr_size(int n, F&& f) {
  switch (n) {
    case 64: return f(Size<64>{});
    case 128: return f(Size<128>{});
    case 192: return f(Size<192>{});
    case 256: return f(Size<256>{});
    case 384: return f(Size<384>{});
    case 512: return f(Size<512>{});
  }
  return fail(FPM_EUNSUPPORTED, "unsupported N");
}

std::vector<float2> twiddles(int n) {
  std::vector<float2> tw(n);
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * (double)m / (double)n;
    tw[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  return tw;
}

// Allocate count elements (adding their bytes to *total) and copy src if given.
template <class T>
int upload(size_t* total, T** dst, const T* src, size_t count) {
  if (hipMalloc((void**)dst, count * sizeof(T)) != hipSuccess) {
    *dst = nullptr;
    return fail(FPM_ENOMEM, "hipMalloc failed");
  }
  *total += count * sizeof(T);
  if (src) FPM_HIP(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  return FPM_OK;
}

enum Kind {
  kPupilBuild, kRowsForward, kCols, kRowsBackward, kPupilGrad, kAdamObject, kAdamScalars,
  kHrRows, kHrCols, kChainFused, kKinds
};
const char* const kKindNames[kKinds] = {"pupil_build", "rows_forward", "cols", "rows_backward",
                                        "pupil_grad", "update", "commit", "hr_rows", "hr_cols",
                                        "chain_fused"};
constexpr size_t kMaxTimed = 65536;

struct TimedLaunch {
  int kind;
  int reps;     // launches inside the bracket
  hipEvent_t start, stop;
};

}  // namespace

struct fpm_plan {
  int device = 0;
  int N = 0, s = 0, M = 0, n_led = 0, max_batch = 0;
  double lambda = 0, na = 0, mag = 0, pixel = 0, dk = 0, radius = 0;
  int ky_lo = 0, ky_hi = -1, nrows = 0, support_px = 0;
  int n_tiles = 0;            // tiles of the Adam rectangle
  int2 tile0 = {0, 0};        // its first tile (row, column), in 32 x 32 HR tiles
  int tile_cols = 0;          // its width in tiles
  bool hr_ok = false;
  size_t device_bytes = 0;    // everything the plan allocated
  std::vector<int2> shifts_h;
  int2* rowext = nullptr;     // [N] (first, last) disk column of each pupil row
  float2* twN = nullptr;      // [N]
  float2* twM = nullptr;      // [M] when the HR transforms are available
  float2* X = nullptr;        // [min(max_batch, kMaxSlots)][N][N] row/column scratch
  float2* gacc = nullptr;     // [M][M] gradient sums of a batch's earlier groups (max_batch > kMaxSlots)
  float2* gP = nullptr;       // [N][N] pupil-gradient accumulator for fpm_step
  float* kappa_tab = nullptr;  // defocus phase per um at integer |u|^2 <= R^2
  std::vector<int2> rowext_h; // host copy of rowext
  double* part = nullptr;     // per-workgroup partial sums (loss | Zernike | pupil_grad)
  double* part_loss = nullptr;
  double* part_z = nullptr;
  double* part_pg = nullptr;
  float* staging = nullptr;   // next pupil-parameter state, written by the update kernel
  double* part_lg = nullptr;  // partials of fpm_loss_grad (column pass | row pass)
  float2* P_ws = nullptr;     // [N][N] pupil built by fpm_loss_grad
  int* oob_ws = nullptr;      // window-clamp counter when the caller passes none
  SubSlot* sub = nullptr;     // [2][max_batch] sub-pixel offsets of a batch (two steps of
                              // fpm_run_multi alternate; fpm_loss_grad uses the first)
  MultiParams* mpar = nullptr;  // [2] parameter blocks of fpm_run_multi
  int* tile_flags = nullptr;  // [(M/32)^2] HR tiles with possibly non-zero Adam moments
  unsigned* counters = nullptr;  // completion counter of pupil_grad's reduction
  int loss_kind = FPM_LOSS_AMPLITUDE;
  bool timing = false;
  int repeat_kind = -1, repeat_n = 1;   // timing: launches of this kind issued repeat_n times
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> event_pool;
};

namespace {

hipEvent_t pool_event(fpm_plan* p) {
  if (!p->event_pool.empty()) {
    hipEvent_t e = p->event_pool.back();
    p->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events when the plan's timing is on. With a repeat
// set for this kind (fpm_timing_repeat), the launch site issues the kernel
// `reps` times back to back inside the bracket.
// Set while fpm_backward_noalloc runs on this thread: its launches are not
// timed, since recording creates events and grows the record on demand.
thread_local bool g_untimed = false;

struct Timed {
  fpm_plan* p;
  int kind;
  hipStream_t st;
  hipEvent_t start = nullptr;
  int reps = 1;
  Timed(fpm_plan* plan, int k, hipStream_t s) : p(plan), kind(k), st(s) {
    if (g_untimed) return;
    if (p->timing && p->repeat_kind == k) reps = p->repeat_n;
    if (p->timing && p->timed.size() < kMaxTimed) {
      start = pool_event(p);
      if (start && hipEventRecord(start, st) != hipSuccess) start = nullptr;
    }
  }
  ~Timed() {
    if (!start) return;
    hipEvent_t stop = pool_event(p);
    if (stop && hipEventRecord(stop, st) == hipSuccess) {
      p->timed.push_back({kind, reps, start, stop});
    } else {
      p->event_pool.push_back(start);
      if (stop) p->event_pool.push_back(stop);
    }
  }
};

void plan_free(fpm_plan* p) {
  for (auto& t : p->timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (auto e : p->event_pool) (void)hipEventDestroy(e);
  (void)hipFree(p->rowext);
  (void)hipFree(p->twN);
  (void)hipFree(p->twM);
  (void)hipFree(p->X);
  (void)hipFree(p->gacc);
  (void)hipFree(p->gP);
  (void)hipFree(p->kappa_tab);
  (void)hipFree(p->part);
  (void)hipFree(p->staging);
  (void)hipFree(p->part_lg);
  (void)hipFree(p->P_ws);
  (void)hipFree(p->oob_ws);
  (void)hipFree(p->mpar);
  (void)hipFree(p->sub);
  (void)hipFree(p->tile_flags);
  (void)hipFree(p->counters);
  delete p;
}

int check_device(const fpm_plan* p) {
  int dev = -1;
  FPM_HIP(hipGetDevice(&dev));
  if (dev != p->device) return fail(FPM_EINVAL, "current HIP device differs from the plan's device");
  return FPM_OK;
}

PupilGeom pupil_geom(const fpm_plan* p) {
  PupilGeom g;
  g.n = p->N;
  g.inv_r = 1.0 / p->radius;
  g.dk2 = p->dk * p->dk;
  g.inv_l = 1.0 / p->lambda;
  return g;
}

int check_batch(const fpm_plan* p, const int32_t* leds, int32_t B) {
  FPM_REQUIRE(B >= 0, "batch size must be >= 0");
  FPM_REQUIRE(B <= p->max_batch, "batch size exceeds the plan's max_batch");
  FPM_REQUIRE(B == 0 || leds != nullptr, "leds must not be NULL");
  for (int b = 0; b < B; ++b) {
    if (leds[b] < 0 || leds[b] >= p->n_led) {
      char buf[96];
      std::snprintf(buf, sizeof buf, "LED id %d at batch position %d is outside [0, %d)", leds[b],
                    b, p->n_led);
      return fail(FPM_EINVAL, buf);
    }
  }
  return FPM_OK;
}

enum { kCounterPupil = 0, kCounters = 1 };

// LED ids (validated by check_batch) and window corners of one batch, by value.
Batch batch_of(const fpm_plan* p, const int32_t* leds, int B) {
  Batch bt{};
  bt.B = B;
  bt.M = p->M;
  bt.intensity = p->loss_kind == FPM_LOSS_INTENSITY;
  const int base = p->M / 2 - p->N / 2;
  for (int b = 0; b < B; ++b) {
    const int2 s = p->shifts_h[leds[b]];
    bt.led[b] = leds[b];
    bt.win[b] = make_int2(base + s.x, base + s.y);
  }
  return bt;
}

// Validate an LED table (every window inside the HR grid) and find the
// rectangle of 32 x 32 HR tiles that bounds the tiles covered by the pupil disk
// of some window (Adam runs over this rectangle: outside the disks the
// gradient and both moments stay zero, so Adam leaves the spectrum there as
// it is, and a workgroup finds its tile from its index alone).
int led_table(fpm_plan* p, const int32_t* shifts_host, std::vector<int2>& shifts,
              int2& tile0, int& tile_rows, int& tile_cols) {
  const int base = p->M / 2 - p->N / 2;
  shifts.assign(p->n_led, make_int2(0, 0));
  for (int i = 0; i < p->n_led; ++i) {
    const int sr = shifts_host[2 * i], sc = shifts_host[2 * i + 1];
    if (base + sr < 0 || base + sr + p->N > p->M || base + sc < 0 || base + sc + p->N > p->M) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "LED %d: window (%d, %d) leaves the %d x %d HR grid", i, sr,
                    sc, p->M, p->M);
      return fail(FPM_EINVAL, buf);
    }
    shifts[i] = make_int2(sr, sc);
  }
  int r0 = INT_MAX, r1 = -1, c0 = INT_MAX, c1 = -1;
  for (int i = 0; i < p->n_led; ++i) {
    const int2 s = shifts[i];
    for (int ky = p->ky_lo; ky <= p->ky_hi; ++ky) {
      const int row = (base + s.x + ky) / 32;
      r0 = std::min(r0, row);
      r1 = std::max(r1, row);
      c0 = std::min(c0, (base + s.y + p->rowext_h[ky].x) / 32);
      c1 = std::max(c1, (base + s.y + p->rowext_h[ky].y) / 32);
    }
  }
  if (r1 < 0) {   // no LED (or no disk row): no tile
    tile0 = make_int2(0, 0);
    tile_rows = tile_cols = 0;
    return FPM_OK;
  }
  tile0 = make_int2(r0, c0);
  tile_rows = r1 - r0 + 1;
  tile_cols = c1 - c0 + 1;
  return FPM_OK;
}

size_t tile_capacity(const fpm_plan* p) {
  const size_t nt = (size_t)(p->M + 31) / 32;
  return nt * nt;
}


Disk disk_of(const fpm_plan* p) {
  Disk d;
  d.rowext = p->rowext;
  d.ky_lo = p->ky_lo;
  d.ky_hi = p->ky_hi;
  d.nrows = p->nrows;
  d.r2i = (int)std::floor(p->radius * p->radius);
  return d;
}

template <int N> constexpr int row_lines() { return kRowThreads / RowPlan<N>::T; }
// the nearest-pixel backward row pass is counted by row_chunks, which also
// sizes the moment-partial buffers
template <int N> constexpr bool bwd_rows_match() { return BwdRow<N>::threads / BwdRow<N>::T == row_lines<N>(); }
static_assert(bwd_rows_match<64>() && bwd_rows_match<128>() && bwd_rows_match<192>() &&
              bwd_rows_match<256>() && bwd_rows_match<384>() && bwd_rows_match<512>(),
              "rows per workgroup of the backward row pass");

struct Grids {
  int slots, row_chunks, col_groups;
  int fwd_chunks;       // chunks of rows_forward (its own workgroup shape)
  int sub_fwd_chunks;   // chunks of rows_forward_sub (its own workgroup shape)
  int sub_bwd_chunks;   // chunks of rows_backward_sub (its own workgroup size)
  int rows() const { return slots * row_chunks; }
  int fwd_rows() const { return slots * fwd_chunks; }
  int sub_fwd_rows() const { return slots * sub_fwd_chunks; }
  int cols() const { return slots * col_groups; }
  int sub_bwd_rows() const { return slots * sub_bwd_chunks; }
};

template <int N>
Grids grids_of(const fpm_plan* p, int B) {
  Grids g;
  g.slots = (B + kXcds - 1) / kXcds * kXcds;
  g.row_chunks = (p->nrows + row_lines<N>() - 1) / row_lines<N>();
  constexpr int fwd_lines = FwdRow<N>::threads / FwdRow<N>::T;
  g.fwd_chunks = (p->nrows + fwd_lines - 1) / fwd_lines;
  constexpr int sub_fwd_lines = SubFwdRow<N>::threads / SubFwdRow<N>::T;
  g.sub_fwd_chunks = (p->nrows + sub_fwd_lines - 1) / sub_fwd_lines;
  g.col_groups = N / ColLines<N>::value;
  constexpr int sub_lines = SubBwdThreads<N>::value / RowPlan<N>::T;
  g.sub_bwd_chunks = (p->nrows + sub_lines - 1) / sub_lines;
  return g;
}

// What a loss-and-gradient pass produces besides g_O.
struct BackwardOut {
  int mode = kGradO;          // rows_backward mode
  float2* gP = nullptr;       // kGradOP
  bool loss = false;          // column pass stores loss partials in part_loss
  int commit = 0;             // rows_forward commits the staged pupil-parameter state
  ScalarState scal{};
  double* loss_part = nullptr;  // where the column pass stores its loss partials (with loss)
  double* zpart = nullptr;      // where the row pass stores its moment partials (kPatchZern)
  float2* X = nullptr;          // row/column scratch; NULL: the plan's
};

template <int N>
int launch_backward(fpm_plan* p, const float2* O, const float2* P, const int32_t* leds, int B,
                    const float* gamma, const float* A, float2* gO, const BackwardOut& o,
                    hipStream_t st) {
  const Grids gr = grids_of<N>(p, B);
  const Batch bt = batch_of(p, leds, B);
  const Disk dk = disk_of(p);
  float2* X = o.X ? o.X : p->X;
  {
    Timed tm(p, kRowsForward, st);
    for (int r = 0; r < tm.reps; ++r)
      rows_forward<N><<<gr.fwd_rows(), FwdRow<N>::threads, 0, st>>>(O, P, bt, dk, gr.fwd_chunks, X,
                                                           p->twN, o.commit, p->staging, o.scal);
  }
  {
    Timed tm(p, kCols, st);
    for (int r = 0; r < tm.reps; ++r)
      cols<N, false><<<gr.cols(), ColLines<N>::value * ColPlan<N>::T, 0, st>>>(
          X, A, gamma, bt, dk, gr.col_groups, o.loss ? o.loss_part : nullptr, nullptr,
          nullptr, p->twN, 1.0f / p->M);
  }
  {
    Timed tm(p, kRowsBackward, st);
    const PupilGeom pg = pupil_geom(p);
    for (int r = 0; r < tm.reps; ++r) switch (o.mode) {
      case kGradO:
        rows_backward<N, kGradO><<<gr.rows(), BwdRow<N>::threads, 0, st>>>(
            X, O, P, bt, dk, pg, gr.row_chunks, gO, nullptr, nullptr, nullptr, p->twN);
        break;
      case kGradOP:
        rows_backward<N, kGradOP><<<gr.rows(), BwdRow<N>::threads, 0, st>>>(
            X, O, P, bt, dk, pg, gr.row_chunks, gO, o.gP, nullptr, nullptr, p->twN);
        break;
      case kPatch:
        rows_backward<N, kPatch><<<gr.rows(), BwdRow<N>::threads, 0, st>>>(
            X, O, P, bt, dk, pg, gr.row_chunks, nullptr, nullptr, nullptr, nullptr, p->twN);
        break;
      default:
        rows_backward<N, kPatchZern><<<gr.rows(), BwdRow<N>::threads, 0, st>>>(
            X, O, P, bt, dk, pg, gr.row_chunks, nullptr, nullptr, o.zpart, p->kappa_tab,
            p->twN);
        break;
    }
  }
  FPM_HIP(hipGetLastError());
  return FPM_OK;
}

template <int N>
int launch_forward(fpm_plan* p, const float2* O, const float2* P, const int32_t* leds, int B,
                   const float* gamma, float* amp, float2* field, hipStream_t st) {
  const Grids gr = grids_of<N>(p, B);
  const Batch bt = batch_of(p, leds, B);
  const Disk dk = disk_of(p);
  {
    Timed tm(p, kRowsForward, st);
    rows_forward<N><<<gr.fwd_rows(), FwdRow<N>::threads, 0, st>>>(O, P, bt, dk, gr.fwd_chunks, p->X,
                                                         p->twN, 0, nullptr, ScalarState{});
  }
  {
    Timed tm(p, kCols, st);
    cols<N, true><<<gr.cols(), ColLines<N>::value * ColPlan<N>::T, 0, st>>>(
        p->X, nullptr, gamma, bt, dk, gr.col_groups, nullptr, amp, field, p->twN, 1.0f / p->M);
  }
  FPM_HIP(hipGetLastError());
  return FPM_OK;
}

// The step's loss and adjoint in one launch (chain_fused) where an N x N image
// fits one CU's LDS: one workgroup per slot, one loss partial and one set of
// moment partials per slot.
bool fused_chain(const fpm_plan* p) { return p->N == 64; }

template <int N>
int launch_fused(fpm_plan* p, const float2* O, const float2* P, const int32_t* leds, int B,
                 const float* gamma, const float* A, const BackwardOut& o, hipStream_t st) {
  if constexpr (!FusedSupported<N>::value) {
    return fail(FPM_EUNSUPPORTED, "the single-launch chain serves N = 64");
  } else {
    const Batch bt = batch_of(p, leds, B);
    const Disk dk = disk_of(p);
    const PupilGeom pg = pupil_geom(p);
    Timed tm(p, kChainFused, st);
    for (int r = 0; r < tm.reps; ++r) {
      if (o.mode == kPatchZern)
        chain_fused<N, kPatchZern><<<B, Fused<N>::threads, 0, st>>>(
            O, P, A, gamma, bt, dk, pg, p->X, p->twN, p->kappa_tab, o.loss_part, o.zpart,
            1.0f / p->M, o.commit, p->staging, o.scal);
      else
        chain_fused<N, kPatch><<<B, Fused<N>::threads, 0, st>>>(
            O, P, A, gamma, bt, dk, pg, p->X, p->twN, p->kappa_tab, o.loss_part, nullptr,
            1.0f / p->M, o.commit, p->staging, o.scal);
    }
    FPM_HIP(hipGetLastError());
    return FPM_OK;
  }
}

int dispatch_backward(fpm_plan* p, const float2* O, const float2* P, const int32_t* leds, int B,
                      const float* gamma, const float* A, float2* gO, const BackwardOut& o,
                      hipStream_t st) {
  return with_lr_size(p->N, [&](auto n) {
    return launch_backward<decltype(n)::value>(p, O, P, leds, B, gamma, A, gO, o, st);
  });
}

// Grid sizes of the reducing kernels at B = max_batch (sizes the partial buffers).
void reduce_grids(const fpm_plan* p, int& rows_grid, int& cols_grid) {
  with_lr_size(p->N, [&](auto n) {
    const Grids g = grids_of<decltype(n)::value>(p, p->max_batch);
    rows_grid = g.rows();
    cols_grid = g.cols();
    return 0;
  });
}

int rows_grid_of(const fpm_plan* p, int B) {
  return with_lr_size(p->N, [&](auto n) { return grids_of<decltype(n)::value>(p, B).rows(); });
}

int cols_grid_of(const fpm_plan* p, int B) {
  return with_lr_size(p->N, [&](auto n) { return grids_of<decltype(n)::value>(p, B).cols(); });
}

// Group g of a batch of B LEDs: kMaxSlots LEDs from position b0 (the last
// group takes the rest). The groups' partial sums are stored one after the
// other, so the partials of the whole batch form one list of
// rows_grid_of(p, B) (cols_grid_of(p, B)) entries, as for a single launch.
struct Group {
  int b0, B, rows_off, cols_off;
};

int n_groups(int B) { return (B + kMaxSlots - 1) / kMaxSlots; }

Group group_of(const fpm_plan* p, int B, int g) {
  Group r;
  r.b0 = g * kMaxSlots;
  r.B = std::min(kMaxSlots, B - r.b0);
  r.rows_off = g * rows_grid_of(p, kMaxSlots);
  r.cols_off = g * cols_grid_of(p, kMaxSlots);
  return r;
}

// Workgroup slots of the pupil part of the update kernels (the kernels derive
// the same count).
int pupil_wgs(const fpm_plan* p) { return pupil_wg_slots(p->N, p->nrows); }

GeomArgs geom_args(const fpm_plan* p, const fpm_led_grid* grid) {
  GeomArgs ga;
  ga.n_side = grid->n_side;
  ga.pitch_mm = grid->pitch_mm;
  ga.height_mm = grid->height_mm;
  ga.roi_x_mm = grid->roi_x_mm;
  ga.roi_y_mm = grid->roi_y_mm;
  ga.base_dx = grid->shift_x_mm;
  ga.base_dy = grid->shift_y_mm;
  ga.base_rot = grid->rot_rad;
  ga.base_dh = grid->dh_mm;
  ga.inv_dk = 1.0 / p->dk;
  ga.lambda = p->lambda;
  ga.N = p->N;
  ga.M = p->M;
  return ga;
}

template <int N>
int launch_loss_grad(fpm_plan* p, const fpm_led_grid* grid, const fpm_params* pr,
                     const int32_t* leds, int B, const float* A, fpm_grads* gr, hipStream_t st) {
  const Grids g = grids_of<N>(p, B);
  const Batch bt = batch_of(p, leds, B);
  const Disk dk = disk_of(p);
  const PupilGeom pg = pupil_geom(p);
  {
    Timed tm(p, kPupilBuild, st);
    pupil_build<<<(p->N * p->N + 255) / 256, 256, 0, st>>>(pg, p->rowext, pr->coeffs,
                                                             pr->coeffs ? kZern : 0, pr->z_um,
                                                             p->P_ws);
  }
  const GeomArgs ga = geom_args(p, grid);
  const float2* O = reinterpret_cast<const float2*>(pr->O);
  double* col_part = p->part_lg;
  double* row_part = p->part_lg + (size_t)g.cols() * 2;
  {
    Timed tm(p, kRowsForward, st);
    rows_forward_sub<N><<<g.sub_fwd_rows(), SubFwdRow<N>::threads, 0, st>>>(
        O, p->P_ws, bt, dk, ga, pr->geom, gr->oob, p->sub, nullptr, g.sub_fwd_chunks, p->X,
                                                          p->twN);
  }
  {
    Timed tm(p, kCols, st);
    cols<N, false, true><<<g.cols(), ColLines<N>::value * ColPlan<N>::T, 0, st>>>(
        p->X, A, pr->gamma, bt, dk, g.col_groups, col_part, nullptr, nullptr, p->twN,
        1.0f / p->M);
  }
  {
    Timed tm(p, kRowsBackward, st);
    rows_backward_sub<N><<<g.sub_bwd_rows(), SubBwdThreads<N>::value, 0, st>>>(
        p->X, O, p->P_ws, bt, dk, pg, p->sub, g.sub_bwd_chunks, row_part, p->kappa_tab,
        p->twN);
  }
  if (gr->g_O) {
    Timed tm(p, kAdamObject, st);
    gather_dense<N><<<(p->M / 32) * (p->M / 32), 256, 0, st>>>(
        p->X, bt, dk, p->sub, reinterpret_cast<float2*>(gr->g_O));
  }
  ReduceArgs ra;
  ra.col_part = col_part;
  ra.col_wgs = g.cols();
  ra.col_chunks = g.col_groups;
  ra.row_part = row_part;
  ra.row_wgs = g.sub_bwd_rows();
  ra.row_chunks = g.sub_bwd_chunks;
  ra.sub = p->sub;
  ra.bt = bt;
  ra.gamma = pr->gamma;
  ra.loss = gr->loss;
  ra.g_par = gr->g_par;
  ra.g_geom = pr->geom ? gr->g_geom : nullptr;
  ra.g_gamma = gr->g_gamma;
  loss_grad_reduce<<<1, 256, 0, st>>>(ra);
  FPM_HIP(hipGetLastError());
  return FPM_OK;
}

static_assert(sizeof(MultiUpdateArgs) <= 4096, "kernel arguments are limited to 4 KiB");
static_assert(sizeof(UpdateArgs) <= 4096, "kernel arguments are limited to 4 KiB");

// One fused multi-parameter step: parameters of this step in block `cur`,
// the next ones written to `next`. The batch's slot offsets live in sub_cur:
// derived there by the forward row pass, or (pre) already by the previous
// step's update kernel, which likewise derives the next batch's (leds_next,
// B_next) into sub_next when there is a next step in this call.
template <int N>
int launch_multi_step(fpm_plan* p, const GeomArgs& ga, fpm_state* s, const fpm_geometry* geo,
                      const fpm_hparams* hp, const int32_t* leds, int B, const float* A,
                      MultiParams* cur, MultiParams* next, SubSlot* sub_cur, bool pre,
                      SubSlot* sub_next, const int32_t* leds_next, int B_next, hipStream_t st) {
  const Grids g = grids_of<N>(p, B);
  const Batch bt = batch_of(p, leds, B);
  const Disk dk = disk_of(p);
  const PupilGeom pg = pupil_geom(p);
  const float2* O = reinterpret_cast<const float2*>(s->O);
  float2* P = reinterpret_cast<float2*>(s->P);
  double* col_part = p->part_lg;
  double* row_part = p->part_lg + (size_t)g.cols() * 2;
  const double* geom = cur->g;
  {
    Timed tm(p, kRowsForward, st);
    for (int r = 0; r < tm.reps; ++r)
      rows_forward_sub<N><<<g.sub_fwd_rows(), SubFwdRow<N>::threads, 0, st>>>(
          O, P, bt, dk, ga, geom, p->oob_ws, sub_cur, pre ? sub_cur : nullptr, g.sub_fwd_chunks,
          p->X, p->twN);
  }
  {
    Timed tm(p, kCols, st);
    for (int r = 0; r < tm.reps; ++r)
      cols<N, false><<<g.cols(), ColLines<N>::value * ColPlan<N>::T, 0, st>>>(
          p->X, A, nullptr, bt, dk, g.col_groups, col_part, nullptr, nullptr, p->twN,
          1.0f / p->M);
  }
  {
    Timed tm(p, kRowsBackward, st);
    for (int r = 0; r < tm.reps; ++r)
      rows_backward_sub<N><<<g.sub_bwd_rows(), SubBwdThreads<N>::value, 0, st>>>(
          p->X, O, P, bt, dk, pg, sub_cur, g.sub_bwd_chunks, row_part, p->kappa_tab, p->twN);
  }
  const int t = s->t + 1;
  const double b1 = hp->beta1, b2 = hp->beta2;
  const double bc1 = 1.0 - std::pow(b1, t), bc2 = 1.0 - std::pow(b2, t);
  MultiUpdateArgs a{};
  a.M = p->M;
  a.tile_flags = p->tile_flags;
  a.O = reinterpret_cast<float*>(s->O);
  a.mO = reinterpret_cast<float*>(s->m_O);
  a.vO = reinterpret_cast<float*>(s->v_O);
  a.c.b1 = hp->beta1;
  a.c.b2 = hp->beta2;
  a.c.eps = hp->eps;
  a.c.step_size = (float)(hp->lr_object / bc1);
  a.c.sqrt_bc2 = (float)std::sqrt(bc2);
  a.X = p->X;
  a.bt = bt;
  a.dk = dk;
  a.sub = sub_cur;
  a.next_sub = sub_next;
  if (sub_next) a.bt_next = batch_of(p, leds_next, B_next);
  a.ga = ga;
  a.loss_part = col_part;
  a.n_loss = g.cols();
  a.loss = s->loss;
  a.row_part = row_part;
  a.n_rows = g.sub_bwd_rows();
  a.row_chunks = g.sub_bwd_chunks;
  a.cur = cur;
  a.next = next;
  a.sa.learn_c = hp->learn_zernike;
  a.sa.learn_z = hp->learn_z;
  a.sa.lr_c = hp->lr_zernike;
  a.sa.lr_z = hp->lr_z;
  a.sa.b1 = b1;
  a.sa.b2 = b2;
  a.sa.eps = hp->eps;
  a.sa.bc1 = bc1;
  a.sa.sqrt_bc2 = std::sqrt(bc2);
  a.learn_geom = geo->learn;
  a.lr_geom[0] = geo->lr_shift_mm;
  a.lr_geom[1] = geo->lr_shift_mm;
  a.lr_geom[2] = geo->lr_rot_rad;
  a.lr_geom[3] = geo->lr_height_mm;
  a.g_par = s->g_par;
  a.g_geom = geo->g_geom;
  a.pg = pg;
  a.P = P;
  const int grid = pupil_wgs(p) + (p->M / 32) * (p->M / 32);
  {
    Timed tm(p, kAdamObject, st);
    for (int r = 0; r < tm.reps; ++r) update_multi<N><<<grid, 256, 0, st>>>(a);
  }
  FPM_HIP(hipGetLastError());
  s->t = t;
  return FPM_OK;
}

// The batch slots that meet each tile row and tile column of the Adam
// rectangle (a slot meets a row of tiles when its window's disk rows overlap
// the row's 32 HR rows; columns alike): a tile's slots are the AND of its row's
// and its column's masks, the bounding-box test of the window's disk.
void tile_masks(const fpm_plan* p, UpdateArgs& a) {
  const int cols = p->tile_cols, rows = cols > 0 ? p->n_tiles / cols : 0;
  for (int i = 0; i < rows && i < kMaxTileSide; ++i) {
    const int lo = 32 * (p->tile0.x + i), hi = lo + 31;
    unsigned long long m = 0ull;
    for (int b = 0; b < a.bt.B; ++b) {
      const int wr = a.bt.win[b].x;
      if (!(hi < wr + p->ky_lo || lo > wr + p->ky_hi)) m |= 1ull << b;
    }
    a.hit_row[i] = m;
  }
  for (int j = 0; j < cols && j < kMaxTileSide; ++j) {
    const int lo = 32 * (p->tile0.y + j), hi = lo + 31;
    unsigned long long m = 0ull;
    for (int b = 0; b < a.bt.B; ++b) {
      const int wc = a.bt.win[b].y;
      if (!(hi < wc + p->ky_lo || lo > wc + p->ky_hi)) m |= 1ull << b;
    }
    a.hit_col[j] = m;
  }
}

int launch_update(fpm_plan* p, const UpdateArgs& a, int grid, hipStream_t st) {
  if (int rc = with_lr_size(p->N, [&](auto n) {
        update<decltype(n)::value><<<grid, 256, 0, st>>>(a);
        return 0;
      }))
    return rc;
  FPM_HIP(hipGetLastError());
  return FPM_OK;
}

template <int M>
int launch_hr(fpm_plan* p, HrArgs a, int row_mode, int dir, int batch, hipStream_t st) {
  constexpr int Lr = HrRowLines<M>::value;
  constexpr int Lc = HrColLines<M>::value;
  constexpr int T = Plan1D<M>::T;
  const dim3 gr(M / Lr, batch), gc(M / Lc, batch);
  {
  Timed tm(p, kHrRows, st);
  switch (row_mode) {
    case kRowFwd: hr_rows<M, kRowFwd><<<gr, Lr * T, 0, st>>>(a, p->twM); break;
    case kRowInv: hr_rows<M, kRowInv><<<gr, Lr * T, 0, st>>>(a, p->twM); break;
    case kRowInit: hr_rows<M, kRowInit><<<gr, Lr * T, 0, st>>>(a, p->twM); break;
    case kRowRefocus: hr_rows<M, kRowRefocus><<<gr, Lr * T, 0, st>>>(a, p->twM); break;
  }
  }
  Timed tm(p, kHrCols, st);
  if (dir < 0)
    hr_cols<M, -1><<<gc, Lc * T, 0, st>>>(a.out, p->twM);
  else
    hr_cols<M, +1><<<gc, Lc * T, 0, st>>>(a.out, p->twM);
  FPM_HIP(hipGetLastError());
  return FPM_OK;
}

// batch > 1 only with kRowRefocus (one distance per transform).
int dispatch_hr(fpm_plan* p, HrArgs a, int row_mode, int dir, hipStream_t st, int batch = 1) {
  switch (p->M) {
    case 256: return launch_hr<256>(p, a, row_mode, dir, batch, st);
    case 512: return launch_hr<512>(p, a, row_mode, dir, batch, st);
    case 768: return launch_hr<768>(p, a, row_mode, dir, batch, st);
    case 1024: return launch_hr<1024>(p, a, row_mode, dir, batch, st);
    case 1536: return launch_hr<1536>(p, a, row_mode, dir, batch, st);
    case 2048: return launch_hr<2048>(p, a, row_mode, dir, batch, st);
  }
  return fail(FPM_EUNSUPPORTED, kHrSizes);
}

}  // namespace

extern "C" {

const char* fpm_strerror(int code) {
  switch (code) {
    case FPM_OK: return "ok";
    case FPM_EINVAL: return "invalid argument";
    case FPM_ENOMEM: return "out of device memory";
    case FPM_EHIP: return "HIP runtime error";
    case FPM_EUNSUPPORTED: return "unsupported size";
    case FPM_ENONFINITE: return "non-finite loss";
  }
  return "unknown error";
}

const char* fpm_last_error(void) { return g_last_error.c_str(); }

#ifndef FPM_BUILD_TAG
#error "FPM_BUILD_TAG (a digest of the sources) is set by the build"
#endif
const char* fpm_build_tag(void) { return FPM_BUILD_TAG; }

int fpm_plan_create(const fpm_desc* d, const int32_t* shifts_host, fpm_plan** out) {
  return guarded([&]() -> int {
    FPM_REQUIRE(d && shifts_host && out, "desc, shifts_host and plan must not be NULL");
    *out = nullptr;
    if (!lr_supported(d->n_lr)) return fail(FPM_EUNSUPPORTED, "n_lr must be 64, 128, 192, 256, 384 or 512");
    FPM_REQUIRE(d->upsample >= 1 && (int64_t)d->upsample * d->n_lr <= 4096, "upsample out of range");
    FPM_REQUIRE(d->n_led >= 1 && d->max_batch >= 1, "n_led and max_batch must be >= 1");
    FPM_REQUIRE(d->max_batch <= kMaxBatch, "max_batch must be <= 1024");
    FPM_REQUIRE(d->wavelength_um > 0 && d->na > 0 && d->mag > 0 && d->pixel_um > 0,
                "optics must be positive");
    fpm_plan* p = new fpm_plan();
    FPM_HIP(hipGetDevice(&p->device));
    p->N = d->n_lr;
    p->s = d->upsample;
    p->M = d->n_lr * d->upsample;
    p->n_led = d->n_led;
    p->max_batch = d->max_batch;
    p->lambda = d->wavelength_um;
    p->na = d->na;
    p->mag = d->mag;
    p->pixel = d->pixel_um;
    const double dx = d->pixel_um / d->mag;
    p->dk = 1.0 / (p->N * dx);
    p->radius = d->na / d->wavelength_um / p->dk;
    if (!(p->radius < p->N / 2 - 1)) {
      delete p;
      return fail(FPM_EINVAL, "pupil disk does not fit the N x N pupil grid");
    }
    // pupil disk: |u|^2 <= R^2, per-row column extents
    std::vector<int2> ext(p->N);
    const double r2 = p->radius * p->radius;
    for (int ky = 0; ky < p->N; ++ky) {
      const double uy = ky - p->N / 2;
      int lo = p->N, hi = -1;
      for (int kx = 0; kx < p->N; ++kx) {
        const double ux = kx - p->N / 2;
        if (uy * uy + ux * ux <= r2) {
          lo = std::min(lo, kx);
          hi = std::max(hi, kx);
          ++p->support_px;
        }
      }
      ext[ky] = make_int2(lo, hi);
      if (hi >= lo) {
        if (p->nrows == 0) p->ky_lo = ky;
        p->ky_hi = ky;
        ++p->nrows;
      }
    }
    // LED table and the rectangle of HR tiles its windows touch
    p->rowext_h = ext;
    int tile_rows = 0;
    if (int rc = led_table(p, shifts_host, p->shifts_h, p->tile0, tile_rows, p->tile_cols)) {
      delete p;
      return rc;
    }
    p->n_tiles = tile_rows * p->tile_cols;
    p->hr_ok = hr_supported(p->M);

    // kappa(|u|^2) = 2 pi (sqrt(1/l^2 - k^2) - 1/l), k^2 = |u|^2 dk^2, cancellation-free form
    std::vector<float> kap((size_t)std::floor(r2) + 1);
    for (size_t q = 0; q < kap.size(); ++q) {
      const double k2 = (double)q * p->dk * p->dk, il = 1.0 / p->lambda;
      kap[q] = (float)(-2.0 * M_PI * k2 / (std::sqrt(il * il - k2) + il));
    }
    int rc = FPM_OK;
    const auto twn = twiddles(p->N);
    if ((rc = upload(&p->device_bytes, &p->rowext, ext.data(), ext.size())) ||
        (rc = upload(&p->device_bytes, &p->twN, twn.data(), twn.size())) ||
        (rc = upload<float2>(&p->device_bytes, &p->X, nullptr,
                             (size_t)std::min(p->max_batch, kMaxSlots) * p->N * p->N)) ||
        (p->max_batch > kMaxSlots &&
         (rc = upload<float2>(&p->device_bytes, &p->gacc, nullptr, (size_t)p->M * p->M))) ||
        (rc = upload<float2>(&p->device_bytes, &p->gP, nullptr, (size_t)p->N * p->N)) ||
        (rc = upload(&p->device_bytes, &p->kappa_tab, kap.data(), kap.size()))) {
      plan_free(p);
      return rc;
    }
    int rows_grid = 0, cols_grid = 0;
    reduce_grids(p, rows_grid, cols_grid);
    const int pg_grid = (p->N * p->N + 255) / 256;
    const size_t n_part = (size_t)cols_grid + (size_t)rows_grid * kPar + (size_t)pg_grid * kPar;
    if ((rc = upload<double>(&p->device_bytes, &p->part, nullptr, n_part)) ||
        (rc = upload<float>(&p->device_bytes, &p->staging, nullptr, kScal)) ||
        (rc = upload<unsigned>(&p->device_bytes, &p->counters, nullptr, kCounters))) {
      plan_free(p);
      return rc;
    }
    if ((rc = upload<double>(&p->device_bytes, &p->part_lg, nullptr, (size_t)cols_grid * 2 + (size_t)rows_grid * kSubPar)) ||
        (rc = upload<float2>(&p->device_bytes, &p->P_ws, nullptr, (size_t)p->N * p->N)) ||
        (rc = upload<int>(&p->device_bytes, &p->oob_ws, nullptr, 1)) ||
        (rc = upload<MultiParams>(&p->device_bytes, &p->mpar, nullptr, 2)) ||
        (rc = upload<SubSlot>(&p->device_bytes, &p->sub, nullptr, 2 * (size_t)p->max_batch)) ||
        (rc = upload<int>(&p->device_bytes, &p->tile_flags, nullptr, tile_capacity(p)))) {
      plan_free(p);
      return rc;
    }
    p->part_loss = p->part;
    p->part_z = p->part + cols_grid;
    p->part_pg = p->part_z + (size_t)rows_grid * kPar;
    if (hipMemset(p->counters, 0, kCounters * sizeof(unsigned)) != hipSuccess) {
      plan_free(p);
      return fail(FPM_EHIP, "hipMemset failed");
    }
    if (p->hr_ok) {
      const auto twm = twiddles(p->M);
      if ((rc = upload(&p->device_bytes, &p->twM, twm.data(), twm.size()))) {
        plan_free(p);
        return rc;
      }
    }
    if (hipMemset(p->gP, 0, (size_t)p->N * p->N * sizeof(float2)) != hipSuccess) {
      plan_free(p);
      return fail(FPM_EHIP, "hipMemset failed");
    }
    *out = p;
    return FPM_OK;
  });
}

int fpm_plan_destroy(fpm_plan* p) {
  if (!p) return FPM_OK;
  plan_free(p);
  return FPM_OK;
}

int fpm_plan_set_shifts(fpm_plan* p, const int32_t* shifts_host, void* stream) {
  return guarded([&]() -> int {
    FPM_REQUIRE(p && shifts_host, "plan and shifts_host must not be NULL");
    if (int rc = check_device(p)) return rc;
    std::vector<int2> shifts;
    int2 tile0;
    int tile_rows = 0, tile_cols = 0;
    if (int rc = led_table(p, shifts_host, shifts, tile0, tile_rows, tile_cols)) return rc;
    (void)stream;   // nothing is uploaded: the table and the rectangle are launch arguments
    p->shifts_h = std::move(shifts);
    p->tile0 = tile0;
    p->tile_cols = tile_cols;
    p->n_tiles = tile_rows * tile_cols;
    return FPM_OK;
  });
}

int fpm_plan_set_loss(fpm_plan* p, int32_t kind) {
  FPM_REQUIRE(p, "plan must not be NULL");
  FPM_REQUIRE(kind == FPM_LOSS_AMPLITUDE || kind == FPM_LOSS_INTENSITY,
              "kind must be FPM_LOSS_AMPLITUDE or FPM_LOSS_INTENSITY");
  p->loss_kind = kind;
  return FPM_OK;
}

int fpm_plan_info(const fpm_plan* p, fpm_info* info) {
  FPM_REQUIRE(p && info, "plan and info must not be NULL");
  info->n_lr = p->N;
  info->m_hr = p->M;
  info->n_led = p->n_led;
  info->max_batch = p->max_batch;
  info->support_px = p->support_px;
  info->support_rows = p->nrows;
  info->adam_tiles = p->n_tiles;
  info->pupil_radius_px = p->radius;
  info->dk = p->dk;
  info->device_bytes = (int64_t)p->device_bytes;
  info->fused_chain = fused_chain(p) ? 1 : 0;
  return FPM_OK;
}

int fpm_led_shifts(const fpm_desc* d, const fpm_led_grid* g, double* k_out, double* s_out,
                   int32_t* nearest_out) {
  FPM_REQUIRE(d && g, "desc and grid must not be NULL");
  FPM_REQUIRE(g->n_side >= 1 && d->n_lr >= 1, "n_side and n_lr must be >= 1");
  FPM_REQUIRE(d->wavelength_um > 0 && d->mag > 0 && d->pixel_um > 0, "optics must be positive");
  const double dk = 1.0 / (d->n_lr * (d->pixel_um / d->mag));
  const double c = (g->n_side - 1) / 2.0;
  const double cr = std::cos(g->rot_rad), sr = std::sin(g->rot_rad);
  for (int row = 0; row < g->n_side; ++row) {
    for (int col = 0; col < g->n_side; ++col) {
      const double i = col - c, j = row - c;
      const double x = g->pitch_mm * (i * cr - j * sr) + g->shift_x_mm - g->roi_x_mm;
      const double y = g->pitch_mm * (i * sr + j * cr) + g->shift_y_mm - g->roi_y_mm;
      const double h = g->height_mm + g->dh_mm;
      const double dist = std::sqrt(x * x + y * y + h * h);
      const double ky = y / dist / d->wavelength_um, kx = x / dist / d->wavelength_um;
      const int led = row * g->n_side + col;
      if (k_out) { k_out[2 * led] = ky; k_out[2 * led + 1] = kx; }
      if (s_out) { s_out[2 * led] = ky / dk; s_out[2 * led + 1] = kx / dk; }
      if (nearest_out) {
        nearest_out[2 * led] = (int32_t)std::floor(ky / dk + 0.5);
        nearest_out[2 * led + 1] = (int32_t)std::floor(kx / dk + 0.5);
      }
    }
  }
  return FPM_OK;
}

int fpm_pupil(fpm_plan* p, const float* coeffs, int32_t n_zern, const float* z_um,
              fpm_c32* P_out, void* stream) {
  FPM_REQUIRE(p && P_out, "plan and P_out must not be NULL");
  FPM_REQUIRE(n_zern >= 0 && n_zern <= kZern, "n_zern must be in [0, 15]");
  if (int rc = check_device(p)) return rc;
  const int nn = p->N * p->N;
  Timed tm(p, kPupilBuild, (hipStream_t)stream);
  pupil_build<<<(nn + 255) / 256, 256, 0, (hipStream_t)stream>>>(
      pupil_geom(p), p->rowext, coeffs, n_zern, z_um, reinterpret_cast<float2*>(P_out));
  FPM_HIP(hipGetLastError());
  return FPM_OK;
}

int fpm_forward(fpm_plan* p, const fpm_c32* O, const fpm_c32* P, const int32_t* leds, int32_t B,
                const float* gamma, float* amp_out, fpm_c32* field_out, void* stream) {
  FPM_REQUIRE(p && O && P && amp_out, "plan, O, P and amp_out must not be NULL");
  if (int rc = check_batch(p, leds, B)) return rc;
  if (int rc = check_device(p)) return rc;
  if (B == 0) return FPM_OK;
  const auto* o = reinterpret_cast<const float2*>(O);
  const auto* pp = reinterpret_cast<const float2*>(P);
  auto* f = reinterpret_cast<float2*>(field_out);
  hipStream_t st = (hipStream_t)stream;
  const size_t nn = (size_t)p->N * p->N;
  for (int g = 0; g < n_groups(B); ++g) {
    const Group gr = group_of(p, B, g);
    if (int rc = with_lr_size(p->N, [&](auto n) {
          return launch_forward<decltype(n)::value>(p, o, pp, leds + gr.b0, gr.B, gamma,
                                                    amp_out + gr.b0 * nn,
                                                    f ? f + gr.b0 * nn : nullptr, st);
        }))
      return rc;
  }
  return FPM_OK;
}

int fpm_backward(fpm_plan* p, const fpm_c32* O, const fpm_c32* P, const int32_t* leds, int32_t B,
                 const float* gamma, const float* meas_amp, fpm_c32* gO, fpm_c32* gP,
                 double* loss, void* stream) {
  FPM_REQUIRE(p && O && P && meas_amp && gO, "plan, O, P, meas_amp and gO must not be NULL");
  if (int rc = check_batch(p, leds, B)) return rc;
  if (int rc = check_device(p)) return rc;
  if (B == 0) return FPM_OK;
  BackwardOut o;
  o.mode = gP ? kGradOP : kGradO;
  o.gP = reinterpret_cast<float2*>(gP);
  o.loss = loss != nullptr;
  hipStream_t st = (hipStream_t)stream;
  for (int g = 0; g < n_groups(B); ++g) {
    const Group gr = group_of(p, B, g);
    o.loss_part = p->part_loss + gr.cols_off;
    if (int rc = dispatch_backward(p, reinterpret_cast<const float2*>(O),
                                   reinterpret_cast<const float2*>(P), leds + gr.b0, gr.B, gamma,
                                   meas_amp, reinterpret_cast<float2*>(gO), o, st))
      return rc;
  }
  if (loss) {   // add the column pass's partials (fixed order)
    UpdateArgs a{};
    a.n = p->N;
    a.loss_part = p->part_loss;
    a.n_loss = cols_grid_of(p, B);
    a.loss = loss;
    Timed tm(p, kAdamObject, st);
    if (int rc = launch_update(p, a, 1, st)) return rc;
  }
  return FPM_OK;
}

}  // extern "C"

namespace {

// Scratch of fpm_backward_noalloc, in a file-scope device array instead of the
// plan's allocations: the row/column intermediate X (kNoAllocXBytes) followed by
// the column pass's loss partials (kNoAllocPartBytes). Each device the library
// runs on holds its own copy from module load to process exit; its host-side
// name is only a stand-in, so host code uses the device address that
// hipGetSymbolAddress returns, looked up once per device.
constexpr size_t kNoAllocXBytes = size_t(16) << 20;
constexpr size_t kNoAllocPartBytes = size_t(256) << 10;
__device__ __align__(256) unsigned char scratch[kNoAllocXBytes + kNoAllocPartBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch (the current device), or an error.
int scratch_of(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FPM_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FPM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch[dev]);
  return FPM_OK;
}

}  // namespace

extern "C" {

int fpm_backward_noalloc(fpm_plan* p, const fpm_c32* O, const fpm_c32* P, const int32_t* leds,
                         int32_t B, const float* gamma, const float* meas_amp, fpm_c32* gO,
                         fpm_c32* gP, double* loss, void* stream) {
  return guarded([&]() -> int {
    FPM_REQUIRE(p && O && P && meas_amp && gO, "plan, O, P, meas_amp and gO must not be NULL");
    if (int rc = check_batch(p, leds, B)) return rc;
    if (int rc = check_device(p)) return rc;
    const size_t x_bytes = (size_t)std::min(B, kMaxSlots) * p->N * p->N * sizeof(float2);
    const size_t part_bytes = (size_t)cols_grid_of(p, B) * sizeof(double);
    if (x_bytes > kNoAllocXBytes || part_bytes > kNoAllocPartBytes) {
      char buf[200];
      std::snprintf(buf, sizeof buf,
                    "batch of %d at N = %d needs %zu + %zu bytes of scratch; the allocation-free "
                    "entry point has %zu + %zu",
                    B, p->N, x_bytes, part_bytes, kNoAllocXBytes, kNoAllocPartBytes);
      return fail(FPM_EINVAL, buf);
    }
    if (B == 0) return FPM_OK;
    unsigned char* base = nullptr;
    if (int rc = scratch_of(p->device, &base)) return rc;
    struct Untimed {   // no timing events: they would be created on demand
      Untimed() { g_untimed = true; }
      ~Untimed() { g_untimed = false; }
    } untimed;
    double* part = reinterpret_cast<double*>(base + kNoAllocXBytes);
    BackwardOut o;
    o.mode = gP ? kGradOP : kGradO;
    o.gP = reinterpret_cast<float2*>(gP);
    o.loss = loss != nullptr;
    o.X = reinterpret_cast<float2*>(base);
    hipStream_t st = (hipStream_t)stream;
    for (int g = 0; g < n_groups(B); ++g) {
      const Group gr = group_of(p, B, g);
      o.loss_part = part + gr.cols_off;
      if (int rc = dispatch_backward(p, reinterpret_cast<const float2*>(O),
                                     reinterpret_cast<const float2*>(P), leds + gr.b0, gr.B,
                                     gamma, meas_amp, reinterpret_cast<float2*>(gO), o, st))
        return rc;
    }
    if (loss) {   // add the column pass's partials (fixed order)
      UpdateArgs a{};
      a.n = p->N;
      a.loss_part = part;
      a.n_loss = cols_grid_of(p, B);
      a.loss = loss;
      if (int rc = launch_update(p, a, 1, st)) return rc;
    }
    return FPM_OK;
  });
}

int fpm_pupil_grad(fpm_plan* p, const fpm_c32* gP, const fpm_c32* P, double* g_par,
                   void* stream) {
  FPM_REQUIRE(p && gP && P && g_par, "plan, gP, P and g_par must not be NULL");
  if (int rc = check_device(p)) return rc;
  const int nn = p->N * p->N;
  Timed tm(p, kPupilGrad, (hipStream_t)stream);
  pupil_grad<<<(nn + 255) / 256, 256, 0, (hipStream_t)stream>>>(
      pupil_geom(p), p->rowext, reinterpret_cast<const float2*>(gP),
      reinterpret_cast<const float2*>(P), Reduction{p->part_pg, p->counters + kCounterPupil},
      g_par);
  FPM_HIP(hipGetLastError());
  return FPM_OK;
}

}  // extern "C"

namespace {

int check_state(fpm_plan* p, const fpm_state* s, const fpm_hparams* hp, const float* meas_amp) {
  FPM_REQUIRE(p && s && hp, "plan, state and hparams must not be NULL");
  FPM_REQUIRE(s->O && s->m_O && s->v_O && s->P && meas_amp,
              "state O, m_O, v_O, P and meas_amp must not be NULL");
  if (hp->learn_zernike) FPM_REQUIRE(s->coeffs && s->m_c && s->v_c, "Zernike state must not be NULL");
  if (hp->learn_z) FPM_REQUIRE(s->z_um && s->m_z && s->v_z, "defocus state must not be NULL");
  FPM_REQUIRE(s->t >= 0, "t must be >= 0");
  return check_device(p);
}

ScalarState scalar_state_of(const fpm_state* s) {
  ScalarState d;
  d.coeffs = s->coeffs; d.m_c = s->m_c; d.v_c = s->v_c;
  d.z = s->z_um; d.m_z = s->m_z; d.v_z = s->v_z;
  return d;
}

// One update: loss and gradients of the batch (projected onto the pupil
// parameters when they are learned), then the update kernel (Adam on the
// spectrum; Adam on the pupil parameters and the pupil rebuilt from them).
// A batch of more than kMaxSlots LEDs runs its passes group by group; every
// group but the last ends with an accumulating launch of the update kernel
// (gradient sums into gacc), the last one with the full update.
// `commit`: the previous step of this call staged a pupil-parameter state.
int step_launches(fpm_plan* p, fpm_state* s, const fpm_hparams* hp, const int32_t* leds, int B,
                  const float* gamma, const float* meas_amp, int commit, hipStream_t st) {
  const bool learn_c = hp->learn_zernike != 0, learn_z = hp->learn_z != 0;
  const bool learn_p = learn_c || learn_z;
  const int t = s->t + 1;
  const double b1 = hp->beta1, b2 = hp->beta2;
  const double bc1 = 1.0 - std::pow(b1, t), bc2 = 1.0 - std::pow(b2, t);
  float2* P = reinterpret_cast<float2*>(s->P);
  const bool fused = fused_chain(p);
  const int G = n_groups(B);
  for (int g = 0; g < G; ++g) {
    const Group gr = group_of(p, B, g);
    const bool last = g == G - 1;
    BackwardOut o;
    o.mode = learn_p ? kPatchZern : kPatch;
    o.loss = s->loss != nullptr;
    o.commit = commit && g == 0;
    o.scal = scalar_state_of(s);
    if (fused) {
      o.loss_part = p->part_loss + gr.b0;
      o.zpart = p->part_z + (size_t)gr.b0 * kPar;
      if (int rc = with_lr_size(p->N, [&](auto n) {
            return launch_fused<decltype(n)::value>(p, reinterpret_cast<const float2*>(s->O), P,
                                                    leds + gr.b0, gr.B, gamma, meas_amp, o, st);
          }))
        return rc;
    } else {
      o.loss_part = p->part_loss + gr.cols_off;
      o.zpart = p->part_z + (size_t)gr.rows_off * kPar;
      if (int rc = dispatch_backward(p, reinterpret_cast<const float2*>(s->O), P, leds + gr.b0,
                                     gr.B, gamma, meas_amp, nullptr, o, st))
        return rc;
    }
    UpdateArgs a{};
    a.X = p->X;
    a.bt = batch_of(p, leds + gr.b0, gr.B);
    a.dk = disk_of(p);
    a.n = p->N;
    a.tile0 = p->tile0;
    a.tile_cols = p->tile_cols;
    a.M = p->M;
    tile_masks(p, a);
    a.gacc = reinterpret_cast<float*>(p->gacc);
    a.acc_in = g > 0;
    a.acc_out = !last;
    if (last) {
      a.O = reinterpret_cast<float*>(s->O);
      a.mO = reinterpret_cast<float*>(s->m_O);
      a.vO = reinterpret_cast<float*>(s->v_O);
      a.c.b1 = hp->beta1;
      a.c.b2 = hp->beta2;
      a.c.eps = hp->eps;
      a.c.step_size = (float)(hp->lr_object / bc1);
      a.c.sqrt_bc2 = (float)std::sqrt(bc2);
      a.loss_part = p->part_loss;
      a.n_loss = fused ? B : cols_grid_of(p, B);
      a.loss = s->loss;
      a.pupil = learn_p;
      a.zpart = p->part_z;
      a.n_zpart = fused ? B : rows_grid_of(p, B);
      a.cur = o.scal;
      a.sa.learn_c = learn_c;
      a.sa.learn_z = learn_z;
      a.sa.lr_c = hp->lr_zernike;
      a.sa.lr_z = hp->lr_z;
      a.sa.b1 = b1;
      a.sa.b2 = b2;
      a.sa.eps = hp->eps;
      a.sa.bc1 = bc1;
      a.sa.sqrt_bc2 = std::sqrt(bc2);
      a.g_par = s->g_par;
      a.staging = p->staging;
      a.pg = pupil_geom(p);
      a.rowext = p->rowext;
      a.P = P;
    }
    const int extra = a.pupil ? pupil_wgs(p) : 1;   // must match the kernel's n_pw
    {
      Timed tm(p, kAdamObject, st);
      for (int r = 0; r < tm.reps; ++r)
        if (int rc = launch_update(p, a, p->n_tiles + extra, st)) return rc;
    }
  }
  FPM_HIP(hipGetLastError());
  s->t = t;
  return FPM_OK;
}

int commit_launch(fpm_plan* p, const fpm_state* s, hipStream_t st) {
  Timed tm(p, kAdamScalars, st);
  commit_scalar_state<<<1, 64, 0, st>>>(p->staging, scalar_state_of(s));
  FPM_HIP(hipGetLastError());
  return FPM_OK;
}

}  // namespace

extern "C" {

int fpm_step(fpm_plan* p, fpm_state* s, const fpm_hparams* hp, const int32_t* leds, int32_t B,
             const float* gamma, const float* meas_amp, void* stream) {
  if (int rc = check_state(p, s, hp, meas_amp)) return rc;
  FPM_REQUIRE(B >= 1, "fpm_step needs a non-empty batch");
  if (int rc = check_batch(p, leds, B)) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (int rc = step_launches(p, s, hp, leds, B, gamma, meas_amp, 0, st)) return rc;
  if (hp->learn_zernike || hp->learn_z) return commit_launch(p, s, st);
  return FPM_OK;
}

int fpm_run(fpm_plan* p, fpm_state* s, const fpm_hparams* hp, const int32_t* leds,
            const int32_t* batch_sizes, int32_t n_steps, const float* gamma,
            const float* meas_amp, void* stream) {
  if (int rc = check_state(p, s, hp, meas_amp)) return rc;
  FPM_REQUIRE(n_steps >= 0, "n_steps must be >= 0");
  FPM_REQUIRE(n_steps == 0 || (leds && batch_sizes), "leds and batch_sizes must not be NULL");
  size_t total = 0;
  for (int i = 0; i < n_steps; ++i) {
    FPM_REQUIRE(batch_sizes[i] >= 1 && batch_sizes[i] <= p->max_batch,
                "every batch size must be in [1, max_batch]");
    if (int rc = check_batch(p, leds + total, batch_sizes[i])) return rc;
    total += batch_sizes[i];
  }
  hipStream_t st = (hipStream_t)stream;
  const bool learn_p = hp->learn_zernike || hp->learn_z;
  size_t off = 0;
  for (int i = 0; i < n_steps; ++i) {
    if (int rc = step_launches(p, s, hp, leds + off, batch_sizes[i], gamma, meas_amp,
                               learn_p && i > 0, st))
      return rc;
    off += batch_sizes[i];
  }
  if (learn_p && n_steps > 0) return commit_launch(p, s, st);
  return FPM_OK;
}

int fpm_loss_grad(fpm_plan* p, const fpm_led_grid* grid, const fpm_params* pr,
                  const int32_t* leds, int32_t B, const float* meas_amp, fpm_grads* gr,
                  void* stream) {
  FPM_REQUIRE(p && grid && pr && gr && pr->O && meas_amp,
              "plan, grid, params, grads, params->O and meas_amp must not be NULL");
  FPM_REQUIRE(grid->n_side >= 1 && grid->n_side * grid->n_side == p->n_led,
              "grid->n_side^2 must equal the plan's n_led");
  if (int rc = check_batch(p, leds, B)) return rc;
  FPM_REQUIRE(B <= kMaxSlots, "the multi-parameter path takes at most 64 LEDs per batch");
  if (int rc = check_device(p)) return rc;
  if (B == 0) return FPM_OK;
  hipStream_t st = (hipStream_t)stream;
  return with_lr_size(p->N, [&](auto n) {
    return launch_loss_grad<decltype(n)::value>(p, grid, pr, leds, B, meas_amp, gr, st);
  });
}

int fpm_run_multi(fpm_plan* p, const fpm_led_grid* grid, fpm_state* s, fpm_geometry* geo,
                  const fpm_hparams* hp, const int32_t* leds, const int32_t* batch_sizes,
                  int32_t n_steps, const float* meas_amp, void* stream) {
  FPM_REQUIRE(p && grid && s && geo && hp, "plan, grid, state, geometry and hparams must not be NULL");
  FPM_REQUIRE(s->O && s->m_O && s->v_O && s->P && meas_amp,
              "state O, m_O, v_O, P and meas_amp must not be NULL");
  FPM_REQUIRE(s->coeffs && s->m_c && s->v_c && s->z_um && s->m_z && s->v_z,
              "the Zernike and defocus state must not be NULL");
  FPM_REQUIRE(geo->geom && geo->m_geom && geo->v_geom, "geometry state must not be NULL");
  FPM_REQUIRE(grid->n_side >= 1 && grid->n_side * grid->n_side == p->n_led,
              "grid->n_side^2 must equal the plan's n_led");
  FPM_REQUIRE(s->t >= 0, "t must be >= 0");
  FPM_REQUIRE(n_steps >= 0, "n_steps must be >= 0");
  FPM_REQUIRE(n_steps == 0 || (leds && batch_sizes), "leds and batch_sizes must not be NULL");
  if (int rc = check_device(p)) return rc;
  size_t off = 0;
  for (int i = 0; i < n_steps; ++i) {
    FPM_REQUIRE(batch_sizes[i] >= 1 && batch_sizes[i] <= p->max_batch,
                "every batch size must be in [1, max_batch]");
    FPM_REQUIRE(batch_sizes[i] <= kMaxSlots,
                "the multi-parameter path takes at most 64 LEDs per batch");
    if (int rc = check_batch(p, leds + off, batch_sizes[i])) return rc;
    off += (size_t)batch_sizes[i];
  }
  if (n_steps == 0) return FPM_OK;
  hipStream_t st = (hipStream_t)stream;
  MultiState ms{s->coeffs, s->m_c, s->v_c, s->z_um, s->m_z, s->v_z,
                geo->geom, geo->m_geom, geo->v_geom};
  multi_params_io<<<1, 64, 0, st>>>(ms, p->mpar, 1);
  tiles_with_moments<<<(p->M / 32) * (p->M / 32), 256, 0, st>>>(
      reinterpret_cast<const float*>(s->m_O), reinterpret_cast<const float*>(s->v_O), p->M,
      p->tile_flags);
  FPM_HIP(hipGetLastError());
  const GeomArgs ga = geom_args(p, grid);
  off = 0;
  for (int i = 0; i < n_steps; ++i) {
    MultiParams* cur = p->mpar + (i & 1);
    MultiParams* next = p->mpar + ((i + 1) & 1);
    SubSlot* sub_cur = p->sub + (size_t)(i & 1) * p->max_batch;
    const bool has_next = i + 1 < n_steps;
    SubSlot* sub_next = has_next ? p->sub + (size_t)((i + 1) & 1) * p->max_batch : nullptr;
    const int B = batch_sizes[i];
    const int rc = with_lr_size(p->N, [&](auto n) {
      return launch_multi_step<decltype(n)::value>(
          p, ga, s, geo, hp, leds + off, B, meas_amp, cur, next, sub_cur, i > 0, sub_next,
          has_next ? leds + off + B : nullptr, has_next ? batch_sizes[i + 1] : 0, st);
    });
    if (rc) return rc;
    off += (size_t)B;
  }
  multi_params_io<<<1, 64, 0, st>>>(ms, p->mpar + (n_steps & 1), 0);
  FPM_HIP(hipGetLastError());
  return FPM_OK;
}

int fpm_hr_transform(fpm_plan* p, const fpm_c32* in, fpm_c32* out, int32_t direction,
                     void* stream) {
  FPM_REQUIRE(p && in && out, "plan, in and out must not be NULL");
  FPM_REQUIRE(direction == 1 || direction == -1, "direction must be +1 or -1");
  if (!p->hr_ok) return fail(FPM_EUNSUPPORTED, kHrSizes);
  if (int rc = check_device(p)) return rc;
  HrArgs a{};
  a.in = reinterpret_cast<const float2*>(in);
  a.out = reinterpret_cast<float2*>(out);
  return dispatch_hr(p, a, direction > 0 ? kRowFwd : kRowInv, direction > 0 ? -1 : +1,
                     (hipStream_t)stream);
}

int fpm_init_spectrum(fpm_plan* p, const float* centre_amp, fpm_c32* O_out, void* stream) {
  FPM_REQUIRE(p && centre_amp && O_out, "plan, centre_amp and O_out must not be NULL");
  if (!p->hr_ok) return fail(FPM_EUNSUPPORTED, kHrSizes);
  if (int rc = check_device(p)) return rc;
  HrArgs a{};
  a.img = centre_amp;
  a.n = p->N;
  a.s = p->s;
  a.out = reinterpret_cast<float2*>(O_out);
  return dispatch_hr(p, a, kRowInit, -1, (hipStream_t)stream);
}

int fpm_refocus(fpm_plan* p, const fpm_c32* O, const float* z_um, int32_t nz, fpm_c32* out,
                void* stream) {
  FPM_REQUIRE(p && O && out && (nz == 0 || z_um), "plan, O, z_um and out must not be NULL");
  FPM_REQUIRE(nz >= 0, "nz must be >= 0");
  if (!p->hr_ok) return fail(FPM_EUNSUPPORTED, kHrSizes);
  if (int rc = check_device(p)) return rc;
  if (nz == 0) return FPM_OK;
  // the distances in batches (grid rows): one row and one column launch each
  constexpr int kBatch = 1024;
  for (int i0 = 0; i0 < nz; i0 += kBatch) {
    HrArgs a{};
    a.in = reinterpret_cast<const float2*>(O);
    a.out = reinterpret_cast<float2*>(out) + (size_t)i0 * p->M * p->M;
    a.z_um = z_um + i0;
    a.dk2 = p->dk * p->dk;
    a.inv_l = 1.0 / p->lambda;
    if (int rc = dispatch_hr(p, a, kRowRefocus, +1, (hipStream_t)stream, std::min(kBatch, nz - i0)))
      return rc;
  }
  return FPM_OK;
}

int fpm_timing_enable(fpm_plan* p, int32_t enable) {
  return guarded([&]() -> int {
    FPM_REQUIRE(p, "plan must not be NULL");
    if (enable) {   // no host allocation inside the launch brackets afterwards
      p->timed.reserve(kMaxTimed);
      p->event_pool.reserve(2 * kMaxTimed);
    }
    p->timing = enable != 0;
    return FPM_OK;
  });
}

int fpm_timing_repeat(fpm_plan* p, int32_t kind, int32_t reps) {
  FPM_REQUIRE(p, "plan must not be NULL");
  FPM_REQUIRE(kind >= -1 && kind < kKinds, "kind must be -1 or a kernel kind index");
  FPM_REQUIRE(reps >= 1 && reps <= 1000, "reps must be in [1, 1000]");
  p->repeat_kind = kind;
  p->repeat_n = reps;
  return FPM_OK;
}

int fpm_timing_collect(fpm_plan* p, int32_t max_kinds, const char** names, double* total_ms,
                       int32_t* counts, int32_t* n_kinds) {
  FPM_REQUIRE(p && names && total_ms && counts && n_kinds, "arguments must not be NULL");
  const int n = std::min<int>(max_kinds, kKinds);
  for (int k = 0; k < n; ++k) {
    names[k] = kKindNames[k];
    total_ms[k] = 0.0;
    counts[k] = 0;
  }
  *n_kinds = n;
  int rc = FPM_OK;
  for (auto& t : p->timed) {
    float ms = 0.f;
    if (hipEventSynchronize(t.stop) != hipSuccess ||
        hipEventElapsedTime(&ms, t.start, t.stop) != hipSuccess)
      rc = fail(FPM_EHIP, "reading a timing event failed");
    if (t.kind < n) {
      total_ms[t.kind] += ms;
      counts[t.kind] += t.reps;
    }
    p->event_pool.push_back(t.start);
    p->event_pool.push_back(t.stop);
  }
  p->timed.clear();
  return rc;
}

}  // extern "C"
