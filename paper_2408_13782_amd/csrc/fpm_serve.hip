// fpm_serve.hip - the tile-reconstruction server: FIFO admission by memory
// footprint, lane threads with one HIP stream each, per-shape slots of
// device state reused across requests. The C ABI is in include/fpm_serve.h;
// the GPU work of a request is the public fpm_* calls of include/fpm.h.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <exception>
#include <new>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fpm.h"
#include "fpm_serve.h"

namespace {

constexpr int kZernTerms = 15;
constexpr int kMaxLanes = 64;

// Shape of a request: sizes and optics (what a plan's allocations depend on).
// The LED table is not part of it: a slot is rebound to another table
// (another tile of the field of view) with fpm_plan_set_shifts.
struct ShapeKey {
  fpm_desc desc;
  bool operator==(const ShapeKey& o) const {
    return desc.n_lr == o.desc.n_lr && desc.upsample == o.desc.upsample &&
           desc.n_led == o.desc.n_led && desc.max_batch == o.desc.max_batch &&
           desc.wavelength_um == o.desc.wavelength_um && desc.na == o.desc.na &&
           desc.mag == o.desc.mag && desc.pixel_um == o.desc.pixel_um;
  }
};

ShapeKey key_of(const fpm_desc* d) {
  ShapeKey k;
  k.desc = *d;
  return k;
}

std::vector<int32_t> table_of(const fpm_desc* d, const int32_t* shifts_host) {
  return std::vector<int32_t>(shifts_host, shifts_host + 2 * (size_t)d->n_led);
}

// Device state of one reconstruction, laid out in one allocation:
// O | m_O | v_O (complex [M][M] each) | P (complex [N][N]) | small block.
struct Slot {
  ShapeKey key;
  std::vector<int32_t> shifts;   // the LED table the plan holds now
  fpm_plan* plan = nullptr;
  void* block = nullptr;
  fpm_c32 *O = nullptr, *m_O = nullptr, *v_O = nullptr, *P = nullptr;
  float *coeffs = nullptr, *m_c = nullptr, *v_c = nullptr, *z = nullptr, *m_z = nullptr,
        *v_z = nullptr;
  double *g_par = nullptr, *loss = nullptr;
  double *geom = nullptr, *m_geom = nullptr, *v_geom = nullptr;
  void* small = nullptr;
  size_t small_bytes = 0;
  int64_t footprint = 0;
  bool busy = false;
};

// Small block: 6 x 16 floats (coeffs, m_c, v_c, z, m_z, v_z), then 16 + 1
// doubles (g_par, loss), then 3 x 4 doubles (LED-array geometry and its moments).
constexpr size_t kSmallFloats = 6 * 16;
constexpr size_t kSmallBytes = kSmallFloats * sizeof(float) + (17 + 12) * sizeof(double);

int64_t state_bytes(const fpm_desc& d) {
  const int64_t M = (int64_t)d.n_lr * d.upsample, N = d.n_lr;
  return 3 * M * M * 8 + N * N * 8 + (int64_t)kSmallBytes;
}

int64_t data_bytes(const fpm_desc& d) { return (int64_t)d.n_led * d.n_lr * d.n_lr * 4; }

struct Job {
  fpm_request req{};
  bool multi = false;          // fused multi-parameter solve on `grid`
  fpm_led_grid grid{};
  ShapeKey key;
  std::vector<int32_t> shifts, leds, sizes;
  int64_t footprint = 0;
  double t_submit = 0.0, t_admit = 0.0;
};

struct Lane {
  std::thread thread;
  std::condition_variable cv;
  std::unique_ptr<Job> job;
  bool busy = false;
};

}  // namespace

namespace fpm {
int set_error(int code, const std::string& msg);   // fpm_last_error()'s message
}

namespace {

int serve_fail(int code, const std::string& msg) { return fpm::set_error(code, msg); }

// Runs the body of an entry point; a C++ exception (a failed host allocation,
// a thread that cannot start) becomes an error code: none crosses the C ABI.
template <class F>
int guarded(F&& body) {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return serve_fail(FPM_ENOMEM, "host memory allocation failed");
  } catch (const std::exception& e) {
    return serve_fail(FPM_EHIP, std::string("host runtime error: ") + e.what());
  }
}

}  // namespace

struct fpm_server {
  int device = 0;
  int64_t budget = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_done;
  std::deque<std::unique_ptr<Job>> queue;
  std::vector<std::unique_ptr<Lane>> lanes;
  std::deque<fpm_completion> done;
  std::vector<std::unique_ptr<Slot>> slots;
  std::vector<std::pair<ShapeKey, int64_t>> footprints;   // per shape, once known
  int64_t bytes_in_use = 0, completed = 0;
  int running = 0, max_running = 0;
  bool stop = false;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
        .count();
  }
};

namespace {

// Free every device allocation of a slot.
void slot_free(Slot* s) {
  if (s->plan) fpm_plan_destroy(s->plan);
  if (s->block) (void)hipFree(s->block);
  s->plan = nullptr;
  s->block = nullptr;
}

// Build a slot of a shape on the current device (allocates).
int slot_create(const ShapeKey& key, const std::vector<int32_t>& shifts,
                std::unique_ptr<Slot>& out) {
  auto s = std::make_unique<Slot>();
  s->key = key;
  s->shifts = shifts;
  if (int rc = fpm_plan_create(&key.desc, shifts.data(), &s->plan))
    return serve_fail(rc, std::string("slot plan: ") + fpm_last_error());
  fpm_info info{};
  fpm_plan_info(s->plan, &info);
  const size_t M = (size_t)key.desc.n_lr * key.desc.upsample, N = key.desc.n_lr;
  const size_t big = M * M * sizeof(fpm_c32), pup = N * N * sizeof(fpm_c32);
  const size_t total = 3 * big + pup + kSmallBytes;
  if (hipMalloc(&s->block, total) != hipSuccess) {
    s->block = nullptr;
    slot_free(s.get());
    return serve_fail(FPM_ENOMEM, "slot state: hipMalloc failed");
  }
  char* b = static_cast<char*>(s->block);
  s->O = reinterpret_cast<fpm_c32*>(b);
  s->m_O = reinterpret_cast<fpm_c32*>(b + big);
  s->v_O = reinterpret_cast<fpm_c32*>(b + 2 * big);
  s->P = reinterpret_cast<fpm_c32*>(b + 3 * big);
  s->small = b + 3 * big + pup;
  float* f = static_cast<float*>(s->small);
  s->coeffs = f;
  s->m_c = f + 16;
  s->v_c = f + 32;
  s->z = f + 48;
  s->m_z = f + 64;
  s->v_z = f + 80;
  s->g_par = reinterpret_cast<double*>(f + kSmallFloats);
  s->loss = s->g_par + 16;
  s->geom = s->loss + 1;
  s->m_geom = s->geom + 4;
  s->v_geom = s->geom + 8;
  s->small_bytes = kSmallBytes;
  s->footprint = state_bytes(key.desc) + info.device_bytes + data_bytes(key.desc);
  out = std::move(s);
  return FPM_OK;
}

// Free the slots no request is using (any shape) and return how many. Their
// work has finished: a lane releases a slot only after waiting for its stream.
int free_idle_slots(fpm_server* sv) {
  std::vector<std::unique_ptr<Slot>> idle;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (auto it = sv->slots.begin(); it != sv->slots.end();) {
      if (!(*it)->busy) {
        idle.push_back(std::move(*it));
        it = sv->slots.erase(it);
      } else {
        ++it;
      }
    }
  }
  for (auto& x : idle) slot_free(x.get());
  return (int)idle.size();
}

// Take a free slot of the job's shape, preferring one that holds the job's LED
// table; another free slot of the shape is rebound to it on the lane's stream;
// with none free, a new slot is created. Idle slots are not part of the
// admission budget: when a new slot does not fit in device memory, the idle
// slots are freed and the creation is tried once more.
int slot_acquire(fpm_server* sv, const Job& j, hipStream_t st, Slot** out) {
  Slot* got = nullptr;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (auto& s : sv->slots)
      if (!s->busy && s->key == j.key && (got == nullptr || s->shifts == j.shifts)) {
        got = s.get();
        if (s->shifts == j.shifts) break;
      }
    if (got) got->busy = true;
  }
  if (got) {
    *out = got;
    if (got->shifts != j.shifts) {
      if (int rc = fpm_plan_set_shifts(got->plan, j.shifts.data(), st))
        return serve_fail(rc, fpm_last_error());
      got->shifts = j.shifts;
    }
    return FPM_OK;
  }
  std::unique_ptr<Slot> s;
  int rc = slot_create(j.key, j.shifts, s);
  if (rc == FPM_ENOMEM && free_idle_slots(sv) > 0) rc = slot_create(j.key, j.shifts, s);
  if (rc) return rc;
  s->busy = true;
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = s.get();
  sv->slots.push_back(std::move(s));
  return FPM_OK;
}

// The whole solve of one request on a slot, enqueued on st; waits for it.
int run_request(const Job& j, Slot* s, hipStream_t st, hipEvent_t ev) {
  const fpm_request& r = j.req;
  const size_t N = r.desc.n_lr, M = N * r.desc.upsample;
  if (hipMemsetAsync(s->m_O, 0, 2 * M * M * sizeof(fpm_c32), st) != hipSuccess ||
      hipMemsetAsync(s->small, 0, s->small_bytes, st) != hipSuccess)
    return serve_fail(FPM_EHIP, "hipMemsetAsync failed");
  if (int rc = fpm_plan_set_loss(s->plan, r.loss_kind)) return serve_fail(rc, fpm_last_error());
  if (int rc = fpm_init_spectrum(s->plan, r.meas_amp + (size_t)r.centre_led * N * N, s->O, st))
    return serve_fail(rc, fpm_last_error());
  if (int rc = fpm_pupil(s->plan, s->coeffs, kZernTerms, s->z, s->P, st))
    return serve_fail(rc, fpm_last_error());
  fpm_state state{};
  state.O = s->O;
  state.m_O = s->m_O;
  state.v_O = s->v_O;
  state.P = s->P;
  state.coeffs = s->coeffs;
  state.m_c = s->m_c;
  state.v_c = s->v_c;
  state.z_um = s->z;
  state.m_z = s->m_z;
  state.v_z = s->v_z;
  state.g_par = s->g_par;
  state.loss = s->loss;
  state.t = 0;
  if (r.n_steps > 0 && j.multi) {
    fpm_geometry geo{};
    geo.geom = s->geom;
    geo.m_geom = s->m_geom;
    geo.v_geom = s->v_geom;
    geo.lr_shift_mm = r.lr_shift_mm;
    geo.lr_rot_rad = r.lr_rot_rad;
    geo.lr_height_mm = r.lr_height_mm;
    geo.learn = r.learn_geometry;
    if (int rc = fpm_run_multi(s->plan, &j.grid, &state, &geo, &r.hp, j.leds.data(),
                               j.sizes.data(), r.n_steps, r.meas_amp, st))
      return serve_fail(rc, fpm_last_error());
  } else if (r.n_steps > 0) {
    if (int rc = fpm_run(s->plan, &state, &r.hp, j.leds.data(), j.sizes.data(), r.n_steps,
                         nullptr, r.meas_amp, st))
      return serve_fail(rc, fpm_last_error());
  }
  if (hipMemcpyAsync(r.O_out, s->O, M * M * sizeof(fpm_c32), hipMemcpyDeviceToDevice, st) !=
      hipSuccess)
    return serve_fail(FPM_EHIP, "result copy failed");
  if (r.coeffs_out && hipMemcpyAsync(r.coeffs_out, s->coeffs, kZernTerms * sizeof(float),
                                     hipMemcpyDeviceToDevice, st) != hipSuccess)
    return serve_fail(FPM_EHIP, "coefficient copy failed");
  if (r.loss_out && hipMemcpyAsync(r.loss_out, s->loss, sizeof(double), hipMemcpyDeviceToDevice,
                                   st) != hipSuccess)
    return serve_fail(FPM_EHIP, "loss copy failed");
  if (r.geom_out && hipMemcpyAsync(r.geom_out, s->geom, 4 * sizeof(double),
                                   hipMemcpyDeviceToDevice, st) != hipSuccess)
    return serve_fail(FPM_EHIP, "geometry copy failed");
  double loss = 0.0;   // the summed loss, for the non-finite guard
  if (hipMemcpyAsync(&loss, s->loss, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
    return serve_fail(FPM_EHIP, "loss read-back failed");
  if (hipEventRecord(ev, st) != hipSuccess || hipEventSynchronize(ev) != hipSuccess)
    return serve_fail(FPM_EHIP, "waiting for the request failed");
  if (!std::isfinite(loss)) return serve_fail(FPM_ENONFINITE, "the solve's loss is not finite");
  return FPM_OK;
}

// Hand queued requests to idle lanes while their footprints fit (FIFO). Lock held.
void admit_locked(fpm_server* sv) {
  while (!sv->queue.empty()) {
    Lane* idle = nullptr;
    for (auto& l : sv->lanes)
      if (!l->busy) {
        idle = l.get();
        break;
      }
    if (!idle) return;
    auto& head = sv->queue.front();
    if (sv->bytes_in_use + head->footprint > sv->budget) return;
    sv->bytes_in_use += head->footprint;
    head->t_admit = sv->now_ms();
    idle->job = std::move(head);
    sv->queue.pop_front();
    idle->busy = true;
    ++sv->running;
    if (sv->running > sv->max_running) sv->max_running = sv->running;
    idle->cv.notify_one();
  }
}

void lane_main(fpm_server* sv, Lane* lane, int index) {
  (void)hipSetDevice(sv->device);
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  const bool ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&ev, hipEventBlockingSync | hipEventDisableTiming) ==
                      hipSuccess;
  for (;;) {
    std::unique_ptr<Job> job;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      lane->cv.wait(lk, [&] { return sv->stop || lane->job != nullptr; });
      if (!lane->job) break;
      job = std::move(lane->job);
    }
    int rc = ok ? FPM_OK : serve_fail(FPM_EHIP, "lane stream or event creation failed");
    Slot* slot = nullptr;
    if (rc == FPM_OK) rc = guarded([&] { return slot_acquire(sv, *job, st, &slot); });
    if (rc == FPM_OK) rc = run_request(*job, slot, st, ev);
    if (rc != FPM_OK && st) (void)hipStreamSynchronize(st);
    const double t_done = sv->now_ms();
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      if (slot) slot->busy = false;
      fpm_completion c{};
      c.tag = job->req.tag;
      c.status = rc;
      c.lane = index;
      c.t_submit_ms = job->t_submit;
      c.t_admit_ms = job->t_admit;
      c.t_done_ms = t_done;
      c.footprint_bytes = job->footprint;
      sv->done.push_back(c);
      sv->bytes_in_use -= job->footprint;
      --sv->running;
      ++sv->completed;
      lane->busy = false;
      admit_locked(sv);
    }
    sv->cv_done.notify_all();
  }
  if (ev) (void)hipEventDestroy(ev);
  if (st) (void)hipStreamDestroy(st);
}

// Footprint of a shape: from a slot or an earlier query, else from a temporary plan.
int footprint_of(fpm_server* sv, const ShapeKey& key, const std::vector<int32_t>& shifts,
                 int64_t* bytes) {
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (auto& f : sv->footprints)
      if (f.first == key) {
        *bytes = f.second;
        return FPM_OK;
      }
  }
  int64_t b = 0;
  if (int rc = fpm_request_footprint(&key.desc, shifts.data(), &b)) return rc;
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->footprints.emplace_back(key, b);
  *bytes = b;
  return FPM_OK;
}

}  // namespace

extern "C" {

int fpm_server_create(const fpm_server_desc* d, fpm_server** out) {
  return guarded([&]() -> int {
    if (!d || !out) return serve_fail(FPM_EINVAL, "desc and server must not be NULL");
    if (d->n_lanes < 1 || d->n_lanes > kMaxLanes)
      return serve_fail(FPM_EINVAL, "n_lanes must be in [1, 64]");
    if (d->hbm_budget_bytes <= 0) return serve_fail(FPM_EINVAL, "hbm_budget_bytes must be > 0");
    auto sv = new fpm_server();
    if (hipGetDevice(&sv->device) != hipSuccess) {
      delete sv;
      return serve_fail(FPM_EHIP, "hipGetDevice failed");
    }
    sv->budget = d->hbm_budget_bytes;
    sv->t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < d->n_lanes; ++i) sv->lanes.push_back(std::make_unique<Lane>());
    for (int i = 0; i < d->n_lanes; ++i)
      sv->lanes[i]->thread = std::thread(lane_main, sv, sv->lanes[i].get(), i);
    *out = sv;
    return FPM_OK;
  });
}

int fpm_server_drain(fpm_server* sv) {
  if (!sv) return serve_fail(FPM_EINVAL, "server must not be NULL");
  std::unique_lock<std::mutex> lk(sv->mu);
  sv->cv_done.wait(lk, [&] { return sv->queue.empty() && sv->running == 0; });
  return FPM_OK;
}

int fpm_server_destroy(fpm_server* sv) {
  if (!sv) return serve_fail(FPM_EINVAL, "server must not be NULL");
  fpm_server_drain(sv);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  for (auto& l : sv->lanes) l->cv.notify_all();
  for (auto& l : sv->lanes)
    if (l->thread.joinable()) l->thread.join();
  for (auto& s : sv->slots) slot_free(s.get());
  delete sv;
  return FPM_OK;
}

int fpm_request_footprint(const fpm_desc* d, const int32_t* shifts_host, int64_t* bytes) {
  return guarded([&]() -> int {
    if (!d || !shifts_host || !bytes)
      return serve_fail(FPM_EINVAL, "desc, shifts_host and bytes must not be NULL");
    fpm_plan* p = nullptr;
    if (int rc = fpm_plan_create(d, shifts_host, &p)) return serve_fail(rc, fpm_last_error());
    fpm_info info{};
    fpm_plan_info(p, &info);
    fpm_plan_destroy(p);
    *bytes = state_bytes(*d) + info.device_bytes + data_bytes(*d);
    return FPM_OK;
  });
}

int fpm_server_reserve(fpm_server* sv, const fpm_desc* d, const int32_t* shifts_host,
                       int32_t count) {
  return guarded([&]() -> int {
    if (!sv || !d || !shifts_host) return serve_fail(FPM_EINVAL, "arguments must not be NULL");
    if (count < 0) return serve_fail(FPM_EINVAL, "count must be >= 0");
    const ShapeKey key = key_of(d);
    const std::vector<int32_t> shifts = table_of(d, shifts_host);
    for (int i = 0; i < count; ++i) {
      std::unique_ptr<Slot> s;
      if (int rc = slot_create(key, shifts, s)) return rc;
      std::lock_guard<std::mutex> lk(sv->mu);
      bool known = false;
      for (auto& f : sv->footprints) known = known || f.first == key;
      if (!known) sv->footprints.emplace_back(key, s->footprint);
      sv->slots.push_back(std::move(s));
    }
    return FPM_OK;
  });
}

int fpm_server_submit(fpm_server* sv, const fpm_request* r) {
  return guarded([&]() -> int {
    if (!sv || !r) return serve_fail(FPM_EINVAL, "server and request must not be NULL");
    const fpm_desc& d = r->desc;
    if (!r->shifts_host || !r->meas_amp || !r->O_out)
      return serve_fail(FPM_EINVAL, "shifts_host, meas_amp and O_out must not be NULL");
    if (d.n_led < 1 || d.max_batch < 1) return serve_fail(FPM_EINVAL, "empty LED table or batch");
    if (r->centre_led < 0 || r->centre_led >= d.n_led)
      return serve_fail(FPM_EINVAL, "centre_led outside [0, n_led)");
    if (r->n_steps < 0) return serve_fail(FPM_EINVAL, "n_steps must be >= 0");
    if (r->loss_kind != FPM_LOSS_AMPLITUDE && r->loss_kind != FPM_LOSS_INTENSITY)
      return serve_fail(FPM_EINVAL, "loss_kind must be FPM_LOSS_AMPLITUDE or FPM_LOSS_INTENSITY");
    if (r->grid && r->grid->n_side * r->grid->n_side != d.n_led)
      return serve_fail(FPM_EINVAL, "grid->n_side^2 must equal n_led");
    if (r->n_steps > 0 && (!r->leds || !r->batch_sizes))
      return serve_fail(FPM_EINVAL, "leds and batch_sizes must not be NULL");
    auto job = std::make_unique<Job>();
    job->req = *r;
    job->key = key_of(&d);
    job->shifts = table_of(&d, r->shifts_host);
    size_t total = 0;
    for (int i = 0; i < r->n_steps; ++i) {
      const int b = r->batch_sizes[i];
      if (b < 1 || b > d.max_batch)
        return serve_fail(FPM_EINVAL, "batch sizes must be in [1, max_batch]");
      if (r->grid && b > 64)
        return serve_fail(FPM_EINVAL, "a multi-parameter request takes at most 64 LEDs per batch");
      total += (size_t)b;
    }
    for (size_t i = 0; i < total; ++i)
      if (r->leds[i] < 0 || r->leds[i] >= d.n_led)
        return serve_fail(FPM_EINVAL, "LED id outside [0, n_led)");
    if (r->n_steps > 0) {
      job->leds.assign(r->leds, r->leds + total);
      job->sizes.assign(r->batch_sizes, r->batch_sizes + r->n_steps);
    }
    if (r->grid) {
      job->multi = true;
      job->grid = *r->grid;
    }
    // the copies own the host arrays from here on
    job->req.grid = nullptr;
    job->req.shifts_host = nullptr;
    job->req.leds = nullptr;
    job->req.batch_sizes = nullptr;
    if (int rc = footprint_of(sv, job->key, job->shifts, &job->footprint)) return rc;
    if (job->footprint > sv->budget)
      return serve_fail(FPM_EINVAL, "the request's footprint exceeds the server's budget");
    std::lock_guard<std::mutex> lk(sv->mu);
    job->t_submit = sv->now_ms();
    sv->queue.push_back(std::move(job));
    admit_locked(sv);
    return FPM_OK;
  });
}

int fpm_server_poll(fpm_server* sv, fpm_completion* out, int32_t max_out, int32_t* n_out,
                    int32_t wait_ms) {
  if (!sv || !n_out || (max_out > 0 && !out))
    return serve_fail(FPM_EINVAL, "server, out and n_out must not be NULL");
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->done.empty() && wait_ms > 0)
    sv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !sv->done.empty(); });
  int n = 0;
  while (n < max_out && !sv->done.empty()) {
    out[n++] = sv->done.front();
    sv->done.pop_front();
  }
  *n_out = n;
  return FPM_OK;
}

double fpm_server_clock_ms(const fpm_server* sv) { return sv ? sv->now_ms() : 0.0; }

int fpm_server_stats(fpm_server* sv, int32_t* queued, int32_t* running, int64_t* completed,
                     int64_t* bytes_in_use, int32_t* max_running, int32_t* slots) {
  if (!sv) return serve_fail(FPM_EINVAL, "server must not be NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (queued) *queued = (int32_t)sv->queue.size();
  if (running) *running = sv->running;
  if (completed) *completed = sv->completed;
  if (bytes_in_use) *bytes_in_use = sv->bytes_in_use;
  if (max_running) *max_running = sv->max_running;
  if (slots) *slots = (int32_t)sv->slots.size();
  return FPM_OK;
}

}  // extern "C"
