// Stand-ins for the libfpm entry points the tile server calls. A "solve"
// sleeps 20 us per step, writes its first LED id into O[0].im, the first entry
// of its plan's LED table into O[1].re and its step count into the loss (NaN
// when the first measured value is NaN); the
// largest number of solves in flight and the LED-table rebinds are counted.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <string>
#include <thread>
#include <atomic>
#include "fpm.h"
namespace fpm { thread_local std::string err; int set_error(int c, const std::string& m) { err = m; return c; } }
#include <vector>
struct fpm_plan { fpm_desc d; std::vector<int32_t> shifts; };
std::atomic<int> rebinds{0};
extern "C" {
const char* fpm_last_error(void) { return fpm::err.c_str(); }
int fpm_plan_create(const fpm_desc* d, const int32_t* sh, fpm_plan** p) {
  *p = new fpm_plan{*d, std::vector<int32_t>(sh, sh + 2 * d->n_led)};
  return 0;
}
int fpm_plan_set_shifts(fpm_plan* p, const int32_t* sh, void*) {
  p->shifts.assign(sh, sh + 2 * p->d.n_led);
  ++rebinds;
  return 0;
}
int fpm_plan_destroy(fpm_plan* p) { delete p; return 0; }
int fpm_plan_set_loss(fpm_plan*, int32_t kind) { return kind == 0 || kind == 1 ? 0 : -1; }
int fpm_plan_info(const fpm_plan* p, fpm_info* i) { i->device_bytes = 1000 * p->d.n_lr; return 0; }
int fpm_init_spectrum(fpm_plan*, const float*, fpm_c32* O, void*) { O[0].re = 1; return 0; }
int fpm_pupil(fpm_plan*, const float*, int32_t, const float*, fpm_c32*, void*) { return 0; }
std::atomic<int> live{0}, peak{0};
int fpm_run(fpm_plan* pl, fpm_state* s, const fpm_hparams*, const int32_t* leds, const int32_t* sizes, int32_t n, const float*, const float* meas, void*) {
  int l = ++live; int p = peak; while (l > p && !peak.compare_exchange_weak(p, l)) {}
  std::this_thread::sleep_for(std::chrono::microseconds(20 * n));
  s->O[0].im = (float)leds[0]; s->loss[0] = n;
  if (std::isnan(meas[0])) s->loss[0] = NAN;   // NaN data give a NaN loss
  s->O[1].re = (float)pl->shifts[0];   // the LED table the solve ran with
  --live; return 0;
}
// the multi-parameter solve: the loss is the step count plus 1000 and the
// first geometry entry the grid size, so the host tests can tell the paths apart
int fpm_run_multi(fpm_plan*, const fpm_led_grid* g, fpm_state* s, fpm_geometry* geo,
                  const fpm_hparams*, const int32_t* leds, const int32_t*, int32_t n,
                  const float*, void*) {
  s->O[0].im = (float)leds[0]; s->loss[0] = n + 1000.0;
  geo->geom[0] = g->n_side;
  return 0;
}
}
