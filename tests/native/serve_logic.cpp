// Scheduling checks of the tile server against the stand-ins in fake_fpm.cpp:
// every request completes with its own result, admission is first-in
// first-out, the footprint budget caps the requests in flight, invalid
// requests are refused, destroy waits for queued work, idle slots of other
// shapes are freed when device memory runs out, a request whose loss is not
// finite fails alone.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <vector>

#include "fpm_serve.h"
#include "hip/hip_runtime.h"

extern std::atomic<int> peak;
extern std::atomic<int> rebinds;

#define CHECK(c)                                          \
  do {                                                    \
    if (!(c)) {                                           \
      std::printf("FAILED %s (line %d)\n", #c, __LINE__); \
      return 1;                                           \
    }                                                     \
  } while (0)

int main() {
  fpm_desc d{64, 4, 9, 4, 0.5, 0.1, 4, 6.5};
  std::vector<int32_t> shifts(18, 0);
  int64_t fp = 0;
  CHECK(fpm_request_footprint(&d, shifts.data(), &fp) == FPM_OK && fp > 0);
  fpm_server_desc sd{4, 3 * fp};   // four lanes, memory for three requests
  fpm_server* sv = nullptr;
  CHECK(fpm_server_create(&sd, &sv) == FPM_OK);
  std::vector<float> amp(9 * 64 * 64);
  const int R = 50;
  std::vector<std::vector<fpm_c32>> outs(R, std::vector<fpm_c32>(256 * 256));
  std::vector<double> loss(R);
  std::vector<int32_t> leds(40), sizes(10, 4);
  for (int i = 0; i < 40; ++i) leds[i] = i % 9;
  for (int i = 0; i < R; ++i) {
    fpm_request r{};
    r.desc = d;
    r.shifts_host = shifts.data();
    r.meas_amp = amp.data();
    r.centre_led = 4;
    leds[0] = i % 9;   // copied at submit: later edits must not reach request i
    r.leds = leds.data();
    r.batch_sizes = sizes.data();
    r.n_steps = 10;
    r.O_out = outs[i].data();
    r.loss_out = &loss[i];
    r.tag = i;
    CHECK(fpm_server_submit(sv, &r) == FPM_OK);
  }
  fpm_request bad{};
  bad.desc = d;
  bad.shifts_host = shifts.data();
  bad.meas_amp = amp.data();
  bad.O_out = outs[0].data();
  bad.centre_led = 99;
  CHECK(fpm_server_submit(sv, &bad) == FPM_EINVAL);
  bad.centre_led = 0;
  bad.loss_kind = 7;   // neither loss
  CHECK(fpm_server_submit(sv, &bad) == FPM_EINVAL);
  bad.loss_kind = 0;
  bad.n_steps = 1;
  bad.leds = leds.data();
  int32_t big_batch = 5;   // > max_batch
  bad.batch_sizes = &big_batch;
  CHECK(fpm_server_submit(sv, &bad) == FPM_EINVAL);
  fpm_desc wide = d;
  wide.n_led = 9;
  wide.n_lr = 128;   // footprint above the budget
  bad.desc = wide;
  bad.n_steps = 0;
  CHECK(fpm_server_submit(sv, &bad) == FPM_EINVAL);

  CHECK(fpm_server_drain(sv) == FPM_OK);
  std::vector<fpm_completion> c(R + 5);
  int32_t n = 0;
  CHECK(fpm_server_poll(sv, c.data(), R + 5, &n, 0) == FPM_OK && n == R);
  int32_t q, run, mr, sl;
  int64_t done, used;
  CHECK(fpm_server_stats(sv, &q, &run, &done, &used, &mr, &sl) == FPM_OK);
  CHECK(q == 0 && run == 0 && done == R && used == 0);
  CHECK(mr == 3 && peak.load() == 3);   // the budget, not the lanes, bounded concurrency
  CHECK(sl == 3);                       // slots reused across requests
  for (int i = 0; i < R; ++i) {
    CHECK(outs[i][0].re == 1.0f && outs[i][0].im == (float)(i % 9) && loss[i] == 10.0);
  }
  std::vector<double> adm(R, -1.0);
  for (int i = 0; i < n; ++i) {
    CHECK(c[i].status == FPM_OK && c[i].footprint_bytes == fp);
    CHECK(c[i].t_submit_ms <= c[i].t_admit_ms && c[i].t_admit_ms <= c[i].t_done_ms);
    adm[c[i].tag] = c[i].t_admit_ms;
  }
  for (int i = 1; i < R; ++i) CHECK(adm[i] >= adm[i - 1]);

  // destroy with work still queued waits for it
  for (int i = 0; i < 8; ++i) {
    fpm_request r{};
    r.desc = d;
    r.shifts_host = shifts.data();
    r.meas_amp = amp.data();
    r.centre_led = 4;
    r.leds = leds.data();
    r.batch_sizes = sizes.data();
    r.n_steps = 10;
    r.O_out = outs[i].data();
    r.loss_out = &loss[i];
    loss[i] = 0.0;
    CHECK(fpm_server_submit(sv, &r) == FPM_OK);
  }
  CHECK(fpm_server_destroy(sv) == FPM_OK);
  for (int i = 0; i < 8; ++i) CHECK(loss[i] == 10.0);

  // tiles of one shape with different LED tables share one slot, rebound per request
  {
    fpm_server_desc one{1, 8 * fp};
    fpm_server* s1 = nullptr;
    CHECK(fpm_server_create(&one, &s1) == FPM_OK);
    std::vector<std::vector<int32_t>> tables(3, std::vector<int32_t>(18, 0));
    for (int k = 0; k < 3; ++k) tables[k][0] = 7 * (k + 1);
    const int order[6] = {0, 0, 1, 2, 2, 0};
    for (int i = 0; i < 6; ++i) {
      fpm_request r{};
      r.desc = d;
      r.shifts_host = tables[order[i]].data();
      r.meas_amp = amp.data();
      r.centre_led = 4;
      r.leds = leds.data();
      r.batch_sizes = sizes.data();
      r.n_steps = 2;
      r.O_out = outs[i].data();
      r.tag = 100 + i;
      CHECK(fpm_server_submit(s1, &r) == FPM_OK);
    }
    CHECK(fpm_server_drain(s1) == FPM_OK);
    int32_t slots1 = 0;
    CHECK(fpm_server_stats(s1, nullptr, nullptr, nullptr, nullptr, nullptr, &slots1) == FPM_OK);
    CHECK(slots1 == 1);
    for (int i = 0; i < 6; ++i) CHECK(outs[i][1].re == (float)(7 * (order[i] + 1)));
    CHECK(rebinds.load() == 3);   // 0 -> 1 -> 2 -> 0
    CHECK(fpm_server_destroy(s1) == FPM_OK);
  }
  // device memory for two slots only: a third shape frees the idle slots
  {
    hip_stub_alloc_cap() = 2;
    fpm_server_desc one{1, 8 * fp};
    fpm_server* s2 = nullptr;
    CHECK(fpm_server_create(&one, &s2) == FPM_OK);
    std::vector<fpm_desc> shapes(3, d);
    shapes[1].wavelength_um = 0.6;
    shapes[2].wavelength_um = 0.7;
    const int order[5] = {0, 1, 2, 0, 1};
    for (int i = 0; i < 5; ++i) {
      fpm_request r{};
      r.desc = shapes[order[i]];
      r.shifts_host = shifts.data();
      r.meas_amp = amp.data();
      r.centre_led = 4;
      r.leds = leds.data();
      r.batch_sizes = sizes.data();
      r.n_steps = 2;
      r.O_out = outs[i].data();
      r.loss_out = &loss[i];
      loss[i] = 0.0;
      r.tag = 200 + i;
      CHECK(fpm_server_submit(s2, &r) == FPM_OK);
    }
    CHECK(fpm_server_drain(s2) == FPM_OK);
    std::vector<fpm_completion> cc(8);
    int32_t nc = 0, slots2 = 0;
    CHECK(fpm_server_poll(s2, cc.data(), 8, &nc, 0) == FPM_OK && nc == 5);
    for (int i = 0; i < nc; ++i) CHECK(cc[i].status == FPM_OK);
    for (int i = 0; i < 5; ++i) CHECK(loss[i] == 2.0);
    CHECK(fpm_server_stats(s2, nullptr, nullptr, nullptr, nullptr, nullptr, &slots2) == FPM_OK);
    CHECK(slots2 <= 2);
    CHECK(fpm_server_destroy(s2) == FPM_OK);
    CHECK(hip_stub_live().load() == 0);
    hip_stub_alloc_cap() = 0;
  }
  // NaN data in one request: that request completes with FPM_ENONFINITE, the
  // others with FPM_OK
  {
    fpm_server_desc two{2, 8 * fp};
    fpm_server* s3 = nullptr;
    CHECK(fpm_server_create(&two, &s3) == FPM_OK);
    std::vector<float> bad_amp(amp);
    bad_amp[0] = NAN;
    for (int i = 0; i < 6; ++i) {
      fpm_request r{};
      r.desc = d;
      r.shifts_host = shifts.data();
      r.meas_amp = i == 3 ? bad_amp.data() : amp.data();
      r.centre_led = 4;
      r.leds = leds.data();
      r.batch_sizes = sizes.data();
      r.n_steps = 2;
      r.O_out = outs[i].data();
      r.loss_out = &loss[i];
      r.tag = 300 + i;
      CHECK(fpm_server_submit(s3, &r) == FPM_OK);
    }
    CHECK(fpm_server_drain(s3) == FPM_OK);
    std::vector<fpm_completion> cc(8);
    int32_t nc = 0;
    CHECK(fpm_server_poll(s3, cc.data(), 8, &nc, 0) == FPM_OK && nc == 6);
    for (int i = 0; i < nc; ++i)
      CHECK(cc[i].status == (cc[i].tag == 303 ? FPM_ENONFINITE : FPM_OK));
    for (int i = 0; i < 6; ++i) CHECK(i == 3 ? std::isnan(loss[i]) : loss[i] == 2.0);
    CHECK(fpm_server_destroy(s3) == FPM_OK);
  }
  // a multi-parameter request (with a grid) runs fpm_run_multi and returns its geometry
  {
    fpm_server_desc one{1, 8 * fp};
    fpm_server* s4 = nullptr;
    CHECK(fpm_server_create(&one, &s4) == FPM_OK);
    fpm_led_grid g{};
    g.n_side = 3;
    std::vector<double> geom_out(4, -1.0);
    fpm_request r{};
    r.desc = d;
    r.shifts_host = shifts.data();
    r.meas_amp = amp.data();
    r.centre_led = 4;
    r.leds = leds.data();
    r.batch_sizes = sizes.data();
    r.n_steps = 3;
    r.O_out = outs[0].data();
    r.loss_out = &loss[0];
    r.grid = &g;
    r.geom_out = geom_out.data();
    r.tag = 400;
    CHECK(fpm_server_submit(s4, &r) == FPM_OK);
    g.n_side = 5;   // the grid was copied at submit
    fpm_request bad2 = r;
    bad2.grid = &g;   // 5 x 5 LEDs for a 9-LED table
    CHECK(fpm_server_submit(s4, &bad2) == FPM_EINVAL);
    CHECK(fpm_server_drain(s4) == FPM_OK);
    CHECK(loss[0] == 1003.0 && geom_out[0] == 3.0);
    CHECK(fpm_server_destroy(s4) == FPM_OK);
  }
  std::printf("OK\n");
  return 0;
}
