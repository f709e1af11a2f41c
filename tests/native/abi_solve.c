/*
 * A whole reconstruction through the C ABI of libfpm from plain C (no Python,
 * no torch): LED table, plan, initial value, pupil, n random-batch steps, and
 * the result copied back. Inputs and outputs are raw little-endian files in
 * one directory:
 *
 *   params.txt  n_lr upsample n_side pitch_mm height_mm wavelength_um na mag
 *               pixel_um max_batch n_steps lr_object lr_zernike learn_zernike
 *   meas.bin    float  [n_led][N][N]  measured amplitudes
 *   sizes.bin   int32  [n_steps]      batch sizes
 *   leds.bin    int32  [sum sizes]    the batches' LED ids, concatenated
 *   O.bin       out: complex64 [M][M] final spectrum
 *   coeffs.bin  out: float [15]       final Zernike coefficients
 *   loss.bin    out: double [1]       loss summed over the steps
 *
 * Exit status 0 on success; otherwise the failing call is printed.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "fpm.h"

#define CHECK_FPM(call)                                                          \
  do {                                                                           \
    int rc_ = (call);                                                            \
    if (rc_ != FPM_OK) {                                                         \
      fprintf(stderr, "%s: %s (%s)\n", #call, fpm_strerror(rc_), fpm_last_error()); \
      return 1;                                                                  \
    }                                                                            \
  } while (0)

#define CHECK_HIP(call)                                                   \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) {                                               \
      fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));          \
      return 1;                                                           \
    }                                                                     \
  } while (0)

static void* read_file(const char* dir, const char* name, size_t bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE* f = fopen(path, "rb");
  if (!f) return NULL;
  void* buf = malloc(bytes ? bytes : 1);
  const size_t got = buf ? fread(buf, 1, bytes, f) : 0;
  fclose(f);
  if (got != bytes) {
    free(buf);
    return NULL;
  }
  return buf;
}

static int write_file(const char* dir, const char* name, const void* data, size_t bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE* f = fopen(path, "wb");
  if (!f) return 1;
  const size_t put = fwrite(data, 1, bytes, f);
  fclose(f);
  return put != bytes;
}

int main(int argc, char** argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: %s <directory>\n", argv[0]);
    return 2;
  }
  const char* dir = argv[1];
  char path[4096];
  snprintf(path, sizeof path, "%s/params.txt", dir);
  FILE* pf = fopen(path, "r");
  if (!pf) {
    fprintf(stderr, "cannot open %s\n", path);
    return 1;
  }
  int n_lr, s, n_side, max_batch, n_steps, learn_zernike;
  double pitch, height, lambda, na, mag, pixel, lr_object, lr_zernike;
  const int nread = fscanf(pf, "%d %d %d %lf %lf %lf %lf %lf %lf %d %d %lf %lf %d", &n_lr, &s,
                           &n_side, &pitch, &height, &lambda, &na, &mag, &pixel, &max_batch,
                           &n_steps, &lr_object, &lr_zernike, &learn_zernike);
  fclose(pf);
  if (nread != 14) {
    fprintf(stderr, "params.txt: expected 14 values, read %d\n", nread);
    return 1;
  }
  const int n_led = n_side * n_side, N = n_lr, M = n_lr * s;

  /* LED table: nearest-pixel spectral offsets from the grid geometry */
  fpm_desc desc = {n_lr, s, n_led, max_batch, lambda, na, mag, pixel};
  fpm_led_grid grid;
  memset(&grid, 0, sizeof grid);
  grid.n_side = n_side;
  grid.pitch_mm = pitch;
  grid.height_mm = height;
  int32_t* shifts = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)n_led);
  CHECK_FPM(fpm_led_shifts(&desc, &grid, NULL, NULL, shifts));
  fpm_plan* plan = NULL;
  CHECK_FPM(fpm_plan_create(&desc, shifts, &plan));

  /* host inputs */
  const size_t img = (size_t)N * N;
  float* meas_h = (float*)read_file(dir, "meas.bin", sizeof(float) * img * (size_t)n_led);
  int32_t* sizes = (int32_t*)read_file(dir, "sizes.bin", sizeof(int32_t) * (size_t)n_steps);
  if (!meas_h || !sizes) {
    fprintf(stderr, "missing or short meas.bin / sizes.bin\n");
    return 1;
  }
  size_t total = 0;
  for (int i = 0; i < n_steps; ++i) total += (size_t)sizes[i];
  int32_t* leds = (int32_t*)read_file(dir, "leds.bin", sizeof(int32_t) * total);
  if (!leds) {
    fprintf(stderr, "missing or short leds.bin\n");
    return 1;
  }

  /* device state: spectrum, Adam moments, pupil, pupil parameters, loss */
  float* meas = NULL;
  fpm_c32 *O = NULL, *mO = NULL, *vO = NULL, *P = NULL;
  float* small = NULL;   /* coeffs | m_c | v_c | z | m_z | v_z, 16 floats each */
  double *g_par = NULL, *loss = NULL;
  CHECK_HIP(hipMalloc((void**)&meas, sizeof(float) * img * (size_t)n_led));
  CHECK_HIP(hipMalloc((void**)&O, sizeof(fpm_c32) * (size_t)M * M));
  CHECK_HIP(hipMalloc((void**)&mO, sizeof(fpm_c32) * (size_t)M * M));
  CHECK_HIP(hipMalloc((void**)&vO, sizeof(fpm_c32) * (size_t)M * M));
  CHECK_HIP(hipMalloc((void**)&P, sizeof(fpm_c32) * img));
  CHECK_HIP(hipMalloc((void**)&small, sizeof(float) * 6 * 16));
  CHECK_HIP(hipMalloc((void**)&g_par, sizeof(double) * 16));
  CHECK_HIP(hipMalloc((void**)&loss, sizeof(double)));
  CHECK_HIP(hipMemcpy(meas, meas_h, sizeof(float) * img * (size_t)n_led, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemset(mO, 0, sizeof(fpm_c32) * (size_t)M * M));
  CHECK_HIP(hipMemset(vO, 0, sizeof(fpm_c32) * (size_t)M * M));
  CHECK_HIP(hipMemset(small, 0, sizeof(float) * 6 * 16));
  CHECK_HIP(hipMemset(g_par, 0, sizeof(double) * 16));
  CHECK_HIP(hipMemset(loss, 0, sizeof(double)));

  /* initial value from the centre LED, pupil from zero coefficients */
  const int centre = (n_side / 2) * n_side + n_side / 2;
  CHECK_FPM(fpm_init_spectrum(plan, meas + (size_t)centre * img, O, NULL));
  CHECK_FPM(fpm_pupil(plan, small, 15, small + 48, P, NULL));

  fpm_state st;
  memset(&st, 0, sizeof st);
  st.O = O;
  st.m_O = mO;
  st.v_O = vO;
  st.P = P;
  st.coeffs = small;
  st.m_c = small + 16;
  st.v_c = small + 32;
  st.z_um = small + 48;
  st.m_z = small + 64;
  st.v_z = small + 80;
  st.g_par = g_par;
  st.loss = loss;
  st.t = 0;
  fpm_hparams hp = {(float)lr_object, (float)lr_zernike, 0.1f, 0.9f, 0.999f, 1e-8f,
                    learn_zernike, 0};
  CHECK_FPM(fpm_run(plan, &st, &hp, leds, sizes, n_steps, NULL, meas, NULL));
  CHECK_HIP(hipDeviceSynchronize());

  fpm_c32* O_h = (fpm_c32*)malloc(sizeof(fpm_c32) * (size_t)M * M);
  float coeffs_h[16];
  double loss_h = 0.0;
  CHECK_HIP(hipMemcpy(O_h, O, sizeof(fpm_c32) * (size_t)M * M, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(coeffs_h, small, sizeof(float) * 15, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(&loss_h, loss, sizeof(double), hipMemcpyDeviceToHost));
  if (write_file(dir, "O.bin", O_h, sizeof(fpm_c32) * (size_t)M * M) ||
      write_file(dir, "coeffs.bin", coeffs_h, sizeof(float) * 15) ||
      write_file(dir, "loss.bin", &loss_h, sizeof(double))) {
    fprintf(stderr, "cannot write the outputs\n");
    return 1;
  }
  printf("steps %d t %d loss %.9e\n", n_steps, st.t, loss_h);
  CHECK_FPM(fpm_plan_destroy(plan));
  hipFree(meas);
  hipFree(O);
  hipFree(mO);
  hipFree(vO);
  hipFree(P);
  hipFree(small);
  hipFree(g_par);
  hipFree(loss);
  free(O_h);
  free(leds);
  free(sizes);
  free(meas_h);
  free(shifts);
  return 0;
}
