/* A C99 client of include/flb.h: the header compiles as C, the library links,
 * and the host-side entry points answer without a GPU (no device calls).
 * Built with FLB_CLIENT_GPU and run with the argument "gpu", it also drives a
 * lattice on the GPU from C: device memory from the HIP runtime's C API,
 * steps in both storage layouts, lattice sums, S(k), populations, and the
 * non-finite check. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "flb.h"

#ifdef FLB_CLIENT_GPU
#include <hip/hip_runtime_api.h>

#define NX 64
#define NY 32
#define NP (5 * NX * NY)

/* D2Q5 lattice NX x NY, float32, local Gaussian noise; returns 0 or an exit code */
static int run_layout(int layout, float* out, double* mass_out, double* sk_out) {
  flb_params p;
  memset(&p, 0, sizeof p);
  p.model = FLB_D2Q5;
  p.precision = 4;
  p.n[0] = NX;
  p.n[1] = NY;
  p.n[2] = 1;
  p.omega[0] = 1.3;
  p.seed = 12345;
  p.layout = layout;
  p.kernel = layout == FLB_LAYOUT_AA ? FLB_KERNEL_FLAT : FLB_KERNEL_AUTO;
  size_t pb = 0, wb = 0;
  if (flb_required_bytes(&p, &pb, &wb) != FLB_OK) return 20;
  if (pb != (size_t)(layout == FLB_LAYOUT_AA ? 1 : 2) * NP * 4) return 21;
  void* d_pop = NULL;
  if (hipMalloc(&d_pop, pb) != hipSuccess) return 22;
  flb_lattice* h = NULL;
  if (flb_create(&p, d_pop, pb, NULL, 0, NULL, &h) != FLB_OK) return 23;
  double w[5];
  flb_lattice_constants(FLB_D2Q5, 0.0, w, NULL);
  float* f0 = (float*)malloc(sizeof(float) * NP);
  for (int i = 0; i < 5; ++i)
    for (int y = 0; y < NY; ++y)
      for (int x = 0; x < NX; ++x) f0[(i * NY + y) * NX + x] = (float)(w[i] * (10.0 + sin(0.3 * x + 0.1 * y)));
  if (flb_set_populations(h, f0, 0, 0) != FLB_OK) return 24;
  const int32_t kv[9] = {1, 0, 0, 0, 1, 0, 2, 3, 0};
  if (flb_set_sampling(h, 2, kv, 3) != FLB_OK) return 25;
  if (flb_step(h, 11) != FLB_OK) return 26;
  int64_t t = 0;
  if (flb_get_step(h, &t) != FLB_OK || t != 11) return 27;
  flb_moments_t m;
  if (flb_moments(h, &m) != FLB_OK) return 28;
  if (fabs(m.mass - m.mass0) > 1e-3 || m.nonfinite != 0) return 29;
  if (flb_structure_factor(h, NULL, 0, FLB_SK_READ, sk_out) != FLB_OK) return 30;
  for (int j = 0; j < 3; ++j)
    if (!(sk_out[j] > 0.0) || !isfinite(sk_out[j])) return 31;
  if (flb_get_populations(h, out, 0) != FLB_OK) return 32;
  double s = 0;
  for (int j = 0; j < NP; ++j) s += out[j];
  if (fabs(s - m.mass) > 1e-3) return 33;
  *mass_out = m.mass;
  /* check mode: a NaN is reported by the next step */
  f0[7] = NAN;
  if (flb_set_populations(h, f0, 0, 0) != FLB_OK) return 34;
  if (flb_set_check(h, 1) != FLB_OK) return 35;
  if (flb_step(h, 3) != FLB_ENONFINITE) return 36;
  if (flb_destroy(h) != FLB_OK) return 37;
  (void)hipFree(d_pop);
  free(f0);
  return 0;
}

static int gpu_main(void) {
  float* a = (float*)malloc(sizeof(float) * NP);
  float* b = (float*)malloc(sizeof(float) * NP);
  double ma = 0, mb = 0, ska[3], skb[3];
  int rc = run_layout(FLB_LAYOUT_TWO_BUFFER, a, &ma, ska);
  if (rc) return rc;
  rc = run_layout(FLB_LAYOUT_AA, b, &mb, skb);
  if (rc) return rc;
  /* the single-buffer layout gives the same bits */
  if (memcmp(a, b, sizeof(float) * NP) != 0 || ma != mb) return 40;
  printf("c client gpu ok: mass %.6f, S(1,0) %.6f, S(0,1) %.6f\n", ma, ska[0], ska[1]);
  free(a);
  free(b);
  return 0;
}
#endif

int main(int argc, char** argv) {
#ifdef FLB_CLIENT_GPU
  if (argc > 1 && strcmp(argv[1], "gpu") == 0) return gpu_main();
#else
  (void)argc;
  (void)argv;
#endif
  if (flb_version() != FLB_ABI_VERSION) return 1;
  double w[5], m[25];
  if (flb_lattice_constants(FLB_D2Q5, 0.0, w, m) != 5) return 2; /* returns Q */
  double s = 0;
  for (int i = 0; i < 5; ++i) s += w[i];
  if (s < 1 - 1e-15 || s > 1 + 1e-15) return 3;
  flb_params p;
  memset(&p, 0, sizeof p);
  p.model = FLB_D2Q5;
  p.precision = 4;
  p.n[0] = 64;
  p.n[1] = 32;
  p.n[2] = 1;
  p.omega[0] = 1.0;
  size_t pb = 0, wb = 0;
  if (flb_required_bytes(&p, &pb, &wb) != FLB_OK) return 4;
  if (pb != (size_t)2 * 5 * 64 * 32 * 4) return 5; /* two buffers of Q planes */
  p.omega[0] = 2.5;
  if (flb_required_bytes(&p, &pb, &wb) != FLB_EINVAL) return 6;
  if (strlen(flb_last_error()) == 0) return 7;
  flb_batch_opts o;
  memset(&o, 0, sizeof o);
  o.width = 96;
  flb_batch* b = NULL;
  if (flb_batch_create(&o, &b) != FLB_EINVAL || b != NULL) return 8;
  printf("c client ok: w0 = %.6f, pop_bytes = %zu, work_bytes = %zu\n", w[0], pb, wb);
  return 0;
}
