/* A C99 client of include/flb.h: the header compiles as C, the library links,
 * and the host-side entry points answer without a GPU (no device calls). */
#include <stdio.h>
#include <string.h>

#include "flb.h"

int main(void) {
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
