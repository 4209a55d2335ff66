/* A plain C client of the C ABI (no Python, no torch): the 1 cm cube of
 * 16^3 voxels in a 32^3 box, n = 20, jc = 1e8 A/m^2, a 0.1 T ramp along z
 * over 1 s, integrated from the virgin state to t = 2 s with the default
 * step control and stopping rule.  Prints the step statistics and the
 * moment at 1 s and 2 s as "key value" lines.  Device memory comes from the
 * HIP runtime; the library owns none of it. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "scfft.h"

#define CHECK(x)                                                                 \
  do {                                                                           \
    scfft_status s_ = (x);                                                       \
    if (s_ < 0) {                                                                \
      fprintf(stderr, "%s: %s (%s)\n", #x, scfft_status_string(s_),              \
              ctx ? scfft_last_error(ctx) : "");                                 \
      return 1;                                                                  \
    }                                                                            \
  } while (0)

int main(void) {
  scfft_ctx* ctx = NULL;
  const double l = 5e-3;
  scfft_grid g = {{32, 32, 32}, {2 * l, 2 * l, 2 * l}};
  scfft_material m = {20.0, 1e8, 1e-4, 20.0, l};
  CHECK(scfft_create(&ctx, &g, &m, SCFFT_F64, NULL));

  size_t ws_bytes = 0;
  CHECK(scfft_workspace_size(ctx, &ws_bytes));
  void* ws = NULL;
  if (hipMalloc(&ws, ws_bytes) != hipSuccess) return 1;
  CHECK(scfft_set_workspace(ctx, ws, ws_bytes));

  scfft_shape cube = {SCFFT_SHAPE_BOX, SCFFT_OP_ADD, 2, 0, {0, 0, 0}, {l, l, l}};
  CHECK(scfft_voxelize(ctx, &cube, 1));
  scfft_drive d = {SCFFT_DRIVE_RAMP_HOLD, 0, {0, 0, 1}, 0.1, 1.0, 0.0, NULL, NULL};
  CHECK(scfft_set_drive(ctx, &d));

  void* h = NULL;
  if (hipMalloc(&h, 3 * 32 * 32 * 32 * sizeof(double)) != hipSuccess) return 1;
  CHECK(scfft_init_state(ctx, 0.0, h));

  scfft_ode_opts o;
  scfft_default_ode_opts(&o);
  scfft_ode_stats st;
  double mom[3];
  const double t_out[2] = {1.0, 2.0};
  double t = 0.0;
  for (int k = 0; k < 2; ++k) {
    CHECK(scfft_integrate(ctx, t, t_out[k], h, &o, NULL, NULL, &st));
    CHECK(scfft_moment(ctx, h, 0, mom));
    printf("t %.3f accepted %lld rejected %lld rhs %lld m_z %.17g\n", t_out[k],
           (long long)st.accepted, (long long)st.rejected, (long long)st.rhs_calls, mom[2]);
    t = t_out[k];
  }
  scfft_destroy(ctx);
  hipFree(h);
  hipFree(ws);
  return 0;
}
