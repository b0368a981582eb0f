/* Host sanitizer driver (CPU, no GPU calls): the library's host-side
 * argument checks and workspace arithmetic, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host code.  Every call here returns
 * before any device work; exits 0 when each returns the expected status. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "mcl.h"

#define EXPECT(cond)                                        \
  do {                                                      \
    if (!(cond)) {                                          \
      fprintf(stderr, "failed: %s (line %d)\n", #cond, __LINE__); \
      return 1;                                             \
    }                                                       \
  } while (0)

int main(void) {
  const int W = 300, H = 170, N = 360;
  uint8_t* occ = (uint8_t*)calloc((size_t)W * H, 1);
  float* table = (float*)calloc((size_t)W * H * N, sizeof(float));
  mcl_map_desc d = {W, H, 0.05, occ, table, N, 10.0};
  mcl_params p = {72, 1.0, 1.0, -1, -1, MCL_F32, MCL_MASK_BEFORE_BLUR | MCL_WALL_NORMALIZE, 0.0, {0}};
  EXPECT(mcl_map_workspace_bytes(&d, &p) > (size_t)W * H * 360 * 2);
  d.width = 0;
  EXPECT(mcl_map_workspace_bytes(&d, &p) == 0);
  d.width = W;
  p.flags = 0x1000u;
  EXPECT(mcl_map_workspace_bytes(&d, &p) == 0);
  p.flags = MCL_MASK_BEFORE_BLUR;
  p.sigma_xy_cells = -1.0;
  EXPECT(mcl_map_workspace_bytes(&d, &p) == 0);
  p.sigma_xy_cells = 1.0;
  for (int n = 1; n <= 65536; n *= 4) EXPECT(mcl_batch_workspace_bytes(n) > 0);
  EXPECT(mcl_batch_workspace_bytes(0) == 0 && mcl_batch_workspace_bytes(70000) == 0);
  mcl_map m = NULL;
  EXPECT(mcl_map_create(&d, &p, NULL, 0, NULL, &m) == MCL_EINVAL);
  EXPECT(mcl_map_create(&d, &p, (void*)16, 1, NULL, &m) == MCL_ENOMEM);
  mcl_filter f = NULL;
  EXPECT(mcl_init_belief(NULL, &p, NULL, 0, NULL, NULL, 0.0, &f) == MCL_EINVAL);
  EXPECT(mcl_step_odometry(NULL, 0.1, 0.0, 0.0) == MCL_EINVAL);
  EXPECT(mcl_apply_scan(NULL, table, N, 0.1) == MCL_EINVAL);
  EXPECT(mcl_normalize(NULL, NULL) == MCL_EINVAL);
  EXPECT(mcl_read_belief(NULL, NULL, NULL, NULL, NULL) == MCL_EINVAL);
  EXPECT(mcl_dither(NULL, 4, 4, NULL, NULL) == MCL_EINVAL);
  EXPECT(mcl_dither(NULL, -1, 4, NULL, NULL) == MCL_EINVAL);
  double dm = 0.0;
  EXPECT(mcl_difficulty(NULL, NULL, NULL, 1, 1.0, &dm) == MCL_EINVAL);
  mcl_batch b = NULL;
  EXPECT(mcl_batch_create(4, (void*)256, mcl_batch_workspace_bytes(4), NULL, &b) == MCL_EINVAL);
  EXPECT(mcl_batch_create(0, NULL, 0, NULL, &b) == MCL_EINVAL);
  EXPECT(mcl_batch_step(NULL, NULL, NULL, 1) == MCL_EINVAL);
  double uvw[3] = {0.1, 0.0, 0.0};
  EXPECT(mcl_step_batch(NULL, uvw, 1, NULL, 0, NULL) == MCL_EINVAL);
  EXPECT(mcl_last_error()[0] != '\0');
  printf("ok\n");
  free(occ);
  free(table);
  return 0;
}
