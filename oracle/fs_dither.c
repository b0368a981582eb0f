/* Floyd-Steinberg error diffusion in raster order, FP32 (Sec. III-B, dithering).
 *
 * TEST INFRASTRUCTURE ONLY: the C form of oracle.sample.floyd_steinberg, for
 * images too large for the Python loop.  It performs the same operations in
 * the same order: cells in raster order; v = intensity + received error;
 * selected if v >= 1/2; the error e = v - (selected ? 1 : 0) is pushed as
 * 7/16 e to the right, 3/16 e below-left, 5/16 e below and 1/16 e below-right
 * (pushes leaving the image are dropped), each push one FP32 product and one
 * FP32 sum rounded to nearest.  Built with -ffp-contract=off so that no
 * product is fused into the following sum.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int oracle_fs_dither(const float* img, int W, int H, uint8_t* out) {
  float* cur = (float*)calloc((size_t)W, sizeof(float));
  float* nxt = (float*)calloc((size_t)W, sizeof(float));
  const float w_right = 7.0f / 16.0f, w_below_left = 3.0f / 16.0f, w_below = 5.0f / 16.0f,
              w_below_right = 1.0f / 16.0f;
  if (!cur || !nxt) {
    free(cur);
    free(nxt);
    return 1;
  }
  for (int j = 0; j < H; ++j) {
    for (int i = 0; i < W; ++i) {
      const float v = img[(size_t)j * W + i] + cur[i];
      const int sel = v >= 0.5f;
      out[(size_t)j * W + i] = (uint8_t)sel;
      const float e = v - (sel ? 1.0f : 0.0f);
      if (i + 1 < W) cur[i + 1] = cur[i + 1] + w_right * e;
      if (j + 1 < H) {
        if (i >= 1) nxt[i - 1] = nxt[i - 1] + w_below_left * e;
        nxt[i] = nxt[i] + w_below * e;
        if (i + 1 < W) nxt[i + 1] = nxt[i + 1] + w_below_right * e;
      }
    }
    float* t = cur;
    cur = nxt;
    nxt = t;
    memset(nxt, 0, (size_t)W * sizeof(float));
  }
  free(cur);
  free(nxt);
  return 0;
}
