/* Host sanitizer driver (CPU): the input generator's ray caster and the C
 * form of the dithering oracle on small inputs, built with AddressSanitizer
 * and UndefinedBehaviorSanitizer.  Exits 0 when every call returns. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void gen_range_table(const uint8_t* occ, int W, int H, double cell, int n_dirs, double max_range, float* out);
int oracle_fs_dither(const float* img, int W, int H, uint8_t* out);

int main(void) {
  const int W = 37, H = 23, N = 64;
  uint8_t* occ = (uint8_t*)calloc((size_t)W * H, 1);
  for (int j = 0; j < H; ++j)
    for (int i = 0; i < W; ++i) occ[j * W + i] = (i == 0 || j == 0 || i == W - 1 || j == H - 1 || (i * 7 + j * 3) % 11 == 0);
  float* table = (float*)malloc(sizeof(float) * (size_t)W * H * N);
  gen_range_table(occ, W, H, 0.1, N, 3.0, table);
  double acc = 0.0;
  for (int i = 0; i < W * H * N; ++i) acc += table[i];
  const int shapes[][2] = {{1, 1}, {1, 9}, {9, 1}, {31, 17}, {64, 3}};
  uint64_t state = 12345;
  for (int s = 0; s < 5; ++s) {
    const int w = shapes[s][0], h = shapes[s][1];
    float* img = (float*)malloc(sizeof(float) * (size_t)w * h);
    uint8_t* mask = (uint8_t*)malloc((size_t)w * h);
    for (int i = 0; i < w * h; ++i) {
      state = state * 6364136223846793005ull + 1442695040888963407ull;
      img[i] = (float)((state >> 40) & 0xffff) / 65536.0f;
    }
    oracle_fs_dither(img, w, h, mask);
    for (int i = 0; i < w * h; ++i) acc += mask[i];
    free(img);
    free(mask);
  }
  printf("ok %.3f\n", acc);
  free(occ);
  free(table);
  return 0;
}
