/* Expected-range ray caster for synthetic laser scans.
 *
 * A ray starts at a world point and walks the occupancy grid cell by cell
 * (grid traversal in the manner of Amanatides and Woo, 1987) until it
 * enters an occupied cell, leaves the grid (the outside counts as
 * occupied) or exceeds max_range; the range is the distance to the entry
 * point of that cell, clamped to max_range.  A ray starting inside an
 * occupied cell has range 0.
 *
 * This is input synthesis only: it plays the role of the simulated LIDAR
 * and of the map-derived expected-range table.
 */
#define _USE_MATH_DEFINES
#include <math.h>
#include <stddef.h>
#include <stdint.h>

static float cast_one(const uint8_t* occ, int W, int H, double cell, double ox, double oy,
                      double ang, double max_range) {
  int ci = (int)floor(ox / cell), cj = (int)floor(oy / cell);
  if (ci < 0 || cj < 0 || ci >= W || cj >= H) return 0.0f;
  if (occ[(size_t)cj * W + ci]) return 0.0f;
  double dx = cos(ang), dy = sin(ang);
  int sx = dx > 0 ? 1 : -1, sy = dy > 0 ? 1 : -1;
  double inf = 1e300;
  double tdx = fabs(dx) > 1e-15 ? cell / fabs(dx) : inf;
  double tdy = fabs(dy) > 1e-15 ? cell / fabs(dy) : inf;
  double nbx = (sx > 0 ? (ci + 1) * cell : ci * cell);
  double nby = (sy > 0 ? (cj + 1) * cell : cj * cell);
  double tmx = fabs(dx) > 1e-15 ? (nbx - ox) / dx : inf;
  double tmy = fabs(dy) > 1e-15 ? (nby - oy) / dy : inf;
  for (;;) {
    double t;
    if (tmx < tmy) {
      t = tmx;
      tmx += tdx;
      ci += sx;
    } else {
      t = tmy;
      tmy += tdy;
      cj += sy;
    }
    if (t >= max_range) return (float)max_range;
    if (ci < 0 || cj < 0 || ci >= W || cj >= H) return (float)t;
    if (occ[(size_t)cj * W + ci]) return (float)t;
  }
}

/* out[(j*W + i)*n_dirs + d]: range from the centre of cell (i, j) along the
 * world direction d * 2 pi / n_dirs. */
void gen_range_table(const uint8_t* occ, int W, int H, double cell, int n_dirs,
                     double max_range, float* out) {
  long n = (long)W * H;
#pragma omp parallel for schedule(dynamic, 64)
  for (long c = 0; c < n; ++c) {
    int i = (int)(c % W), j = (int)(c / W);
    double ox = (i + 0.5) * cell, oy = (j + 0.5) * cell;
    float* row = out + (size_t)c * n_dirs;
    for (int d = 0; d < n_dirs; ++d)
      row[d] = cast_one(occ, W, H, cell, ox, oy, d * (2.0 * M_PI / n_dirs), max_range);
  }
}

/* out[b]: range along heading + b * 2 pi / n_beams from world point (x, y). */
void gen_scan(const uint8_t* occ, int W, int H, double cell, double x, double y,
              double heading, int n_beams, double max_range, float* out) {
  for (int b = 0; b < n_beams; ++b)
    out[b] = cast_one(occ, W, H, cell, x, y, heading + b * (2.0 * M_PI / n_beams), max_range);
}
