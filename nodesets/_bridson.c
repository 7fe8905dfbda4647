/*
 * Bridson Poisson-disk sampling in a disk of radius R0 (input generator for
 * the tests and the benchmark; holds none of the RBF-FD arithmetic).
 *
 * Every random number comes from the caller's stream u[0..nu) (uniform in
 * [0,1)), consumed in order, so the node set is fixed by the seed of that
 * stream.  Points are written in generation order.
 * Returns 0 on success, 1 if the stream or the output capacity ran out.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

int bridson_disk(double R0, double r, int ntries, const double* u, int64_t nu,
                 double* out, int64_t cap, int64_t* count) {
  const double cs = r / sqrt(2.0);
  const int64_t g = (int64_t)ceil(2.0 * R0 / cs) + 1;
  int64_t* grid = (int64_t*)malloc(sizeof(int64_t) * g * g);
  int64_t* active = (int64_t*)malloc(sizeof(int64_t) * cap);
  for (int64_t i = 0; i < g * g; i++) grid[i] = -1;
  int64_t np = 0, na = 0, iu = 0;
  int rc = 0;
#define NEXT_U() (iu < nu ? u[iu++] : (rc = 1, 0.5))
  /* first point: uniform in the disk by rejection */
  for (;;) {
    double px = (2.0 * NEXT_U() - 1.0) * R0, py = (2.0 * NEXT_U() - 1.0) * R0;
    if (rc) goto done;
    if (px * px + py * py <= R0 * R0) {
      out[0] = px;
      out[1] = py;
      break;
    }
  }
  np = 1;
  active[na++] = 0;
  grid[(int64_t)((out[1] + R0) / cs) * g + (int64_t)((out[0] + R0) / cs)] = 0;
  while (na > 0) {
    int64_t ai = (int64_t)(NEXT_U() * (double)na);
    if (ai >= na) ai = na - 1;
    int64_t i = active[ai];
    int placed = 0;
    for (int t = 0; t < ntries; t++) {
      double rr = r * sqrt(1.0 + 3.0 * NEXT_U());
      double th = 6.283185307179586 * NEXT_U();
      if (rc) goto done;
      double px = out[2 * i] + rr * cos(th), py = out[2 * i + 1] + rr * sin(th);
      if (px * px + py * py > R0 * R0) continue;
      int64_t cx = (int64_t)((px + R0) / cs), cy = (int64_t)((py + R0) / cs);
      int ok = 1;
      for (int64_t yy = cy - 2; yy <= cy + 2 && ok; yy++)
        for (int64_t xx = cx - 2; xx <= cx + 2; xx++) {
          if (xx < 0 || yy < 0 || xx >= g || yy >= g) continue;
          int64_t o = grid[yy * g + xx];
          if (o < 0) continue;
          double dx = out[2 * o] - px, dy = out[2 * o + 1] - py;
          if (dx * dx + dy * dy < r * r) {
            ok = 0;
            break;
          }
        }
      if (!ok) continue;
      if (np >= cap) {
        rc = 1;
        goto done;
      }
      out[2 * np] = px;
      out[2 * np + 1] = py;
      grid[cy * g + cx] = np;
      active[na++] = np;
      np++;
      placed = 1;
      break;
    }
    if (!placed) active[ai] = active[--na];
  }
done:
  *count = np;
  free(grid);
  free(active);
  return rc;
#undef NEXT_U
}
