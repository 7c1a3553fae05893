/*
 * Node placement for variable resolution (the paper's section "Variable
 * resolution and node generation"): sweep the box in steps of s_min/4 and
 * place a node at a sweep point when no node already placed lies within
 * s(r)/sqrt(2) of it, s(r) the prescribed local spacing. Used only to
 * generate synthetic input node sets.
 *
 * The spacing field is given on a regular grid (nearest-sample lookup); the
 * box is periodic in both directions; sweep points inside obstacles carry a
 * spacing <= 0 and are skipped.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
  int ncx, ncy, cap;
  double w;
  int32_t* count;
  int32_t* idx;
} Grid;

static int wrapi(int a, int n) { return ((a % n) + n) % n; }

static double wrapd(double d, double L) {
  if (d > 0.5 * L) return d - L;
  if (d < -0.5 * L) return d + L;
  return d;
}

/* Returns the number of nodes written to (x, y), at most max_nodes, or -1
 * when a grid cell overflows. */
int64_t place_nodes(double L, double smin, const double* sgrid, int ng, double* x, double* y,
                    int64_t max_nodes) {
  const double step = 0.25 * smin;
  const int nsweep = (int)floor(L / step);
  double smax = 0.0;
  for (int64_t k = 0; k < (int64_t)ng * ng; ++k)
    if (sgrid[k] > smax) smax = sgrid[k];
  Grid g;
  const double reach = smax / sqrt(2.0);
  g.ncx = g.ncy = (int)fmax(1.0, floor(L / reach));
  g.w = L / g.ncx;
  /* a cell of width w holds at most (w / (smin/sqrt2) + 1)^2 nodes */
  g.cap = (int)pow(g.w / (smin / sqrt(2.0)) + 2.0, 2.0) + 4;
  g.count = (int32_t*)calloc((size_t)g.ncx * g.ncy, sizeof(int32_t));
  g.idx = (int32_t*)malloc((size_t)g.ncx * g.ncy * g.cap * sizeof(int32_t));
  if (!g.count || !g.idx) return -2;
  int64_t n = 0;
  for (int j = 0; j < nsweep; ++j) {
    const double py = (j + 0.5) * step;
    for (int i = 0; i < nsweep; ++i) {
      const double px = (i + 0.5) * step;
      int gi = (int)(px / L * ng), gj = (int)(py / L * ng);
      if (gi >= ng) gi = ng - 1;
      if (gj >= ng) gj = ng - 1;
      const double s = sgrid[(int64_t)gj * ng + gi];
      if (s <= 0.0) continue;
      const double r2 = 0.5 * s * s; /* (s / sqrt2)^2 */
      const int cx = (int)(px / g.w) % g.ncx, cy = (int)(py / g.w) % g.ncy;
      int free_ = 1;
      for (int dy = -1; dy <= 1 && free_; ++dy) {
        for (int dx = -1; dx <= 1 && free_; ++dx) {
          const int c = wrapi(cy + dy, g.ncy) * g.ncx + wrapi(cx + dx, g.ncx);
          for (int k = 0; k < g.count[c]; ++k) {
            const int32_t q = g.idx[(int64_t)c * g.cap + k];
            const double ddx = wrapd(x[q] - px, L), ddy = wrapd(y[q] - py, L);
            if (ddx * ddx + ddy * ddy < r2) {
              free_ = 0;
              break;
            }
          }
        }
      }
      if (!free_) continue;
      if (n >= max_nodes) continue;
      const int c = cy * g.ncx + cx;
      if (g.count[c] >= g.cap) {
        free(g.count);
        free(g.idx);
        return -1;
      }
      x[n] = px;
      y[n] = py;
      g.idx[(int64_t)c * g.cap + g.count[c]++] = (int32_t)n;
      ++n;
    }
  }
  free(g.count);
  free(g.idx);
  return n;
}
