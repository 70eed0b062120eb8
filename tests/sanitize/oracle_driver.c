/* The FP64 oracle's entry points on small inputs (whole, grid and box
 * partitions, early termination, MIP, mask, perspective, candidates,
 * gradient, composite, ranges), for builds with AddressSanitizer and
 * UndefinedBehaviorSanitizer.  The oracle's own types are restated here as
 * its callers see them; exits non-zero on an error return. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double R[9];
  int W, H;
  double extent, eye_dist;
} or_view;
typedef struct {
  double lo[3], hi[3];
  int closed[3];
} or_box;
typedef struct {
  const float *vol;
  int64_t n[3];
  const float *tf;
  int M;
  double vmin, vmax, step, tau;
  int nboxes;
  const or_box *boxes;
  int grid;
  int64_t gb[3];
  int gnb[3];
  double ert_margin, geom_margin;
  int mode;
  const float *mask;
} or_scene;

int or_render_images(const or_scene *, const or_view *, int, double *, uint8_t *, int64_t *, int);
int or_render_candidates(const or_scene *, const or_view *, int, const int32_t *, const int32_t *, const int32_t *,
                         int64_t, double *, uint8_t *, int64_t *, int64_t *, int, double *, int32_t *, int);
int or_render_grad(const or_scene *, const or_view *, const double *, double *, double *, double *, int);
int or_minmax(const float *, int64_t, double *, double *, int64_t *, int);
int or_box_minmax(const float *, const int64_t *, const int64_t *, const int64_t *, double *, double *);
int or_composite(const double *, int, int64_t, double *);

int main(void) {
  enum { N1 = 13, N2 = 11, N3 = 17, M = 16, W = 24, H = 20 };
  float *vol = malloc(sizeof(float) * N1 * N2 * N3);
  uint64_t s = 12345;
  for (int i = 0; i < N1 * N2 * N3; i++) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    vol[i] = (float)((s >> 33) % 1000) / 250.0f;
  }
  float tf[4 * M], mask[N3];
  for (int i = 0; i < M; i++) {
    const float t = (float)i / (M - 1);
    tf[4 * i] = t;
    tf[4 * i + 1] = 1 - t;
    tf[4 * i + 2] = 0.5f;
    tf[4 * i + 3] = 0.3f * t;
  }
  for (int i = 0; i < N3; i++) mask[i] = (i % 4) ? 1.0f : 0.25f;
  const double c = cos(0.6), sn = sin(0.6);
  or_view views[2] = {{{1, 0, 0, 0, 1, 0, 0, 0, 1}, W, H, 0.0, 0.0},
                      {{c, 0, -sn, 0, 1, 0, sn, 0, c}, W, H, 0.0, 0.0}};
  or_box boxes[2] = {{{0, 0, 0}, {N1 - 1, N2 - 1, 8}, {1, 1, 0}}, {{0, 0, 8}, {N1 - 1, N2 - 1, N3 - 1}, {1, 1, 1}}};
  or_scene sc;
  memset(&sc, 0, sizeof sc);
  sc.vol = vol;
  sc.n[0] = N1;
  sc.n[1] = N2;
  sc.n[2] = N3;
  sc.tf = tf;
  sc.M = M;
  sc.vmin = 0.0;
  sc.vmax = 4.0;
  sc.step = 0.5;
  sc.ert_margin = 1e-2;
  sc.geom_margin = 1e-9;
  double *img = malloc(sizeof(double) * 2 * W * H * 4);
  uint8_t *fl = malloc(2 * W * H);
  int64_t tot = 0;
  int bad = 0;
  for (int variant = 0; variant < 8; variant++) {
    sc.tau = (variant & 1) ? 0.6 : 2.0;
    sc.nboxes = (variant & 2) ? 2 : 0;
    sc.boxes = (variant & 2) ? boxes : NULL;
    sc.mode = (variant & 4) ? 1 : 0;
    sc.mask = (variant == 7) ? mask : NULL;
    views[1].eye_dist = (variant == 5) ? 40.0 : 0.0;
    bad |= or_render_images(&sc, views, 2, img, fl, &tot, 2) != 0;
    int32_t rv[W], ru[W], rr[W];
    for (int i = 0; i < W; i++) {
      rv[i] = i & 1;
      ru[i] = i;
      rr[i] = (i * 7) % H;
    }
    double rgba[4 * W], cand[4 * W * 8];
    int32_t nc[W];
    int64_t ns[W], ne[W];
    uint8_t f2[W];
    bad |= or_render_candidates(&sc, views, 2, rv, ru, rr, W, rgba, f2, ns, ne, 8, cand, nc, 2) != 0;
  }
  sc.tau = 2.0;
  sc.nboxes = 0;
  sc.boxes = NULL;
  sc.mode = 0;
  sc.mask = NULL;
  double *g = calloc(W * H * 4, sizeof(double));
  for (int i = 0; i < W * H * 4; i++) g[i] = (double)(i % 7) - 3.0;
  double gtf[4 * M] = {0};
  double *gvol = calloc(N1 * N2 * N3, sizeof(double));
  bad |= or_render_grad(&sc, &views[1], g, gtf, gvol, img, 2) != 0;
  double mn, mx;
  int64_t nf;
  bad |= or_minmax(vol, N1 * N2 * N3, &mn, &mx, &nf, 2) != 0;
  const int64_t n3[3] = {N1, N2, N3}, lo[3] = {1, 2, 3}, hi[3] = {N1 - 1, N2 - 2, N3 - 4};
  bad |= or_box_minmax(vol, n3, lo, hi, &mn, &mx) != 0;
  bad |= or_composite(img, 2, W * H / 2, g) != 0;
  printf("oracle driver: %s\n", bad ? "an entry point failed" : "ok");
  free(vol);
  free(img);
  free(fl);
  free(g);
  free(gvol);
  return bad;
}
