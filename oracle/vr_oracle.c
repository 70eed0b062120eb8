/*
 * vr_oracle.c -- FP64 CPU oracle for bricked ray-cast volume rendering with
 * sort-last "over" compositing (Hassan, Fluke & Barnes, "Interactive
 * Visualization of the Largest Radioastronomy Cubes", arXiv:1008.0135).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark, and by nothing
 * else.  It shares no code, header, table or helper with the HIP
 * implementation: it is a plain, slow, obviously correct restatement of what a
 * ray-casting renderer computes, evaluated in double precision.
 *
 * What it computes (paper Sec. 2 "Ray casting", Sec. 2.4 "Ray-Casting
 * Process", Sec. 2.5 "Image Composition"):
 *   - one ray per pixel, cast through the volume (Sec. 2);
 *   - a ray/box test against the data portion; rays that miss contribute
 *     nothing, rays that hit are sampled between the entry and exit points
 *     (Sec. 2.4);
 *   - each sample's scalar value is mapped to colour and opacity by a transfer
 *     function and accumulated front to back into an aggregate colour and
 *     opacity (Sec. 2, after Levoy 1990);
 *   - early ray termination once the accumulated opacity reaches its maximum
 *     (Sec. 2.4), read here as "stop after the sample for which 1 - T >= tau";
 *   - object-space partitioning into sub-volumes (Sec. 2.3), each rendered on
 *     its own with its own accumulation, and the partial images combined with
 *     the associative alpha-blending operator in depth order (Sec. 2.5).
 *
 * Readings taken where the paper is silent (all in voxel units):
 *   - voxel centres sit at integer coordinates; the domain box is
 *     [0,n1-1] x [0,n2-1] x [0,n3-1];
 *   - orthographic camera: view axes are the rows of R; pixel (u,v) maps to
 *     x = ((u+1/2)/W - 1/2) S, y = ((v+1/2)/H - 1/2) S H/W with S the extent
 *     (box diagonal when 0), the ray starts at c + x e1 + y e2 - S e3 and runs
 *     along e3;
 *   - spectral-channel masking (the user may enable or disable spectral channels,
 *     Sec. 2.2): an optional weight m[k] in [0, 1] per index k along axis 3 (the
 *     spectral axis); a sample's opacity (its normalised value under MIP) is
 *     multiplied by m interpolated linearly along axis 3 with the sample's own
 *     trilinear weight, (1 - f3) m[i3] + f3 m[i3 + 1];
 *   - perspective camera (the projection a render request may carry, Sec. 2.2;
 *     evaluated in Sec. 3): the eye sits at c - D e3 (D = eye distance, larger
 *     than half the box diagonal so the whole box lies in front of it), the
 *     pixel grid above lies on the plane through c normal to e3, and the ray of
 *     pixel (u,v) starts at the eye and runs along the unit vector of
 *     x e1 + y e2 + D e3; samples are still a step apart along the ray;
 *   - samples sit on one global lattice per ray anchored at the whole-volume
 *     entry: t_k = t_in + (k + 1/2) step while t_k < t_out;
 *   - trilinear interpolation with the cell index clamped to [0, n-2];
 *   - s = clamp((v - vmin)/(vmax - vmin), 0, 1) (s = 0 when vmax == vmin),
 *     u = s (M-1), i = min(floor(u), M-2), linear interpolation of the RGBA
 *     table (non-premultiplied colour);
 *   - C += T a rgb, T *= (1 - a); the pixel is (C, 1 - T), premultiplied;
 *   - a sub-volume owns the half-open box [lo, hi) along each axis (closed at
 *     the far face of the volume); a lattice sample belongs to the sub-volume
 *     whose box contains it; each sub-volume accumulates from T = 1 and stops
 *     on its own (sort-last: the paper's GPUs never see each other's opacity);
 *   - the partial images of one ray are combined front to back in the order
 *     of the first sample each sub-volume received.
 *
 * Where several results are correct (an opacity that lands within rounding
 * distance of tau, a sample within rounding distance of a face), the oracle
 * flags the pixel; for early-termination ties it lists every valid image (one
 * per combination of valid stopping samples) so that a caller can accept a
 * result that matches one of them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_FLAG_ERT 1  /* several stops are valid: opacity within rounding of tau */
#define OR_FLAG_GEOM 2 /* sample count or ownership decided within rounding of a face */

typedef struct {
  double R[9]; /* row-major rotation; row i is view axis e_{i+1} in volume coordinates */
  int W, H;
  double extent;   /* S; <= 0 means the box diagonal */
  double eye_dist; /* D: 0 = orthographic, > 0 = perspective with the eye at c - D e3 */
} or_view;

typedef struct {
  double lo[3], hi[3]; /* ownership box [lo, hi) per axis */
  int closed[3];       /* 1 where hi is the far face of the volume (owned, <=) */
} or_box;

typedef struct {
  const float *vol; /* [n3][n2][n1] */
  int64_t n[3];     /* n1, n2, n3 */
  const float *tf;  /* [M][4] RGBA, non-premultiplied */
  int M;
  double vmin, vmax;
  double step, tau;
  int nboxes;          /* 0: whole volume as one chain */
  const or_box *boxes; /* sub-volume ownership boxes (a partition of the domain) */
  int grid;            /* 1: boxes form the regular grid below (fast owner lookup) */
  int64_t gb[3];       /* grid brick size per axis (cells) */
  int gnb[3];          /* grid brick count per axis; box index = (k3*gnb2 + k2)*gnb1 + k1 */
  double ert_margin;   /* opacity window around tau treated as a tie */
  double geom_margin;  /* distance (voxels) treated as a geometric tie */
  int mode;            /* OR_MODE_DVR or OR_MODE_MIP */
  const float *mask;   /* [n3] channel weights along axis 3, or NULL (all 1) */
} or_scene;

/*
 * Maximum intensity projection (Sec. 2.4: the kernel's output is the maximum
 * scalar value recorded along each ray; termination once the pixel value
 * reaches its maximum).  Read here as: M = max over the ray's samples of the
 * normalised value s = clamp((v - vmin) / (vmax - vmin), 0, 1) (s = 0 when
 * vmax = vmin; M = 0 without samples), written as (M, M, M, M).  Sub-volume
 * images combine with the element-wise maximum, in any order.
 */
#define OR_MODE_DVR 0
#define OR_MODE_MIP 1

typedef struct {
  double c[3], e1[3], e2[3], e3[3], S, D;
  int W, H;
} camera;

static void make_camera(const or_scene *sc, const or_view *vw, camera *cam) {
  double diag = 0.0;
  for (int i = 0; i < 3; i++) {
    cam->c[i] = 0.5 * (double)(sc->n[i] - 1);
    diag += (double)(sc->n[i] - 1) * (double)(sc->n[i] - 1);
    cam->e1[i] = vw->R[0 + i];
    cam->e2[i] = vw->R[3 + i];
    cam->e3[i] = vw->R[6 + i];
  }
  cam->S = vw->extent > 0.0 ? vw->extent : sqrt(diag);
  cam->D = vw->eye_dist > 0.0 ? vw->eye_dist : 0.0;
  cam->W = vw->W;
  cam->H = vw->H;
}

/* Ray through the centre of pixel (u, v). */
static void pixel_ray(const camera *cam, int u, int v, double o[3], double d[3]) {
  double x = (((double)u + 0.5) / (double)cam->W - 0.5) * cam->S;
  double y = (((double)v + 0.5) / (double)cam->H - 0.5) * cam->S * (double)cam->H / (double)cam->W;
  if (cam->D > 0.0) {
    double w[3], len = 0.0;
    for (int i = 0; i < 3; i++) {
      o[i] = cam->c[i] - cam->D * cam->e3[i];
      w[i] = x * cam->e1[i] + y * cam->e2[i] + cam->D * cam->e3[i];
      len += w[i] * w[i];
    }
    len = sqrt(len);
    for (int i = 0; i < 3; i++) d[i] = w[i] / len;
    return;
  }
  for (int i = 0; i < 3; i++) {
    o[i] = cam->c[i] + x * cam->e1[i] + y * cam->e2[i] - cam->S * cam->e3[i];
    d[i] = cam->e3[i];
  }
}

/* Slab test against the closed box [lo, hi].  Returns 1 on a hit (t_in < t_out). */
static int slab(const double o[3], const double d[3], const double lo[3], const double hi[3],
                double *tin, double *tout, int *near_tie, double gm) {
  double a = -INFINITY, b = INFINITY;
  for (int i = 0; i < 3; i++) {
    if (d[i] == 0.0) {
      if (o[i] < lo[i] || o[i] > hi[i]) {
        if (fabs(o[i] - lo[i]) < gm || fabs(o[i] - hi[i]) < gm) *near_tie = 1;
        return 0;
      }
      if (fabs(o[i] - lo[i]) < gm || fabs(o[i] - hi[i]) < gm) *near_tie = 1;
      continue;
    }
    double t1 = (lo[i] - o[i]) / d[i], t2 = (hi[i] - o[i]) / d[i];
    double tn = t1 < t2 ? t1 : t2, tf = t1 < t2 ? t2 : t1;
    if (tn > a) a = tn;
    if (tf < b) b = tf;
  }
  *tin = a;
  *tout = b;
  if (fabs(b - a) < gm) *near_tie = 1;
  return a < b;
}

static double voxel(const or_scene *sc, int64_t x, int64_t y, int64_t z) {
  return (double)sc->vol[(z * sc->n[1] + y) * sc->n[0] + x];
}

/* Trilinear reconstruction at p; also returns the base corner and fractions. */
static double trilinear(const or_scene *sc, const double p[3], int64_t i0[3], double f[3]) {
  for (int i = 0; i < 3; i++) {
    double fl = floor(p[i]);
    int64_t k = (int64_t)fl;
    if (k < 0) k = 0;
    if (k > sc->n[i] - 2) k = sc->n[i] - 2;
    i0[i] = k;
    f[i] = p[i] - (double)k;
  }
  double v = 0.0;
  for (int dz = 0; dz < 2; dz++)
    for (int dy = 0; dy < 2; dy++)
      for (int dx = 0; dx < 2; dx++) {
        double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
        v += w * voxel(sc, i0[0] + dx, i0[1] + dy, i0[2] + dz);
      }
  return v;
}

/* Channel weight at a sample: the mask interpolated along axis 3 with the
 * sample's trilinear weight (1 without a mask). */
static double mask_at(const or_scene *sc, const int64_t i0[3], const double f[3]) {
  if (!sc->mask) return 1.0;
  return (1.0 - f[2]) * (double)sc->mask[i0[2]] + f[2] * (double)sc->mask[i0[2] + 1];
}

/* Transfer-function lookup: value -> non-premultiplied RGBA. */
static void classify(const or_scene *sc, double v, double rgba[4], int *ti, double *tw, double *sraw) {
  double s = 0.0;
  if (sc->vmax > sc->vmin) s = (v - sc->vmin) / (sc->vmax - sc->vmin);
  *sraw = s;
  if (s < 0.0) s = 0.0;
  if (s > 1.0) s = 1.0;
  double u = s * (double)(sc->M - 1);
  int i = (int)floor(u);
  if (i > sc->M - 2) i = sc->M - 2;
  double w = u - (double)i;
  for (int c = 0; c < 4; c++)
    rgba[c] = (1.0 - w) * (double)sc->tf[4 * i + c] + w * (double)sc->tf[4 * (i + 1) + c];
  *ti = i;
  *tw = w;
}

/* One accumulation chain (the whole ray, or one sub-volume's share of it).
 *
 * With early termination on, an FP32 renderer may stop a chain at any sample
 * whose FP64 opacity lies within ert_margin of tau: at the first sample with
 * A >= tau - margin at the earliest, at the first with A >= tau + margin at the
 * latest.  Every stop in that range is a correct result.  The chain keeps the
 * state (C, T) after each of those samples (continuing past the FP64 stop) so
 * that a caller can list every valid image. */
#define OR_MAXST 48
typedef struct {
  double C[3], T;   /* accumulated colour and transmittance (stops at ERT) */
  double Ct[3], Tt; /* continued past the stop (tie window only) */
  int stopped, lo_seen, hi_seen, used, nst, overflow;
  double stC[OR_MAXST][3], stT[OR_MAXST]; /* states after each sample of the tie window */
  double tfirst;
} chain;

static void chain_reset(chain *ch) {
  for (int c = 0; c < 3; c++) ch->C[c] = ch->Ct[c] = 0.0;
  ch->T = 1.0;
  ch->Tt = 1.0;
  ch->stopped = ch->lo_seen = ch->hi_seen = ch->used = ch->nst = ch->overflow = 0;
  ch->tfirst = 0.0;
}

/* Feed one sample.  Returns 0 once nothing more can change the chain's outputs. */
static int chain_feed(const or_scene *sc, chain *ch, const double rgba[4]) {
  int ert = sc->tau < 1.0;
  double a = rgba[3];
  if (!ert) {
    for (int c = 0; c < 3; c++) ch->C[c] += ch->T * a * rgba[c];
    ch->T *= (1.0 - a);
    return 1;
  }
  if (ch->hi_seen) return 0;
  if (!ch->stopped) {
    for (int c = 0; c < 3; c++) ch->C[c] += ch->T * a * rgba[c];
    ch->T *= (1.0 - a);
    if (1.0 - ch->T >= sc->tau) ch->stopped = 1;
  }
  for (int c = 0; c < 3; c++) ch->Ct[c] += ch->Tt * a * rgba[c];
  ch->Tt *= (1.0 - a);
  double A = 1.0 - ch->Tt;
  if (A >= sc->tau - sc->ert_margin) ch->lo_seen = 1;
  /* a sample of zero opacity repeats the previous state: listed once */
  if (ch->lo_seen && (ch->nst == 0 || a > 0.0)) {
    if (ch->nst < OR_MAXST) {
      for (int c = 0; c < 3; c++) ch->stC[ch->nst][c] = ch->Ct[c];
      ch->stT[ch->nst] = ch->Tt;
      ch->nst++;
    } else {
      ch->overflow = 1;
    }
  }
  if (A >= sc->tau + sc->ert_margin) ch->hi_seen = 1;
  return !ch->hi_seen;
}

/* Number of valid stops of a chain (1 when its stop is not a tie). */
static int chain_nstates(const chain *ch) { return ch->nst >= 2 ? ch->nst : 1; }

/* State j of a chain's valid stops: colour and transmittance. */
static void chain_state(const chain *ch, int j, double C[3], double *T) {
  if (ch->nst >= 2) {
    for (int c = 0; c < 3; c++) C[c] = ch->stC[j][c];
    *T = ch->stT[j];
  } else {
    for (int c = 0; c < 3; c++) C[c] = ch->C[c];
    *T = ch->T;
  }
}

/* Owner of a sample: index into sc->boxes, or -1. */
static int owner(const or_scene *sc, const double p[3], int *near_tie) {
  if (sc->grid) {
    int k[3];
    for (int i = 0; i < 3; i++) {
      double q = p[i] / (double)sc->gb[i];
      int64_t j = (int64_t)floor(q);
      if (j < 0) j = 0;
      if (j > sc->gnb[i] - 1) j = sc->gnb[i] - 1;
      k[i] = (int)j;
      /* interior faces are multiples of the brick size */
      double r = p[i] - (double)(j * sc->gb[i]);
      if (j > 0 && fabs(r) < sc->geom_margin) *near_tie = 1;
      if (j < sc->gnb[i] - 1 && fabs((double)((j + 1) * sc->gb[i]) - p[i]) < sc->geom_margin) *near_tie = 1;
    }
    return (k[2] * sc->gnb[1] + k[1]) * sc->gnb[0] + k[0];
  }
  int found = -1;
  for (int b = 0; b < sc->nboxes && found < 0; b++) {
    const or_box *bx = &sc->boxes[b];
    int in = 1;
    for (int i = 0; i < 3 && in; i++) {
      if (p[i] < bx->lo[i]) in = 0;
      else if (bx->closed[i] ? p[i] > bx->hi[i] : p[i] >= bx->hi[i]) in = 0;
    }
    if (in) found = b;
  }
  if (found >= 0) {
    const or_box *bx = &sc->boxes[found];
    for (int i = 0; i < 3; i++) {
      if (bx->lo[i] > 0.0 && fabs(p[i] - bx->lo[i]) < sc->geom_margin) *near_tie = 1;
      if (!bx->closed[i] && fabs(p[i] - bx->hi[i]) < sc->geom_margin) *near_tie = 1;
    }
  }
  return found;
}

typedef struct {
  chain *chains; /* one per box (or one for the whole volume) */
  int *touched;  /* indices of chains used by the current ray */
  int ntouched;
} ray_scratch;

/*
 * Every valid image of one ray when early termination makes several correct:
 * the over-composite, in depth order, of one valid stop per chain, for every
 * combination of the chains' valid stops.  Writes at most maxc candidates
 * (RGBA each) and returns their number, or -1 when there are more than maxc
 * (or a chain's tie window held more samples than it keeps).
 */
static int ray_candidates(const ray_scratch *rs, double *cand, int maxc) {
  int64_t total = 1;
  for (int a = 0; a < rs->ntouched; a++) {
    const chain *ch = &rs->chains[rs->touched[a]];
    if (ch->overflow) return -1;
    total *= chain_nstates(ch);
    if (total > maxc) return -1;
  }
  for (int64_t q = 0; q < total; q++) {
    int64_t rest = q;
    double C[3] = {0, 0, 0}, A = 0.0;
    for (int a = 0; a < rs->ntouched; a++) {
      const chain *ch = &rs->chains[rs->touched[a]];
      int ns = chain_nstates(ch);
      double Cb[3], Tb;
      chain_state(ch, (int)(rest % ns), Cb, &Tb);
      rest /= ns;
      for (int c = 0; c < 3; c++) C[c] = C[c] + (1.0 - A) * Cb[c];
      A = A + (1.0 - A) * (1.0 - Tb);
    }
    for (int c = 0; c < 3; c++) cand[4 * q + c] = C[c];
    cand[4 * q + 3] = A;
  }
  return (int)total;
}

/* Render one ray.  out[4] = (C, A); returns flags.  With cand != NULL, also
 * lists the ray's valid images (see ray_candidates) and their count in *ncand. */
static int trace(const or_scene *sc, const camera *cam, int u, int v, ray_scratch *rs, double out[4],
                 int64_t *nsamp, int64_t *neval, double *cand, int maxc, int *ncand) {
  double o[3], d[3], lo[3], hi[3];
  int flags = 0, gtie = 0;
  pixel_ray(cam, u, v, o, d);
  for (int i = 0; i < 3; i++) {
    lo[i] = 0.0;
    hi[i] = (double)(sc->n[i] - 1);
  }
  for (int c = 0; c < 4; c++) out[c] = 0.0;
  *nsamp = 0;
  *neval = 0;
  if (ncand) *ncand = 0;
  double tin, tout;
  int hit = slab(o, d, lo, hi, &tin, &tout, &gtie, sc->geom_margin);
  if (!hit) return gtie ? OR_FLAG_GEOM : 0;
  double X = (tout - tin) / sc->step - 0.5;
  int64_t n = (int64_t)ceil(X);
  if (n < 0) n = 0;
  if (fabs(X - floor(X + 0.5)) < sc->geom_margin / sc->step) gtie = 1;
  *nsamp = n;

  if (sc->mode == OR_MODE_MIP) {
    double m = 0.0;
    for (int64_t k = 0; k < n; k++) {
      double t = tin + ((double)k + 0.5) * sc->step;
      double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
      if (sc->nboxes > 0 && owner(sc, p, &gtie) < 0) {
        gtie = 1;
        continue;
      }
      int64_t i0[3];
      double f[3];
      double val = trilinear(sc, p, i0, f);
      double s = sc->vmax > sc->vmin ? (val - sc->vmin) / (sc->vmax - sc->vmin) : 0.0;
      if (s < 0.0) s = 0.0;
      if (s > 1.0) s = 1.0;
      s *= mask_at(sc, i0, f);
      if (m < 1.0) (*neval)++; /* evaluated: the maximum had not reached 1 */
      if (s > m) m = s;
    }
    for (int c = 0; c < 4; c++) out[c] = m;
    if (gtie) flags |= OR_FLAG_GEOM;
    return flags;
  }
  rs->ntouched = 0;
  for (int64_t k = 0; k < n; k++) {
    double t = tin + ((double)k + 0.5) * sc->step;
    double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
    int b = 0;
    if (sc->nboxes > 0) {
      b = owner(sc, p, &gtie);
      if (b < 0) {
        gtie = 1;
        continue;
      }
    }
    chain *ch = &rs->chains[b];
    if (!ch->used) {
      chain_reset(ch);
      ch->used = 1;
      ch->tfirst = t;
      rs->touched[rs->ntouched++] = b;
    }
    if (sc->tau < 1.0 && ch->hi_seen) continue;
    int64_t i0[3];
    double f[3], rgba[4], tw, sraw;
    int ti;
    double val = trilinear(sc, p, i0, f);
    classify(sc, val, rgba, &ti, &tw, &sraw);
    rgba[3] *= mask_at(sc, i0, f);
    if (!ch->stopped) (*neval)++;
    chain_feed(sc, ch, rgba);
    if (sc->nboxes == 0 && sc->tau < 1.0 && ch->hi_seen) break;
  }
  /* order the touched chains by their first sample (insertion sort, few entries) */
  for (int a = 1; a < rs->ntouched; a++) {
    int key = rs->touched[a], j = a - 1;
    while (j >= 0 && rs->chains[rs->touched[j]].tfirst > rs->chains[key].tfirst) {
      rs->touched[j + 1] = rs->touched[j];
      j--;
    }
    rs->touched[j + 1] = key;
  }
  double C[3] = {0, 0, 0}, A = 0.0;
  for (int a = 0; a < rs->ntouched; a++) {
    chain *ch = &rs->chains[rs->touched[a]];
    if (chain_nstates(ch) > 1 || ch->overflow) flags |= OR_FLAG_ERT;
    for (int c = 0; c < 3; c++) C[c] = C[c] + (1.0 - A) * ch->C[c];
    A = A + (1.0 - A) * (1.0 - ch->T);
  }
  for (int c = 0; c < 3; c++) out[c] = C[c];
  out[3] = A;
  if (cand && ncand) *ncand = ray_candidates(rs, cand, maxc);
  for (int a = 0; a < rs->ntouched; a++) rs->chains[rs->touched[a]].used = 0;
  if (gtie) flags |= OR_FLAG_GEOM;
  return flags;
}

int or_render_candidates(const or_scene *sc, const or_view *views, int nviews, const int32_t *ray_view,
                         const int32_t *ray_u, const int32_t *ray_v, int64_t nrays, double *rgba, uint8_t *flags,
                         int64_t *nsamp, int64_t *neval, int maxc, double *cand, int32_t *ncand, int nthreads);

static int scene_ok(const or_scene *sc) {
  if (!sc || !sc->vol || !sc->tf || sc->M < 2 || sc->step <= 0.0) return 0;
  for (int i = 0; i < 3; i++)
    if (sc->n[i] < 2) return 0;
  return 1;
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

/*
 * Render a list of rays.  ray_view/ray_u/ray_v select (view, pixel).  Outputs
 * per ray: rgba[4] (premultiplied colour, opacity), flags, nsamp (lattice
 * samples inside the volume box), neval (samples evaluated: those of each
 * chain up to its stop).  Any output pointer may be NULL.  Returns 0 on
 * success, -1 on bad input.
 */
int or_render_rays(const or_scene *sc, const or_view *views, int nviews, const int32_t *ray_view,
                   const int32_t *ray_u, const int32_t *ray_v, int64_t nrays, double *rgba, uint8_t *flags,
                   int64_t *nsamp, int64_t *neval, int nthreads) {
  return or_render_candidates(sc, views, nviews, ray_view, ray_u, ray_v, nrays, rgba, flags, nsamp, neval, 0,
                              NULL, NULL, nthreads);
}

/*
 * As or_render_rays, and with cand != NULL also every valid image of each ray
 * (early-termination ties): cand is [nrays][maxc][4], ncand[r] the number
 * written for ray r (1 without a tie, 0 for a ray that misses or an MIP ray,
 * -1 when there are more than maxc).
 */
int or_render_candidates(const or_scene *sc, const or_view *views, int nviews, const int32_t *ray_view,
                         const int32_t *ray_u, const int32_t *ray_v, int64_t nrays, double *rgba, uint8_t *flags,
                         int64_t *nsamp, int64_t *neval, int maxc, double *cand, int32_t *ncand, int nthreads) {
  if (!scene_ok(sc) || nviews < 1 || (cand && (maxc < 1 || !ncand))) return -1;
  set_threads(nthreads);
  camera *cams = (camera *)malloc(sizeof(camera) * (size_t)nviews);
  for (int i = 0; i < nviews; i++) make_camera(sc, &views[i], &cams[i]);
  int nch = sc->nboxes > 0 ? sc->nboxes : 1;
  int err = 0;
#pragma omp parallel
  {
    ray_scratch rs;
    rs.chains = (chain *)calloc((size_t)nch, sizeof(chain));
    rs.touched = (int *)malloc(sizeof(int) * (size_t)nch);
#pragma omp for schedule(dynamic, 64)
    for (int64_t r = 0; r < nrays; r++) {
      int vi = ray_view ? ray_view[r] : 0;
      if (vi < 0 || vi >= nviews) {
        err = 1;
        continue;
      }
      double o4[4];
      int64_t ns, ne;
      int nc = 0;
      int fl = trace(sc, &cams[vi], ray_u[r], ray_v[r], &rs, o4, &ns, &ne,
                     cand ? cand + 4 * (int64_t)maxc * r : NULL, maxc, &nc);
      if (rgba) memcpy(rgba + 4 * r, o4, sizeof(o4));
      if (flags) flags[r] = (uint8_t)fl;
      if (nsamp) nsamp[r] = ns;
      if (neval) neval[r] = ne;
      if (cand) ncand[r] = nc;
    }
    free(rs.chains);
    free(rs.touched);
  }
  free(cams);
  return err ? -1 : 0;
}

/* Render full images: rgba is [nviews][H][W][4] doubles, flags [nviews][H][W]. */
int or_render_images(const or_scene *sc, const or_view *views, int nviews, double *rgba, uint8_t *flags,
                     int64_t *nsamp_total, int nthreads) {
  if (!scene_ok(sc) || nviews < 1) return -1;
  set_threads(nthreads);
  int nch = sc->nboxes > 0 ? sc->nboxes : 1;
  int64_t total = 0, off = 0;
  for (int vi = 0; vi < nviews; vi++) {
    camera cam;
    make_camera(sc, &views[vi], &cam);
    int64_t npix = (int64_t)cam.W * cam.H, vtotal = 0;
#pragma omp parallel reduction(+ : vtotal)
    {
      ray_scratch rs;
      rs.chains = (chain *)calloc((size_t)nch, sizeof(chain));
      rs.touched = (int *)malloc(sizeof(int) * (size_t)nch);
#pragma omp for schedule(dynamic, 16)
      for (int64_t q = 0; q < npix; q++) {
        int u = (int)(q % cam.W), v = (int)(q / cam.W);
        double o4[4];
        int64_t ns, ne;
        int fl = trace(sc, &cam, u, v, &rs, o4, &ns, &ne, NULL, 0, NULL);
        if (rgba) memcpy(rgba + 4 * (off + q), o4, sizeof(o4));
        if (flags) flags[off + q] = (uint8_t)fl;
        vtotal += ns;
      }
      free(rs.chains);
      free(rs.touched);
    }
    total += vtotal;
    off += npix;
  }
  if (nsamp_total) *nsamp_total = total;
  return 0;
}

/*
 * Exact gradient of L = 1/2 sum (I - I*)^2 -- here of sum(grad_out * I) -- with
 * respect to the transfer-function table and the voxel values, for the
 * whole-volume (single chain) render.  Derivative of the discrete forward
 * model above, evaluated with full per-sample arrays (no checkpointing):
 *   dC/dc_k = T_{k-1} a_k,   dC/da_k = T_{k-1} (c_k - R_k),
 *   dA/da_k = T_{k-1} (1 - Q_k),
 *   R_{k-1} = a_k c_k + (1 - a_k) R_k,  Q_{k-1} = a_k + (1 - a_k) Q_k,
 *   R_n = Q_n = 0.
 * With ERT on, the termination index is frozen (samples after the stop are
 * excluded).  The window [vmin, vmax] is a constant.  grad_tf ([M][4]) and
 * grad_vol ([n3][n2][n1]) are accumulated into (caller zeroes them).
 * Optional out ([H][W][4]) receives the forward image.
 */
int or_render_grad(const or_scene *sc, const or_view *view, const double *grad_out, double *grad_tf,
                   double *grad_vol, double *out, int nthreads) {
  if (!scene_ok(sc) || sc->nboxes != 0 || sc->mask) return -1;
  set_threads(nthreads);
  camera cam;
  make_camera(sc, view, &cam);
  int64_t npix = (int64_t)cam.W * cam.H;
  int M = sc->M;
  double dsdv = sc->vmax > sc->vmin ? 1.0 / (sc->vmax - sc->vmin) : 0.0;
#pragma omp parallel
  {
    double *gtf = (double *)calloc((size_t)M * 4, sizeof(double));
    int64_t cap = 0;
    double *Tm1 = NULL, *rg = NULL, *sr = NULL, *tw = NULL, *fr = NULL;
    int *ti = NULL;
    int64_t *base = NULL;
#pragma omp for schedule(dynamic, 16)
    for (int64_t q = 0; q < npix; q++) {
      int u = (int)(q % cam.W), v = (int)(q / cam.W);
      double o[3], d[3], lo[3] = {0, 0, 0}, hi[3];
      for (int i = 0; i < 3; i++) hi[i] = (double)(sc->n[i] - 1);
      pixel_ray(&cam, u, v, o, d);
      double tin, tout;
      int tie = 0;
      if (out)
        for (int c = 0; c < 4; c++) out[4 * q + c] = 0.0;
      if (!slab(o, d, lo, hi, &tin, &tout, &tie, 0.0)) continue;
      int64_t n = (int64_t)ceil((tout - tin) / sc->step - 0.5);
      if (n <= 0) continue;
      if (n > cap) {
        cap = n;
        Tm1 = (double *)realloc(Tm1, sizeof(double) * cap);
        rg = (double *)realloc(rg, sizeof(double) * 4 * cap);
        sr = (double *)realloc(sr, sizeof(double) * cap);
        tw = (double *)realloc(tw, sizeof(double) * cap);
        fr = (double *)realloc(fr, sizeof(double) * 3 * cap);
        ti = (int *)realloc(ti, sizeof(int) * cap);
        base = (int64_t *)realloc(base, sizeof(int64_t) * 3 * cap);
      }
      /* forward, keeping every sample */
      double T = 1.0, C[3] = {0, 0, 0};
      int64_t used = 0;
      for (int64_t k = 0; k < n; k++) {
        double t = tin + ((double)k + 0.5) * sc->step;
        double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
        int64_t i0[3];
        double f[3], rgba[4];
        double val = trilinear(sc, p, i0, f);
        classify(sc, val, rgba, &ti[k], &tw[k], &sr[k]);
        for (int c = 0; c < 4; c++) rg[4 * k + c] = rgba[c];
        for (int i = 0; i < 3; i++) {
          base[3 * k + i] = i0[i];
          fr[3 * k + i] = f[i];
        }
        Tm1[k] = T;
        for (int c = 0; c < 3; c++) C[c] += T * rgba[3] * rgba[c];
        T *= (1.0 - rgba[3]);
        used = k + 1;
        if (sc->tau < 1.0 && 1.0 - T >= sc->tau) break;
      }
      if (out) {
        for (int c = 0; c < 3; c++) out[4 * q + c] = C[c];
        out[4 * q + 3] = 1.0 - T;
      }
      const double *g = grad_out + 4 * q;
      double R[3] = {0, 0, 0}, Q = 0.0;
      for (int64_t k = used - 1; k >= 0; k--) {
        double a = rg[4 * k + 3], Tp = Tm1[k];
        double gk[4];
        for (int c = 0; c < 3; c++) gk[c] = g[c] * Tp * a;
        gk[3] = g[3] * Tp * (1.0 - Q);
        for (int c = 0; c < 3; c++) gk[3] += g[c] * Tp * (rg[4 * k + c] - R[c]);
        for (int c = 0; c < 3; c++) R[c] = a * rg[4 * k + c] + (1.0 - a) * R[c];
        Q = a + (1.0 - a) * Q;
        int i = ti[k];
        double w = tw[k];
        double gu = 0.0;
        for (int c = 0; c < 4; c++) {
          gtf[4 * i + c] += (1.0 - w) * gk[c];
          gtf[4 * (i + 1) + c] += w * gk[c];
          gu += gk[c] * ((double)sc->tf[4 * (i + 1) + c] - (double)sc->tf[4 * i + c]);
        }
        if (grad_vol && sr[k] > 0.0 && sr[k] < 1.0) {
          double gv = gu * (double)(M - 1) * dsdv;
          const double *f = &fr[3 * k];
          const int64_t *i0 = &base[3 * k];
          for (int dz = 0; dz < 2; dz++)
            for (int dy = 0; dy < 2; dy++)
              for (int dx = 0; dx < 2; dx++) {
                double wt = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
                int64_t idx = ((i0[2] + dz) * sc->n[1] + (i0[1] + dy)) * sc->n[0] + (i0[0] + dx);
#pragma omp atomic
                grad_vol[idx] += gv * wt;
              }
        }
      }
    }
#pragma omp critical
    {
      for (int j = 0; j < M * 4; j++) grad_tf[j] += gtf[j];
    }
    free(gtf);
    free(Tm1);
    free(rg);
    free(sr);
    free(tw);
    free(fr);
    free(ti);
    free(base);
  }
  return 0;
}

/* Global min/max and non-finite count of n floats. */
int or_minmax(const float *x, int64_t n, double *mn, double *mx, int64_t *nonfinite, int nthreads) {
  set_threads(nthreads);
  double a = INFINITY, b = -INFINITY;
  int64_t bad = 0;
#pragma omp parallel for reduction(min : a) reduction(max : b) reduction(+ : bad)
  for (int64_t i = 0; i < n; i++) {
    double v = (double)x[i];
    if (!isfinite(v)) {
      bad++;
      continue;
    }
    if (v < a) a = v;
    if (v > b) b = v;
  }
  *mn = a;
  *mx = b;
  if (nonfinite) *nonfinite = bad;
  return 0;
}

/* Min/max over the voxel range [lo, hi] (inclusive, per axis) of the volume. */
int or_box_minmax(const float *vol, const int64_t n[3], const int64_t lo[3], const int64_t hi[3], double *mn,
                  double *mx) {
  double a = INFINITY, b = -INFINITY;
  for (int64_t z = lo[2]; z <= hi[2]; z++)
    for (int64_t y = lo[1]; y <= hi[1]; y++)
      for (int64_t x = lo[0]; x <= hi[0]; x++) {
        double v = (double)vol[(z * n[1] + y) * n[0] + x];
        if (v < a) a = v;
        if (v > b) b = v;
      }
  *mn = a;
  *mx = b;
  return 0;
}

/*
 * Over-composite n premultiplied RGBA layers, front (index 0) to back, per
 * pixel: (C, A) <- (C + (1 - A) C_b, A + (1 - A) A_b).  layers: [n][npix][4].
 */
int or_composite(const double *layers, int n, int64_t npix, double *out) {
  for (int64_t q = 0; q < npix; q++) {
    double C[3] = {0, 0, 0}, A = 0.0;
    for (int b = 0; b < n; b++) {
      const double *L = layers + 4 * ((int64_t)b * npix + q);
      for (int c = 0; c < 3; c++) C[c] = C[c] + (1.0 - A) * L[c];
      A = A + (1.0 - A) * L[3];
    }
    for (int c = 0; c < 3; c++) out[4 * q + c] = C[c];
    out[4 * q + 3] = A;
  }
  return 0;
}

int or_version(void) { return 1; }
