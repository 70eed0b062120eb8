// plan.cpp -- host-side planning of libvr (see plan.h).
#include "plan.h"

#include <algorithm>
#include <cmath>

namespace vr {

bool make_grid(const int64_t n[3], const int64_t size[3], Partition& out, std::string& err) {
  out = Partition();
  out.mode = VR_BRICK_GRID;
  int64_t total = 1;
  for (int i = 0; i < 3; i++) {
    if (size[i] < 1) {
      err = "brick size must be >= 1 along every axis";
      return false;
    }
    out.gsize[i] = size[i];
    int64_t c = (n[i] - 1 + size[i] - 1) / size[i];
    if (c < 1) c = 1;
    out.gcount[i] = (int32_t)std::min<int64_t>(c, 1 << 20);
    total *= c;
  }
  if (total > 65536) {
    err = "more than 65536 bricks";
    return false;
  }
  out.boxes.reserve((size_t)total);
  for (int32_t k3 = 0; k3 < out.gcount[2]; k3++)
    for (int32_t k2 = 0; k2 < out.gcount[1]; k2++)
      for (int32_t k1 = 0; k1 < out.gcount[0]; k1++) {
        Box b;
        const int32_t k[3] = {k1, k2, k3};
        for (int i = 0; i < 3; i++) {
          b.lo[i] = (int64_t)k[i] * size[i];
          const bool last = k[i] == out.gcount[i] - 1;
          b.hi[i] = last ? n[i] - 1 : (int64_t)(k[i] + 1) * size[i];
          b.closed[i] = last ? 1 : 0;
        }
        out.boxes.push_back(b);
      }
  return true;
}

static void kd_rec(Partition& P, const int64_t lo[3], const int64_t hi[3], const int32_t cl[3], int32_t p,
                   int32_t node) {
  if (p == 1) {
    Box b;
    for (int i = 0; i < 3; i++) {
      b.lo[i] = lo[i];
      b.hi[i] = hi[i];
      b.closed[i] = cl[i];
    }
    P.nodes[node].leaf = (int32_t)P.boxes.size();
    P.boxes.push_back(b);
    return;
  }
  int ax = 0;
  for (int i = 1; i < 3; i++)
    if (hi[i] - lo[i] > hi[ax] - lo[ax]) ax = i;
  const int32_t pl = p / 2;
  const int64_t ext = hi[ax] - lo[ax];
  int64_t cut = lo[ax] + (int64_t)std::nearbyint((double)(ext * pl) / (double)p);
  cut = std::min(std::max(cut, lo[ax] + 1), hi[ax] - 1);
  P.nodes[node].axis = ax;
  P.nodes[node].plane = cut;
  P.nodes[node].leaf = -1;
  const int32_t left = (int32_t)P.nodes.size();
  P.nodes.push_back(KdNode{0, 0, -1, -1, -1});
  const int32_t right = (int32_t)P.nodes.size();
  P.nodes.push_back(KdNode{0, 0, -1, -1, -1});
  P.nodes[node].left = left;
  P.nodes[node].right = right;
  int64_t hl[3] = {hi[0], hi[1], hi[2]}, lr[3] = {lo[0], lo[1], lo[2]};
  int32_t cll[3] = {cl[0], cl[1], cl[2]};
  hl[ax] = cut;
  cll[ax] = 0;
  lr[ax] = cut;
  kd_rec(P, lo, hl, cll, pl, left);
  kd_rec(P, lr, hi, cl, p - pl, right);
}

bool make_kd(const int64_t n[3], int32_t nparts, Partition& out, std::string& err) {
  out = Partition();
  out.mode = VR_BRICK_LONGEST_AXIS;
  if (nparts < 1 || nparts > 4096) {
    err = "nparts must be in [1, 4096]";
    return false;
  }
  // every split needs an extent of at least 2 cells on the chosen axis
  int64_t cells = (n[0] - 1) * (n[1] - 1) * (n[2] - 1);
  if (cells < nparts) {
    err = "volume too small for that many sub-volumes";
    return false;
  }
  const int64_t lo[3] = {0, 0, 0}, hi[3] = {n[0] - 1, n[1] - 1, n[2] - 1};
  const int32_t cl[3] = {1, 1, 1};
  out.nodes.push_back(KdNode{0, 0, -1, -1, -1});
  kd_rec(out, lo, hi, cl, nparts, 0);
  for (const Box& b : out.boxes)
    for (int i = 0; i < 3; i++)
      if (b.hi[i] <= b.lo[i]) {
        err = "longest-axis split produced an empty sub-volume";
        return false;
      }
  return true;
}

void permute_partition(const Partition& p, const int64_t n_twin[3], Partition& out) {
  // axis a of the volume is axis t[a] of the copy
  static const int t[3] = {2, 0, 1};
  if (p.mode == VR_BRICK_GRID) {
    int64_t size[3];
    for (int a = 0; a < 3; a++) size[t[a]] = p.gsize[a];
    std::string err;
    make_grid(n_twin, size, out, err);  // cannot fail: the same counts as p
    return;
  }
  out = Partition();
  out.mode = p.mode;
  out.boxes.resize(p.boxes.size());
  for (size_t b = 0; b < p.boxes.size(); b++)
    for (int a = 0; a < 3; a++) {
      out.boxes[b].lo[t[a]] = p.boxes[b].lo[a];
      out.boxes[b].hi[t[a]] = p.boxes[b].hi[a];
      out.boxes[b].closed[t[a]] = p.boxes[b].closed[a];
    }
  out.nodes = p.nodes;
  for (KdNode& nd : out.nodes)
    if (nd.leaf < 0) nd.axis = t[nd.axis];
}

void stored_box(const Box& b, const int64_t n[3], int64_t slo[3], int64_t shi[3]) {
  for (int i = 0; i < 3; i++) {
    slo[i] = std::max<int64_t>(0, b.lo[i] - 1);
    shi[i] = std::min<int64_t>(n[i] - 1, b.hi[i] + 1);
  }
}

Rect brick_rect(const Camera& cam, const Box& b) {
  double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
  const double k = (double)cam.W / cam.S;  // pixels per voxel
  for (int c = 0; c < 8; c++) {
    double p[3];
    for (int i = 0; i < 3; i++)
      p[i] = (double)(((c >> i) & 1) ? b.hi[i] : b.lo[i]) - (cam.persp ? cam.eye[i] : cam.c[i]);
    double x = p[0] * cam.e1[0] + p[1] * cam.e1[1] + p[2] * cam.e1[2];
    double y = p[0] * cam.e2[0] + p[1] * cam.e2[1] + p[2] * cam.e2[2];
    if (cam.persp) {
      // pinhole projection onto the pixel plane at distance D (every corner
      // lies in front of the eye: D exceeds half the box diagonal)
      const double z = p[0] * cam.e3[0] + p[1] * cam.e3[1] + p[2] * cam.e3[2];
      x *= cam.D / z;
      y *= cam.D / z;
    }
    const double u = x * k + 0.5 * cam.W - 0.5, v = y * k + 0.5 * cam.H - 0.5;
    umin = std::min(umin, u);
    umax = std::max(umax, u);
    vmin = std::min(vmin, v);
    vmax = std::max(vmax, v);
  }
  Rect r{0, 0, 0, 0};
  const double x0 = std::max(0.0, std::floor(umin) - 1.0), x1 = std::min((double)cam.W - 1, std::ceil(umax) + 1.0);
  const double y0 = std::max(0.0, std::floor(vmin) - 1.0), y1 = std::min((double)cam.H - 1, std::ceil(vmax) + 1.0);
  if (x1 < x0 || y1 < y0) return r;
  r.x0 = (int32_t)x0;
  r.y0 = (int32_t)y0;
  r.w = (int32_t)(x1 - x0) + 1;
  r.h = (int32_t)(y1 - y0) + 1;
  return r;
}

// Slab of the eye along each axis of a grid (-1 before the first slab, the
// slab count past the last): rays from the eye move away from it.
static void eye_slabs(const Partition& p, const Camera& cam, int32_t e[3]) {
  for (int i = 0; i < 3; i++) {
    const double q = cam.eye[i];
    const int32_t c = p.gcount[i];
    if (q < 0.0) e[i] = -1;
    else if (q >= (double)p.boxes.back().hi[i]) e[i] = c;
    else e[i] = std::min<int32_t>(c - 1, (int32_t)std::floor(q / (double)p.gsize[i]));
  }
}

// Near child first: for parallel rays the side the rays come from; for rays
// from an eye the side that holds the eye (a ray crosses a plane at most once,
// leaving the eye's side).
static void kd_order(const Partition& P, int32_t node, const Camera& cam, std::vector<int32_t>& order) {
  const KdNode& nd = P.nodes[node];
  if (nd.leaf >= 0) {
    order.push_back(nd.leaf);
    return;
  }
  const bool low_first = cam.persp ? cam.eye[nd.axis] < (double)nd.plane : cam.e3[nd.axis] >= 0.0;
  kd_order(P, low_first ? nd.left : nd.right, cam, order);
  kd_order(P, low_first ? nd.right : nd.left, cam, order);
}

void depth_order(const Partition& p, const Camera& cam, std::vector<int32_t>& order) {
  order.clear();
  if (p.mode == VR_BRICK_LONGEST_AXIS) {
    kd_order(p, 0, cam, order);
    return;
  }
  if (cam.persp) {
    // rays from an eye move away from it along every axis, so a ray's slab
    // distance |k_i - e_i| from the eye's slab e_i never decreases; sorting
    // by the distances along axes 3, 2, 1 (lexicographically) puts every
    // brick a ray meets after the ones it met before
    int32_t e[3];
    eye_slabs(p, cam, e);
    const int32_t* c = p.gcount;
    std::vector<std::pair<int64_t, int32_t>> key;
    key.reserve(p.boxes.size());
    const int64_t m1 = (int64_t)c[0] + 2, m2 = (int64_t)c[1] + 2;
    for (int32_t k3 = 0; k3 < c[2]; k3++)
      for (int32_t k2 = 0; k2 < c[1]; k2++)
        for (int32_t k1 = 0; k1 < c[0]; k1++) {
          const int64_t d1 = std::abs(k1 - e[0]), d2 = std::abs(k2 - e[1]), d3 = std::abs(k3 - e[2]);
          key.emplace_back((d3 * m2 + d2) * m1 + d1, (k3 * c[1] + k2) * c[0] + k1);
        }
    std::sort(key.begin(), key.end());
    order.reserve(key.size());
    for (const auto& kv : key) order.push_back(kv.second);
    return;
  }
  const double* d = cam.e3;
  // grid: visit slabs along axis 3, then 2, then 1, each in the ray's direction;
  // a ray crosses the grid monotonically along every axis, so this lexicographic
  // order puts every brick a ray meets after the ones it met before.
  const int32_t* c = p.gcount;
  order.reserve(p.boxes.size());
  for (int32_t a3 = 0; a3 < c[2]; a3++) {
    const int32_t k3 = d[2] >= 0.0 ? a3 : c[2] - 1 - a3;
    for (int32_t a2 = 0; a2 < c[1]; a2++) {
      const int32_t k2 = d[1] >= 0.0 ? a2 : c[1] - 1 - a2;
      for (int32_t a1 = 0; a1 < c[0]; a1++) {
        const int32_t k1 = d[0] >= 0.0 ? a1 : c[0] - 1 - a1;
        order.push_back((k3 * c[1] + k2) * c[0] + k1);
      }
    }
  }
}

int32_t brick_waves(const Partition& p, const Camera& cam, std::vector<int32_t>& wave) {
  const int32_t nb = (int32_t)p.boxes.size();
  wave.assign((size_t)nb, 0);
  int32_t nw = 0;
  if (p.mode == VR_BRICK_GRID) {
    const int32_t* c = p.gcount;
    int32_t e[3] = {0, 0, 0};
    if (cam.persp) eye_slabs(p, cam, e);
    for (int32_t b = 0; b < nb; b++) {
      const int32_t k[3] = {b % c[0], (b / c[0]) % c[1], b / (c[0] * c[1])};
      int32_t w = 0;
      for (int i = 0; i < 3; i++) {
        if (cam.persp) w += std::abs(k[i] - e[i]);
        else w += cam.e3[i] >= 0.0 ? k[i] : c[i] - 1 - k[i];
      }
      wave[b] = w;
      nw = std::max(nw, w + 1);
    }
    return nw;
  }
  std::vector<int32_t> order;
  depth_order(p, cam, order);
  std::vector<Rect> r((size_t)nb);
  for (int32_t b = 0; b < nb; b++) r[b] = brick_rect(cam, p.boxes[b]);
  for (size_t i = 0; i < order.size(); i++) {
    const int32_t b = order[i];
    int32_t w = 0;
    if (r[b].w > 0 && r[b].h > 0)
      for (size_t j = 0; j < i; j++) {
        const int32_t q = order[j];
        if (r[q].w == 0 || r[q].h == 0) continue;
        const bool overlap = r[q].x0 < r[b].x0 + r[b].w && r[b].x0 < r[q].x0 + r[q].w && r[q].y0 < r[b].y0 + r[b].h &&
                             r[b].y0 < r[q].y0 + r[q].h;
        if (overlap) w = std::max(w, wave[q] + 1);
      }
    wave[b] = w;
    nw = std::max(nw, w + 1);
  }
  return nw;
}

bool brick_transparent(float bmin, float bmax, const float* tf, int32_t M, double vmin, double vmax) {
  if (!std::isfinite(bmin) || !std::isfinite(bmax)) return false;
  auto ucoord = [&](double v) {
    double s = vmax > vmin ? (v - vmin) / (vmax - vmin) : 0.0;
    s = std::min(1.0, std::max(0.0, s));
    return s * (double)(M - 1);
  };
  int64_t i0 = (int64_t)std::floor(ucoord(bmin)) - 1, i1 = (int64_t)std::ceil(ucoord(bmax)) + 1;
  i0 = std::max<int64_t>(0, i0);
  i1 = std::min<int64_t>(M - 1, i1);
  for (int64_t i = i0; i <= i1; i++)
    if (tf[4 * i + 3] != 0.0f) return false;
  return true;
}

bool choose_slab(const Camera& cam, int32_t tw, int32_t th, int32_t budget, int32_t& axis, int32_t& T) {
  if (cam.persp) return false;  // the slab march assumes parallel rays
  const double p = cam.S / (double)cam.W;  // pixel pitch in voxels
  double best = INFINITY;
  bool found = false;
  for (int b = 1; b <= 2; b++) {
    const int g = 3 - b;
    const double db = cam.e3[b];
    if (std::fabs(db) < 1e-3) continue;
    const double rf = cam.e3[0] / db, rg = cam.e3[g] / db;
    // footprint of the tile's corner rays on one plane of constant axis b
    const double Wf = p * ((tw - 1) * std::fabs(cam.e1[0] - cam.e1[b] * rf) + (th - 1) * std::fabs(cam.e2[0] - cam.e2[b] * rf));
    const double Wg = p * ((tw - 1) * std::fabs(cam.e1[g] - cam.e1[b] * rg) + (th - 1) * std::fabs(cam.e2[g] - cam.e2[b] * rg));
    for (int t = 64; t >= 1; t--) {
      // box: cells floor(q) .. floor(q)+1 over the footprint widened by 0.05 each side
      const double nf = std::floor(Wf + t * std::fabs(rf) + 0.11) + 2.0;
      const double ng = std::floor(Wg + t * std::fabs(rg) + 0.11) + 2.0;
      const double pitch = 4.0 * std::ceil(nf / 4.0);
      const double size = pitch * ng * (double)(t + 1);
      if (size > (double)budget) continue;
      // voxels loaded per sample: box / (rays x samples per ray in t layers)
      const double cost = size / ((double)(tw * th) * (double)t / (0.5 * std::fabs(db)));
      if (cost < best) {
        best = cost;
        axis = b;
        T = t;
        found = true;
      }
      break;
    }
  }
  return found;
}

int ring_waves_per_block(int32_t slot, int32_t M, int32_t max_waves, int32_t* waves_per_cu, int32_t nslots) {
  const int64_t lds = 160 * 1024;
  int best_w = 1, best_waves = -1;
  for (int w : {4, 2, 1}) {
    const int64_t per_block = 16 * (int64_t)M + 4 * (int64_t)nslots * w * slot;
    int64_t blocks = lds / per_block;
    if (blocks * w > max_waves) blocks = max_waves / w;
    const int waves = (int)(blocks * w);
    if (waves > best_waves) {
      best_waves = waves;
      best_w = w;
    }
  }
  if (waves_per_cu) *waves_per_cu = best_waves;
  return best_w;
}

bool choose_ring(const Camera& cam, int32_t cap, int32_t M, int32_t max_waves, int32_t want_waves,
                 int32_t min_waves, int32_t& axis, int32_t& slot, int32_t& wpb, int32_t nslots,
                 int32_t* waves_per_cu) {
  const double p = cam.S / (double)cam.W;
  // ray directions to size the window for: the view direction (parallel
  // rays), or the rays of the image's corners and centre (perspective; a
  // tile's footprint also grows with depth, by at most (D + r) / D for the
  // box's circumradius r)
  double dirs[5][3];
  int ndir = 1;
  double scale = 1.0;
  for (int i = 0; i < 3; i++) dirs[0][i] = cam.e3[i];
  if (cam.persp) {
    const int us[5] = {cam.W / 2, 0, cam.W - 1, 0, cam.W - 1}, vs[5] = {cam.H / 2, 0, 0, cam.H - 1, cam.H - 1};
    for (int k = 0; k < 5; k++) {
      double o[3];
      pixel_ray(cam, us[k], vs[k], o, dirs[k]);
    }
    ndir = 5;
    double r2 = 0.0;
    for (int i = 0; i < 3; i++) r2 += cam.c[i] * cam.c[i];
    scale = (cam.D + std::sqrt(r2)) / cam.D;
  }
  double best = INFINITY;
  bool found = false;
  for (int b = 1; b <= 2; b++) {
    const int g = 3 - b;
    const double db = dirs[0][b];
    if (std::fabs(db) < 1e-3) continue;
    double nf = 0.0, ng = 0.0;
    bool ok = true;
    for (int k = 0; k < ndir && ok; k++) {
      const double* d = dirs[k];
      if (std::fabs(d[b]) < 1e-3 || (d[b] > 0.0) != (db > 0.0)) {
        ok = false;
        break;
      }
      const double rf = d[0] / d[b], rg = d[g] / d[b];
      const double Wf = scale * p * 7.0 * (std::fabs(cam.e1[0] - cam.e1[b] * rf) + std::fabs(cam.e2[0] - cam.e2[b] * rf));
      const double Wg = scale * p * 7.0 * (std::fabs(cam.e1[g] - cam.e1[b] * rg) + std::fabs(cam.e2[g] - cam.e2[b] * rg));
      // the kernel's bound is floor(span + 0.2) + 3 per axis; one more for rounding
      nf = std::max(nf, std::floor(Wf + 2.0 * std::fabs(rf) + 0.2) + 4.0);
      ng = std::max(ng, std::floor(Wg + 2.0 * std::fabs(rg) + 0.2) + 4.0);
    }
    if (!ok) continue;
    const double pitch = 4.0 * std::ceil(nf / 4.0);
    const double size = pitch * ng;
    if (size > (double)cap || pitch > 256.0) continue;
    int32_t waves = 0;
    const int w = ring_waves_per_block((int32_t)size, M, max_waves, &waves, nslots);
    if (waves < min_waves) continue;
    // window floats per sample (one window per layer, 2 / |db| samples per ray
    // and layer), weighted by the occupancy shortfall
    const double cost = size * std::fabs(db) * std::max(1.0, (double)want_waves / (double)waves);
    if (cost < best) {
      best = cost;
      axis = b;
      slot = (int32_t)size;
      wpb = w;
      if (waves_per_cu) *waves_per_cu = waves;
      found = true;
    }
  }
  return found;
}

// Most pixels any cell of Tf x Tg holds, over 32 placements of the cell grid
// against the pixel lattice (Halton points): (su_f, sv_f) and (su_g, sv_g) are
// the cell coordinates f / Tf and g / Tg per pixel step along u and v.  When a
// cell edge runs nearly along a lattice direction the counts jump by whole
// rows, so a mean well below 64 can still leave many cells above it.
static int32_t foot_max_pixels(double su_f, double sv_f, double su_g, double sv_g) {
  const double det = su_f * sv_g - sv_f * su_g;
  if (!(std::fabs(det) > 1e-12)) return 1 << 30;
  int32_t worst = 0;
  for (int i = 1; i <= 32; i++) {
    double a = 0.0, b = 0.0;
    for (int n = i, f2 = 2; n > 0; n /= 2, f2 *= 2) a += (double)(n % 2) / f2;
    for (int n = i, f3 = 3; n > 0; n /= 3, f3 *= 3) b += (double)(n % 3) / f3;
    // pixel box of the cell 0 <= a + F < 1, 0 <= b + G < 1
    double ulo = INFINITY, uhi = -INFINITY, vlo = INFINITY, vhi = -INFINITY;
    for (int c = 0; c < 4; c++) {
      const double F = (double)(c & 1) - a, G = (double)(c >> 1) - b;
      const double u = (F * sv_g - G * sv_f) / det, v = (G * su_f - F * su_g) / det;
      ulo = std::min(ulo, u);
      uhi = std::max(uhi, u);
      vlo = std::min(vlo, v);
      vhi = std::max(vhi, v);
    }
    if ((uhi - ulo + 1.0) * (vhi - vlo + 1.0) > 1e5) return 1 << 30;
    int32_t n = 0;
    for (int v = (int)std::floor(vlo); v <= (int)std::ceil(vhi); v++)
      for (int u = (int)std::floor(ulo); u <= (int)std::ceil(uhi); u++) {
        const double F = a + u * su_f + v * sv_f, G = b + u * su_g + v * sv_g;
        n += (F >= 0.0 && F < 1.0 && G >= 0.0 && G < 1.0) ? 1 : 0;
      }
    worst = std::max(worst, n);
  }
  return worst;
}

int32_t window_loads(int32_t pitch, int32_t ng) {
  const int32_t rows = 64 / std::max(1, pitch / 4);
  return rows > 0 ? (ng + rows - 1) / rows : 1 << 30;
}

bool choose_foot(const Camera& cam, int32_t cap, int32_t M, int32_t max_waves, int32_t want_waves, double rays,
                 int32_t nslots_rule, FootShape& out, int32_t pad, int32_t kmax, int32_t reg_waves,
                 int32_t reg_loads, int32_t max_px_in) {
  if (cam.persp) return false;
  const double p = cam.S / (double)cam.W;
  const double* e1 = cam.e1;
  const double* e2 = cam.e2;
  const double* d = cam.e3;
  // pixels a wavefront marches: one or two per lane
  const int32_t max_px = max_px_in > 0 ? max_px_in : (rays > 64.0 ? 128 : 64);
  double best = INFINITY;
  bool found = false;
  for (int b = 1; b <= 2; b++) {
    const int g = 3 - b;
    if (std::fabs(d[b]) < 0.05) continue;  // windows grow as 1 / |d_b|
    const double rf = d[0] / d[b], rg = d[g] / d[b];
    // cell coordinates (f, g on the plane b = 0) per pixel step: the ray
    // origin moves by p e1 per column and p e2 per row
    const double au = p * (e1[0] - e1[b] * rf), av = p * (e2[0] - e2[b] * rf);
    const double bu = p * (e1[g] - e1[b] * rg), bv = p * (e2[g] - e2[b] * rg);
    const double det = au * bv - av * bu;  // plane area per pixel (signed)
    if (!(std::fabs(det) > 1e-9)) continue;
    // rows along f of the window: the cell, the slant over two layers and the
    // margin, about a whole number of 32-float lines
    for (int k = 1; k <= kmax; k++) {
      const double Tf = std::max(4.0, 32.0 * k - 2.0 * std::fabs(rf) - 3.5);
      double Tg = std::max(1.0, rays * std::fabs(det) / Tf);
      // shrink the cells until (nearly) none holds more than 64 pixels: the
      // pixels past the 64th are marched by gathers
      for (int it = 0; it < 8; it++) {
        const int32_t most = foot_max_pixels(au / Tf, av / Tf, bu / Tg, bv / Tg);
        if (most <= max_px || Tg <= 1.0) break;
        Tg = std::max(1.0, Tg * std::min(0.98, (double)max_px / most));
      }
      const int32_t nf = (int32_t)std::floor(Tf + 2.0 * std::fabs(rf) + 0.25) + 3 + pad;
      const int32_t ng = (int32_t)std::floor(Tg + 2.0 * std::fabs(rg) + 0.25) + 3;
      const int32_t pitch = (nf + 3) & ~3;
      const int64_t slot = (int64_t)pitch * ng;
      if (slot > cap || pitch > 256) continue;
      // image rows a cell spans: v extent of the cell's two edge vectors
      const double rows = std::fabs(bu * Tf / det) + std::fabs(au * Tg / det) + 3.0;
      if (rows > 62.0) continue;
      int32_t waves3 = 0, waves2 = 0;
      const int w3 = ring_waves_per_block((int32_t)slot, M, max_waves, &waves3, 3);
      const bool reg = reg_waves > 0 && window_loads(pitch, ng) <= reg_loads;
      const int w2 = ring_waves_per_block((int32_t)slot, M, reg ? std::min(max_waves, reg_waves) : max_waves,
                                          &waves2, 2);
      const bool two = reg || nslots_rule == 2 || (nslots_rule == 0 && waves2 > waves3);
      const int32_t waves = two ? waves2 : waves3;
      if (waves < 2) continue;
      // 128-byte lines per window row (a row starts anywhere in a line), per
      // ray, per unit of ray length (|d_b| layers)
      const double lines = (double)ng * ((double)pitch + 31.0) / 32.0;
      const double cell_rays = Tf * Tg / std::fabs(det);  // mean pixels per cell
      const double cost = lines / cell_rays * std::fabs(d[b]) * std::max(1.0, (double)want_waves / (double)waves);
      if (cost < best) {
        best = cost;
        found = true;
        out.axis = b;
        out.Tf = Tf;
        out.Tg = Tg;
        out.nf = nf;
        out.ng = ng;
        out.slot = (int32_t)slot;
        out.wpb = two ? w2 : w3;
        out.nslots = two ? 2 : 3;
        out.reg = reg ? 1 : 0;
        out.waves = waves;
        out.rf = rf;
        out.rg = rg;
        out.fa_u = au / Tf;
        out.fa_v = av / Tf;
        out.fb_u = bu / Tg;
        out.fb_v = bv / Tg;
        out.rays = cell_rays;
      }
    }
  }
  return found;
}

bool choose_foot_block(const Camera& cam, FootShape& fs, const int64_t ext[3], int32_t M, int32_t max_waves,
                       int32_t want_waves, int32_t reg_loads, int32_t force_f, int32_t force_g) {
  if (cam.persp || fs.axis == 0) return false;
  const int b = fs.axis, g = 3 - b;
  // cells of a typical brick
  Box box;
  for (int i = 0; i < 3; i++) {
    box.lo[i] = 0;
    box.hi[i] = ext[i];
    box.closed[i] = 0;
  }
  int32_t cf0, cg0, ncf, ncg;
  double fa0, fb0;
  foot_cells(cam, fs, box, cf0, cg0, ncf, ncg, fa0, fb0);
  (void)g;
  const double rays = fs.rays;
  // a wavefront per cell: lines per ray and layer
  const int32_t pitch1 = (fs.nf + 3) & ~3;
  const double base_cost = (double)fs.ng * ((double)pitch1 + 31.0) / 32.0 / rays *
                           std::max(1.0, (double)want_waves / std::max(1, fs.waves));
  double best = base_cost;
  bool found = false;
  for (int bf = 1; bf <= 8; bf++)
    for (int bg = 1; bf * bg <= 8; bg++) {
      if (bf * bg < 2) continue;
      if (force_f > 0 && (bf != force_f || bg != force_g)) continue;
      const int32_t nf = (int32_t)std::floor(bf * fs.Tf + 2.0 * std::fabs(fs.rf) + 0.25) + 3;
      const int32_t ng = (int32_t)std::floor(bg * fs.Tg + 2.0 * std::fabs(fs.rg) + 0.25) + 3;
      const int32_t pitch = (nf + 3) & ~3;
      if (pitch > 256 || pitch > ext[0] + 1) continue;
      const int32_t nw = bf * bg;
      const int32_t loads = (window_loads(pitch, ng) + nw - 1) / nw;
      if (loads > reg_loads) continue;
      const int64_t slot = (int64_t)pitch * ng;
      const int64_t lds_wg = 16 * (int64_t)M + 8 * slot + 128;
      int64_t wgs = (160 * 1024) / lds_wg;
      if (wgs * nw > max_waves) wgs = max_waves / nw;
      const int32_t waves = (int32_t)(wgs * nw);
      if (waves < nw || waves < 4) continue;
      // cells the blocks of a typical brick hold, over the cells it has
      const double pad = (double)(((ncf + bf - 1) / bf) * bf) * (double)(((ncg + bg - 1) / bg) * bg) /
                         ((double)ncf * (double)ncg);
      const double lines = (double)ng * ((double)pitch + 31.0) / 32.0;
      const double cost = lines / (nw * rays) * pad * std::max(1.0, (double)want_waves / waves);
      if (cost < best || force_f > 0) {
        best = cost;
        found = true;
        fs.blk_f = bf;
        fs.blk_g = bg;
        fs.blk_nf = nf;
        fs.blk_ng = ng;
        fs.blk_slot = (int32_t)slot;
        fs.blk_waves = waves;
      }
    }
  return found;
}

void foot_cells(const Camera& cam, const FootShape& fs, const Box& box, int32_t& cf0, int32_t& cg0, int32_t& ncf,
                int32_t& ncg, double& fa0, double& fb0) {
  const int b = fs.axis, g = 3 - b;
  // a point q (brick-local) lies on the ray that crosses the plane b = 0 at
  // f = q_f - q_b rf, g = q_g - q_b rg
  double flo = INFINITY, fhi = -INFINITY, glo = INFINITY, ghi = -INFINITY;
  for (int c = 0; c < 8; c++) {
    double q[3];
    for (int i = 0; i < 3; i++) q[i] = (c >> i) & 1 ? (double)(box.hi[i] - box.lo[i]) : 0.0;
    const double f = q[0] - q[b] * fs.rf, gg = q[g] - q[b] * fs.rg;
    flo = std::min(flo, f);
    fhi = std::max(fhi, f);
    glo = std::min(glo, gg);
    ghi = std::max(ghi, gg);
  }
  cf0 = (int32_t)std::floor(flo / fs.Tf - 1e-6);
  cg0 = (int32_t)std::floor(glo / fs.Tg - 1e-6);
  ncf = (int32_t)std::floor(fhi / fs.Tf + 1e-6) - cf0 + 1;
  ncg = (int32_t)std::floor(ghi / fs.Tg + 1e-6) - cg0 + 1;
  double o[3];
  pixel_origin(cam, 0, 0, o);
  const double ob = o[b] - (double)box.lo[b];
  fa0 = ((o[0] - (double)box.lo[0]) - ob * fs.rf) / fs.Tf;
  fb0 = ((o[g] - (double)box.lo[g]) - ob * fs.rg) / fs.Tg;
}

bool persp_cells(const Camera& cam, int b, const Box& box, const Rect& rect, double rays, int32_t kmax,
                 int32_t cap, int32_t reg_loads, PerspCells& out, int32_t max_px) {
  if (!cam.persp || rect.w <= 0 || rect.h <= 0) return false;
  const int g = 3 - b;
  double E[3], ext[3];
  for (int i = 0; i < 3; i++) {
    E[i] = cam.eye[i] - (double)box.lo[i];
    ext[i] = (double)(box.hi[i] - box.lo[i]);
  }
  // the eye well outside the brick's slab along b: every ray of the brick
  // then crosses the planes b = const one way, in front of the eye
  if (!(E[b] < -8.0 || E[b] > ext[b] + 8.0)) return false;
  const double sgn = E[b] < 0.0 ? 1.0 : -1.0;  // sign of w_b toward the brick
  const double px0 = rect.x0 - 0.5, py0 = rect.y0 - 0.5, px1 = rect.x0 + rect.w - 0.5, py1 = rect.y0 + rect.h - 0.5;
  for (int c = 0; c < 4; c++) {
    const double u = (c & 1) ? px1 : px0, v = (c & 2) ? py1 : py0;
    const double x = ((u + 0.5) / (double)cam.W - 0.5) * cam.S;
    const double y = ((v + 0.5) / (double)cam.H - 0.5) * cam.S * (double)cam.H / (double)cam.W;
    const double wb = x * cam.e1[b] + y * cam.e2[b] + cam.D * cam.e3[b];
    if (!(sgn * wb > 1e-3 * cam.D)) return false;
  }
  // the brick seen from the eye on the plane b = 0 (its corners, one voxel of
  // margin): every ray through the brick crosses the plane in this box
  double flo = INFINITY, fhi = -INFINITY, glo = INFINITY, ghi = -INFINITY;
  for (int c = 0; c < 8; c++) {
    double q[3];
    for (int i = 0; i < 3; i++) q[i] = (c >> i) & 1 ? ext[i] + 1.0 : -1.0;
    const double t = -E[b] / (q[b] - E[b]);
    const double f = E[0] + t * (q[0] - E[0]), gg = E[g] + t * (q[g] - E[g]);
    flo = std::min(flo, f);
    fhi = std::max(fhi, f);
    glo = std::min(glo, gg);
    ghi = std::max(ghi, gg);
  }
  // scale of the plane b = V against b = 0 about the eye's foot point, over
  // the voxel layers a window can cover
  const double s_a = 1.0 - (-2.0) / E[b], s_b = 1.0 - (ext[b] + 3.0) / E[b];
  const double s_max = std::max(s_a, s_b);
  // growth of a window over its two layers: the scale changes by 2 / |E_b|
  // across them, times the distance from the eye's foot point
  const double slant_f = 2.0 * std::max(std::fabs(flo - E[0]), std::fabs(fhi - E[0])) / std::fabs(E[b]);
  const double slant_g = 2.0 * std::max(std::fabs(glo - E[g]), std::fabs(ghi - E[g])) / std::fabs(E[b]);
  // plane coordinates per pixel step at the rectangle's corners and centre;
  // the densest point sizes the cells, the one with the most image rows per
  // cell bounds the rows a cell spans
  double su_f = 0, sv_f = 0, su_g = 0, sv_g = 0, det_min = INFINITY, rows_f = 0.0, rows_g = 0.0;
  for (int c = 0; c < 5; c++) {
    const double u = c == 4 ? 0.5 * (px0 + px1) : ((c & 1) ? px1 : px0);
    const double v = c == 4 ? 0.5 * (py0 + py1) : ((c & 2) ? py1 : py0);
    double f0, g0, fu, gu, fv, gv;
    persp_plane_point(cam, E, b, g, u, v, f0, g0);
    persp_plane_point(cam, E, b, g, u + 1.0, v, fu, gu);
    persp_plane_point(cam, E, b, g, u, v + 1.0, fv, gv);
    const double au = fu - f0, av = fv - f0, bu = gu - g0, bv = gv - g0;
    const double det = au * bv - av * bu;
    if (!(std::fabs(det) > 1e-12)) return false;
    if (std::fabs(det) < det_min) {
      det_min = std::fabs(det);
      su_f = au;
      sv_f = av;
      su_g = bu;
      sv_g = bv;
    }
    // image rows per unit of f and of g (the inverse map's v row)
    rows_f = std::max(rows_f, std::fabs(bu / det));
    rows_g = std::max(rows_g, std::fabs(au / det));
  }
  double best = INFINITY;
  bool found = false;
  // fewer rays per cell shrink the windows of far bricks (sparse rays), which
  // lets more wavefronts share a compute unit: the cost weighs the lines per
  // ray by the occupancy shortfall below 16 wavefronts
  for (int k = 1; k <= kmax; k++)
  for (const double rr : {rays, 0.8 * rays, 0.65 * rays, 0.5 * rays}) {
    const double Tf = (32.0 * k - slant_f - 3.5) / s_max;
    if (Tf < 4.0) continue;
    double Tg = std::max(1.0, rr * det_min / Tf);
    int32_t most = 0;
    for (int it = 0; it < 8; it++) {
      most = foot_max_pixels(su_f / Tf, sv_f / Tf, su_g / Tg, sv_g / Tg);
      if (most <= max_px || Tg <= 1.0) break;
      Tg = std::max(1.0, Tg * std::min(0.98, (double)max_px / most));
    }
    if (most > max_px) continue;  // too many pixels even in the thinnest cells of this width
    // the cells of the grid's first and last columns and rows reach up to
    // two cells past the brick's box: their distance from the foot point
    const double wf = 2.0 * std::max(std::fabs(flo - 2.0 * Tf - E[0]), std::fabs(fhi + 2.0 * Tf - E[0])) /
                      std::fabs(E[b]);
    const double wg = 2.0 * std::max(std::fabs(glo - 2.0 * Tg - E[g]), std::fabs(ghi + 2.0 * Tg - E[g])) /
                      std::fabs(E[b]);
    const int32_t nf = (int32_t)std::floor(s_max * Tf + wf + 0.25) + 3;
    const int32_t ng = (int32_t)std::floor(s_max * Tg + wg + 0.25) + 3;
    const int32_t pitch = (nf + 3) & ~3;
    if ((int64_t)pitch * ng > cap || pitch > 256 || window_loads(pitch, ng) > reg_loads) continue;
    if (rows_f * Tf + rows_g * Tg + 4.0 > 60.0) continue;
    const double cell_rays = Tf * Tg / det_min;
    int32_t waves = 0;
    ring_waves_per_block(pitch * ng, 256, 16, &waves, 2);
    const double cost = (double)ng * ((double)pitch + 31.0) / 32.0 / cell_rays * std::max(1.0, 16.0 / std::max(1, waves));
    if (cost < best) {
      best = cost;
      found = true;
      out.Tf = Tf;
      out.Tg = Tg;
      out.pitch = pitch;
      out.ng = ng;
      out.rays = cell_rays;
    }
  }
  if (!found) return false;
  out.cf0 = (int32_t)std::floor(flo / out.Tf) - 1;
  out.cg0 = (int32_t)std::floor(glo / out.Tg) - 1;
  out.ncf = (int32_t)std::floor(fhi / out.Tf) + 1 - out.cf0 + 1;
  out.ncg = (int32_t)std::floor(ghi / out.Tg) + 1 - out.cg0 + 1;
  return true;
}

void foot_traffic(const Camera& cam, const FootShape& fs, const Box& box, const int64_t n[3], FootTraffic& t) {
  const int b = fs.axis, g = 3 - b;
  int64_t ext[3];
  for (int i = 0; i < 3; i++) ext[i] = box.hi[i] - box.lo[i];
  t.own += 4.0 * (double)(ext[0] + (box.closed[0] ? 1 : 0)) * (double)(ext[1] + (box.closed[1] ? 1 : 0)) *
           (double)(ext[2] + (box.closed[2] ? 1 : 0));
  // clamps of the local cell index, as on the device: the brick's stored
  // range (its box and one ghost voxel each side, inside the volume) - lo, the
  // last cell one short of the last stored voxel
  int64_t slo[3], shi[3];
  stored_box(box, n, slo, shi);
  const int64_t cloF = slo[0] - box.lo[0], chiF = shi[0] - 1 - box.lo[0];
  const int64_t cloG = slo[g] - box.lo[g], chiG = shi[g] - 1 - box.lo[g];
  const int64_t cloB = slo[b] - box.lo[b], chiB = shi[b] - 1 - box.lo[b];
  const int64_t pitch = (fs.nf + 3) & ~3;
  const int64_t NG = std::min<int64_t>(fs.ng, chiG + 2 - cloG);
  const int64_t sG = g == 1 ? n[0] : n[0] * n[1], sB = b == 1 ? n[0] : n[0] * n[1];
  const double rf = fs.rf, rg = fs.rg, arf = std::fabs(rf), arg = std::fabs(rg);
  int32_t cf0, cg0, ncf, ncg;
  double fa0, fb0;
  foot_cells(cam, fs, box, cf0, cg0, ncf, ncg, fa0, fb0);
  // per (voxel layer, window row): the f range any window covers
  const int64_t v_lo = std::max<int64_t>(cloB, -2), v_hi = std::min<int64_t>(chiB + 1, ext[b] + 2);
  const int64_t g_lo = cloG, g_hi = chiG + 1;
  if (v_hi < v_lo || g_hi < g_lo) return;
  const int64_t nv = v_hi - v_lo + 1, nrow = std::min<int64_t>(g_hi - g_lo + 1, ext[g] + 2 * NG + 8);
  const int64_t g_base = std::max<int64_t>(g_lo, -NG - 4);
  std::vector<int64_t> fmin((size_t)(nv * nrow), INT64_MAX), fmax((size_t)(nv * nrow), INT64_MIN);
  const double eb = (double)ext[b] + (box.closed[b] ? 1.0 : 0.0);
  for (int32_t cj = cg0; cj < cg0 + ncg; cj++)
    for (int32_t ci = cf0; ci < cf0 + ncf; ci++) {
      const double F0 = ci * fs.Tf, F1 = (ci + 1) * fs.Tf, G0 = cj * fs.Tg, G1 = (cj + 1) * fs.Tg;
      // cell layers c (samples with c <= q_b < c + 1) in which some ray of
      // the cell is inside the box along f and g
      int64_t c0 = INT64_MAX, c1 = INT64_MIN;
      for (int64_t c = 0; c < (int64_t)std::ceil(eb); c++) {
        const double lo_b = (double)c, hi_b = std::min((double)(c + 1), eb);
        const double f_lo = F0 + std::min(lo_b * rf, hi_b * rf), f_hi = F1 + std::max(lo_b * rf, hi_b * rf);
        const double gg_lo = G0 + std::min(lo_b * rg, hi_b * rg), gg_hi = G1 + std::max(lo_b * rg, hi_b * rg);
        if (f_hi <= 0.0 || f_lo >= (double)ext[0] + (box.closed[0] ? 1e-9 : 0.0)) continue;
        if (gg_hi <= 0.0 || gg_lo >= (double)ext[g] + (box.closed[g] ? 1e-9 : 0.0)) continue;
        c0 = std::min(c0, c);
        c1 = std::max(c1, c);
      }
      if (c1 < c0) continue;
      t.cells += 1.0;
      // voxel layers c0 .. c1 + 1, whichever way the rays run
      for (int64_t V = c0; V <= c1 + 1; V++) {
        t.layers += 1.0;
        const int64_t flo = std::max<int64_t>((int64_t)std::floor(F0 + V * rf - arf - 0.05), cloF);
        const int64_t glo = std::max<int64_t>((int64_t)std::floor(G0 + V * rg - arg - 0.05), cloG);
        const int64_t f0 = std::max(cloF, std::min(flo, chiF + 2 - pitch));
        const int64_t g0 = std::max(cloG, std::min(glo, chiG + 2 - NG));
        t.win += 4.0 * (double)(pitch * NG);
        const int64_t iv = V - v_lo;
        for (int64_t r = 0; r < NG; r++) {
          const int64_t row = box.lo[0] + (box.lo[g] + g0 + r) * sG + (box.lo[b] + V) * sB;
          const int64_t a0 = row + f0;
          t.line += 128.0 * (double)((a0 + pitch - 1) / 32 - a0 / 32 + 1);
          t.seg += 64.0 * (double)((a0 + pitch - 1) / 16 - a0 / 16 + 1);
          const int64_t ir = g0 + r - g_base;
          if (iv < 0 || iv >= nv || ir < 0 || ir >= nrow) continue;
          const size_t k = (size_t)(iv * nrow + ir);
          fmin[k] = std::min(fmin[k], a0);
          fmax[k] = std::max(fmax[k], a0 + pitch);
        }
      }
    }
  for (size_t k = 0; k < fmin.size(); k++)
    if (fmax[k] > fmin[k]) t.uni += 128.0 * (double)((fmax[k] - 1) / 32 - fmin[k] / 32 + 1);
}

// Window floats of the perspective ring march for the 8 x 8 tile with corner
// pixels (cx, cy) .. (ex, ey) over box r, on the better of axes 2 and 3 (the
// kernel's choice, bounded over the box's layers); infinity when neither suits.
static double persp_tile_window(const Camera& cam, const TileRegion& r, int cx, int cy, int ex, int ey) {
  double oc[3], dc[4][3];
  for (int k = 0; k < 4; k++) pixel_ray(cam, (k & 1) ? ex : cx, (k & 2) ? ey : cy, oc, dc[k]);
  double best = INFINITY;
  for (int b = 1; b <= 2; b++) {
    const int g = 3 - b;
    bool ok = true;
    for (int k = 0; k < 4 && ok; k++)
      ok = std::fabs(dc[k][b]) > 1e-6 && (dc[k][b] > 0.0) == (dc[0][b] > 0.0);
    if (!ok) continue;
    const double Va = (double)r.lo[b] - 1.0, Vb = (double)r.hi[b] + 1.0;
    double wf = 0.0, wg = 0.0;
    for (double V : {Va, Vb}) {
      double lf = INFINITY, hf = -INFINITY, lg = INFINITY, hg = -INFINITY;
      for (int k = 0; k < 4; k++) {
        const double rf = dc[k][0] / dc[k][b], rg = dc[k][g] / dc[k][b];
        for (double P : {V - 1.0, V + 1.0}) {
          const double f = oc[0] + (P - oc[b]) * rf, q = oc[g] + (P - oc[b]) * rg;
          lf = std::min(lf, f);
          hf = std::max(hf, f);
          lg = std::min(lg, q);
          hg = std::max(hg, q);
        }
      }
      wf = std::max(wf, hf - lf);
      wg = std::max(wg, hg - lg);
    }
    if (!(wf < 4096.0 && wg < 4096.0)) continue;
    const double pitch = 4.0 * std::ceil((std::floor(wf + 0.2) + 3.0) / 4.0);
    const double ng = std::min(std::floor(wg + 0.2) + 3.0, (double)(r.hi[g] - r.lo[g]) + 4.0);
    best = std::min(best, pitch * ng);
  }
  return best;
}

double persp_region_window(const Camera& cam, const TileRegion& r) {
  if (r.w <= 0 || r.h <= 0) return 0.0;
  const int ntx = (r.w + 7) / 8, nty = (r.h + 7) / 8;
  const int sx[5] = {0, ntx - 1, 0, ntx - 1, ntx / 2}, sy[5] = {0, 0, nty - 1, nty - 1, nty / 2};
  double worst = 0.0;
  for (int k = 0; k < 5; k++) {
    const int cx = r.x0 + 8 * sx[k], cy = r.y0 + 8 * sy[k];
    const int ex = std::min(cx + 7, r.x0 + r.w - 1), ey = std::min(cy + 7, r.y0 + r.h - 1);
    worst = std::max(worst, persp_tile_window(cam, r, cx, cy, ex, ey));
  }
  return worst;
}

bool choose_ring_persp(const Camera& cam, const std::vector<TileRegion>& regs, int32_t cap, int32_t M,
                       int32_t max_waves, int32_t min_waves, int32_t& slot, int32_t& wpb, double fit) {
  std::vector<std::pair<double, double>> est;  // (window of the region's worst sampled tile, tiles)
  double total = 0.0;
  for (const TileRegion& r : regs) {
    if (r.w <= 0 || r.h <= 0) continue;
    const int ntx = (r.w + 7) / 8, nty = (r.h + 7) / 8;
    est.emplace_back(persp_region_window(cam, r), (double)ntx * nty);
    total += (double)ntx * nty;
  }
  if (est.empty()) return false;
  std::sort(est.begin(), est.end());
  double acc = 0.0, need = INFINITY;
  for (const auto& e : est) {
    acc += e.second;
    if (acc >= fit * total) {
      need = e.first;
      break;
    }
  }
  if (!(need <= (double)cap)) {
    // windows past the cap read global memory; worthwhile only for a minority
    double fit = 0.0;
    for (const auto& e : est)
      if (e.first <= (double)cap) fit += e.second;
    if (fit < 0.5 * total) return false;
    need = (double)cap;
  }
  slot = (int32_t)(4.0 * std::ceil(need / 4.0));
  int32_t waves = 0;
  wpb = ring_waves_per_block(slot, M, max_waves, &waves);
  return waves >= min_waves;
}

int64_t count_samples(const Camera& cam, const int64_t n[3], double step) {
  const double hi[3] = {(double)(n[0] - 1), (double)(n[1] - 1), (double)(n[2] - 1)};
  int64_t total = 0;
  for (int v = 0; v < cam.H; v++)
    for (int u = 0; u < cam.W; u++) {
      double o[3], d[3], tin;
      int64_t k;
      pixel_ray(cam, u, v, o, d);
      if (ray_lattice(o, d, hi, step, tin, k)) total += k;
    }
  return total;
}

}  // namespace vr
