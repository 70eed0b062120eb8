// Host-only planning code of libvr (partitions, rendering rectangles, depth
// order, front-to-back waves, march shape choices, sample counts) driven over
// a range of volumes, partitions and views, for builds with AddressSanitizer
// and UndefinedBehaviorSanitizer.  Exits non-zero when an invariant fails.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "plan.h"

using namespace vr;

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static double urand() {  // splitmix64 -> [0, 1)
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// rotation from a random unit quaternion
static void rand_rotation(double R[9]) {
  double q[4], s = 0.0;
  for (double& x : q) {
    x = urand() * 2.0 - 1.0;
    s += x * x;
  }
  s = std::sqrt(s);
  for (double& x : q) x /= s;
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  const double M[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - z * w),     2 * (x * z + y * w),
                       2 * (x * y + z * w),     1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                       2 * (x * z - y * w),     2 * (y * z + x * w),     1 - 2 * (x * x + y * y)};
  for (int i = 0; i < 9; i++) R[i] = M[i];
}

static int fails = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      fails++;                                                        \
    }                                                                 \
  } while (0)

int main() {
  const int64_t dims[][3] = {{2, 2, 2}, {17, 9, 33}, {64, 64, 64}, {300, 257, 129}, {2048, 2048, 1536}};
  const float tf[4 * 8] = {0, 0, 0, 0, 0, 0, 0, 0, 0.1f, 0.1f, 0.1f, 0.01f, 0.2f, 0.2f, 0.2f, 0.02f,
                           0.3f, 0.3f, 0.3f, 0.03f, 0.4f, 0.4f, 0.4f, 0.04f, 0.5f, 0.5f, 0.5f, 0.05f, 1, 1, 1, 0.1f};
  for (const auto& n : dims) {
    std::vector<Partition> parts;
    {
      Partition g;
      std::string err;
      const int64_t bs[3] = {std::max<int64_t>(1, (n[0] - 1) / 3), std::max<int64_t>(1, (n[1] - 1) / 2),
                             std::max<int64_t>(1, n[2] / 5)};
      if (make_grid(n, bs, g, err)) parts.push_back(g);
      Partition k;
      if (make_kd(n, 7, k, err)) parts.push_back(k);
      Partition one;
      if (make_kd(n, 1, one, err)) parts.push_back(one);
    }
    CHECK(!parts.empty());
    for (const Partition& P : parts) {
      // ownership boxes tile the volume's cells
      double vol = 0.0;
      for (const Box& b : P.boxes) {
        double v = 1.0;
        for (int i = 0; i < 3; i++) {
          CHECK(b.lo[i] >= 0 && b.hi[i] <= n[i] - 1 && b.lo[i] < b.hi[i]);
          v *= (double)(b.hi[i] - b.lo[i]);
        }
        vol += v;
        int64_t slo[3], shi[3];
        stored_box(b, n, slo, shi);
        for (int i = 0; i < 3; i++) CHECK(slo[i] >= 0 && shi[i] <= n[i] - 1 && slo[i] <= shi[i]);
      }
      CHECK(std::fabs(vol - (double)(n[0] - 1) * (n[1] - 1) * (n[2] - 1)) < 0.5);
      Partition tw;
      const int64_t nt[3] = {n[1], n[2], n[0]};
      permute_partition(P, nt, tw);
      CHECK(tw.boxes.size() == P.boxes.size());
      for (int k = 0; k < 12; k++) {
        vr_view view;
        rand_rotation(view.R);
        view.W = 1 + (int)(urand() * 200);
        view.H = 1 + (int)(urand() * 200);
        view.extent = 0.0;
        view.eye_dist = (k % 3 == 2) ? 2.0 * std::sqrt((double)(n[0] * n[0] + n[1] * n[1] + n[2] * n[2])) : 0.0;
        Camera cam;
        make_camera(view, n, cam);
        for (const Box& b : P.boxes) {
          const Rect r = brick_rect(cam, b);
          CHECK(r.w >= 0 && r.h >= 0 && r.x0 >= 0 && r.y0 >= 0 && r.x0 + r.w <= view.W && r.y0 + r.h <= view.H);
          (void)brick_transparent(-1.f, 2.f, tf, 8, 0.0, 1.0);
        }
        std::vector<int32_t> order, wave;
        depth_order(P, cam, order);
        CHECK(order.size() == P.boxes.size());
        std::vector<int> seen(P.boxes.size(), 0);
        for (int32_t b : order) {
          CHECK(b >= 0 && b < (int32_t)P.boxes.size());
          if (b >= 0 && b < (int32_t)P.boxes.size()) seen[b]++;
        }
        for (int s : seen) CHECK(s == 1);
        const int32_t nw = brick_waves(P, cam, wave);
        CHECK(nw >= 1 && wave.size() == P.boxes.size());
        for (int32_t w : wave) CHECK(w >= 0 && w < nw);
        int32_t ax = 0, T = 0, slot = 0, wpb = 0, waves = 0;
        (void)choose_slab(cam, 8, 8, 4096, ax, T);
        (void)choose_ring(cam, 8192, 256, 24, 12, 2, ax, slot, wpb, 3, &waves);
        if (cam.persp) {
          std::vector<TileRegion> regs;
          for (const Box& b : P.boxes) {
            const Rect r = brick_rect(cam, b);
            if (r.w == 0 || r.h == 0) continue;
            TileRegion t;
            for (int i = 0; i < 3; i++) {
              t.lo[i] = b.lo[i];
              t.hi[i] = b.hi[i];
            }
            t.x0 = r.x0;
            t.y0 = r.y0;
            t.w = r.w;
            t.h = r.h;
            regs.push_back(t);
          }
          (void)choose_ring_persp(cam, regs, 8192, 256, 24, 2, slot, wpb);
        } else {
          FootShape fs;
          if (choose_foot(cam, 8192, 256, 24, 12, 60.0, 0, fs)) {
            CHECK(fs.slot > 0 && fs.slot <= 8192 && fs.Tf > 0 && fs.Tg > 0);
            for (const Box& b : P.boxes) {
              int32_t cf0, cg0, ncf, ncg;
              double fa0, fb0;
              foot_cells(cam, fs, b, cf0, cg0, ncf, ncg, fa0, fb0);
              CHECK(ncf >= 1 && ncg >= 1 && std::isfinite(fa0) && std::isfinite(fb0));
            }
          }
        }
        if (n[0] * n[1] * n[2] < 1000000) CHECK(count_samples(cam, n, 0.5) >= 0);
      }
    }
  }
  std::printf("plan driver: %d failed checks\n", fails);
  return fails == 0 ? 0 : 1;
}
