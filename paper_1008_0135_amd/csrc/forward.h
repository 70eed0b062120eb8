// forward.h -- forward-path planning and launch sequence shared by the
// forward, differentiable and autotuning entry points.
#pragma once

#include <vector>

#include "runtime.h"

namespace vr {

struct ViewPlan {
  std::vector<DevBrickView> bv;       // rendered bricks, launch order
  std::vector<int32_t> layers_order;  // indices into bv, front to back
  int32_t ntiles = 0;
  int64_t pixels = 0;                 // brick-image pixels of this view
  // opacity tested over the whole ray: bv grouped into front-to-back waves,
  // wave w = bv[wave_begin[w] .. wave_begin[w + 1]) with tile_begin counted
  // from the wave's first brick and wave_tiles[w] tiles
  std::vector<int32_t> wave_begin, wave_tiles;
  // perspective ring march: bv grouped into classes of bricks with similar
  // windows, class c = bv[class_begin[c] .. class_begin[c + 1]) with
  // tile_begin counted from the class's first brick and class_tiles[c] tiles
  // (empty: one launch for the view)
  std::vector<int32_t> class_begin, class_tiles;
  // perspective views on footprint cells sized per brick (pfoot): bv counts
  // cells, grouped into the classes above by window size; paxis = slab axis
  bool pfoot = false;
  int32_t paxis = 0;
  // ring march over footprint cells (parallel rays): bv counts cells, not tiles
  bool foot = false;
  FootShape fs;
};

// Hook that replaces the march launch (the differentiable forward saves
// per-ray state from its own kernel variant).
struct ForwardExtras {
  virtual ~ForwardExtras() {}
  virtual void prepare(MarchArgs& a, int32_t view) = 0;
  virtual hipError_t launch(const MarchArgs& a, hipStream_t s) = 0;
  double vmin = 0.0, vmax = 0.0;
};

// Footprint-cell shape of one parallel view of a volume of size n, as the
// forward picks it: plain = the plain march (no macrocell skipping, no mask),
// reg_on = register staging allowed, nslots = the ring-slot rule (0, 2 or 3),
// cells of about `rays` pixels with window rows of at most kmax 128-byte
// lines (+ pad floats).  False when the view has no suitable slab axis.
bool pick_foot(const Camera& cam, const int64_t n[3], int32_t M, bool plain, bool reg_on, int32_t nslots,
               double rays, int32_t pad, int32_t kmax, FootShape& fs, int32_t max_px = 0);

void plan_bricked_view(const vr_volume* vol, const Camera& cam, const vr_params* p, int32_t tile_w, const float* tf,
                       int32_t M, double vmin, double vmax, ViewPlan& vp, bool waves = false);
int render_forward(vr_ctx* ctx, vr_volume* vol, const vr_view* views, int32_t nviews, const vr_params* p, float* out,
                   hipStream_t s, ForwardExtras* extras);
int validate_render(vr_ctx* ctx, const vr_volume* vol, const vr_view* views, int32_t nviews, const vr_params* p);
int render_with_state(vr_ctx* ctx, vr_volume* vol, const vr_view* views, int32_t nviews, const vr_params* p,
                      float* out, hipStream_t s, vr_state** save);

}  // namespace vr
