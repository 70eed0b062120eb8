// forward.cpp -- forward rendering entry points: vr_render (whole volume or
// bricks + composite), vr_render_bricks and vr_composite (the two halves of
// sort-last compositing, paper Sec. 2.4 and 2.5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "forward.h"
#include "plan.h"
#include "runtime.h"
#include "vr_internal.h"

namespace vr {

namespace {

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// Ring march limits: window floats per slot, and wavefronts per compute unit
// the kernel's registers allow (78 VGPRs: 6 per SIMD).
constexpr int32_t kRingCap = 8192;
constexpr int32_t kRingMaxWaves = 24;
constexpr int32_t kRingWantWaves = 12;  // below this the march starts to wait on its loads
constexpr int32_t kRingMinWaves = 2;
// register-staged cells march: its registers leave room for 4 wavefronts per SIMD
constexpr int32_t kRingRegWaves = 16;
constexpr int32_t kLdsPerCu = 160 * 1024;

}  // namespace

bool pick_foot(const Camera& cam, const int64_t n[3], int32_t M, bool plain, bool reg_on, int32_t nslots,
               double rays, int32_t pad, int32_t kmax, FootShape& fs, int32_t max_px) {
  // register-staged cells: a lane's offset inside a window's rows (at most
  // kRingRegLoads instructions of up to 16 rows) must stay below 4 GiB
  const int64_t row_stride = std::max(n[0], n[0] * n[1]);
  const bool reg = plain && reg_on && nslots != 3 && ((int64_t)kRingRegLoads * 16 * row_stride + 256) * 4 < ((int64_t)1 << 32);
  const bool two = rays > 64.0;  // two pixels per lane: half the wavefronts, twice the window loads
  const int32_t rw = two ? kRingRegWaves / 2 : kRingRegWaves;
  return choose_foot(cam, kRingCap, M, kRingMaxWaves, reg ? rw : kRingWantWaves, rays, plain ? nslots : 3, fs, pad,
                     kmax, reg ? rw : 0, two ? 2 * kRingRegLoads : kRingRegLoads, max_px);
}

// Plan one view of a bricked volume: rectangles, culling (empty rectangle or
// transparent brick), launch order (brick index order, which keeps
// neighbouring bricks together), arena offsets and the front-to-back layers.
void plan_bricked_view(const vr_volume* vol, const Camera& cam, const vr_params* p, int32_t tile_w,
                       const float* tf, int32_t M, double vmin, double vmax, ViewPlan& vp, bool waves) {
  const Partition& P = vol->part;
  const int32_t nb = (int32_t)P.boxes.size();
  const int32_t tile_h = 64 / tile_w;
  std::vector<Rect> rects((size_t)nb);
  std::vector<int32_t> slot((size_t)nb, -1);
  vp.bv.clear();
  vp.layers_order.clear();
  int32_t tiles = 0;
  int64_t pix = 0;
  for (int32_t b = 0; b < nb; b++) {
    rects[b] = brick_rect(cam, P.boxes[b]);
    if (rects[b].w == 0 || rects[b].h == 0) continue;
    if (p->ess && p->mode == VR_MODE_DVR &&
        brick_transparent(vol->bricks[b].vmin, vol->bricks[b].vmax, tf, M, vmin, vmax))
      continue;
    DevBrickView v;
    std::memset(&v, 0, sizeof v);
    v.brick = b;
    v.x0 = rects[b].x0;
    v.y0 = rects[b].y0;
    v.w = rects[b].w;
    v.h = rects[b].h;
    v.tiles_x = (v.w + tile_w - 1) / tile_w;
    v.tile_begin = tiles;
    v.img_off = pix;
    tiles += v.tiles_x * ((v.h + tile_h - 1) / tile_h);
    pix += (int64_t)v.w * v.h;
    slot[b] = (int32_t)vp.bv.size();
    vp.bv.push_back(v);
  }
  std::vector<int32_t> order;
  depth_order(P, cam, order);
  for (int32_t b : order)
    if (slot[b] >= 0) vp.layers_order.push_back(slot[b]);
  vp.ntiles = tiles;
  vp.pixels = pix;
  vp.wave_begin.clear();
  vp.wave_tiles.clear();
  if (waves) {
    std::vector<int32_t> wave;
    const int32_t nw = brick_waves(P, cam, wave);
    std::vector<DevBrickView> by_wave;
    by_wave.reserve(vp.bv.size());
    for (int32_t w = 0; w < nw; w++) {
      const int32_t first = (int32_t)by_wave.size();
      int32_t t = 0;
      for (const DevBrickView& b : vp.bv)
        if (wave[b.brick] == w) {
          DevBrickView c = b;
          c.tile_begin = t;
          t += c.tiles_x * ((c.h + tile_h - 1) / tile_h);
          by_wave.push_back(c);
        }
      if (t == 0) continue;
      vp.wave_begin.push_back(first);
      vp.wave_tiles.push_back(t);
    }
    vp.wave_begin.push_back((int32_t)by_wave.size());
    vp.bv.swap(by_wave);
    vp.layers_order.clear();  // no brick images to composite
  }
}

int render_forward(vr_ctx* ctx, vr_volume* vol, const vr_view* views, int32_t nviews, const vr_params* p,
                   float* out, hipStream_t s, ForwardExtras* extras) {
  const bool bricked = vol->bricked;
  const int32_t W = views[0].W, H = views[0].H;
  double vmin, vmax;
  VR_TRY(resolve_window(ctx, vol, s, vmin, vmax));
  MarchArgs base;
  std::memset(&base, 0, sizeof base);
  int32_t tuned_tile, budget, mode;
  tuned_shape(ctx, vol, W, H, p, tuned_tile, budget, mode);
  vr_params pt = *p;
  pt.tile = tuned_tile;
  fill_march_common(base, vol, &pt, vmin, vmax, ctx->d_tf, ctx->tf_m);
  if (ctx->mask_n > 0) {
    if (vol->n[vol->spectral_axis] != ctx->mask_n)
      return fail(VR_EINVAL, "mask length %d differs from the volume's axis-3 size %lld", ctx->mask_n,
                  (long long)vol->n[vol->spectral_axis]);
    base.mask = ctx->d_mask;
  }
  if (!extras) VR_TRY(prepare_macrocells(ctx, vol, p, vmin, vmax, base, s));
  const int32_t tw = base.tile_w, th = base.tile_h;
  // opacity tested over the whole ray: bricks marched in front-to-back waves
  // straight into the frame, each ray carrying its state from brick to brick
  const bool global = bricked && out && !extras && !base.mip && p->ert_scope == VR_ERT_GLOBAL;

  std::vector<ViewPlan> plans((size_t)nviews);
  std::vector<Camera> cams((size_t)nviews);
  int64_t arena_pix = 0;
  for (int32_t v = 0; v < nviews; v++) {
    make_camera(views[v], vol->n, cams[v]);
    ViewPlan& vp = plans[v];
    if (bricked) {
      plan_bricked_view(vol, cams[v], p, tw, ctx->h_tf.data(), ctx->tf_m, vmin, vmax, vp, global);
      if (!global) arena_pix = std::max(arena_pix, vp.pixels);
    } else {
      DevBrickView b;
      std::memset(&b, 0, sizeof b);
      b.brick = 0;
      b.w = W;
      b.h = H;
      b.tiles_x = (W + tw - 1) / tw;
      b.tile_begin = 0;
      b.img_off = (int64_t)v * W * H;
      vp.bv.assign(1, b);
      vp.ntiles = b.tiles_x * ((H + th - 1) / th);
      vp.pixels = (int64_t)W * H;
    }
  }
  // perspective views on the ring march: rays from the eye spread with depth,
  // so the 8 x 8 tiles of far bricks need windows about twice those of near
  // ones, and one slot sized for nearly all tiles leaves the near bricks at a
  // fraction of the wavefronts their windows allow.  Bricks are grouped into
  // classes of similar window (about equal tile counts), launched one class
  // at a time with a slot of its own.
  // bricks of a view grouped into ncls classes of about equal work by a size
  // key (the window), launched one class at a time; items(b): the work items
  // (tiles or cells) of brick view b
  auto group_classes = [&](ViewPlan& vp, const std::vector<double>& key, int32_t ncls, auto items) {
    std::vector<int32_t> idx(vp.bv.size());
    int64_t total = 0;
    for (int32_t i = 0; i < (int32_t)vp.bv.size(); i++) {
      idx[i] = i;
      total += items(vp.bv[i]);
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return key[x] < key[y]; });
    // class boundaries at about equal work; within a class, brick order
    std::vector<int32_t> cls(vp.bv.size(), 0);
    int64_t acc = 0;
    for (int32_t i : idx) {
      cls[i] = (int32_t)std::min<int64_t>(ncls - 1, acc * ncls / std::max<int64_t>(1, total));
      acc += items(vp.bv[i]);
    }
    std::vector<DevBrickView> nbv;
    std::vector<int32_t> where(vp.bv.size(), -1);
    nbv.reserve(vp.bv.size());
    vp.class_begin.clear();
    vp.class_tiles.clear();
    for (int32_t c = 0; c < ncls; c++) {
      const int32_t first = (int32_t)nbv.size();
      int32_t t = 0;
      for (int32_t i = 0; i < (int32_t)vp.bv.size(); i++)
        if (cls[i] == c) {
          DevBrickView b = vp.bv[i];
          b.tile_begin = t;
          t += (int32_t)items(b);
          where[i] = (int32_t)nbv.size();
          nbv.push_back(b);
        }
      if (t == 0) continue;
      vp.class_begin.push_back(first);
      vp.class_tiles.push_back(t);
    }
    vp.class_begin.push_back((int32_t)nbv.size());
    for (int32_t& l : vp.layers_order) l = where[l];
    vp.bv.swap(nbv);
  };
  // perspective views on footprint cells sized per brick (the plain march of
  // emission-absorption or MIP, register-staged): one slab axis for the view,
  // the one along which the eye lies outside every brick's slab.  A view
  // where some brick does not suit keeps the 8 x 8 tiles.
  for (int32_t v = 0; v < nviews; v++) {
    ViewPlan& vp = plans[v];
    vp.pfoot = false;
    if (!bricked || global || extras || !cams[v].persp || !(mode == 0 || mode == 3) || tw != 8 ||
        !ctx->persp_cells || base.mc != 0 || base.mask || ctx->ring_reg <= 0 || ctx->ring_nslots == 3 ||
        vp.bv.empty())
      continue;
    const int first_axis = std::fabs(cams[v].e3[1]) >= std::fabs(cams[v].e3[2]) ? 1 : 2;
    std::vector<PerspCells> pcs(vp.bv.size());
    int axis = 0;
    for (int tryax : {first_axis, 3 - first_axis}) {
      bool all = true;
      for (size_t i = 0; i < vp.bv.size() && all; i++) {
        const DevBrickView& b = vp.bv[i];
        Rect rc;
        rc.x0 = b.x0;
        rc.y0 = b.y0;
        rc.w = b.w;
        rc.h = b.h;
        all = persp_cells(cams[v], tryax, vol->part.boxes[b.brick], rc, ctx->foot_rays, ctx->persp_kmax, kRingCap,
                          kRingRegLoads, pcs[i], ctx->foot_maxpx);
      }
      if (all) {
        axis = tryax;
        break;
      }
    }
    if (axis == 0) continue;
    std::vector<double> key(vp.bv.size());
    for (size_t i = 0; i < vp.bv.size(); i++) {
      DevBrickView& b = vp.bv[i];
      const PerspCells& pc = pcs[i];
      b.tiles_x = pc.ncf;
      b.cf0 = pc.cf0;
      b.cg0 = pc.cg0;
      b.blocks_x = pc.ncg;  // cells along g (the cell count is tiles_x x blocks_x)
      b.pTf = pc.Tf;
      b.pTg = pc.Tg;
      b.ppitch = pc.pitch;
      b.png = pc.ng;
      key[i] = (double)pc.pitch * pc.ng;
    }
    // one launch: the cell shapes are chosen for the occupancy their windows
    // allow, so their slots differ little (three launches measured slower)
    group_classes(vp, key, 1, [](const DevBrickView& b) { return (int64_t)b.tiles_x * b.blocks_x; });
    vp.pfoot = true;
    vp.paxis = axis;
    int64_t cells = 0;
    for (int32_t t : vp.class_tiles) cells += t;
    vp.ntiles = (int32_t)cells;
  }
  // perspective views on the ring march's 8 x 8 tiles: rays from the eye
  // spread with depth, so the tiles of far bricks need windows about twice
  // those of near ones, and one slot sized for nearly all tiles leaves the
  // near bricks at a fraction of the wavefronts their windows allow.  Bricks
  // are grouped into classes of similar window (about equal tile counts),
  // launched one class at a time with a slot of its own.
  for (int32_t v = 0; v < nviews; v++) {
    ViewPlan& vp = plans[v];
    if (vp.pfoot) continue;
    vp.class_begin.clear();
    vp.class_tiles.clear();
    const int32_t ncls = ctx->persp_classes;
    if (!bricked || global || extras || !cams[v].persp || !(mode == 0 || mode == 3) || tw != 8 || ncls < 2 ||
        vp.bv.size() < (size_t)(2 * ncls))
      continue;
    std::vector<double> key(vp.bv.size());
    for (int32_t i = 0; i < (int32_t)vp.bv.size(); i++) {
      const DevBrickView& b = vp.bv[i];
      TileRegion r;
      for (int k = 0; k < 3; k++) {
        r.lo[k] = vol->part.boxes[b.brick].lo[k];
        r.hi[k] = vol->part.boxes[b.brick].hi[k];
      }
      r.x0 = b.x0;
      r.y0 = b.y0;
      r.w = b.w;
      r.h = b.h;
      key[i] = persp_region_window(cams[v], r);
    }
    group_classes(vp, key, ncls, [th](const DevBrickView& b) { return (int64_t)b.tiles_x * ((b.h + th - 1) / th); });
  }
  // parallel rays on the ring march: footprint cells instead of 8 x 8 pixel
  // tiles (the cell counts replace the tile counts of the plan)
  const bool plain_ring = base.mc == 0 && !base.mask;
  for (int32_t v = 0; v < nviews; v++) {
    ViewPlan& vp = plans[v];
    if (extras || cams[v].persp || !ctx->foot || !(mode == 0 || mode == 3) || tw != 8) continue;
    FootShape fs;
    if (!pick_foot(cams[v], vol->n, base.M, plain_ring, ctx->ring_reg > 0, ctx->ring_nslots, ctx->foot_rays,
                   ctx->foot_pad, ctx->foot_kmax, fs, ctx->foot_maxpx))
      continue;
    Box whole;
    for (int i = 0; i < 3; i++) {
      whole.lo[i] = 0;
      whole.hi[i] = vol->n[i] - 1;
      whole.closed[i] = 1;
    }
    // blocks of cells (the plain march, emission-absorption or MIP): one
    // workgroup per block, one window per layer; the window's rows must fit
    // inside every brick along axis 1
    if (plain_ring && ctx->foot_block != 0) {
      int64_t ext[3] = {INT64_MAX, 0, 0};
      for (const DevBrickView& b : vp.bv) {
        const Box& bx = bricked ? vol->part.boxes[b.brick] : whole;
        ext[0] = std::min<int64_t>(ext[0], bx.hi[0] - bx.lo[0]);
        for (int i = 1; i < 3; i++) ext[i] = std::max<int64_t>(ext[i], bx.hi[i] - bx.lo[i]);
      }
      const Box& b0 = bricked ? vol->part.boxes[vp.bv.empty() ? 0 : vp.bv[0].brick] : whole;
      int64_t typ[3];
      for (int i = 0; i < 3; i++) typ[i] = b0.hi[i] - b0.lo[i];
      typ[0] = std::min(typ[0], ext[0]);
      choose_foot_block(cams[v], fs, typ, base.M, kRingRegWaves, kRingRegWaves, kRingRegLoads,
                        ctx->foot_block > 0 ? ctx->foot_block_f : 0, ctx->foot_block > 0 ? ctx->foot_block_g : 0);
    }
    if (ctx->debug_plan)
      std::fprintf(stderr, "[vr] view %d: cells axis %d Tf %.1f Tg %.2f nf %d ng %d slot %d nslots %d reg %d wpb %d waves %d rf %.3f rg %.3f blocks %dx%d nf %d ng %d waves %d\n",
                   v, fs.axis, fs.Tf, fs.Tg, fs.nf, fs.ng, fs.slot, fs.nslots, fs.reg, fs.wpb, fs.waves, fs.rf, fs.rg,
                   fs.blk_f, fs.blk_g, fs.blk_nf, fs.blk_ng, fs.blk_waves);
    vp.foot = true;
    vp.fs = fs;
    int32_t tiles = 0;
    size_t w = 0;  // wave of the brick (whole-ray termination)
    for (size_t i = 0; i < vp.bv.size(); i++) {
      DevBrickView& b = vp.bv[i];
      if (global) {
        while (w + 1 < vp.wave_begin.size() && (int32_t)i >= vp.wave_begin[w + 1]) w++;
        if ((int32_t)i == vp.wave_begin[w]) tiles = 0;
      }
      int32_t ncf, ncg;
      foot_cells(cams[v], fs, bricked ? vol->part.boxes[b.brick] : whole, b.cf0, b.cg0, ncf, ncg, b.fa0, b.fb0);
      b.tiles_x = ncf;
      b.tile_begin = tiles;
      if (fs.blk_f > 0) {
        b.blocks_x = (ncf + fs.blk_f - 1) / fs.blk_f;
        tiles += b.blocks_x * ((ncg + fs.blk_g - 1) / fs.blk_g);
      } else {
        b.blocks_x = 0;
        tiles += ncf * ncg;
      }
      if (global) vp.wave_tiles[w] = tiles;
    }
    if (!global) vp.ntiles = tiles;
  }
  if (bricked && arena_pix > 0) VR_TRY(ensure_device(&ctx->d_arena, &ctx->arena_bytes, (size_t)arena_pix * 16));
  // overflow lists of the footprint-cell marches: one per stream a view may use
  int64_t foot_tiles = 0;  // cells of a launch (a block holds blk_f x blk_g)
  for (const ViewPlan& vp : plans) {
    if (vp.foot) {
      const int64_t per = vp.fs.blk_f > 0 ? (int64_t)vp.fs.blk_f * vp.fs.blk_g : 1;
      foot_tiles = std::max<int64_t>(foot_tiles, vp.ntiles * per);
      for (int32_t t : vp.wave_tiles) foot_tiles = std::max<int64_t>(foot_tiles, t * per);
    }
    if (vp.pfoot)
      for (int32_t t : vp.class_tiles) foot_tiles = std::max<int64_t>(foot_tiles, t);
  }
  const size_t ovf_stride = align16(256 + 4 * (size_t)foot_tiles);
  if (foot_tiles > 0) VR_TRY(ensure_device(&ctx->d_ovf, &ctx->ovf_bytes, ovf_stride * vr_ctx::kAux));
  float4* arena = reinterpret_cast<float4*>(ctx->d_arena);

  // pack: [whole-volume brick] then per view [DevBrickView...][CompLayer...]
  std::vector<size_t> off_bv((size_t)nviews), off_cl((size_t)nviews);
  size_t bytes = align16(sizeof(DevBrick));
  for (int32_t v = 0; v < nviews; v++) {
    off_bv[v] = bytes;
    bytes = align16(bytes + sizeof(DevBrickView) * plans[v].bv.size());
    off_cl[v] = bytes;
    bytes = align16(bytes + sizeof(CompLayer) * plans[v].layers_order.size());
  }
  std::vector<unsigned char> host(bytes, 0);
  std::memcpy(host.data(), &vol->whole, sizeof(DevBrick));
  for (int32_t v = 0; v < nviews; v++) {
    const ViewPlan& vp = plans[v];
    std::memcpy(host.data() + off_bv[v], vp.bv.data(), sizeof(DevBrickView) * vp.bv.size());
    CompLayer* cl = reinterpret_cast<CompLayer*>(host.data() + off_cl[v]);
    for (size_t i = 0; i < vp.layers_order.size(); i++) {
      const DevBrickView& b = vp.bv[vp.layers_order[i]];
      cl[i].x0 = b.x0;
      cl[i].y0 = b.y0;
      cl[i].w = b.w;
      cl[i].h = b.h;
      cl[i].rgba = arena + b.img_off;
    }
  }
  void* dtab = nullptr;
  VR_TRY(stage_begin(ctx, VR_STAGE_SETUP, s));
  VR_TRY(upload_tables(ctx, s, host.data(), bytes, &dtab));
  VR_TRY(stage_end(ctx, s));
  unsigned char* dt = reinterpret_cast<unsigned char*>(dtab);

  // views with the opacity test over whole rays write disjoint frames and use
  // no shared arena: their wave sequences run side by side on the side streams
  // (small front and back waves of one view leave most of the chip idle)
  if (global) {
    VR_TRY(stage_begin(ctx, VR_STAGE_MARCH, s));
    VR_TRY(aux_fork(ctx, s));
  }
  // LDS slot, slots per wavefront and register staging of the perspective
  // ring march for the bricks bv[first .. first + count) of view v; false
  // when the windows do not fit (gather march)
  auto persp_shape = [&](int32_t v, int32_t first, int32_t count, MarchArgs& a, int& wpb) {
    const ViewPlan& vp = plans[v];
    std::vector<TileRegion> regs;
    for (int32_t k = first; k < first + count; k++) {
      const DevBrickView& b = vp.bv[k];
      TileRegion r;
      for (int i = 0; i < 3; i++) {
        r.lo[i] = bricked ? vol->part.boxes[b.brick].lo[i] : 0;
        r.hi[i] = bricked ? vol->part.boxes[b.brick].hi[i] : vol->n[i] - 1;
      }
      r.x0 = b.x0;
      r.y0 = b.y0;
      r.w = b.w;
      r.h = b.h;
      regs.push_back(r);
    }
    a.slab_axis = std::fabs(cams[v].e3[1]) >= std::fabs(cams[v].e3[2]) ? 1 : 2;
    const bool ok = choose_ring_persp(cams[v], regs, kRingCap, a.M, kRingMaxWaves, kRingMinWaves, a.ring_slot, wpb,
                                      ctx->persp_fit);
    a.ring_nslots = 3;
    a.ring_reg = 0;
    // two slots wherever they fit more wavefronts (as for parallel rays)
    if (ok && a.mc == 0 && !a.mask && ctx->ring_nslots != 3) {
      int32_t waves3 = 0, waves2 = 0;
      ring_waves_per_block(a.ring_slot, a.M, kRingMaxWaves, &waves3, 3);
      const int32_t wpb2 = ring_waves_per_block(a.ring_slot, a.M, kRingMaxWaves, &waves2, 2);
      if (ctx->ring_nslots == 2 || waves2 > waves3) {
        wpb = wpb2;
        a.ring_nslots = 2;
      }
    }
    // the layer after next staged in registers (emission-absorption)
    if (ok && a.ring_nslots == 2 && !a.mip && a.mc == 0 && !a.mask && ctx->ring_reg) a.ring_reg = 1;
    return ok;
  };
  for (int32_t v = 0; v < nviews; v++) {
    const ViewPlan& vp = plans[v];
    MarchArgs a = base;
    a.cam = cams[v];
    a.nbv = (int32_t)vp.bv.size();
    a.ntiles = vp.ntiles;
    a.bv = reinterpret_cast<const DevBrickView*>(dt + off_bv[v]);
    if (bricked) {
      a.bricks = vol->d_bricks;
      a.img = arena;
    } else {
      a.bricks = reinterpret_cast<const DevBrick*>(dt);
      a.img = reinterpret_cast<float4*>(out);
    }
    if (extras) extras->prepare(a, v);
    bool lds = false, ring = false;
    int ring_wpb = 4;
    a.lds_budget = budget;
    if (vp.foot) {
      const FootShape& fs = vp.fs;
      ring = true;
      a.foot = 1;
      a.slab_axis = fs.axis;
      a.ring_slot = fs.slot;
      a.ring_nslots = fs.nslots;
      a.ring_reg = fs.reg;
      ring_wpb = fs.reg && ctx->cells_wpb > 0 ? ctx->cells_wpb : fs.wpb;
      if (fs.reg && ctx->cells_waves > 0) {
        // at most cells_waves wavefronts per compute unit: reserve LDS so that
        // one workgroup more would not fit (more wavefronts ran slower: their
        // windows crowd each other out of the caches)
        const int32_t nwg = std::max(1, ctx->cells_waves / ring_wpb);
        a.lds_floor = kLdsPerCu / (nwg + 1) + 1024;
      }
      a.foot_nf = fs.nf;
      a.foot_ng = fs.ng;
      a.foot_Tf = fs.Tf;
      a.foot_Tg = fs.Tg;
      if (fs.blk_f > 0) {
        // one window per block: its rows and slot replace the cell's
        a.blk_f = fs.blk_f;
        a.blk_g = fs.blk_g;
        a.foot_nf = fs.blk_nf;
        a.foot_ng = fs.blk_ng;
        a.ring_slot = fs.blk_slot;
        a.ring_nslots = 2;
      }
      a.fa_u = fs.fa_u;
      a.fa_v = fs.fa_v;
      a.fb_u = fs.fb_u;
      a.fb_v = fs.fb_v;
      unsigned char* ovf = reinterpret_cast<unsigned char*>(ctx->d_ovf) + (global ? (size_t)(v % vr_ctx::kAux) * ovf_stride : 0);
      a.ovf_count = reinterpret_cast<unsigned int*>(ovf);
      a.ovf_tiles = reinterpret_cast<int32_t*>(ovf + 256);
      // pixels of the brick images (or of the frame) whose rays have no
      // sample are not written by the cells: clear them first
      if (!global) {
        VR_HIP(launch_zero(bricked ? arena : reinterpret_cast<float4*>(out) + (int64_t)v * W * H,
                           bricked ? vp.pixels : (int64_t)W * H, s));
      }
    } else if (!extras && (mode == 0 || mode == 3) && a.tile_w == 8) {
      if (cams[v].persp) {
        if (vp.class_begin.empty()) {
          ring = persp_shape(v, 0, (int32_t)vp.bv.size(), a, ring_wpb);
        } else {
          ring = true;  // shapes per class at the launch
        }
      } else {
        int32_t waves3 = 0;
        ring = choose_ring(cams[v], kRingCap, a.M, kRingMaxWaves, kRingWantWaves, kRingMinWaves, a.slab_axis,
                           a.ring_slot, ring_wpb, 3, &waves3);
        a.ring_nslots = 3;
        // two LDS slots per wavefront (the next layer's loads no longer overlap
        // the wavefront's own sampling, but more wavefronts fit): taken
        // whenever they fit more wavefronts on a compute unit than three (on
        // 24 GiB cubes the march follows the wavefront count, not the
        // lookahead: 12 -> 16 wavefronts took one view from 12.1 to 9.3 ms, a
        // fourth slot at fewer wavefronts cost 35 %), or when forced; plain
        // march and maximum intensity projection only
        const bool plain = a.mc == 0 && !a.mask;
        if (ring && plain && ctx->ring_nslots != 3) {
          int32_t ax2 = 0, slot2 = 0, wpb2 = 4, waves2 = 0;
          if (choose_ring(cams[v], kRingCap, a.M, kRingMaxWaves, kRingWantWaves, kRingMinWaves, ax2, slot2, wpb2, 2,
                          &waves2) &&
              (ctx->ring_nslots == 2 || waves2 > waves3)) {
            a.slab_axis = ax2;
            a.ring_slot = slot2;
            ring_wpb = wpb2;
            a.ring_nslots = 2;
          }
        }
      }
    }
    if (ring && !vp.foot && ctx->debug_plan)
      std::fprintf(stderr, "[vr] view %d: tiles axis %d slot %d nslots %d wpb %d\n", v, a.slab_axis, a.ring_slot,
                   a.ring_nslots, ring_wpb);
    if (ring) {
      a.tile_order = ctx->tile_order;
      a.tile_bw = ctx->tile_bw;
      a.tile_bh = ctx->tile_bh;
    }
    if (!ring && !extras && mode != 1 && !a.mip && !a.mask) {  // (the slab march has no MIP and no mask)
      lds = choose_slab(cams[v], a.tile_w, a.tile_h, budget, a.slab_axis, a.slab_T);
      // rays nearly parallel to axis 1 need a wider slab box: retry with twice the budget
      if (!lds && budget < 8192 && choose_slab(cams[v], a.tile_w, a.tile_h, 8192, a.slab_axis, a.slab_T)) {
        lds = true;
        a.lds_budget = 8192;
      }
    }
    if (global) {
      // waves in order, each continuing the rays the previous left in the frame
      float4* frame = reinterpret_cast<float4*>(out) + (int64_t)v * W * H;
      hipStream_t vs = ctx->aux[v % vr_ctx::kAux];
      lds = false;  // the slab march does not carry state
      a.carry = 1;
      a.img = frame;
      VR_HIP(launch_carry(frame, (int64_t)W * H, false, vs));
      const DevBrickView* wbv = a.bv;
      for (size_t w = 0; w + 1 < vp.wave_begin.size(); w++) {
        a.bv = wbv + vp.wave_begin[w];
        a.nbv = vp.wave_begin[w + 1] - vp.wave_begin[w];
        a.ntiles = vp.wave_tiles[w];
        VR_HIP(ring ? launch_march_ring(a, ring_wpb, vs) : launch_march(a, vs));
      }
      VR_HIP(launch_carry(frame, (int64_t)W * H, true, vs));
      continue;
    }
    VR_TRY(stage_begin(ctx, VR_STAGE_MARCH, s));
    if (vp.pfoot) {
      // perspective footprint cells: the brick images' pixels without samples
      // are not written, so the arena is cleared first; one launch per class
      // of window size, the class's largest window as the slot
      VR_HIP(launch_zero(arena, vp.pixels, s));
      const DevBrickView* cbv = a.bv;
      for (size_t c = 0; c + 1 < vp.class_begin.size(); c++) {
        MarchArgs ac = a;
        const int32_t first = vp.class_begin[c], count = vp.class_begin[c + 1] - first;
        int32_t slot = 0, mpitch = 0, mng = 0;
        for (int32_t k = first; k < first + count; k++) {
          slot = std::max(slot, vp.bv[k].ppitch * vp.bv[k].png);
          mpitch = std::max(mpitch, vp.bv[k].ppitch);
          mng = std::max(mng, vp.bv[k].png);
        }
        ac.bv = cbv + first;
        ac.nbv = count;
        ac.ntiles = vp.class_tiles[c];
        ac.foot = 1;
        ac.blk_f = ac.blk_g = 0;
        ac.slab_axis = vp.paxis;
        ac.ring_slot = slot;
        ac.ring_nslots = 2;
        ac.ring_reg = 1;
        ac.foot_nf = mpitch;
        ac.foot_ng = mng;
        int32_t waves = 0;
        int cwpb = ring_waves_per_block(slot, ac.M, kRingRegWaves, &waves, 2);
        if (ctx->cells_wpb > 0) cwpb = ctx->cells_wpb;
        if (ctx->cells_waves > 0) {
          const int32_t nwg = std::max(1, ctx->cells_waves / cwpb);
          ac.lds_floor = kLdsPerCu / (nwg + 1) + 1024;
        }
        unsigned char* ovf = reinterpret_cast<unsigned char*>(ctx->d_ovf);
        ac.ovf_count = reinterpret_cast<unsigned int*>(ovf);
        ac.ovf_tiles = reinterpret_cast<int32_t*>(ovf + 256);
        if (ctx->debug_plan)
          std::fprintf(stderr, "[vr] view %d cells class %zu: bricks %d cells %d axis %d slot %d pitch<=%d ng<=%d wpb %d waves %d\n",
                       v, c, count, ac.ntiles, vp.paxis, slot, mpitch, mng, cwpb, waves);
        VR_HIP(launch_march_ring(ac, cwpb, s));
      }
    } else if (!vp.class_begin.empty()) {
      // perspective classes: one launch each, with the class's own slot
      const DevBrickView* cbv = a.bv;
      for (size_t c = 0; c + 1 < vp.class_begin.size(); c++) {
        MarchArgs ac = a;
        int cwpb = 4;
        const int32_t first = vp.class_begin[c], count = vp.class_begin[c + 1] - first;
        const bool cring = persp_shape(v, first, count, ac, cwpb);
        ac.bv = cbv + first;
        ac.nbv = count;
        ac.ntiles = vp.class_tiles[c];
        if (ctx->debug_plan)
          std::fprintf(stderr, "[vr] view %d class %zu: bricks %d tiles %d ring %d slot %d nslots %d reg %d wpb %d\n", v, c,
                       count, ac.ntiles, cring ? 1 : 0, ac.ring_slot, ac.ring_nslots, ac.ring_reg, cwpb);
        VR_HIP(cring ? launch_march_ring(ac, cwpb, s) : launch_march(ac, s));
      }
    } else {
      VR_HIP(extras ? extras->launch(a, s)
                    : (ring ? launch_march_ring(a, ring_wpb, s) : (lds ? launch_march_lds(a, s) : launch_march(a, s))));
    }
    VR_TRY(stage_end(ctx, s));
    if (bricked && out) {
      CompArgs c;
      std::memset(&c, 0, sizeof c);
      c.layers = reinterpret_cast<const CompLayer*>(dt + off_cl[v]);
      c.n = (int32_t)vp.layers_order.size();
      c.W = W;
      c.H = H;
      c.mip = base.mip;
      c.out = reinterpret_cast<float4*>(out) + (int64_t)v * W * H;
      VR_TRY(stage_begin(ctx, VR_STAGE_COMPOSITE, s));
      VR_HIP(launch_composite(c, s));
      VR_TRY(stage_end(ctx, s));
    }
  }
  if (global) {
    VR_TRY(aux_join(ctx, s));
    VR_TRY(stage_end(ctx, s));
  }
  if (extras) {
    extras->vmin = vmin;
    extras->vmax = vmax;
  }
  return VR_OK;
}

int validate_render(vr_ctx* ctx, const vr_volume* vol, const vr_view* views, int32_t nviews, const vr_params* p) {
  if (!ctx || !vol || !views) return fail(VR_EINVAL, "ctx, vol and views must be non-NULL");
  if (vol->ctx != ctx) return fail(VR_EINVAL, "volume belongs to another context");
  if (nviews < 1) return fail(VR_EINVAL, "nviews must be >= 1");
  VR_TRY(check_params(p));
  for (int32_t v = 0; v < nviews; v++) {
    VR_TRY(check_view(&views[v], vol->n));
    if (views[v].W != views[0].W || views[v].H != views[0].H)
      return fail(VR_EINVAL, "all views of one call must share W and H");
  }
  if (!ctx->tf_set) return fail(VR_ESTATE, "no transfer function set (vr_tf_set)");
  if (!vol->bricked && vol->n[0] * vol->n[1] * vol->n[2] >= ((int64_t)1 << 31))
    return fail(VR_EUNSUPPORTED, "unbricked rendering needs fewer than 2^31 voxels; brick the volume");
  return VR_OK;
}

}  // namespace vr

using namespace vr;

extern "C" {

int vr_render(vr_ctx* ctx, const vr_volume* cvol, const vr_view* views, int32_t nviews, const vr_params* p,
              float* out, uintptr_t stream, vr_state** save) {
  clear_error();
  VR_TRY(validate_render(ctx, cvol, views, nviews, p));
  if (!out) return fail(VR_EINVAL, "out is NULL");
  vr_volume* vol = const_cast<vr_volume*>(cvol);
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  if (save) return render_with_state(ctx, vol, views, nviews, p, out, s, save);
  VR_TRY(ctx_begin(ctx, s));
  if (!vol->twin || !vol->bricked) {
    VR_TRY(render_forward(ctx, vol, views, nviews, p, out, s, nullptr));
    return ctx_end(ctx, s);
  }
  // views looking mostly along axis 1 (the contiguous one) are rendered from
  // the permuted copy, whose contiguous axis is axis 2: the same rays in
  // permuted coordinates (view axes permuted like the volume's)
  auto along1 = [](const vr_view& v) {
    return std::fabs(v.R[6]) > std::max(std::fabs(v.R[7]), std::fabs(v.R[8]));
  };
  const int64_t frame = (int64_t)views[0].W * views[0].H * 4;
  for (int32_t v0 = 0; v0 < nviews;) {
    const bool tw = along1(views[v0]);
    int32_t v1 = v0 + 1;
    while (v1 < nviews && along1(views[v1]) == tw) v1++;
    if (tw) {
      std::vector<vr_view> pv(views + v0, views + v1);
      for (vr_view& q : pv)
        for (int r = 0; r < 3; r++) {
          const double x = q.R[3 * r], y = q.R[3 * r + 1], z = q.R[3 * r + 2];
          q.R[3 * r] = y;
          q.R[3 * r + 1] = z;
          q.R[3 * r + 2] = x;
        }
      VR_TRY(render_forward(ctx, vol->twin, pv.data(), v1 - v0, p, out + v0 * frame, s, nullptr));
    } else {
      VR_TRY(render_forward(ctx, vol, views + v0, v1 - v0, p, out + v0 * frame, s, nullptr));
    }
    v0 = v1;
  }
  return ctx_end(ctx, s);
}

int vr_render_bricks(vr_ctx* ctx, const vr_volume* cvol, const vr_view* view, const vr_params* p,
                     vr_brick_image* imgs, int32_t* nimg, int32_t* order, uintptr_t stream) {
  clear_error();
  VR_TRY(validate_render(ctx, cvol, view, 1, p));
  if (!imgs || !nimg || !order) return fail(VR_EINVAL, "imgs, nimg and order must be non-NULL");
  if (!cvol->bricked) return fail(VR_ESTATE, "volume is not bricked (vr_volume_brick)");
  if (p->ert_scope == VR_ERT_GLOBAL)
    return fail(VR_EUNSUPPORTED, "per-brick images exist only with VR_ERT_LOCAL (global termination carries rays "
                                 "across bricks)");
  vr_volume* vol = const_cast<vr_volume*>(cvol);
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  VR_TRY(ctx_begin(ctx, s));
  // plan first to check capacity
  double vmin, vmax;
  VR_TRY(resolve_window(ctx, vol, s, vmin, vmax));
  Camera cam;
  make_camera(*view, vol->n, cam);
  ViewPlan vp;
  int32_t tw, budget, mode;
  tuned_shape(ctx, vol, view->W, view->H, p, tw, budget, mode);
  plan_bricked_view(vol, cam, p, tw, ctx->h_tf.data(), ctx->tf_m, vmin, vmax, vp);
  if ((int32_t)vp.bv.size() > *nimg)
    return fail(VR_EINVAL, "capacity %d below the %d rendered bricks", *nimg, (int)vp.bv.size());
  VR_TRY(render_forward(ctx, vol, view, 1, p, nullptr, s, nullptr));
  float4* arena = reinterpret_cast<float4*>(ctx->d_arena);
  for (size_t i = 0; i < vp.bv.size(); i++) {
    const DevBrickView& b = vp.bv[i];
    imgs[i].brick = b.brick;
    imgs[i].x0 = b.x0;
    imgs[i].y0 = b.y0;
    imgs[i].w = b.w;
    imgs[i].h = b.h;
    imgs[i].reserved = 0;
    imgs[i].rgba = reinterpret_cast<float*>(arena + b.img_off);
  }
  for (size_t i = 0; i < vp.layers_order.size(); i++) order[i] = vp.layers_order[i];
  *nimg = (int32_t)vp.bv.size();
  return ctx_end(ctx, s);
}

int vr_composite(vr_ctx* ctx, const vr_brick_image* imgs, int32_t n, const int32_t* order, int32_t W, int32_t H,
                 float* out, uintptr_t stream) {
  clear_error();
  if (!ctx || !out || (n > 0 && !imgs)) return fail(VR_EINVAL, "ctx, out (and imgs when n > 0) must be non-NULL");
  if (n < 0) return fail(VR_EINVAL, "n must be >= 0");
  if (W < 1 || H < 1 || W > 16384 || H > 16384) return fail(VR_EINVAL, "image size outside [1, 16384]");
  std::vector<CompLayer> layers((size_t)n);
  std::vector<char> seen((size_t)n, 0);
  for (int32_t i = 0; i < n; i++) {
    const int32_t j = order ? order[i] : i;
    if (j < 0 || j >= n) return fail(VR_EINVAL, "order[%d] = %d out of range", i, j);
    if (seen[j]) return fail(VR_EINVAL, "order lists image %d twice", j);
    seen[j] = 1;
    const vr_brick_image& im = imgs[j];
    if (im.w < 0 || im.h < 0 || im.x0 < 0 || im.y0 < 0 || (int64_t)im.x0 + im.w > W || (int64_t)im.y0 + im.h > H)
      return fail(VR_EINVAL, "image %d rectangle (%d,%d,%d,%d) outside %dx%d", j, im.x0, im.y0, im.w, im.h, W, H);
    if (im.w > 0 && im.h > 0 && !im.rgba) return fail(VR_EINVAL, "image %d has no pixels pointer", j);
    layers[i] = CompLayer{im.x0, im.y0, im.w, im.h, reinterpret_cast<const float4*>(im.rgba)};
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  VR_TRY(ctx_begin(ctx, s));
  void* d = nullptr;
  CompLayer dummy{0, 0, 0, 0, nullptr};
  VR_TRY(upload_tables(ctx, s, n > 0 ? (const void*)layers.data() : (const void*)&dummy,
                       sizeof(CompLayer) * (size_t)std::max(n, 1), &d));
  CompArgs c;
  std::memset(&c, 0, sizeof c);
  c.layers = reinterpret_cast<const CompLayer*>(d);
  c.n = n;
  c.W = W;
  c.H = H;
  c.out = reinterpret_cast<float4*>(out);
  VR_TRY(stage_begin(ctx, VR_STAGE_COMPOSITE, s));
  VR_HIP(launch_composite(c, s));
  VR_TRY(stage_end(ctx, s));
  return ctx_end(ctx, s);
}

}  // extern "C"
