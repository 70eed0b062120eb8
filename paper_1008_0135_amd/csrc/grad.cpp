// grad.cpp -- the differentiable forward (vr_render with save) and
// vr_render_backward: state ownership, validation and launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "forward.h"
#include "plan.h"
#include "runtime.h"
#include "vr_internal.h"

struct vr_state {
  vr_ctx* ctx = nullptr;
  const vr_volume* vol = nullptr;
  uint64_t vol_version = 0, tf_version = 0;
  std::vector<vr_view> views;
  vr_params p;
  double vmin = 0.0, vmax = 0.0;
  int32_t W = 0, H = 0, nviews = 0, K = 32, nseg = 0;
  // per view: checkpoint layout.  Ring views keep, per group of L cell layers
  // of each 8 x 8 tile, T and the sample cursor at the group's start; the
  // others keep T before every K-th sample.
  struct View {
    bool ring = false;
    int32_t axis = 0, slot = 0, fwd_wpb = 4, bwd_wpb = 1, L = 0, smax = 0, ngrp = 0;
    int64_t off = 0;  // offset of this view's checkpoints (floats / ints) in d_ckpt / d_ckpt_j
    int32_t band[9] = {};  // ring adjoint: tile groups per XCD (all zero: equal counts)
  };
  std::vector<View> vs;
  float* d_ckpt = nullptr;     // checkpoints, all views
  int32_t* d_ckpt_j = nullptr; // ring views: sample cursors at group starts
  int32_t* d_nused = nullptr;  // [view][pixel], then the adjoint's bound flag
  size_t ckpt_bytes = 0, ckpt_j_bytes = 0, nused_bytes = 0;  // allocated sizes
  int32_t* d_flag = nullptr;   // set by the adjoint when a group held more samples than its bound
};

namespace vr {

namespace {

// Device tables of one view of a whole-volume render: [DevBrick][DevBrickView].
struct WholeTables {
  size_t bytes = 0, off_bv = 0;
};

void pack_whole(const vr_volume* vol, int32_t W, int32_t H, int32_t tw, int32_t th, int32_t nviews,
                std::vector<unsigned char>& host, std::vector<size_t>& off_bv) {
  size_t bytes = (sizeof(DevBrick) + 15) & ~(size_t)15;
  off_bv.resize((size_t)nviews);
  for (int32_t v = 0; v < nviews; v++) {
    off_bv[v] = bytes;
    bytes += (sizeof(DevBrickView) + 15) & ~(size_t)15;
  }
  host.assign(bytes, 0);
  std::memcpy(host.data(), &vol->whole, sizeof(DevBrick));
  for (int32_t v = 0; v < nviews; v++) {
    DevBrickView b;
    std::memset(&b, 0, sizeof b);
    b.w = W;
    b.h = H;
    b.tiles_x = (W + tw - 1) / tw;
    b.img_off = (int64_t)v * W * H;
    std::memcpy(host.data() + off_bv[v], &b, sizeof b);
  }
}

int ntiles_of(int32_t W, int32_t H, int32_t tw, int32_t th) { return ((W + tw - 1) / tw) * ((H + th - 1) / th); }

// Estimated work of each 8 x 8 tile of a whole-volume view, for splitting a
// ring march's tile groups into XCD bands: a fixed set-up plus the samples of
// the tile's longest ray, taken as the longest of its four corner rays through
// the volume (a wavefront walks its tile's rays in lockstep).
std::vector<double> tile_costs(const Camera& cam, const double hi[3], double step, int32_t W, int32_t H) {
  const int tx_n = (W + 7) / 8, ty_n = (H + 7) / 8;
  std::vector<int64_t> cn((size_t)(tx_n + 1) * (ty_n + 1), 0);  // samples of the corner rays
  for (int cy = 0; cy <= ty_n; cy++)
    for (int cx = 0; cx <= tx_n; cx++) {
      double o[3], tin;
      int64_t n = 0;
      pixel_origin(cam, std::min(cx * 8, W - 1), std::min(cy * 8, H - 1), o);
      if (ray_lattice(o, cam.e3, hi, step, tin, n)) cn[(size_t)cy * (tx_n + 1) + cx] = n;
    }
  std::vector<double> c((size_t)tx_n * ty_n);
  for (int t = 0; t < tx_n * ty_n; t++) {
    const size_t i = (size_t)(t / tx_n) * (tx_n + 1) + (size_t)(t % tx_n);
    c[(size_t)t] = 32.0 + (double)std::max(std::max(cn[i], cn[i + 1]), std::max(cn[i + tx_n + 1], cn[i + tx_n + 2]));
  }
  return c;
}

// Tile groups (wpb consecutive tiles) in 8 contiguous bands of about equal
// work, one per XCD.  Equal counts of groups leave the XCDs holding the
// image's border idle while those holding its middle, where rays are
// longest, still work.
void xcd_bands(const std::vector<double>& cost, int wpb, int32_t band[9]) {
  const int nt = (int)cost.size(), ng = (nt + wpb - 1) / wpb;
  std::vector<double> pre((size_t)ng + 1, 0.0);
  for (int g = 0; g < ng; g++) {
    double c = 0.0;
    for (int t = g * wpb; t < std::min(nt, (g + 1) * wpb); t++) c += cost[(size_t)t];
    pre[g + 1] = pre[g] + c;
  }
  band[0] = 0;
  for (int x = 1; x < 8; x++) {
    const double target = pre[ng] * (double)x / 8.0;
    const int b = (int)(std::lower_bound(pre.begin(), pre.end(), target) - pre.begin());
    band[x] = std::max(band[x - 1], std::min(b, ng));
  }
  band[8] = ng;
}

// Ring layout for the differentiable pair of one view: slab axis, window slot,
// forward launch shape, cell layers per checkpoint group (about K samples),
// and the adjoint's wavefronts per workgroup under 160 KB of LDS.  False when
// the view needs the sample-segment kernels.
bool plan_ring_view(const Camera& cam, const vr_params* p, int32_t M, const int64_t n[3], int layer_cap,
                    vr_state::View& rv) {
  if (p->tile != 0 && p->tile != 8) return false;
  if (cam.persp) return false;  // the ring adjoint assumes parallel rays
  int32_t axis = 0, slot = 0, wpb = 4;
  if (!choose_ring(cam, 4096, M, 24, 12, 2, axis, slot, wpb)) return false;
  const double db = std::fabs(cam.e3[axis]);
  // layers per group: about K samples, at most `layer_cap` (LDS per wavefront
  // grows with the group and occupancy falls)
  const int Lmax = std::max(1, std::min(layer_cap, (int)std::lround((double)p->ckpt_K * p->step * db)));
  for (int L = Lmax; L >= 1; L = L > 1 ? L / 2 : 0) {
    const int smax = (int)std::floor((double)L / (p->step * db)) + 3;
    const double per_wave = 4.0 * (2.0 * (L + 1) * slot + 64.0 + 64.0 * smax);
    const double fixed = 48.0 * M;  // table (float4) and table gradients (double x 4)
    int best_w = 0, best_waves = 0;
    for (int w : {4, 2, 1}) {
      const double lds = fixed + w * per_wave;
      if (lds > 160.0 * 1024.0) continue;
      int blocks = (int)std::floor(160.0 * 1024.0 / lds);
      blocks = std::min(blocks, 16 / w);  // 99 VGPRs: 4 wavefronts per SIMD
      if (blocks * w > best_waves) {
        best_waves = blocks * w;
        best_w = w;
      }
    }
    if (best_w == 0) continue;
    rv.ring = true;
    rv.axis = axis;
    rv.slot = slot;
    rv.fwd_wpb = wpb;
    rv.bwd_wpb = best_w;
    rv.L = L;
    rv.smax = smax;
    rv.ngrp = (int32_t)((n[axis] - 1 + L - 1) / L) + 1;
    return true;
  }
  return false;
}

}  // namespace

int render_with_state(vr_ctx* ctx, vr_volume* vol, const vr_view* views, int32_t nviews, const vr_params* p,
                      float* out, hipStream_t s, vr_state** save) {
  if (vol->bricked) return fail(VR_EUNSUPPORTED, "saving forward state needs an unbricked volume");
  if (p->mode != VR_MODE_DVR) return fail(VR_EUNSUPPORTED, "the adjoint implements VR_MODE_DVR only");
  if (ctx->mask_n > 0) return fail(VR_EUNSUPPORTED, "the adjoint takes no channel mask (vr_mask_set(ctx, NULL, 0))");
  if (p->ckpt_K > 64) return fail(VR_EINVAL, "ckpt_K must be <= 64");
  const int32_t W = views[0].W, H = views[0].H;
  VR_TRY(ctx_begin(ctx, s));
  double vmin, vmax;
  VR_TRY(resolve_window(ctx, vol, s, vmin, vmax));
  vr_state* st = new (std::nothrow) vr_state();
  if (!st) return fail(VR_ENOMEM, "out of host memory");
  st->ctx = ctx;
  st->vol = vol;
  st->vol_version = vol->version;
  st->tf_version = ctx->tf_version;
  st->views.assign(views, views + nviews);
  st->p = *p;
  st->vmin = vmin;
  st->vmax = vmax;
  st->W = W;
  st->H = H;
  st->nviews = nviews;
  st->K = p->ckpt_K;
  double diag = 0.0;
  for (int i = 0; i < 3; i++) diag += (double)(vol->n[i] - 1) * (double)(vol->n[i] - 1);
  const int64_t nmax = (int64_t)std::ceil(std::sqrt(diag) / p->step) + 2;
  st->nseg = (int32_t)((nmax + st->K - 1) / st->K);
  const int64_t npix = (int64_t)W * H;
  // per-view layout and checkpoint offsets
  std::vector<Camera> cams((size_t)nviews);
  st->vs.assign((size_t)nviews, vr_state::View());
  int64_t ck_total = 0, ckj_total = 0;
  for (int32_t v = 0; v < nviews; v++) {
    make_camera(views[v], vol->n, cams[v]);
    vr_state::View& rv = st->vs[v];
    if (ctx->march_mode != 1 && plan_ring_view(cams[v], p, ctx->tf_m, vol->n, ctx->bwd_layer_cap, rv)) {
      rv.off = ck_total;
      ck_total += (int64_t)rv.ngrp * npix;
      ckj_total += (int64_t)rv.ngrp * npix;
    } else {
      rv.off = ck_total;
      ck_total += (int64_t)st->nseg * npix;
    }
  }
  const size_t ck_bytes = sizeof(float) * (size_t)std::max<int64_t>(ck_total, 1);
  const size_t ckj_bytes = ckj_total > 0 ? sizeof(int32_t) * (size_t)ck_total : 0;
  const size_t nu_bytes = sizeof(int32_t) * ((size_t)nviews * npix + 64);
  // the buffers of the last destroyed state when they are large enough
  vr_ctx::StateBufs& sp = ctx->spare;
  if (sp.ckpt && sp.ckpt_bytes >= ck_bytes && sp.nused_bytes >= nu_bytes && sp.ckpt_j_bytes >= ckj_bytes) {
    st->d_ckpt = sp.ckpt;
    st->d_ckpt_j = sp.ckpt_j;
    st->d_nused = sp.nused;
    st->ckpt_bytes = sp.ckpt_bytes;
    st->ckpt_j_bytes = sp.ckpt_j_bytes;
    st->nused_bytes = sp.nused_bytes;
    sp = vr_ctx::StateBufs();
  } else {
    st->ckpt_bytes = ck_bytes;
    st->ckpt_j_bytes = ckj_bytes;
    st->nused_bytes = nu_bytes;
    if (hipMalloc(&st->d_ckpt, ck_bytes) != hipSuccess || hipMalloc(&st->d_nused, nu_bytes) != hipSuccess ||
        (ckj_bytes > 0 && hipMalloc(&st->d_ckpt_j, ckj_bytes) != hipSuccess)) {
      (void)hipGetLastError();
      vr_state_destroy(st);
      return fail(VR_ENOMEM, "hipMalloc for %zu bytes of checkpoints failed", ck_bytes);
    }
  }
  st->d_flag = st->d_nused + (size_t)nviews * npix;
  {
    const hipError_t e = launch_fill(reinterpret_cast<float*>(st->d_flag), 1, 0.f, s);
    if (e != hipSuccess) {
      vr_state_destroy(st);
      return fail(VR_EHIP, "flag clear: %s", hipGetErrorString(e));
    }
  }
  MarchArgs base;
  std::memset(&base, 0, sizeof base);
  fill_march_common(base, vol, p, vmin, vmax, ctx->d_tf, ctx->tf_m);
  std::vector<unsigned char> host;
  std::vector<size_t> off_bv;
  pack_whole(vol, W, H, base.tile_w, base.tile_h, nviews, host, off_bv);
  void* dtab = nullptr;
  int rc = upload_tables(ctx, s, host.data(), host.size(), &dtab);
  // views write disjoint frames and checkpoints: side by side on the side
  // streams, as the adjoint runs them
  const bool side = ctx->bwd_side && nviews > 1;
  if (rc == VR_OK && side) rc = stage_begin(ctx, VR_STAGE_MARCH, s);
  if (rc == VR_OK && side) rc = aux_fork(ctx, s);
  for (int32_t v = 0; v < nviews && rc == VR_OK; v++) {
    const hipStream_t vs = side ? ctx->aux[v % vr_ctx::kAux] : s;
    const vr_state::View& rv = st->vs[v];
    MarchArgs a = base;
    a.cam = cams[v];
    a.nbv = 1;
    a.ntiles = ntiles_of(W, H, a.tile_w, a.tile_h);
    a.bricks = reinterpret_cast<const DevBrick*>(dtab);
    a.bv = reinterpret_cast<const DevBrickView*>(reinterpret_cast<unsigned char*>(dtab) + off_bv[v]);
    a.img = reinterpret_cast<float4*>(out);
    SaveArgs sa;
    std::memset(&sa, 0, sizeof sa);
    sa.ckpt = st->d_ckpt + rv.off;
    sa.ckpt_j = rv.ring ? st->d_ckpt_j + rv.off : nullptr;
    sa.nused = st->d_nused + (int64_t)v * npix;
    sa.K = rv.ring ? rv.L : st->K;
    sa.npix = (int32_t)npix;
    if (rv.ring && ctx->bwd_bands) {
      // XCD bands of this view's forward and adjoint (the host plans view v
      // while the GPU marches view v - 1)
      const std::vector<double> cost = tile_costs(cams[v], base.hi, p->step, W, H);
      xcd_bands(cost, rv.fwd_wpb, sa.band);
      xcd_bands(cost, rv.bwd_wpb, st->vs[v].band);
    }
    if (!side) rc = stage_begin(ctx, VR_STAGE_MARCH, s);
    if (rc == VR_OK) {
      hipError_t e;
      if (rv.ring) {
        a.slab_axis = rv.axis;
        a.ring_slot = rv.slot;
        e = launch_march_ring_save(a, sa, rv.fwd_wpb, vs);
      } else {
        e = launch_fwd_save(a, sa, vs);
      }
      if (e != hipSuccess) rc = fail(VR_EHIP, "forward launch: %s", hipGetErrorString(e));
    }
    if (rc == VR_OK && !side) rc = stage_end(ctx, s);
  }
  if (rc == VR_OK && side) rc = aux_join(ctx, s);
  if (rc == VR_OK && side) rc = stage_end(ctx, s);
  if (rc == VR_OK) rc = ctx_end(ctx, s);
  if (rc != VR_OK) {
    vr_state_destroy(st);
    return rc;
  }
  *save = st;
  return VR_OK;
}

}  // namespace vr

using namespace vr;

extern "C" {

int vr_state_destroy(vr_state* st) {
  if (!st) return VR_OK;
  DeviceGuard g(st->ctx->device);
  vr_ctx::StateBufs& sp = st->ctx->spare;
  if (!sp.ckpt && st->d_ckpt && st->d_nused) {
    // kept for the context's next forward with state (calls on a context are
    // ordered, so no work of this state can still be reading them then)
    sp.ckpt = st->d_ckpt;
    sp.ckpt_j = st->d_ckpt_j;
    sp.nused = st->d_nused;
    sp.ckpt_bytes = st->ckpt_bytes;
    sp.ckpt_j_bytes = st->ckpt_j_bytes;
    sp.nused_bytes = st->nused_bytes;
  } else {
    (void)hipDeviceSynchronize();
    if (st->d_ckpt) (void)hipFree(st->d_ckpt);
    if (st->d_ckpt_j) (void)hipFree(st->d_ckpt_j);
    if (st->d_nused) (void)hipFree(st->d_nused);
  }
  delete st;
  return VR_OK;
}

int vr_state_info(const vr_state* st, int32_t view, int32_t* ring, int32_t* layers_per_group, double* samples_per_group) {
  clear_error();
  if (!st || view < 0 || view >= st->nviews) return fail(VR_EINVAL, "state NULL or view out of range");
  const vr_state::View& rv = st->vs[view];
  if (ring) *ring = rv.ring ? 1 : 0;
  if (layers_per_group) *layers_per_group = rv.ring ? rv.L : 0;
  if (samples_per_group) {
    if (rv.ring) {
      const double* e3 = st->views[view].R + 6;
      *samples_per_group = (double)rv.L / (st->p.step * std::fabs(e3[rv.axis]));
    } else {
      *samples_per_group = (double)st->K;
    }
  }
  return VR_OK;
}

int vr_render_backward(vr_ctx* ctx, const vr_volume* vol, const vr_state* st, const float* grad_out, float* grad_tf,
                       float* grad_vol, int accumulate, uintptr_t stream) {
  clear_error();
  if (!ctx || !vol || !st || !grad_out || !grad_tf)
    return fail(VR_EINVAL, "ctx, vol, st, grad_out and grad_tf must be non-NULL");
  if (st->ctx != ctx || st->vol != vol) return fail(VR_ESTATE, "state belongs to another context or volume");
  if (st->vol_version != vol->version) return fail(VR_ESTATE, "volume was re-bricked since the forward");
  if (st->tf_version != ctx->tf_version) return fail(VR_ESTATE, "transfer function changed since the forward");
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  VR_TRY(ctx_begin(ctx, s));
  const int32_t M = ctx->tf_m, W = st->W, H = st->H;
  const int64_t npix = (int64_t)W * H;
  if (!accumulate) {
    VR_HIP(launch_fill(grad_tf, (int64_t)M * 4, 0.f, s));
    if (grad_vol) VR_HIP(launch_fill(grad_vol, vol->n[0] * vol->n[1] * vol->n[2], 0.f, s));
  }
  MarchArgs base;
  std::memset(&base, 0, sizeof base);
  vr_params p = st->p;
  p.tile = 8;
  fill_march_common(base, vol, &p, st->vmin, st->vmax, ctx->d_tf, M);
  std::vector<unsigned char> host;
  std::vector<size_t> off_bv;
  pack_whole(vol, W, H, base.tile_w, base.tile_h, st->nviews, host, off_bv);
  void* dtab = nullptr;
  VR_TRY(upload_tables(ctx, s, host.data(), host.size(), &dtab));
  MarchArgs a0 = base;
  a0.ntiles = ntiles_of(W, H, base.tile_w, base.tile_h);
  // every view's workgroups write their table partials into a region of their
  // own, so the views can run side by side (a view's tiles differ in ray
  // length; alone, its launch leaves compute units idle at its tail) and one
  // fixed-order reduction sums them all
  std::vector<int64_t> pbase((size_t)st->nviews + 1, 0);
  for (int32_t v = 0; v < st->nviews; v++) {
    const vr_state::View& rv = st->vs[v];
    BwdArgs bb;
    std::memset(&bb, 0, sizeof bb);
    std::memcpy(bb.band, rv.band, sizeof bb.band);
    pbase[v + 1] = pbase[v] + (rv.ring ? bwd_ring_blocks(a0, bb, rv.bwd_wpb) : bwd_blocks(a0));
  }
  const bool side = ctx->bwd_side && st->nviews > 1;
  int64_t nslots = 1;
  for (int32_t v = 0; v < st->nviews; v++) nslots = std::max(nslots, pbase[v + 1] - pbase[v]);
  if (side) nslots = std::max<int64_t>(pbase.back(), 1);
  VR_TRY(ensure_device(&ctx->d_scratch, &ctx->scratch_bytes,
                       sizeof(double) * 4 * (size_t)M * ((size_t)nslots + (size_t)tf_reduce_slices())));
  double* part = reinterpret_cast<double*>(ctx->d_scratch);
  double* slices = part + 4 * (size_t)M * (size_t)nslots;
  VR_TRY(stage_begin(ctx, VR_STAGE_BACKWARD, s));
  if (side) VR_TRY(aux_fork(ctx, s));
  for (int32_t v = 0; v < st->nviews; v++) {
    const vr_state::View& rv = st->vs[v];
    const hipStream_t vs = side ? ctx->aux[v % vr_ctx::kAux] : s;
    MarchArgs a = base;
    make_camera(st->views[v], vol->n, a.cam);
    a.nbv = 1;
    a.ntiles = a0.ntiles;
    a.bricks = reinterpret_cast<const DevBrick*>(dtab);
    a.bv = reinterpret_cast<const DevBrickView*>(reinterpret_cast<unsigned char*>(dtab) + off_bv[v]);
    BwdArgs ba;
    std::memset(&ba, 0, sizeof ba);
    ba.ckpt = st->d_ckpt + rv.off;
    ba.ckpt_j = rv.ring ? st->d_ckpt_j + rv.off : nullptr;
    ba.nused = st->d_nused + (int64_t)v * npix;
    ba.gout = reinterpret_cast<const float4*>(grad_out) + (int64_t)v * npix;
    ba.gvol = grad_vol;
    ba.tf_part = part + (side ? 4 * (size_t)M * (size_t)pbase[v] : 0);
    ba.vmin = st->vmin;
    ba.inv_range = st->vmax > st->vmin ? 1.0 / (st->vmax - st->vmin) : 0.0;
    ba.K = rv.ring ? rv.L : st->K;
    ba.npix = (int32_t)npix;
    ba.smax = rv.smax;
    std::memcpy(ba.band, rv.band, sizeof ba.band);
    ba.flag = st->d_flag;
    if (rv.ring) {
      a.slab_axis = rv.axis;
      a.ring_slot = rv.slot;
      VR_HIP(launch_bwd_ring(a, ba, rv.bwd_wpb, vs));
    } else {
      VR_HIP(launch_bwd(a, ba, vs));
    }
    if (!side) VR_HIP(launch_tf_reduce(part, (int)(pbase[v + 1] - pbase[v]), M * 4, grad_tf, slices, s));
  }
  if (side) {
    VR_TRY(aux_join(ctx, s));
    VR_HIP(launch_tf_reduce(part, (int)pbase.back(), M * 4, grad_tf, slices, s));
  }
  VR_TRY(stage_end(ctx, s));
  VR_TRY(ctx_end(ctx, s));
  // the ring adjoint's bound on the samples of one ray in one checkpoint group
  // holds by construction; a group that exceeded it is reported, not clamped
  int32_t flag = 0;
  VR_HIP(hipMemcpyAsync(&flag, st->d_flag, sizeof flag, hipMemcpyDeviceToHost, s));
  VR_HIP(hipStreamSynchronize(s));
  if (flag) return fail(VR_EHIP, "adjoint: a ray held more samples in one checkpoint group than the planned bound");
  return VR_OK;
}

}  // extern "C"
