// grad.cpp -- the differentiable forward (vr_render with save) and
// vr_render_backward: state ownership, validation and launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "forward.h"
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
  float* d_ckpt = nullptr;     // [view][segment][pixel]
  int32_t* d_nused = nullptr;  // [view][pixel]
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

}  // namespace

int render_with_state(vr_ctx* ctx, vr_volume* vol, const vr_view* views, int32_t nviews, const vr_params* p,
                      float* out, hipStream_t s, vr_state** save) {
  if (vol->bricked) return fail(VR_EUNSUPPORTED, "saving forward state needs an unbricked volume");
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
  const size_t ck_bytes = sizeof(float) * (size_t)nviews * (size_t)st->nseg * (size_t)npix;
  if (hipMalloc(&st->d_ckpt, ck_bytes) != hipSuccess || hipMalloc(&st->d_nused, sizeof(int32_t) * nviews * npix) != hipSuccess) {
    (void)hipGetLastError();
    vr_state_destroy(st);
    return fail(VR_ENOMEM, "hipMalloc for %zu bytes of checkpoints failed", ck_bytes);
  }
  MarchArgs base;
  std::memset(&base, 0, sizeof base);
  fill_march_common(base, vol, p, vmin, vmax, ctx->d_tf, ctx->tf_m);
  std::vector<unsigned char> host;
  std::vector<size_t> off_bv;
  pack_whole(vol, W, H, base.tile_w, base.tile_h, nviews, host, off_bv);
  void* dtab = nullptr;
  int rc = upload_tables(ctx, s, host.data(), host.size(), &dtab);
  for (int32_t v = 0; v < nviews && rc == VR_OK; v++) {
    MarchArgs a = base;
    make_camera(views[v], vol->n, a.cam);
    a.nbv = 1;
    a.ntiles = ntiles_of(W, H, a.tile_w, a.tile_h);
    a.bricks = reinterpret_cast<const DevBrick*>(dtab);
    a.bv = reinterpret_cast<const DevBrickView*>(reinterpret_cast<unsigned char*>(dtab) + off_bv[v]);
    a.img = reinterpret_cast<float4*>(out);
    SaveArgs sa;
    sa.ckpt = st->d_ckpt + (int64_t)v * st->nseg * npix;
    sa.nused = st->d_nused + (int64_t)v * npix;
    sa.K = st->K;
    sa.npix = (int32_t)npix;
    rc = stage_begin(ctx, VR_STAGE_MARCH, s);
    if (rc == VR_OK) {
      hipError_t e = launch_fwd_save(a, sa, s);
      if (e != hipSuccess) rc = fail(VR_EHIP, "forward launch: %s", hipGetErrorString(e));
    }
    if (rc == VR_OK) rc = stage_end(ctx, s);
  }
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
  (void)hipDeviceSynchronize();
  if (st->d_ckpt) (void)hipFree(st->d_ckpt);
  if (st->d_nused) (void)hipFree(st->d_nused);
  delete st;
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
  const int nblocks = bwd_blocks(a0);
  VR_TRY(ensure_device(&ctx->d_scratch, &ctx->scratch_bytes, sizeof(double) * 4 * (size_t)M * (size_t)std::max(nblocks, 1)));
  double* part = reinterpret_cast<double*>(ctx->d_scratch);
  for (int32_t v = 0; v < st->nviews; v++) {
    MarchArgs a = base;
    make_camera(st->views[v], vol->n, a.cam);
    a.nbv = 1;
    a.ntiles = a0.ntiles;
    a.bricks = reinterpret_cast<const DevBrick*>(dtab);
    a.bv = reinterpret_cast<const DevBrickView*>(reinterpret_cast<unsigned char*>(dtab) + off_bv[v]);
    BwdArgs ba;
    ba.ckpt = st->d_ckpt + (int64_t)v * st->nseg * npix;
    ba.nused = st->d_nused + (int64_t)v * npix;
    ba.gout = reinterpret_cast<const float4*>(grad_out) + (int64_t)v * npix;
    ba.gvol = grad_vol;
    ba.tf_part = part;
    ba.vmin = st->vmin;
    ba.inv_range = st->vmax > st->vmin ? 1.0 / (st->vmax - st->vmin) : 0.0;
    ba.K = st->K;
    ba.npix = (int32_t)npix;
    VR_TRY(stage_begin(ctx, VR_STAGE_BACKWARD, s));
    VR_HIP(launch_bwd(a, ba, s));
    VR_HIP(launch_tf_reduce(part, nblocks, M * 4, grad_tf, s));
    VR_TRY(stage_end(ctx, s));
  }
  return ctx_end(ctx, s);
}

}  // extern "C"
