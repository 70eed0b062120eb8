// api.cpp -- the extern "C" entry points of libvr (declared in include/vr.h):
// argument validation, device memory ownership, per-view planning and the
// launch sequence of the forward path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "forward.h"
#include "plan.h"
#include "runtime.h"
#include "vr_internal.h"

using namespace vr;

namespace vr {

static thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

void clear_error() { g_err.clear(); }

DeviceGuard::DeviceGuard(int dev) {
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  if (prev != dev) (void)hipSetDevice(dev);
  target = dev;
}
DeviceGuard::~DeviceGuard() {
  if (prev >= 0 && prev != target) (void)hipSetDevice(prev);
}

// ---------------------------------------------------------------- ctx helpers
int ctx_begin(vr_ctx* ctx, hipStream_t s) {
  if (ctx->done_valid) VR_HIP(hipStreamWaitEvent(s, ctx->done, 0));
  if (ctx->prof) {
    for (auto& t : ctx->timed) {
      ctx->event_pool.push_back(t.a);
      ctx->event_pool.push_back(t.b);
    }
    ctx->timed.clear();
    ctx->prof_stream = s;
  }
  return VR_OK;
}

int ctx_end(vr_ctx* ctx, hipStream_t s) {
  VR_HIP(hipEventRecord(ctx->done, s));
  ctx->done_valid = true;
  return VR_OK;
}

static hipEvent_t pool_event(vr_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int stage_begin(vr_ctx* ctx, int stage, hipStream_t s) {
  if (!ctx->prof) return VR_OK;
  vr_ctx::Timed t{stage, pool_event(ctx), pool_event(ctx)};
  if (!t.a || !t.b) return fail(VR_EHIP, "hipEventCreate failed");
  VR_HIP(hipEventRecord(t.a, s));
  ctx->timed.push_back(t);
  return VR_OK;
}

int aux_fork(vr_ctx* ctx, hipStream_t s) {
  if (!ctx->aux_fork_ev) {
    for (int i = 0; i < vr_ctx::kAux; i++) {
      VR_HIP(hipStreamCreateWithFlags(&ctx->aux[i], hipStreamNonBlocking));
      VR_HIP(hipEventCreateWithFlags(&ctx->aux_join_ev[i], hipEventDisableTiming));
    }
    VR_HIP(hipEventCreateWithFlags(&ctx->aux_fork_ev, hipEventDisableTiming));
  }
  VR_HIP(hipEventRecord(ctx->aux_fork_ev, s));
  for (int i = 0; i < vr_ctx::kAux; i++) VR_HIP(hipStreamWaitEvent(ctx->aux[i], ctx->aux_fork_ev, 0));
  return VR_OK;
}

int aux_join(vr_ctx* ctx, hipStream_t s) {
  for (int i = 0; i < vr_ctx::kAux; i++) {
    VR_HIP(hipEventRecord(ctx->aux_join_ev[i], ctx->aux[i]));
    VR_HIP(hipStreamWaitEvent(s, ctx->aux_join_ev[i], 0));
  }
  return VR_OK;
}

int stage_end(vr_ctx* ctx, hipStream_t s) {
  if (!ctx->prof) return VR_OK;
  VR_HIP(hipEventRecord(ctx->timed.back().b, s));
  return VR_OK;
}

int ensure_device(void** p, size_t* cap, size_t need) {
  if (need <= *cap && *p) return VR_OK;
  if (*p) {
    hipError_t e = hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (e != hipSuccess) return fail(VR_EHIP, "hipFree: %s", hipGetErrorString(e));
  }
  size_t bytes = std::max<size_t>(need, 256);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(VR_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
  }
  *cap = bytes;
  return VR_OK;
}

int upload_tables(vr_ctx* ctx, hipStream_t s, const void* data, size_t bytes, void** dev) {
  vr_ctx::Slot& sl = ctx->ring[ctx->ring_next];
  ctx->ring_next = (ctx->ring_next + 1) % vr_ctx::kRing;
  if (sl.used) VR_HIP(hipEventSynchronize(sl.copied));
  if (bytes > sl.bytes || !sl.h || !sl.d) {
    if (sl.h) VR_HIP(hipHostFree(sl.h));
    if (sl.d) VR_HIP(hipFree(sl.d));
    sl.h = sl.d = nullptr;
    sl.bytes = 0;
    size_t cap = std::max<size_t>(bytes, 4096);
    cap = (cap + 4095) & ~(size_t)4095;
    if (hipHostMalloc(&sl.h, cap, hipHostMallocDefault) != hipSuccess) {
      sl.h = nullptr;
      return fail(VR_ENOMEM, "hipHostMalloc(%zu) failed", cap);
    }
    if (hipMalloc(&sl.d, cap) != hipSuccess) {
      sl.d = nullptr;
      return fail(VR_ENOMEM, "hipMalloc(%zu) failed", cap);
    }
    sl.bytes = cap;
  }
  std::memcpy(sl.h, data, bytes);
  VR_HIP(hipMemcpyAsync(sl.d, sl.h, bytes, hipMemcpyHostToDevice, s));
  VR_HIP(hipEventRecord(sl.copied, s));
  sl.used = true;
  *dev = sl.d;
  return VR_OK;
}

// Global (min, max, non-finite count) of n floats at x, read back to the host.
int reduce_minmax(vr_ctx* ctx, const float* x, int64_t n, hipStream_t s, float out3[3]) {
  int32_t nb = (int32_t)std::min<int64_t>(2048, std::max<int64_t>(1, n / (256 * 16)));
  VR_TRY(ensure_device(&ctx->d_small, &ctx->small_bytes, (size_t)nb * 16 + 64));
  float* part = reinterpret_cast<float*>(ctx->d_small);
  float* res = reinterpret_cast<float*>(reinterpret_cast<char*>(ctx->d_small) + (size_t)nb * 16);
  VR_HIP(launch_minmax(x, n, part, nb, s));
  VR_HIP(launch_minmax_final(part, nb, res, s));
  VR_HIP(hipMemcpyAsync(out3, res, 3 * sizeof(float), hipMemcpyDeviceToHost, s));
  VR_HIP(hipStreamSynchronize(s));
  return VR_OK;
}

static bool finite_view(const vr_view& v) {
  for (int i = 0; i < 9; i++)
    if (!std::isfinite(v.R[i])) return false;
  return std::isfinite(v.extent) && std::isfinite(v.eye_dist);
}

int check_view(const vr_view* v, const int64_t n[3]) {
  if (!v) return fail(VR_EINVAL, "view is NULL");
  if (v->W < 1 || v->H < 1 || v->W > 16384 || v->H > 16384)
    return fail(VR_EINVAL, "image size %dx%d outside [1, 16384]", v->W, v->H);
  if (!finite_view(*v)) return fail(VR_EINVAL, "view has non-finite entries");
  double e3 = v->R[6] * v->R[6] + v->R[7] * v->R[7] + v->R[8] * v->R[8];
  if (!(e3 > 0.0)) return fail(VR_EINVAL, "view direction (third row of R) is zero");
  if (v->eye_dist < 0.0) return fail(VR_EINVAL, "eye_dist must be >= 0");
  if (v->eye_dist > 0.0) {
    double diag = 0.0;
    for (int i = 0; i < 3; i++) diag += (double)(n[i] - 1) * (double)(n[i] - 1);
    if (!(v->eye_dist > 0.5 * std::sqrt(diag)))
      return fail(VR_EINVAL, "eye_dist %g must exceed half the box diagonal (%g)", v->eye_dist, 0.5 * std::sqrt(diag));
  }
  return VR_OK;
}

int check_params(const vr_params* p) {
  if (!p) return fail(VR_EINVAL, "params is NULL");
  if (!(p->step > 0.0) || !std::isfinite(p->step)) return fail(VR_EINVAL, "step must be > 0");
  if (!(p->tau > 0.0) || !std::isfinite(p->tau)) return fail(VR_EINVAL, "tau must be > 0 (>= 1 disables)");
  if (p->ert_scope != VR_ERT_LOCAL && p->ert_scope != VR_ERT_GLOBAL) return fail(VR_EINVAL, "unknown ert_scope %d", p->ert_scope);
  if (p->mode != VR_MODE_DVR && p->mode != VR_MODE_MIP) return fail(VR_EINVAL, "unknown mode %d", p->mode);
  if (p->ckpt_K < 1) return fail(VR_EINVAL, "ckpt_K must be >= 1");
  if (p->tile != 0 && p->tile != 4 && p->tile != 8 && p->tile != 16)
    return fail(VR_EINVAL, "tile must be 0, 4, 8 or 16");
  return VR_OK;
}

// Normalisation window of a render: the table's, or the volume's range.
int resolve_window(vr_ctx* ctx, vr_volume* vol, hipStream_t s, double& vmin, double& vmax) {
  if (ctx->tf_vmin == 0.0 && ctx->tf_vmax == 0.0) {
    VR_TRY(volume_range(vol, s));
    vmin = vol->vmin;
    vmax = vol->vmax;
  } else {
    vmin = ctx->tf_vmin;
    vmax = ctx->tf_vmax;
  }
  return VR_OK;
}

int volume_range(vr_volume* vol, hipStream_t s) {
  if (vol->have_range) return VR_OK;
  float r[3];
  VR_TRY(reduce_minmax(vol->ctx, vol->data, vol->n[0] * vol->n[1] * vol->n[2], s, r));
  vol->vmin = r[0];
  vol->vmax = r[1];
  vol->nonfinite = (int64_t)r[2];
  vol->have_range = true;
  return VR_OK;
}

void fill_march_common(MarchArgs& a, const vr_volume* vol, const vr_params* p, double vmin, double vmax,
                       const float4* tf, int32_t M) {
  for (int i = 0; i < 3; i++) a.hi[i] = (double)(vol->n[i] - 1);
  a.step = p->step;
  a.tau = p->tau >= 1.0 ? 2.0f : (float)p->tau;
  a.ert = p->tau < 1.0;
  a.vmin = (float)vmin;
  a.inv_range = vmax > vmin ? (float)(1.0 / (vmax - vmin)) : 0.0f;
  a.M = M;
  a.tf = tf;
  a.mip = p->mode == VR_MODE_MIP ? 1 : 0;
  a.mask_axis = vol->spectral_axis;
  a.mask = nullptr;  // set by the callers that take a mask
  a.tile_w = p->tile ? p->tile : 8;
  a.tile_h = 64 / a.tile_w;
}

// (Re)build the macrocell grid of edge mc over the whole volume (mc = 0: drop it).
int build_macrocells(vr_volume* vol, int32_t mc, hipStream_t s) {
  if (vol->d_mc_mm || vol->d_mc_clear) {
    VR_HIP(hipStreamSynchronize(s));
    if (vol->d_mc_mm) VR_HIP(hipFree(vol->d_mc_mm));
    if (vol->d_mc_clear) VR_HIP(hipFree(vol->d_mc_clear));
  }
  vol->d_mc_mm = nullptr;
  vol->d_mc_clear = nullptr;
  vol->d_mc_count = nullptr;
  vol->mc_nclear = 0;
  vol->mc = 0;
  vol->mc_classified = false;
  for (int i = 0; i < 3; i++) vol->mcn[i] = 0;
  if (mc == 0) return VR_OK;
  int64_t c[3];
  for (int i = 0; i < 3; i++) c[i] = (vol->n[i] - 1 + mc - 1) / mc;
  const int64_t count = c[0] * c[1] * c[2];
  if (count >= ((int64_t)1 << 31)) return fail(VR_EINVAL, "%lld macrocells: too many", (long long)count);
  const size_t cbytes = ((size_t)count + 255) & ~(size_t)255;  // flags, then the clear-cell counter
  if (hipMalloc(&vol->d_mc_mm, (size_t)count * 8) != hipSuccess ||
      hipMalloc(&vol->d_mc_clear, cbytes + 256) != hipSuccess) {
    (void)hipGetLastError();
    if (vol->d_mc_mm) (void)hipFree(vol->d_mc_mm);
    vol->d_mc_mm = nullptr;
    vol->d_mc_clear = nullptr;
    return fail(VR_ENOMEM, "hipMalloc for %lld macrocells failed", (long long)count);
  }
  vol->d_mc_count = reinterpret_cast<unsigned int*>(vol->d_mc_clear + cbytes);
  VR_HIP(launch_mc_minmax(vol->data, vol->n, mc, c, vol->d_mc_mm, s));
  VR_HIP(hipStreamSynchronize(s));
  vol->mc = mc;
  for (int i = 0; i < 3; i++) vol->mcn[i] = c[i];
  return VR_OK;
}

int prepare_macrocells(vr_ctx* ctx, vr_volume* vol, const vr_params* p, double vmin, double vmax, MarchArgs& a,
                       hipStream_t s) {
  a.mc = 0;
  a.mc_clear = nullptr;
  for (int i = 0; i < 3; i++) a.mcn[i] = 0;
  // nothing to skip unless a run of at least three table entries is fully
  // transparent (a macrocell's entry range spans three or more entries);
  // maximum intensity projection does not use the table
  if (!p->ess || p->mode != VR_MODE_DVR || vol->mc <= 0 || ctx->tf_zero_run < 3) return VR_OK;
  if (!vol->mc_classified || vol->mc_tf_version != ctx->tf_version || vol->mc_vmin != vmin || vol->mc_vmax != vmax) {
    VR_HIP(launch_mc_classify(vol->d_mc_mm, vol->mcn[0] * vol->mcn[1] * vol->mcn[2], ctx->d_tf_nz, ctx->tf_m, vmin,
                              vmax, vol->d_mc_clear, vol->d_mc_count, s));
    // one read-back per table or window change: with no clear macrocell the
    // marches skip the per-slab test altogether
    unsigned int nclear = 0;
    VR_HIP(hipMemcpyAsync(&nclear, vol->d_mc_count, sizeof nclear, hipMemcpyDeviceToHost, s));
    VR_HIP(hipStreamSynchronize(s));
    vol->mc_nclear = nclear;
    vol->mc_classified = true;
    vol->mc_tf_version = ctx->tf_version;
    vol->mc_vmin = vmin;
    vol->mc_vmax = vmax;
  }
  if (vol->mc_nclear == 0) return VR_OK;
  a.mc = vol->mc;
  a.mc_clear = vol->d_mc_clear;
  for (int i = 0; i < 3; i++) a.mcn[i] = (int32_t)vol->mcn[i];
  return VR_OK;
}

}  // namespace vr

// ====================================================================== ABI
extern "C" {

const char* vr_last_error(void) { return g_err.c_str(); }

int vr_version(void) { return 2; }

void vr_params_default(vr_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->step = 0.5;
  p->tau = 0.99;
  p->ess = 1;
  p->ert_scope = VR_ERT_LOCAL;
  p->mode = VR_MODE_DVR;
  p->ckpt_K = 32;
  p->tile = 0;
}

int vr_create(int device, vr_ctx** out) {
  clear_error();
  if (!out) return fail(VR_EINVAL, "out is NULL");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(VR_EHIP, "no HIP device available (%s)", hipGetErrorString(e));
  }
  if (device < 0 || device >= ndev) return fail(VR_EHIP, "device %d out of range (have %d)", device, ndev);
  DeviceGuard g(device);
  vr_ctx* ctx = new (std::nothrow) vr_ctx();
  if (!ctx) return fail(VR_ENOMEM, "out of host memory");
  ctx->device = device;
  if (const char* m = std::getenv("VR_TILE_ORDER")) {
    if (!std::strcmp(m, "row")) ctx->tile_order = 0;
    if (!std::strcmp(m, "col")) ctx->tile_order = 1;
    int bw = 0, bh = 0;
    if (std::sscanf(m, "blk%dx%d", &bw, &bh) == 2 && bw >= 1 && bh >= 1 && bw * bh <= 64) {
      ctx->tile_order = 2;
      ctx->tile_bw = bw;
      ctx->tile_bh = bh;
    }
  }
  if (const char* m = std::getenv("VR_RING_SLOTS")) {
    const int k = std::atoi(m);
    if (k == 2 || k == 3) ctx->ring_nslots = k;
  }
  if (const char* m = std::getenv("VR_FOOT")) ctx->foot = std::atoi(m) != 0 ? 1 : 0;
  if (const char* m = std::getenv("VR_RING_REG")) ctx->ring_reg = std::atoi(m) != 0 ? 1 : 0;
  if (const char* m = std::getenv("VR_CELLS_WAVES")) ctx->cells_waves = std::max(0, std::min(32, std::atoi(m)));
  if (const char* m = std::getenv("VR_FOOT_BLOCK")) {
    int bf = 0, bg = 0;
    if (std::sscanf(m, "%dx%d", &bf, &bg) == 2 && bf >= 1 && bg >= 1 && bf * bg >= 2 && bf * bg <= 8) {
      ctx->foot_block = 1;
      ctx->foot_block_f = bf;
      ctx->foot_block_g = bg;
    } else {
      ctx->foot_block = std::atoi(m) != 0 ? -1 : 0;
    }
  }
  if (const char* m = std::getenv("VR_FOOT_PAD")) ctx->foot_pad = std::max(0, std::min(32, std::atoi(m)));
  if (const char* m = std::getenv("VR_FOOT_KMAX")) ctx->foot_kmax = std::max(1, std::min(4, std::atoi(m)));
  if (const char* m = std::getenv("VR_PERSP_CLASSES")) ctx->persp_classes = std::max(1, std::min(4, std::atoi(m)));
  if (const char* m = std::getenv("VR_PERSP_CELLS")) ctx->persp_cells = std::atoi(m) != 0 ? 1 : 0;
  if (const char* m = std::getenv("VR_PERSP_KMAX")) ctx->persp_kmax = std::max(1, std::min(4, std::atoi(m)));
  if (const char* m = std::getenv("VR_CELLS_WPB")) {
    const int k = std::atoi(m);
    ctx->cells_wpb = (k == 1 || k == 2 || k == 4) ? k : 0;
  }
  if (const char* m = std::getenv("VR_DEBUG_PLAN")) ctx->debug_plan = std::atoi(m) != 0;
  if (const char* m = std::getenv("VR_PERSP_FIT")) {
    const double f = std::atof(m);
    if (f >= 0.3 && f <= 1.0) ctx->persp_fit = f;
  }
  if (const char* m = std::getenv("VR_FOOT_MAXPX")) ctx->foot_maxpx = std::max(16, std::min(4096, std::atoi(m)));
  if (const char* m = std::getenv("VR_FOOT_RAYS")) {
    const double r = std::atof(m);
    if (r >= 16.0 && r <= 64.0) ctx->foot_rays = r;
  }
  if (const char* m = std::getenv("VR_BWD_LAYERS")) {
    const int k = std::atoi(m);
    if (k >= 1 && k <= 16) ctx->bwd_layer_cap = k;
  }
  if (const char* m = std::getenv("VR_BWD_BANDS")) ctx->bwd_bands = std::atoi(m) != 0 ? 1 : 0;
  if (const char* m = std::getenv("VR_BWD_SIDE")) ctx->bwd_side = std::atoi(m) != 0 ? 1 : 0;
  if (const char* m = std::getenv("VR_MARCH"))
    ctx->march_mode = std::strcmp(m, "gather") == 0 ? 1 : std::strcmp(m, "slab") == 0 ? 2 : std::strcmp(m, "ring") == 0 ? 3 : 0;
  if (const char* b = std::getenv("VR_LDS_BUDGET")) {
    const long v = std::strtol(b, nullptr, 10);
    if (v >= 256 && v <= 32768) ctx->lds_budget = (int32_t)v;
  }
  tune_load(ctx);
  if (hipEventCreateWithFlags(&ctx->done, hipEventDisableTiming) != hipSuccess) {
    delete ctx;
    return fail(VR_EHIP, "hipEventCreate failed");
  }
  for (auto& sl : ctx->ring)
    if (hipEventCreateWithFlags(&sl.copied, hipEventDisableTiming) != hipSuccess) {
      vr_destroy(ctx);
      return fail(VR_EHIP, "hipEventCreate failed");
    }
  // set-up of the allocation-free batched path: the device's scratch address,
  // a pinned staging buffer for its descriptors and the event of their copy
  if (int rc = noalloc_init(device); rc != VR_OK) {
    vr_destroy(ctx);
    return rc;
  }
  if (hipHostMalloc(&ctx->na_host, kNoAllocBytes, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->na_copied, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    vr_destroy(ctx);
    return fail(VR_ENOMEM, "pinned staging for the allocation-free batch failed");
  }
  *out = ctx;
  return VR_OK;
}

int vr_destroy(vr_ctx* ctx) {
  if (!ctx) return VR_OK;
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& sl : ctx->ring) {
    if (sl.h) (void)hipHostFree(sl.h);
    if (sl.d) (void)hipFree(sl.d);
    if (sl.copied) (void)hipEventDestroy(sl.copied);
  }
  if (ctx->d_tf) (void)hipFree(ctx->d_tf);
  if (ctx->d_tf_nz) (void)hipFree(ctx->d_tf_nz);
  if (ctx->d_mask) (void)hipFree(ctx->d_mask);
  if (ctx->d_arena) (void)hipFree(ctx->d_arena);
  if (ctx->d_small) (void)hipFree(ctx->d_small);
  if (ctx->d_scratch) (void)hipFree(ctx->d_scratch);
  if (ctx->d_ovf) (void)hipFree(ctx->d_ovf);
  if (ctx->spare.ckpt) (void)hipFree(ctx->spare.ckpt);
  if (ctx->spare.ckpt_j) (void)hipFree(ctx->spare.ckpt_j);
  if (ctx->spare.nused) (void)hipFree(ctx->spare.nused);
  for (auto& t : ctx->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  if (ctx->done) (void)hipEventDestroy(ctx->done);
  for (int i = 0; i < vr_ctx::kAux; i++) {
    if (ctx->aux[i]) (void)hipStreamDestroy(ctx->aux[i]);
    if (ctx->aux_join_ev[i]) (void)hipEventDestroy(ctx->aux_join_ev[i]);
  }
  if (ctx->aux_fork_ev) (void)hipEventDestroy(ctx->aux_fork_ev);
  if (ctx->na_host) (void)hipHostFree(ctx->na_host);
  if (ctx->na_copied) (void)hipEventDestroy(ctx->na_copied);
  delete ctx;
  return VR_OK;
}

int vr_set_profiling(vr_ctx* ctx, int on) {
  clear_error();
  if (!ctx) return fail(VR_EINVAL, "ctx is NULL");
  ctx->prof = on != 0;
  return VR_OK;
}

int vr_stage_times(vr_ctx* ctx, double* ms, int32_t* launches) {
  clear_error();
  if (!ctx) return fail(VR_EINVAL, "ctx is NULL");
  DeviceGuard g(ctx->device);
  double acc[VR_NSTAGES] = {0};
  int32_t cnt[VR_NSTAGES] = {0};
  for (auto& t : ctx->timed) {
    VR_HIP(hipEventSynchronize(t.b));
    float f = 0.f;
    VR_HIP(hipEventElapsedTime(&f, t.a, t.b));
    if (t.stage >= 0 && t.stage < VR_NSTAGES) {
      acc[t.stage] += f;
      cnt[t.stage]++;
    }
  }
  for (int i = 0; i < VR_NSTAGES; i++) {
    if (ms) ms[i] = acc[i];
    if (launches) launches[i] = cnt[i];
  }
  return VR_OK;
}

// ---------------------------------------------------------------- volumes
static int make_whole_brick(vr_volume* vol) {
  DevBrick b;
  std::memset(&b, 0, sizeof b);
  b.base = vol->data;
  b.sy = (int32_t)vol->n[0];
  b.sz = (int32_t)(vol->n[0] * vol->n[1]);
  for (int i = 0; i < 3; i++) {
    b.lo[i] = 0;
    b.hi[i] = (int32_t)(vol->n[i] - 1);
    b.clo[i] = 0;
    b.chi[i] = (int32_t)(vol->n[i] - 2);
  }
  b.closed = 7;
  b.vmin = vol->vmin;
  b.vmax = vol->vmax;
  b.slack = vol->owned ? 1 : 0;
  vol->whole = b;
  return VR_OK;
}

static int check_dims(int64_t n1, int64_t n2, int64_t n3) {
  if (n1 < 2 || n2 < 2 || n3 < 2) return fail(VR_EINVAL, "every dimension must be >= 2 (got %lld x %lld x %lld)",
                                               (long long)n1, (long long)n2, (long long)n3);
  if (n1 > (1 << 24) || n2 > (1 << 24) || n3 > (1 << 24)) return fail(VR_EINVAL, "dimension above 2^24");
  if (n1 * n2 > ((int64_t)1 << 31) - 1) return fail(VR_EINVAL, "n1*n2 must be below 2^31");
  return VR_OK;
}

int vr_volume_create(vr_ctx* ctx, const float* src, int src_on_device, int64_t n1, int64_t n2, int64_t n3,
                     const int64_t* sub_origin, const int64_t* sub_extent, uintptr_t stream, vr_volume** out) {
  clear_error();
  if (!ctx || !src || !out) return fail(VR_EINVAL, "ctx, src and out must be non-NULL");
  VR_TRY(check_dims(n1, n2, n3));
  int64_t so[3] = {0, 0, 0}, dn[3] = {n1, n2, n3};
  const int64_t sn[3] = {n1, n2, n3};
  if ((sub_origin == nullptr) != (sub_extent == nullptr))
    return fail(VR_EINVAL, "sub_origin and sub_extent must both be given or both NULL");
  if (sub_origin) {
    for (int i = 0; i < 3; i++) {
      so[i] = sub_origin[i];
      dn[i] = sub_extent[i];
      if (so[i] < 0 || dn[i] < 2 || so[i] + dn[i] > sn[i])
        return fail(VR_EINVAL, "sub-cube axis %d [%lld, %lld) outside [0, %lld) or extent < 2", i + 1,
                    (long long)so[i], (long long)(so[i] + dn[i]), (long long)sn[i]);
    }
    VR_TRY(check_dims(dn[0], dn[1], dn[2]));
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  VR_TRY(ctx_begin(ctx, s));
  vr_volume* vol = new (std::nothrow) vr_volume();
  if (!vol) return fail(VR_ENOMEM, "out of host memory");
  vol->ctx = ctx;
  for (int i = 0; i < 3; i++) vol->n[i] = dn[i];
  const int64_t count = dn[0] * dn[1] * dn[2];
  const size_t bytes = (size_t)count * sizeof(float);
  // 64 floats of slack after the voxels: staged loads may read past a row's end
  if (hipMalloc(&vol->data, bytes + 256) != hipSuccess) {
    (void)hipGetLastError();
    delete vol;
    return fail(VR_ENOMEM, "hipMalloc(%zu bytes) for the volume failed", bytes);
  }
  vol->owned = true;
  int rc = VR_OK;
  hipError_t e = hipSuccess;
  const bool whole = !sub_origin || (so[0] == 0 && so[1] == 0 && so[2] == 0 && dn[0] == n1 && dn[1] == n2 && dn[2] == n3);
  if (whole) {
    e = hipMemcpyAsync(vol->data, src, bytes, src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
  } else if (src_on_device) {
    e = launch_copy_box(src, sn, so, vol->data, dn, s);
  } else {
    for (int64_t z = 0; z < dn[2] && e == hipSuccess; z++) {
      const float* sp = src + ((so[2] + z) * n2 + so[1]) * n1 + so[0];
      e = hipMemcpy2DAsync(vol->data + z * dn[0] * dn[1], (size_t)dn[0] * 4, sp, (size_t)n1 * 4, (size_t)dn[0] * 4,
                           (size_t)dn[1], hipMemcpyHostToDevice, s);
    }
  }
  if (e != hipSuccess) rc = fail(VR_EHIP, "volume upload: %s", hipGetErrorString(e));
  if (rc == VR_OK) rc = volume_range(vol, s);
  if (rc == VR_OK && vol->nonfinite > 0)
    rc = fail(VR_ENONFINITE, "volume holds %lld non-finite voxels", (long long)vol->nonfinite);
  if (rc == VR_OK) rc = make_whole_brick(vol);
  if (rc == VR_OK) rc = ctx_end(ctx, s);
  if (rc != VR_OK) {
    vr_volume_destroy(vol);
    return rc;
  }
  *out = vol;
  return VR_OK;
}

int vr_volume_wrap(vr_ctx* ctx, float* dev_ptr, int64_t n1, int64_t n2, int64_t n3, uintptr_t stream,
                   vr_volume** out) {
  clear_error();
  (void)stream;
  if (!ctx || !dev_ptr || !out) return fail(VR_EINVAL, "ctx, dev_ptr and out must be non-NULL");
  VR_TRY(check_dims(n1, n2, n3));
  hipPointerAttribute_t attr;
  {
    DeviceGuard g(ctx->device);
    if (hipPointerGetAttributes(&attr, dev_ptr) != hipSuccess) {
      (void)hipGetLastError();
      return fail(VR_EINVAL, "dev_ptr is not a HIP allocation");
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
      return fail(VR_EINVAL, "dev_ptr is not device memory");
  }
  vr_volume* vol = new (std::nothrow) vr_volume();
  if (!vol) return fail(VR_ENOMEM, "out of host memory");
  vol->ctx = ctx;
  vol->n[0] = n1;
  vol->n[1] = n2;
  vol->n[2] = n3;
  vol->data = dev_ptr;
  vol->owned = false;
  make_whole_brick(vol);
  *out = vol;
  return VR_OK;
}

int vr_volume_destroy(vr_volume* vol) {
  if (!vol) return VR_OK;
  DeviceGuard g(vol->ctx->device);
  (void)hipDeviceSynchronize();
  if (vol->owned && vol->data) (void)hipFree(vol->data);
  if (vol->d_bricks) (void)hipFree(vol->d_bricks);
  if (vol->d_store) (void)hipFree(vol->d_store);
  if (vol->d_mc_mm) (void)hipFree(vol->d_mc_mm);
  if (vol->d_mc_clear) (void)hipFree(vol->d_mc_clear);
  if (vol->twin) vr_volume_destroy(vol->twin);
  delete vol;
  return VR_OK;
}

int vr_volume_minmax(vr_volume* vol, float* vmin, float* vmax) {
  clear_error();
  if (!vol || !vmin || !vmax) return fail(VR_EINVAL, "vol, vmin and vmax must be non-NULL");
  DeviceGuard g(vol->ctx->device);
  if (!vol->owned) vol->have_range = false;  // borrowed data may have changed
  VR_TRY(volume_range(vol, nullptr));
  if (vol->nonfinite > 0) return fail(VR_ENONFINITE, "volume holds non-finite voxels");
  *vmin = vol->vmin;
  *vmax = vol->vmax;
  vol->whole.vmin = vol->vmin;
  vol->whole.vmax = vol->vmax;
  return VR_OK;
}

int vr_volume_dims(const vr_volume* vol, int64_t n[3]) {
  clear_error();
  if (!vol || !n) return fail(VR_EINVAL, "vol and n must be non-NULL");
  for (int i = 0; i < 3; i++) n[i] = vol->n[i];
  return VR_OK;
}

// Brick records, storage and ranges of partition P for vol (and its
// macrocells); the caller holds the context's call order.
static int brick_volume(vr_volume* vol, Partition& P, bool materialize, int32_t macrocell, hipStream_t s) {
  vr_ctx* ctx = vol->ctx;
  const int32_t nb = (int32_t)P.boxes.size();
  const int64_t* n = vol->n;
  // storage: virtual (strided view of the volume) unless asked, or unless a
  // brick's local offsets would not fit 32-bit indices
  bool mat = materialize;
  std::vector<int64_t> sboxes(6 * (size_t)nb);
  for (int32_t b = 0; b < nb; b++) {
    int64_t slo[3], shi[3];
    stored_box(P.boxes[b], n, slo, shi);
    for (int i = 0; i < 3; i++) {
      sboxes[6 * b + i] = slo[i];
      sboxes[6 * b + 3 + i] = shi[i];
    }
    const int64_t span = (shi[2] - slo[2] + 1) * n[0] * n[1];
    if (span >= ((int64_t)1 << 31)) mat = true;
  }
  // free previous partition storage
  if (vol->d_store) {
    VR_HIP(hipStreamSynchronize(s));
    VR_HIP(hipFree(vol->d_store));
    vol->d_store = nullptr;
  }
  std::vector<int64_t> store_off((size_t)nb, 0);
  if (mat) {
    int64_t total = 0;
    for (int32_t b = 0; b < nb; b++) {
      store_off[b] = total;
      int64_t c = 1;
      for (int i = 0; i < 3; i++) c *= sboxes[6 * b + 3 + i] - sboxes[6 * b + i] + 1;
      total += (c + 63) & ~(int64_t)63;
    }
    total += 64;  // slack after the last brick
    if (hipMalloc(&vol->d_store, (size_t)total * sizeof(float)) != hipSuccess) {
      (void)hipGetLastError();
      vol->d_store = nullptr;
      return fail(VR_ENOMEM, "hipMalloc(%lld floats) for materialised bricks failed", (long long)total);
    }
    for (int32_t b = 0; b < nb; b++) {
      const int64_t so[3] = {sboxes[6 * b], sboxes[6 * b + 1], sboxes[6 * b + 2]};
      const int64_t dn[3] = {sboxes[6 * b + 3] - so[0] + 1, sboxes[6 * b + 4] - so[1] + 1, sboxes[6 * b + 5] - so[2] + 1};
      VR_HIP(launch_copy_box(vol->data, n, so, vol->d_store + store_off[b], dn, s));
    }
  }
  // per-brick (min, max) over stored voxels
  int zper = 4, zmax = 1;
  for (int32_t b = 0; b < nb; b++) zmax = std::max<int>(zmax, (int)(sboxes[6 * b + 5] - sboxes[6 * b + 2] + 1));
  const int zgroups = (zmax + zper - 1) / zper;
  const size_t need = (size_t)nb * 48 + (size_t)nb * zgroups * 8 + (size_t)nb * 8 + 1024;
  VR_TRY(ensure_device(&ctx->d_scratch, &ctx->scratch_bytes, need));
  char* sc = reinterpret_cast<char*>(ctx->d_scratch);
  int64_t* d_boxes = reinterpret_cast<int64_t*>(sc);
  float* d_part = reinterpret_cast<float*>(sc + (size_t)nb * 48);
  float* d_mm = reinterpret_cast<float*>(sc + (size_t)nb * 48 + (size_t)nb * zgroups * 8);
  VR_HIP(hipMemcpyAsync(d_boxes, sboxes.data(), (size_t)nb * 48, hipMemcpyHostToDevice, s));
  VR_HIP(launch_brick_minmax_parts(vol->data, n, d_boxes, nb, zgroups, zper, d_part, d_mm, s));
  std::vector<float> mm(2 * (size_t)nb);
  VR_HIP(hipMemcpyAsync(mm.data(), d_mm, (size_t)nb * 8, hipMemcpyDeviceToHost, s));
  VR_HIP(hipStreamSynchronize(s));
  // brick records
  std::vector<DevBrick> recs((size_t)nb);
  vol->bdesc.assign((size_t)nb, vr_brick_desc());
  for (int32_t b = 0; b < nb; b++) {
    const Box& bx = P.boxes[b];
    DevBrick& r = recs[b];
    std::memset(&r, 0, sizeof r);
    const int64_t* slo = &sboxes[6 * b];
    const int64_t* shi = &sboxes[6 * b + 3];
    if (mat) {
      const int64_t d1 = shi[0] - slo[0] + 1, d2 = shi[1] - slo[1] + 1;
      r.sy = (int32_t)d1;
      r.sz = (int32_t)(d1 * d2);
      r.base = vol->d_store + store_off[b] + ((bx.lo[2] - slo[2]) * d2 + (bx.lo[1] - slo[1])) * d1 + (bx.lo[0] - slo[0]);
    } else {
      r.sy = (int32_t)n[0];
      r.sz = (int32_t)(n[0] * n[1]);
      r.base = vol->data + (bx.lo[2] * n[1] + bx.lo[1]) * n[0] + bx.lo[0];
    }
    r.closed = 0;
    for (int i = 0; i < 3; i++) {
      r.lo[i] = (int32_t)bx.lo[i];
      r.hi[i] = (int32_t)bx.hi[i];
      if (bx.closed[i]) r.closed |= 1 << i;
      r.clo[i] = (int32_t)(slo[i] - bx.lo[i]);
      r.chi[i] = (int32_t)(shi[i] - 1 - bx.lo[i]);
    }
    r.vmin = mm[2 * b];
    r.vmax = mm[2 * b + 1];
    r.slack = (mat || vol->owned) ? 1 : 0;
    vr_brick_desc& d = vol->bdesc[b];
    for (int i = 0; i < 3; i++) {
      d.lo[i] = bx.lo[i];
      d.hi[i] = bx.hi[i];
      d.closed[i] = bx.closed[i];
      d.slo[i] = slo[i];
      d.shi[i] = shi[i];
    }
    d.vmin = r.vmin;
    d.vmax = r.vmax;
  }
  if (vol->d_bricks) {
    VR_HIP(hipFree(vol->d_bricks));
    vol->d_bricks = nullptr;
  }
  if (hipMalloc(&vol->d_bricks, sizeof(DevBrick) * (size_t)nb) != hipSuccess) {
    (void)hipGetLastError();
    vol->d_bricks = nullptr;
    return fail(VR_ENOMEM, "hipMalloc for the brick table failed");
  }
  VR_HIP(hipMemcpy(vol->d_bricks, recs.data(), sizeof(DevBrick) * (size_t)nb, hipMemcpyHostToDevice));
  vol->bricks = std::move(recs);
  vol->part = std::move(P);
  vol->bricked = true;
  vol->materialized = mat;
  vol->version++;
  return build_macrocells(vol, macrocell, s);
}

static void destroy_twin(vr_volume* vol) {
  if (vol->twin) {
    vr_volume_destroy(vol->twin);
    vol->twin = nullptr;
  }
}

// The permuted copy of vol (axes 1, 2, 3 = vol's axes 2, 3, 1), bricked with
// the permuted partition of vol.
static int make_twin(vr_volume* vol, int32_t macrocell, hipStream_t s) {
  const int64_t* n = vol->n;
  vr_volume* t = vol->twin;
  if (!t) {
    t = new vr_volume;
    t->ctx = vol->ctx;
    t->n[0] = n[1];
    t->n[1] = n[2];
    t->n[2] = n[0];
    t->spectral_axis = 1;  // the volume's axis 3 is the copy's axis 2
    if (hipMalloc(&t->data, sizeof(float) * (size_t)(n[0] * n[1] * n[2]) + 256) != hipSuccess) {
      (void)hipGetLastError();
      delete t;
      return fail(VR_ENOMEM, "hipMalloc for the permuted copy (%lld floats) failed", (long long)(n[0] * n[1] * n[2]));
    }
    t->owned = true;
    vol->twin = t;
  }
  VR_HIP(launch_twin(vol->data, n, t->data, s));
  t->have_range = vol->have_range;
  t->vmin = vol->vmin;
  t->vmax = vol->vmax;
  t->nonfinite = vol->nonfinite;
  VR_TRY(make_whole_brick(t));
  Partition P;
  permute_partition(vol->part, t->n, P);
  VR_TRY(brick_volume(t, P, false, macrocell, s));
  t->version++;
  return VR_OK;
}

int vr_volume_brick(vr_volume* vol, const vr_brick_spec* spec, uintptr_t stream) {
  clear_error();
  if (!vol || !spec) return fail(VR_EINVAL, "vol and spec must be non-NULL");
  if (spec->ghost != 1) return fail(VR_EINVAL, "ghost must be 1");
  if (spec->macrocell != 0 && (spec->macrocell < 2 || spec->macrocell > 1024))
    return fail(VR_EINVAL, "macrocell %d outside {0} U [2, 1024]", spec->macrocell);
  if (spec->twin != 0 && spec->twin != 1) return fail(VR_EINVAL, "twin must be 0 or 1");
  Partition P;
  std::string err;
  if (spec->mode == VR_BRICK_GRID) {
    if (!make_grid(vol->n, spec->size, P, err)) return fail(VR_EINVAL, "%s", err.c_str());
  } else if (spec->mode == VR_BRICK_LONGEST_AXIS) {
    if (!make_kd(vol->n, spec->nparts, P, err)) return fail(VR_EINVAL, "%s", err.c_str());
  } else {
    return fail(VR_EINVAL, "unknown brick mode %d", spec->mode);
  }
  vr_ctx* ctx = vol->ctx;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  VR_TRY(ctx_begin(ctx, s));
  VR_TRY(brick_volume(vol, P, spec->materialize != 0, spec->macrocell, s));
  if (spec->twin) {
    VR_TRY(make_twin(vol, spec->macrocell, s));
  } else if (vol->twin) {
    VR_HIP(hipStreamSynchronize(s));
    destroy_twin(vol);
  }
  return ctx_end(ctx, s);
}

int vr_volume_brick_info(const vr_volume* vol, int32_t* nb, vr_brick_desc* out) {
  clear_error();
  if (!vol || !nb) return fail(VR_EINVAL, "vol and nb must be non-NULL");
  const int32_t have = vol->bricked ? (int32_t)vol->bdesc.size() : 0;
  if (out) {
    if (*nb < have) return fail(VR_EINVAL, "capacity %d below brick count %d", *nb, have);
    for (int32_t i = 0; i < have; i++) out[i] = vol->bdesc[i];
  }
  *nb = have;
  return VR_OK;
}

int vr_volume_macrocell_info(const vr_volume* vol, int32_t* edge, int64_t count[3], float* minmax) {
  clear_error();
  if (!vol || !edge || !count) return fail(VR_EINVAL, "vol, edge and count must be non-NULL");
  *edge = vol->mc;
  for (int i = 0; i < 3; i++) count[i] = vol->mcn[i];
  if (minmax && vol->mc > 0) {
    DeviceGuard g(vol->ctx->device);
    VR_HIP(hipMemcpy(minmax, vol->d_mc_mm, (size_t)(vol->mcn[0] * vol->mcn[1] * vol->mcn[2]) * 8,
                     hipMemcpyDeviceToHost));
  }
  return VR_OK;
}

// ---------------------------------------------------------------- spectral-channel mask
int vr_mask_set(vr_ctx* ctx, const float* mask, int32_t n, int src_on_device, uintptr_t stream) {
  clear_error();
  if (!ctx) return fail(VR_EINVAL, "ctx is NULL");
  if (!mask || n == 0) {
    ctx->mask_n = 0;
    return VR_OK;
  }
  if (n < 2 || n > (1 << 20)) return fail(VR_EINVAL, "mask length %d outside [2, 2^20]", n);
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  std::vector<float> h((size_t)n);
  if (src_on_device) {
    VR_HIP(hipMemcpyAsync(h.data(), mask, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, s));
    VR_HIP(hipStreamSynchronize(s));
  } else {
    std::memcpy(h.data(), mask, sizeof(float) * (size_t)n);
  }
  for (int32_t i = 0; i < n; i++)
    if (!(h[i] >= 0.f && h[i] <= 1.f)) return fail(VR_EINVAL, "mask[%d] = %g outside [0, 1]", i, (double)h[i]);
  VR_TRY(ctx_begin(ctx, s));
  if (n > ctx->mask_cap) {
    if (ctx->d_mask) VR_HIP(hipFree(ctx->d_mask));
    ctx->d_mask = nullptr;
    ctx->mask_cap = 0;
    if (hipMalloc(&ctx->d_mask, sizeof(float) * (size_t)n) != hipSuccess) {
      (void)hipGetLastError();
      ctx->d_mask = nullptr;
      return fail(VR_ENOMEM, "hipMalloc for the mask failed");
    }
    ctx->mask_cap = n;
  }
  // synchronous copy: the host vector dies with this call
  VR_HIP(hipMemcpyAsync(ctx->d_mask, h.data(), sizeof(float) * (size_t)n, hipMemcpyHostToDevice, s));
  VR_HIP(hipStreamSynchronize(s));
  ctx->mask_n = n;
  return ctx_end(ctx, s);
}

// ---------------------------------------------------------------- transfer function
int vr_tf_set(vr_ctx* ctx, const float* rgba, int32_t m, double vmin, double vmax, int src_on_device,
              uintptr_t stream) {
  clear_error();
  if (!ctx || !rgba) return fail(VR_EINVAL, "ctx and rgba must be non-NULL");
  if (m < 2 || m > 4096) return fail(VR_EINVAL, "table size %d outside [2, 4096]", m);
  if (!std::isfinite(vmin) || !std::isfinite(vmax) || vmax < vmin)
    return fail(VR_EINVAL, "window must be finite with vmax >= vmin");
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  std::vector<float> h((size_t)m * 4);
  if (src_on_device) {
    VR_HIP(hipMemcpyAsync(h.data(), rgba, h.size() * 4, hipMemcpyDeviceToHost, s));
    VR_HIP(hipStreamSynchronize(s));
  } else {
    std::memcpy(h.data(), rgba, h.size() * 4);
  }
  for (size_t i = 0; i < h.size(); i++)
    if (!(h[i] >= 0.0f && h[i] <= 1.0f)) return fail(VR_EINVAL, "table entry %zu = %g outside [0, 1]", i, (double)h[i]);
  VR_TRY(ctx_begin(ctx, s));
  if (m > ctx->tf_cap) {
    if (ctx->d_tf) VR_HIP(hipFree(ctx->d_tf));
    ctx->d_tf = nullptr;
    if (hipMalloc(&ctx->d_tf, sizeof(float4) * (size_t)m) != hipSuccess) {
      (void)hipGetLastError();
      ctx->d_tf = nullptr;
      ctx->tf_cap = 0;
      return fail(VR_ENOMEM, "hipMalloc for the table failed");
    }
    ctx->tf_cap = m;
  }
  // prefix count of entries with opacity != 0 (macrocell classification)
  std::vector<int32_t> nz((size_t)m + 1, 0);
  for (int32_t i = 0; i < m; i++) nz[i + 1] = nz[i] + (h[4 * (size_t)i + 3] != 0.0f ? 1 : 0);
  if (m + 1 > ctx->tf_nz_cap) {
    if (ctx->d_tf_nz) VR_HIP(hipFree(ctx->d_tf_nz));
    ctx->d_tf_nz = nullptr;
    if (hipMalloc(&ctx->d_tf_nz, sizeof(int32_t) * ((size_t)m + 1)) != hipSuccess) {
      (void)hipGetLastError();
      ctx->d_tf_nz = nullptr;
      ctx->tf_nz_cap = 0;
      return fail(VR_ENOMEM, "hipMalloc for the table's opacity prefix failed");
    }
    ctx->tf_nz_cap = m + 1;
  }
  // synchronous copies: the host vectors die with this call
  VR_HIP(hipMemcpyAsync(ctx->d_tf, h.data(), h.size() * 4, hipMemcpyHostToDevice, s));
  VR_HIP(hipMemcpyAsync(ctx->d_tf_nz, nz.data(), nz.size() * 4, hipMemcpyHostToDevice, s));
  VR_HIP(hipStreamSynchronize(s));
  ctx->tf_zero = m - nz[(size_t)m];
  int32_t run = 0, best_run = 0;
  for (int32_t i = 0; i < m; i++) {
    run = h[4 * (size_t)i + 3] == 0.0f ? run + 1 : 0;
    best_run = std::max(best_run, run);
  }
  ctx->tf_zero_run = best_run;
  ctx->h_tf = std::move(h);
  ctx->tf_m = m;
  ctx->tf_vmin = vmin;
  ctx->tf_vmax = vmax;
  ctx->tf_set = true;
  ctx->tf_version++;
  VR_TRY(ctx_end(ctx, s));
  return VR_OK;
}

// ---------------------------------------------------------------- host-only helpers
int vr_plan_view(const int64_t dims[3], const vr_brick_spec* spec, const vr_view* view, int32_t* nb, int32_t* rects,
                 int32_t* order, int32_t* waves) {
  clear_error();
  if (!dims || !spec || !view || !nb) return fail(VR_EINVAL, "dims, spec, view and nb must be non-NULL");
  VR_TRY(check_dims(dims[0], dims[1], dims[2]));
  VR_TRY(check_view(view, dims));
  Partition P;
  std::string err;
  if (spec->mode == VR_BRICK_GRID) {
    if (!make_grid(dims, spec->size, P, err)) return fail(VR_EINVAL, "%s", err.c_str());
  } else if (spec->mode == VR_BRICK_LONGEST_AXIS) {
    if (!make_kd(dims, spec->nparts, P, err)) return fail(VR_EINVAL, "%s", err.c_str());
  } else {
    return fail(VR_EINVAL, "unknown brick mode %d", spec->mode);
  }
  const int32_t have = (int32_t)P.boxes.size();
  if ((rects || order || waves) && *nb < have) return fail(VR_EINVAL, "capacity %d below brick count %d", *nb, have);
  Camera cam;
  make_camera(*view, dims, cam);
  if (rects)
    for (int32_t b = 0; b < have; b++) {
      Rect r = brick_rect(cam, P.boxes[b]);
      rects[4 * b] = r.x0;
      rects[4 * b + 1] = r.y0;
      rects[4 * b + 2] = r.w;
      rects[4 * b + 3] = r.h;
    }
  if (order) {
    std::vector<int32_t> o;
    depth_order(P, cam, o);
    std::copy(o.begin(), o.end(), order);
  }
  if (waves) {
    std::vector<int32_t> w;
    brick_waves(P, cam, w);
    std::copy(w.begin(), w.end(), waves);
  }
  *nb = have;
  return VR_OK;
}

int vr_partition(const int64_t dims[3], const vr_brick_spec* spec, int32_t* nb, vr_brick_desc* out) {
  clear_error();
  if (!dims || !spec || !nb) return fail(VR_EINVAL, "dims, spec and nb must be non-NULL");
  VR_TRY(check_dims(dims[0], dims[1], dims[2]));
  Partition P;
  std::string err;
  if (spec->mode == VR_BRICK_GRID) {
    if (!make_grid(dims, spec->size, P, err)) return fail(VR_EINVAL, "%s", err.c_str());
  } else if (spec->mode == VR_BRICK_LONGEST_AXIS) {
    if (!make_kd(dims, spec->nparts, P, err)) return fail(VR_EINVAL, "%s", err.c_str());
  } else {
    return fail(VR_EINVAL, "unknown brick mode %d", spec->mode);
  }
  const int32_t have = (int32_t)P.boxes.size();
  if (out) {
    if (*nb < have) return fail(VR_EINVAL, "capacity %d below brick count %d", *nb, have);
    for (int32_t b = 0; b < have; b++) {
      vr_brick_desc d;
      std::memset(&d, 0, sizeof d);
      int64_t slo[3], shi[3];
      stored_box(P.boxes[b], dims, slo, shi);
      for (int i = 0; i < 3; i++) {
        d.lo[i] = P.boxes[b].lo[i];
        d.hi[i] = P.boxes[b].hi[i];
        d.closed[i] = P.boxes[b].closed[i];
        d.slo[i] = slo[i];
        d.shi[i] = shi[i];
      }
      out[b] = d;
    }
  }
  *nb = have;
  return VR_OK;
}

int vr_count_samples(const int64_t dims[3], const vr_view* view, double step, int64_t* nominal) {
  clear_error();
  if (!dims || !view || !nominal) return fail(VR_EINVAL, "dims, view and nominal must be non-NULL");
  VR_TRY(check_dims(dims[0], dims[1], dims[2]));
  VR_TRY(check_view(view, dims));
  if (!(step > 0.0)) return fail(VR_EINVAL, "step must be > 0");
  Camera cam;
  make_camera(*view, dims, cam);
  *nominal = count_samples(cam, dims, step);
  return VR_OK;
}

int vr_plan_cells(const int64_t dims[3], const vr_brick_spec* spec, const vr_view* view, double rays, int32_t kmax,
                  int32_t tf_entries, vr_cell_traffic* out) {
  clear_error();
  if (!dims || !spec || !view || !out) return fail(VR_EINVAL, "dims, spec, view and out must be non-NULL");
  VR_TRY(check_dims(dims[0], dims[1], dims[2]));
  VR_TRY(check_view(view, dims));
  if (view->eye_dist > 0.0) return fail(VR_EINVAL, "the cell march renders parallel views only");
  if (!(rays >= 0.0) || rays > 128.0) return fail(VR_EINVAL, "rays must be in [0, 128] (0: default)");
  if (kmax < 0 || kmax > 4) return fail(VR_EINVAL, "kmax must be in [0, 4] (0: default)");
  if (tf_entries < 0 || tf_entries > 4096) return fail(VR_EINVAL, "tf_entries must be in [0, 4096] (0: 256)");
  Partition P;
  std::string err;
  if (spec->mode == VR_BRICK_GRID) {
    if (!make_grid(dims, spec->size, P, err)) return fail(VR_EINVAL, "%s", err.c_str());
  } else if (spec->mode == VR_BRICK_LONGEST_AXIS) {
    if (!make_kd(dims, spec->nparts, P, err)) return fail(VR_EINVAL, "%s", err.c_str());
  } else {
    return fail(VR_EINVAL, "unknown brick mode %d", spec->mode);
  }
  vr_ctx defaults;  // the library's defaults (no device state is made)
  vr_view v = *view;
  int64_t n[3] = {dims[0], dims[1], dims[2]};
  // a view mostly along axis 1 is rendered from the copy with axes (2, 3, 1)
  const bool tw = spec->twin && std::fabs(v.R[6]) > std::max(std::fabs(v.R[7]), std::fabs(v.R[8]));
  if (tw) {
    for (int r = 0; r < 3; r++) {
      const double x = v.R[3 * r], y = v.R[3 * r + 1], z = v.R[3 * r + 2];
      v.R[3 * r] = y;
      v.R[3 * r + 1] = z;
      v.R[3 * r + 2] = x;
    }
    n[0] = dims[1];
    n[1] = dims[2];
    n[2] = dims[0];
    Partition Q;
    permute_partition(P, n, Q);
    P = Q;
  }
  Camera cam;
  make_camera(v, n, cam);
  FootShape fs;
  if (!pick_foot(cam, n, tf_entries > 0 ? tf_entries : 256, true, defaults.ring_reg > 0, defaults.ring_nslots,
                 rays > 0.0 ? rays : defaults.foot_rays, defaults.foot_pad, kmax > 0 ? kmax : defaults.foot_kmax, fs))
    return fail(VR_EUNSUPPORTED, "no slab axis suits the cell march for this view");
  FootTraffic t;
  for (const Box& b : P.boxes) {
    const Rect r = brick_rect(cam, b);
    if (r.w <= 0 || r.h <= 0) continue;
    foot_traffic(cam, fs, b, n, t);
  }
  std::memset(out, 0, sizeof *out);
  out->own_bytes = t.own;
  out->union_bytes = t.uni;
  out->window_bytes = t.win;
  out->line_bytes = t.line;
  out->segment_bytes = t.seg;
  out->cells = t.cells;
  out->cell_layers = t.layers;
  out->rays_per_cell = fs.rays;
  out->Tf = fs.Tf;
  out->Tg = fs.Tg;
  out->axis = fs.axis + 1;
  out->row_floats = (fs.nf + 3) & ~3;
  out->rows = fs.ng;
  out->twin = tw ? 1 : 0;
  return VR_OK;
}

}  // extern "C"
