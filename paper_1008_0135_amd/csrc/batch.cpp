// batch.cpp -- vr_render_batch: descriptor table, longest-first work order,
// HIP-graph capture of [descriptor copy -> counter reset -> persistent
// kernel] on a private stream, and replay on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "runtime.h"
#include "vr_internal.h"

struct vr_batch {
  vr_ctx* ctx = nullptr;
  // shape key: a graph is reused while these match
  std::vector<const vr_volume*> vols;
  std::vector<int32_t> W, H, M;
  double step = 0.0;
  float tau = 0.f;
  int32_t blocks = 0;
  // device and pinned host descriptor tables
  vr::BatchReq* d_reqs = nullptr;
  vr::BatchReq* h_reqs = nullptr;
  unsigned int* d_counter = nullptr;
  int32_t total_items = 0, max_M = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t launched = nullptr;
  bool pending = false;
  int64_t replays = 0;
};

namespace vr {

static void batch_free(vr_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->d_reqs) (void)hipFree(b->d_reqs);
  if (b->d_counter) (void)hipFree(b->d_counter);
  if (b->h_reqs) (void)hipHostFree(b->h_reqs);
  if (b->launched) (void)hipEventDestroy(b->launched);
  b->exec = nullptr;
  b->graph = nullptr;
  b->cap = nullptr;
  b->d_reqs = nullptr;
  b->d_counter = nullptr;
  b->h_reqs = nullptr;
  b->launched = nullptr;
  b->pending = false;
}

int batch_blocks(vr_ctx* ctx) {
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  const int wpc = ctx->tune_waves_per_cu > 0 ? ctx->tune_waves_per_cu : 8;
  return std::max(1, cus * wpc / 4);  // 4 wavefronts per block
}

// Estimated samples per pixel of a request: box volume / (pixel area x step), per pixel.
static double pixel_cost(const vr_volume* v, const vr_view& view, double step) {
  double diag = 0.0, vol = 1.0;
  for (int i = 0; i < 3; i++) {
    diag += (double)(v->n[i] - 1) * (double)(v->n[i] - 1);
    vol *= (double)(v->n[i] - 1);
  }
  const double S = view.extent > 0.0 ? view.extent : std::sqrt(diag);
  const double pitch = S / view.W;
  return vol / (pitch * pitch * step) / ((double)view.W * view.H);
}

static int log2_floor(double x) {
  int c = 0;
  while (c < 62 && std::ldexp(1.0, c + 1) <= x) c++;
  return c;
}

// Size class of a batched request for the autotuner: volume size class
// (floor(log2 voxels) / 3, i.e. per doubling of every axis) and image class
// (floor(log2 pixels) / 2, i.e. per doubling of each side).
std::string batch_key(const vr_volume* v, int32_t W, int32_t H) {
  char buf[64];
  snprintf(buf, sizeof buf, "batch/v%d/i%d", log2_floor((double)v->n[0] * v->n[1] * v->n[2]) / 3,
           log2_floor((double)W * H) / 2);
  return buf;
}

// Tile width of a batched request: the autotuner's choice for its size class, else 8.
int32_t batch_tile(const vr_ctx* ctx, const vr_volume* v, int32_t W, int32_t H) {
  const std::string key = batch_key(v, W, H);
  for (const auto& e : ctx->tune)
    if (e.key == key) return e.tile;
  return 8;
}

int check_batch(vr_ctx* ctx, const vr_request* reqs, int32_t n, const vr_params* p) {
  if (p && p->mode != VR_MODE_DVR) return fail(VR_EUNSUPPORTED, "batched rendering implements VR_MODE_DVR only");
  if (ctx->mask_n > 0) return fail(VR_EUNSUPPORTED, "batched rendering takes no channel mask");
  for (int32_t i = 0; i < n; i++) {
    const vr_request& r = reqs[i];
    if (!r.vol || !r.tf || !r.out) return fail(VR_EINVAL, "request %d: vol, tf and out must be non-NULL", i);
    if (r.vol->ctx != ctx) return fail(VR_EINVAL, "request %d: volume belongs to another context", i);
    if (r.vol->bricked) return fail(VR_EINVAL, "request %d: batched requests take unbricked volumes", i);
    if (r.vol->n[0] * r.vol->n[1] * r.vol->n[2] >= ((int64_t)1 << 31))
      return fail(VR_EUNSUPPORTED, "request %d: volume of 2^31 voxels or more", i);
    VR_TRY(check_view(&r.view, r.vol->n));
    if (r.m < 2 || r.m > 4096) return fail(VR_EINVAL, "request %d: table size %d outside [2, 4096]", i, r.m);
    if (!std::isfinite(r.vmin) || !std::isfinite(r.vmax) || r.vmax < r.vmin)
      return fail(VR_EINVAL, "request %d: window must be finite with vmax >= vmin", i);
  }
  return VR_OK;
}

// Descriptor table of a batch: requests in longest-first order (estimated
// samples per tile), each with its tile shape, and the work-item count.
// tiles: per-request tile width (4, 8, 16 or 32), or null for the tuned ones.
// Requests whose window defaults to the volume range need that range: with
// may_reduce = false they fail (VR_ESTATE) instead of computing it.
int plan_batch(vr_ctx* ctx, const vr_request* reqs, int32_t n, const vr_params* p, const int32_t* tiles,
               bool may_reduce, hipStream_t s, std::vector<BatchReq>& desc, int32_t& items, int32_t& maxM) {
  std::vector<double> vmin((size_t)n), vmax((size_t)n);
  std::vector<int32_t> tw((size_t)n);
  for (int32_t i = 0; i < n; i++) {
    vmin[i] = reqs[i].vmin;
    vmax[i] = reqs[i].vmax;
    if (vmin[i] == 0.0 && vmax[i] == 0.0) {
      vr_volume* v = const_cast<vr_volume*>(reqs[i].vol);
      if (!v->have_range && !may_reduce)
        return fail(VR_ESTATE, "request %d: the volume's range is not known yet; give the window", i);
      VR_TRY(volume_range(v, s));
      vmin[i] = v->vmin;
      vmax[i] = v->vmax;
    }
    tw[i] = tiles ? tiles[i] : batch_tile(ctx, reqs[i].vol, reqs[i].view.W, reqs[i].view.H);
    if (tw[i] != 4 && tw[i] != 8 && tw[i] != 16 && tw[i] != 32)
      return fail(VR_EINVAL, "request %d: tile width %d not 4, 8, 16 or 32", i, tw[i]);
  }
  std::vector<int32_t> order((size_t)n);
  std::iota(order.begin(), order.end(), 0);
  std::vector<double> cost((size_t)n);
  for (int32_t i = 0; i < n; i++) cost[i] = 64.0 * pixel_cost(reqs[i].vol, reqs[i].view, p->step);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
  desc.assign((size_t)n, BatchReq());
  items = 0;
  maxM = 2;
  for (int32_t k = 0; k < n; k++) {
    const int32_t i = order[k];
    const vr_request& r = reqs[i];
    BatchReq& d = desc[k];
    std::memset(&d, 0, sizeof d);
    make_camera(r.view, r.vol->n, d.cam);
    d.br = r.vol->whole;
    for (int a = 0; a < 3; a++) d.hi[a] = (double)(r.vol->n[a] - 1);
    d.vmin = (float)vmin[i];
    d.inv_range = vmax[i] > vmin[i] ? (float)(1.0 / (vmax[i] - vmin[i])) : 0.0f;
    d.tf = reinterpret_cast<const float4*>(r.tf);
    d.out = reinterpret_cast<float4*>(r.out);
    d.M = r.m;
    int sh = 0;
    while ((1 << sh) < tw[i]) sh++;
    d.tile_shift = sh;
    d.tiles_x = (r.view.W + tw[i] - 1) / tw[i];
    const int32_t th = 64 / tw[i];
    d.ntiles = d.tiles_x * ((r.view.H + th - 1) / th);
    d.item_begin = items;
    items += d.ntiles;
    maxM = std::max(maxM, r.m);
  }
  return VR_OK;
}

int render_batch(vr_ctx* ctx, const vr_request* reqs, int32_t n, const vr_params* p, vr_batch** cache,
                 hipStream_t s, int32_t force_blocks, const int32_t* tiles) {
  VR_TRY(check_batch(ctx, reqs, n, p));
  vr_batch* b = *cache;
  if (b && b->ctx != ctx) return fail(VR_EINVAL, "batch cache belongs to another context");
  const int32_t blocks = force_blocks > 0 ? force_blocks : batch_blocks(ctx);
  // shape key
  bool match = b && (int32_t)b->vols.size() == n && b->step == p->step && b->tau == (float)(p->tau >= 1.0 ? 2.0 : p->tau) &&
               b->blocks == blocks;
  for (int32_t i = 0; match && i < n; i++)
    match = b->vols[i] == reqs[i].vol && b->W[i] == reqs[i].view.W && b->H[i] == reqs[i].view.H && b->M[i] == reqs[i].m;
  std::vector<BatchReq> desc;
  int32_t items = 0, maxM = 2;
  VR_TRY(plan_batch(ctx, reqs, n, p, tiles, true, s, desc, items, maxM));
  if (b && match && (b->total_items != items || b->max_M != maxM)) match = false;
  if (!match) {
    if (!b) {
      b = new (std::nothrow) vr_batch();
      if (!b) return fail(VR_ENOMEM, "out of host memory");
      b->ctx = ctx;
      *cache = b;
    } else {
      VR_HIP(hipDeviceSynchronize());
      batch_free(b);
    }
    b->vols.assign((size_t)n, nullptr);
    b->W.assign((size_t)n, 0);
    b->H.assign((size_t)n, 0);
    b->M.assign((size_t)n, 0);
    for (int32_t i = 0; i < n; i++) {
      b->vols[i] = reqs[i].vol;
      b->W[i] = reqs[i].view.W;
      b->H[i] = reqs[i].view.H;
      b->M[i] = reqs[i].m;
    }
    b->step = p->step;
    b->tau = (float)(p->tau >= 1.0 ? 2.0 : p->tau);
    b->blocks = blocks;
    b->total_items = items;
    b->max_M = maxM;
    const size_t bytes = sizeof(BatchReq) * (size_t)std::max(n, 1);
    if (hipMalloc(&b->d_reqs, bytes) != hipSuccess || hipMalloc(&b->d_counter, 256) != hipSuccess ||
        hipHostMalloc(&b->h_reqs, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      batch_free(b);
      return fail(VR_ENOMEM, "batch tables allocation failed");
    }
    VR_HIP(hipEventCreateWithFlags(&b->launched, hipEventDisableTiming));
    VR_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    std::memcpy(b->h_reqs, desc.data(), sizeof(BatchReq) * (size_t)n);
    BatchArgs a;
    std::memset(&a, 0, sizeof a);
    a.reqs = b->d_reqs;
    a.counter = b->d_counter;
    a.nreq = n;
    a.total_items = items;
    a.max_M = maxM;
    a.step = p->step;
    a.tau = b->tau;
    VR_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = hipMemcpyAsync(b->d_reqs, b->h_reqs, sizeof(BatchReq) * (size_t)n, hipMemcpyHostToDevice, b->cap);
    hipError_t e2 = e1 == hipSuccess ? launch_batch(a, blocks, b->cap) : e1;
    hipError_t e3 = hipStreamEndCapture(b->cap, &b->graph);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
      (void)hipGetLastError();
      batch_free(b);
      return fail(VR_EHIP, "graph capture failed: %s", hipGetErrorString(e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3)));
    }
    VR_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  } else {
    // the previous replay may still be reading the pinned descriptors
    if (b->pending) VR_HIP(hipEventSynchronize(b->launched));
    std::memcpy(b->h_reqs, desc.data(), sizeof(BatchReq) * (size_t)n);
  }
  VR_TRY(stage_begin(ctx, VR_STAGE_BATCH, s));
  VR_HIP(hipGraphLaunch(b->exec, s));
  VR_TRY(stage_end(ctx, s));
  VR_HIP(hipEventRecord(b->launched, s));
  b->pending = true;
  b->replays++;
  return VR_OK;
}

}  // namespace vr

using namespace vr;

extern "C" {

int vr_render_batch(vr_ctx* ctx, const vr_request* reqs, int32_t n, const vr_params* p, vr_batch** cache,
                    uintptr_t stream) {
  clear_error();
  if (!ctx || !reqs || !cache || n < 1) return fail(VR_EINVAL, "ctx, reqs and cache must be non-NULL, n >= 1");
  VR_TRY(check_params(p));
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  VR_TRY(ctx_begin(ctx, s));
  VR_TRY(render_batch(ctx, reqs, n, p, cache, s, 0, nullptr));
  return ctx_end(ctx, s);
}

int vr_render_batch_noalloc(vr_ctx* ctx, const vr_request* reqs, int32_t n, const vr_params* p, uintptr_t stream) {
  clear_error();
  if (!ctx || !reqs || n < 1) return fail(VR_EINVAL, "ctx and reqs must be non-NULL, n >= 1");
  if (n > kNoAllocMaxReq)
    return fail(VR_EINVAL, "%d requests exceed the allocation-free batch's limit of %d", n, kNoAllocMaxReq);
  VR_TRY(check_params(p));
  VR_TRY(check_batch(ctx, reqs, n, p));
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  unsigned char* dev = static_cast<unsigned char*>(noalloc_scratch(ctx->device));
  if (!dev || !ctx->na_host) return fail(VR_ESTATE, "allocation-free batch not set up on device %d", ctx->device);
  std::vector<BatchReq> desc;
  int32_t items = 0, maxM = 2;
  VR_TRY(plan_batch(ctx, reqs, n, p, nullptr, false, s, desc, items, maxM));
  VR_TRY(ctx_begin(ctx, s));
  // the previous call's copy out of the pinned staging must be done before it is overwritten
  if (ctx->na_pending) VR_HIP(hipEventSynchronize(ctx->na_copied));
  const size_t bytes = sizeof(BatchReq) * (size_t)n;
  std::memcpy(ctx->na_host, desc.data(), bytes);
  VR_HIP(hipMemcpyAsync(dev, ctx->na_host, bytes, hipMemcpyHostToDevice, s));
  VR_HIP(hipEventRecord(ctx->na_copied, s));
  ctx->na_pending = true;
  BatchArgs a;
  std::memset(&a, 0, sizeof a);
  a.reqs = reinterpret_cast<const BatchReq*>(dev);
  a.counter = reinterpret_cast<unsigned int*>(dev + sizeof(BatchReq) * (size_t)kNoAllocMaxReq);
  a.nreq = n;
  a.total_items = items;
  a.max_M = maxM;
  a.step = p->step;
  a.tau = (float)(p->tau >= 1.0 ? 2.0 : p->tau);
  // the work counter is cleared by a kernel of the launch sequence (no memset)
  VR_HIP(launch_batch(a, batch_blocks(ctx), s));
  return ctx_end(ctx, s);
}

int vr_batch_destroy(vr_batch* b) {
  if (!b) return VR_OK;
  DeviceGuard g(b->ctx->device);
  (void)hipDeviceSynchronize();
  batch_free(b);
  delete b;
  return VR_OK;
}

}  // extern "C"
