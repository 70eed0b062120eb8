// tune.cpp -- the autotuner: times candidate launch shapes on the caller's
// data and keeps the fastest per shape class (volume size class, image size)
// in the context, optionally persisted to the file named by VR_TUNE_CACHE.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "forward.h"
#include "runtime.h"
#include "vr_internal.h"

namespace vr {

static int size_class(int64_t n) {
  int c = 0;
  while ((int64_t)1 << (c + 1) <= n) c++;
  return c;  // floor(log2 n)
}

std::string tune_key(const vr_volume* vol, int32_t W, int32_t H, int32_t mode) {
  char buf[128];
  snprintf(buf, sizeof buf, "render/%d.%d.%d/%s/%dx%d%s", size_class(vol->n[0]), size_class(vol->n[1]),
           size_class(vol->n[2]), vol->bricked ? "bricked" : "whole", W, H, mode == VR_MODE_MIP ? "/mip" : "");
  return buf;
}

void tuned_shape(const vr_ctx* ctx, const vr_volume* vol, int32_t W, int32_t H, const vr_params* p, int32_t& tile,
                 int32_t& budget, int32_t& mode) {
  tile = p->tile ? p->tile : 8;
  budget = ctx->lds_budget;
  mode = ctx->march_mode;
  if (p->tile) return;
  const std::string key = tune_key(vol, W, H, p->mode);
  for (const auto& e : ctx->tune)
    if (e.key == key) {
      tile = e.tile;
      budget = e.lds_budget;
      mode = e.march_mode;
      return;
    }
}

void tune_load(vr_ctx* ctx) {
  const char* path = std::getenv("VR_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char key[256];
  int tile, budget, mode;
  double ms;
  while (std::fscanf(f, "%255s %d %d %d %lf", key, &tile, &budget, &mode, &ms) == 5) {
    if (std::strcmp(key, "batch/waves_per_cu") == 0) {
      ctx->tune_waves_per_cu = tile;
      continue;
    }
    if (std::strncmp(key, "batch/", 6) == 0) {
      if (tile == 4 || tile == 8 || tile == 16 || tile == 32) ctx->tune.push_back(vr_ctx::TuneEntry{key, tile, 0, 1, ms});
      continue;
    }
    if ((tile == 4 || tile == 8 || tile == 16) && budget >= 256 && budget <= 32768 && mode >= 0 && mode <= 3)
      ctx->tune.push_back(vr_ctx::TuneEntry{key, tile, budget, mode, ms});
  }
  std::fclose(f);
}

static void tune_save(const vr_ctx* ctx) {
  const char* path = std::getenv("VR_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  for (const auto& e : ctx->tune) std::fprintf(f, "%s %d %d %d %.6f\n", e.key.c_str(), e.tile, e.lds_budget, e.march_mode, e.ms);
  if (ctx->tune_waves_per_cu > 0) std::fprintf(f, "batch/waves_per_cu %d 0 0 0\n", ctx->tune_waves_per_cu);
  std::fclose(f);
}

// Average time (ms) of `reps` calls of fn on stream s, after one warm-up call.
template <class F>
static int time_ms(hipStream_t s, int reps, F fn, double& ms) {
  VR_TRY(fn());
  hipEvent_t a, b;
  VR_HIP(hipEventCreate(&a));
  VR_HIP(hipEventCreate(&b));
  int rc = VR_OK;
  if (hipEventRecord(a, s) != hipSuccess) rc = fail(VR_EHIP, "hipEventRecord failed");
  for (int i = 0; i < reps && rc == VR_OK; i++) rc = fn();
  float f = 0.f;
  if (rc == VR_OK && (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                      hipEventElapsedTime(&f, a, b) != hipSuccess))
    rc = fail(VR_EHIP, "event timing failed");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  ms = (double)f / reps;
  return rc;
}

}  // namespace vr

using namespace vr;

extern "C" {

int vr_autotune(vr_ctx* ctx, const vr_volume* cvol, const vr_view* view, const vr_params* p, vr_tune_result* out,
                uintptr_t stream) {
  clear_error();
  VR_TRY(validate_render(ctx, cvol, view, 1, p));
  if (!out) return fail(VR_EINVAL, "out is NULL");
  vr_volume* vol = const_cast<vr_volume*>(cvol);
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  float* img = nullptr;
  if (hipMalloc(&img, sizeof(float) * 4 * (size_t)view->W * view->H) != hipSuccess) {
    (void)hipGetLastError();
    return fail(VR_ENOMEM, "hipMalloc for the tuning image failed");
  }
  const std::string key = tune_key(vol, view->W, view->H, p->mode);
  // drop a previous entry for this key so the candidates run as given
  for (size_t i = 0; i < ctx->tune.size(); i++)
    if (ctx->tune[i].key == key) {
      ctx->tune.erase(ctx->tune.begin() + (long)i);
      break;
    }
  const int32_t saved_mode = ctx->march_mode, saved_budget = ctx->lds_budget;
  struct Cand {
    int32_t tile, budget, mode;
  };
  // default (ring, else slabs), slab-only budgets, slab tiles, gathers
  std::vector<Cand> cands = {{8, 4096, 0}, {8, 4096, 2}, {8, 2048, 2}, {8, 6144, 2}, {8, 8192, 2},
                             {4, 4096, 2}, {16, 4096, 2}, {8, 0, 1}, {4, 0, 1}, {16, 0, 1}};
  double best = INFINITY, dflt = INFINITY;
  Cand pick = cands[0];
  int rc = VR_OK;
  for (size_t c = 0; c < cands.size() && rc == VR_OK; c++) {
    ctx->march_mode = cands[c].mode;
    if (cands[c].budget) ctx->lds_budget = cands[c].budget;
    vr_params q = *p;
    q.tile = cands[c].tile;
    double ms = 0.0;
    rc = time_ms(s, 3, [&]() {
      VR_TRY(ctx_begin(ctx, s));
      VR_TRY(render_forward(ctx, vol, view, 1, &q, img, s, nullptr));
      return ctx_end(ctx, s);
    }, ms);
    ctx->march_mode = saved_mode;
    ctx->lds_budget = saved_budget;
    if (rc != VR_OK) break;
    if (c == 0) dflt = ms;
    if (ms < best) {
      best = ms;
      pick = cands[c];
      if (!pick.budget) pick.budget = saved_budget;
    }
  }
  (void)hipFree(img);
  if (rc != VR_OK) return rc;
  ctx->tune.push_back(vr_ctx::TuneEntry{key, pick.tile, pick.budget, pick.mode, best});
  tune_save(ctx);
  out->tile = pick.tile;
  out->waves_per_cu = ctx->tune_waves_per_cu;
  out->ms = best;
  out->ms_default = dflt;
  out->lds_budget = pick.budget;
  out->march_mode = pick.mode;
  return VR_OK;
}

int vr_autotune_batch(vr_ctx* ctx, const vr_request* reqs, int32_t n, const vr_params* p, vr_batch** cache,
                      vr_tune_result* out, uintptr_t stream) {
  clear_error();
  if (!ctx || !reqs || !cache || !out || n < 1) return fail(VR_EINVAL, "ctx, reqs, cache and out must be non-NULL");
  VR_TRY(check_params(p));
  VR_TRY(check_batch(ctx, reqs, n, p));
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  // 1. tile shape per size class: the requests of one class rendered as a
  //    batch of their own with each candidate tile (same grid as the default)
  std::vector<std::string> keys((size_t)n);
  for (int32_t i = 0; i < n; i++) keys[i] = batch_key(reqs[i].vol, reqs[i].view.W, reqs[i].view.H);
  std::vector<std::string> classes;
  for (const std::string& k : keys)
    if (std::find(classes.begin(), classes.end(), k) == classes.end()) classes.push_back(k);
  int32_t ntile_wins[4] = {0, 0, 0, 0};
  for (const std::string& key : classes) {
    std::vector<vr_request> sub;
    for (int32_t i = 0; i < n; i++)
      if (keys[i] == key) sub.push_back(reqs[i]);
    const int32_t m = (int32_t)sub.size();
    const int32_t tcand[] = {8, 16, 4, 32};
    double best = INFINITY;
    int32_t pick = 8;
    vr_batch* tmp = nullptr;
    int rc = VR_OK;
    for (int32_t t : tcand) {
      std::vector<int32_t> tiles((size_t)m, t);
      double ms = 0.0;
      rc = time_ms(s, 3, [&]() {
        VR_TRY(ctx_begin(ctx, s));
        VR_TRY(render_batch(ctx, sub.data(), m, p, &tmp, s, 0, tiles.data()));
        return ctx_end(ctx, s);
      }, ms);
      if (rc != VR_OK) break;
      if (ms < best) {
        best = ms;
        pick = t;
      }
    }
    (void)vr_batch_destroy(tmp);
    if (rc != VR_OK) return rc;
    for (size_t i = 0; i < ctx->tune.size(); i++)
      if (ctx->tune[i].key == key) {
        ctx->tune.erase(ctx->tune.begin() + (long)i);
        break;
      }
    ctx->tune.push_back(vr_ctx::TuneEntry{key, pick, 0, 1, best});
    ntile_wins[pick == 4 ? 0 : pick == 8 ? 1 : pick == 16 ? 2 : 3]++;
  }
  // 2. persistent-grid occupancy for the whole batch with the tuned tiles
  const int32_t cands[] = {8, 2, 4, 16, 32};
  double best = INFINITY, dflt = INFINITY;
  int32_t pick = 8;
  for (int32_t wpc : cands) {
    double ms = 0.0;
    VR_TRY(time_ms(s, 3, [&]() {
      VR_TRY(ctx_begin(ctx, s));
      VR_TRY(render_batch(ctx, reqs, n, p, cache, s, std::max(1, cus * wpc / 4), nullptr));
      return ctx_end(ctx, s);
    }, ms));
    if (wpc == 8) dflt = ms;
    if (ms < best) {
      best = ms;
      pick = wpc;
    }
  }
  ctx->tune_waves_per_cu = pick;
  tune_save(ctx);
  // leave the cache holding the graph of the chosen grid and tiles
  VR_TRY(ctx_begin(ctx, s));
  VR_TRY(render_batch(ctx, reqs, n, p, cache, s, 0, nullptr));
  VR_TRY(ctx_end(ctx, s));
  // the most frequent tile choice over the classes
  int32_t most = 1;
  for (int32_t k = 0; k < 4; k++)
    if (ntile_wins[k] > ntile_wins[most]) most = k;
  out->tile = 4 << most;
  out->waves_per_cu = pick;
  out->ms = best;
  out->ms_default = dflt;
  out->lds_budget = 0;
  out->march_mode = 1;
  return VR_OK;
}

/*
 * Tile width each request of a batch runs with (the tuned choice of its size
 * class, else 8): tiles[i] for reqs[i].
 */
int vr_batch_tiles(const vr_ctx* ctx, const vr_request* reqs, int32_t n, int32_t* tiles) {
  clear_error();
  if (!ctx || !reqs || !tiles || n < 0) return fail(VR_EINVAL, "ctx, reqs and tiles must be non-NULL");
  for (int32_t i = 0; i < n; i++) {
    if (!reqs[i].vol) return fail(VR_EINVAL, "request %d has no volume", i);
    tiles[i] = batch_tile(ctx, reqs[i].vol, reqs[i].view.W, reqs[i].view.H);
  }
  return VR_OK;
}

}  // extern "C"
