// runtime.h -- host-side objects behind the opaque handles of vr.h and the
// helpers the entry points share (errors, device guard, stream ordering,
// table uploads, stage timers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "plan.h"
#include "vr_internal.h"

namespace vr {

int fail(int code, const char* fmt, ...);
void clear_error();

#define VR_TRY(expr)                 \
  do {                               \
    int rc_ = (expr);                \
    if (rc_ != VR_OK) return rc_;    \
  } while (0)

#define VR_HIP(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      (void)hipGetLastError();                                                          \
      return ::vr::fail(VR_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));        \
    }                                                                                   \
  } while (0)

// Makes `dev` current for the scope and restores the caller's device.
struct DeviceGuard {
  int prev = -1, target = -1;
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
};

}  // namespace vr

struct vr_ctx {
  int device = 0;
  // transfer function slot
  float4* d_tf = nullptr;
  int32_t tf_cap = 0, tf_m = 0;
  std::vector<float> h_tf;
  double tf_vmin = 0.0, tf_vmax = 0.0;
  bool tf_set = false;
  // spectral-channel mask: weights along the volume's axis 3 (mask_n = 0: none)
  float* d_mask = nullptr;
  int32_t mask_n = 0, mask_cap = 0;
  uint64_t tf_version = 0;
  int32_t* d_tf_nz = nullptr;  // [M + 1] prefix count of entries with opacity != 0
  int32_t tf_nz_cap = 0;
  int32_t tf_zero = 0;         // entries with opacity == 0
  int32_t tf_zero_run = 0;     // longest run of consecutive entries with opacity == 0
  // brick-image arena and general scratch
  void* d_arena = nullptr;
  size_t arena_bytes = 0;
  void* d_small = nullptr;
  size_t small_bytes = 0;
  void* d_scratch = nullptr;
  size_t scratch_bytes = 0;
  // device buffers of the last destroyed forward state (checkpoints, sample
  // cursors, samples used + the adjoint's bound flag), kept for the next one
  struct StateBufs {
    float* ckpt = nullptr;
    int32_t* ckpt_j = nullptr;
    int32_t* nused = nullptr;
    size_t ckpt_bytes = 0, ckpt_j_bytes = 0, nused_bytes = 0;
  } spare;
  // footprint-cell marches: per side stream, a count and the work items of
  // cells with more than 64 pixels
  void* d_ovf = nullptr;
  size_t ovf_bytes = 0;
  // per-call table uploads: pinned staging + device copy, reused round-robin
  static constexpr int kRing = 4;
  struct Slot {
    void* h = nullptr;
    void* d = nullptr;
    size_t bytes = 0;
    hipEvent_t copied = nullptr;
    bool used = false;
  } ring[kRing];
  int ring_next = 0;
  // calls on this context are ordered, whatever stream they use
  hipEvent_t done = nullptr;
  bool done_valid = false;
  // side streams (default priority) for work of one call that is independent
  // (the views of a render with the opacity test over whole rays), forked
  // from and joined back into the caller's stream; created on first use
  static constexpr int kAux = 4;
  hipStream_t aux[kAux] = {};
  hipEvent_t aux_fork_ev = nullptr, aux_join_ev[kAux] = {};
  // stage timers
  bool prof = false;
  struct Timed {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> event_pool;
  hipStream_t prof_stream = nullptr;
  // march selection: 0 = automatic (per-layer ring when its windows fit, else
  // LDS-staged slabs when a slab fits, else gather); 1 = gather only;
  // 2 = LDS-staged slabs (else gather); 3 = same as 0
  int32_t march_mode = 0;
  int32_t lds_budget = 4096;  // floats of LDS for one slab's voxel box
  int32_t bwd_layer_cap = 3;  // adjoint on the ring layout: cell layers per checkpoint group, at most
  // ring march: tiles of a brick numbered along rows (0), down columns (1) or in
  // blocks of tile_bw x tile_bh tiles (2)
  int32_t tile_order = 2, tile_bw = 2, tile_bh = 4;
  int32_t ring_nslots = 0;    // forward ring march (plain orthographic): LDS slots per wavefront, 3 or 2; 0 = by occupancy
  int32_t foot = 1;           // forward ring march, parallel rays: footprint cells (1) or 8 x 8 pixel tiles (0)
  int32_t cells_waves = 16;   // cells march: wavefronts per compute unit at most (0 = as LDS allows)
  int32_t ring_reg = 1;       // footprint cells, plain march: the layer after next staged in registers (1)
  double foot_rays = 60.0;    // footprint cells: mean pixels per cell (each holds at most 64 in one pass)
  int32_t foot_pad = 0;       // footprint cells: extra floats per window row (LDS bank spread)
  int32_t foot_kmax = 2;      // footprint cells: window rows of at most this many 128-byte lines
  int32_t bwd_bands = 1;      // ring adjoint: tile groups in XCD bands of equal estimated work (0: equal counts)
  int32_t bwd_side = 1;       // differentiable pair: views side by side on the side streams (one table reduction)
  int32_t foot_maxpx = 64;    // footprint cells: pixels of a cell at most, as sized (past 64: marched by gathers)
  int32_t cells_wpb = 0;      // register-staged cells march: wavefronts per workgroup (0: the plan's)
  int32_t foot_block = 0;     // blocks of cells per workgroup: -1 = by cost, 0 = off, 1 = foot_block_f x _g
  int32_t foot_block_f = 0, foot_block_g = 0;
  bool debug_plan = false;    // print each view's march shape to stderr
  double persp_fit = 0.95;    // perspective ring march: fraction of tiles whose windows the slot holds
  int32_t persp_classes = 3;  // perspective ring march: launches per view, bricks grouped by window size
  int32_t persp_cells = 1;    // perspective views: footprint cells sized per brick (0: 8 x 8 pixel tiles)
  int32_t persp_kmax = 1;     // perspective footprint cells: window rows of at most this many 128-byte lines
  // autotune cache: render shapes -> (tile edge, LDS budget, march mode)
  struct TuneEntry {
    std::string key;
    int32_t tile, lds_budget, march_mode;
    double ms;
  };
  std::vector<TuneEntry> tune;
  int32_t tune_waves_per_cu = 0;  // persistent-grid occupancy of the batched path (0 = default 8)
  // allocation-free batched path: pinned staging for its descriptor table
  // (made at creation) and the event of the last copy out of it
  void* na_host = nullptr;
  hipEvent_t na_copied = nullptr;
  bool na_pending = false;
};

struct vr_volume {
  vr_ctx* ctx = nullptr;
  int64_t n[3] = {0, 0, 0};
  float* data = nullptr;
  bool owned = false;
  bool have_range = false;
  float vmin = 0.f, vmax = 0.f;
  int64_t nonfinite = 0;
  vr::DevBrick whole;  // the whole volume as one brick (unbricked rendering)
  bool bricked = false, materialized = false;
  vr::Partition part;
  std::vector<vr::DevBrick> bricks;
  std::vector<vr_brick_desc> bdesc;
  vr::DevBrick* d_bricks = nullptr;
  float* d_store = nullptr;  // materialised brick storage
  // macrocells (empty-space skipping): edge in cells, counts, (min, max), and the
  // per-table "opacity is 0 over the range" flags with the table they were made for
  int32_t mc = 0;
  int64_t mcn[3] = {0, 0, 0};
  float* d_mc_mm = nullptr;
  uint8_t* d_mc_clear = nullptr;
  unsigned int* d_mc_count = nullptr;  // clear macrocells of the last classification
  int64_t mc_nclear = 0;
  bool mc_classified = false;
  uint64_t mc_tf_version = 0;
  double mc_vmin = 0.0, mc_vmax = 0.0;
  uint64_t version = 0;
  // permuted copy (axes 1, 2, 3 = this volume's axes 2, 3, 1), bricked with the
  // permuted partition, for views that look along axis 1 (owned; or null)
  vr_volume* twin = nullptr;
  int32_t spectral_axis = 2;  // the axis the channel mask runs along (1 in the permuted copy)
};

namespace vr {

int ctx_begin(vr_ctx* ctx, hipStream_t s);
int ctx_end(vr_ctx* ctx, hipStream_t s);
int stage_begin(vr_ctx* ctx, int stage, hipStream_t s);
// make the side streams wait for the work queued on s so far / s wait for theirs
int aux_fork(vr_ctx* ctx, hipStream_t s);
int aux_join(vr_ctx* ctx, hipStream_t s);
int stage_end(vr_ctx* ctx, hipStream_t s);
int ensure_device(void** p, size_t* cap, size_t need);
int upload_tables(vr_ctx* ctx, hipStream_t s, const void* data, size_t bytes, void** dev);
int reduce_minmax(vr_ctx* ctx, const float* x, int64_t n, hipStream_t s, float out3[3]);
int volume_range(vr_volume* vol, hipStream_t s);
int check_view(const vr_view* v, const int64_t n[3]);
int check_params(const vr_params* p);
int resolve_window(vr_ctx* ctx, vr_volume* vol, hipStream_t s, double& vmin, double& vmax);
void fill_march_common(MarchArgs& a, const vr_volume* vol, const vr_params* p, double vmin, double vmax,
                       const float4* tf, int32_t M);
// Macrocell skipping for a forward march: classifies the macrocells for the
// context's table and window when needed and fills a.mc* (a.mc = 0: off).
int prepare_macrocells(vr_ctx* ctx, vr_volume* vol, const vr_params* p, double vmin, double vmax, MarchArgs& a,
                       hipStream_t s);
// Tuned launch shape for a render (tile edge, LDS budget, march mode); defaults when untuned.
void tuned_shape(const vr_ctx* ctx, const vr_volume* vol, int32_t W, int32_t H, const vr_params* p, int32_t& tile,
                 int32_t& budget, int32_t& mode);
std::string tune_key(const vr_volume* vol, int32_t W, int32_t H, int32_t mode);
void tune_load(vr_ctx* ctx);
int render_batch(vr_ctx* ctx, const vr_request* reqs, int32_t n, const vr_params* p, vr_batch** cache, hipStream_t s,
                 int32_t force_blocks, const int32_t* tiles);
int check_batch(vr_ctx* ctx, const vr_request* reqs, int32_t n, const vr_params* p);
int plan_batch(vr_ctx* ctx, const vr_request* reqs, int32_t n, const vr_params* p, const int32_t* tiles,
               bool may_reduce, hipStream_t s, std::vector<BatchReq>& desc, int32_t& items, int32_t& maxM);
std::string batch_key(const vr_volume* v, int32_t W, int32_t H);
int32_t batch_tile(const vr_ctx* ctx, const vr_volume* v, int32_t W, int32_t H);
int batch_blocks(vr_ctx* ctx);
// Allocation-free batched path: look up the device's scratch address once
// (device current; called by vr_create), and return it (null before init).
int noalloc_init(int device);
void* noalloc_scratch(int device);

}  // namespace vr
