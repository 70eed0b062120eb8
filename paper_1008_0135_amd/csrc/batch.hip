// batch.hip -- batched rendering of many independent requests in one
// persistent launch (gfx950).
//
// Each request is a whole (unbricked) volume with its own view, transfer
// function, window and output image.  Work items are (request, pixel tile)
// pairs numbered in the host's order (requests with the most samples per tile
// first, so the longest items start first); a request's tile is 64 pixels,
// 4 x 16, 8 x 8, 16 x 4 or 32 x 2, as the autotuner chose for its size
// class.  A grid sized to the device pulls items from one atomic counter, one
// item per wavefront per
// pull, until the queue is empty: every wavefront reaches the exit test after
// each item, so the grid drains by itself.  A wavefront keeps the table of
// the request it is working on in its own LDS slot and reloads it only when
// the next item belongs to another request.  The per-sample arithmetic is the
// one of every other march (sample.h).
#include <mutex>

#include "runtime.h"
#include "sample.h"
#include "vr_internal.h"

namespace vr {

// Device scratch of the allocation-free batched entry point
// (vr_render_batch_noalloc): the descriptor table of at most
// kNoAllocMaxReq requests, then the work counter.  Each device holds its own
// copy for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress returns for that device.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(VR_EUNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return VR_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(VR_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device, hipGetErrorString(e));
  }
  g_scratch_ptr[device] = p;
  return VR_OK;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

namespace {

typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));
typedef const float __attribute__((address_space(1))) gfloat;

__device__ __forceinline__ f2u ld_pair(gfloat* p) {
  return *reinterpret_cast<const f2u __attribute__((address_space(1)))*>(p);
}

__global__ void k_batch_reset(unsigned int* counter) { *counter = 0u; }

__global__ __launch_bounds__(256) void k_batch(BatchArgs ba) {
  extern __shared__ float4 smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float4* s_tf = smem + (size_t)wave * ba.max_M;
  int cur = -1;  // request whose table sits in this wavefront's slot
  for (;;) {
    unsigned int item = 0;
    if (lane == 0) item = atomicAdd(ba.counter, 1u);
    item = __builtin_amdgcn_readfirstlane(item);
    if (item >= (unsigned)ba.total_items) break;
    // request owning the item: last with item_begin <= item
    int lo = 0, hi = ba.nreq - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ba.reqs[mid].item_begin <= (int)item) lo = mid;
      else hi = mid - 1;
    }
    const BatchReq& rq = ba.reqs[lo];
    if (lo != cur) {
      for (int i = lane; i < rq.M; i += 64) s_tf[i] = rq.tf[i];
      cur = lo;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    const int t = (int)item - rq.item_begin;
    const int tx = t % rq.tiles_x, ty = t / rq.tiles_x;
    const int sh = rq.tile_shift;
    const int u = (tx << sh) + (lane & ((1 << sh) - 1)), v = ty * (64 >> sh) + (lane >> sh);
    if (u < rq.cam.W && v < rq.cam.H) {
      double o[3], d[3];
      pixel_ray(rq.cam, u, v, o, d);
      float Cr = 0.f, Cg = 0.f, Cb = 0.f, T = 1.f;
      double tin;
      int64_t n;
      if (ray_lattice(o, d, rq.hi, ba.step, tin, n)) {
        const float px = (float)(o[0] + (tin + 0.5 * ba.step) * d[0]);
        const float py = (float)(o[1] + (tin + 0.5 * ba.step) * d[1]);
        const float pz = (float)(o[2] + (tin + 0.5 * ba.step) * d[2]);
        const float sx = (float)(ba.step * d[0]), sy = (float)(ba.step * d[1]), sz = (float)(ba.step * d[2]);
        const int cnt = (int)n;
        const DevBrick& br = rq.br;
        gfloat* base = (gfloat*)br.base;
        const int ys = br.sy, zs = br.sz;
        for (int j = 0; j < cnt; ++j) {
          const Cell c = cell_of(sample_pos(j, px, py, pz, sx, sy, sz), br);
          gfloat* p = base + (c.iz * zs + c.iy * ys + c.ix);
          const f2u a00 = ld_pair(p), a01 = ld_pair(p + ys), a10 = ld_pair(p + zs), a11 = ld_pair(p + zs + ys);
          const float val = trilerp(a00.x, a00.y, a01.x, a01.y, a10.x, a10.y, a11.x, a11.y, c);
          accumulate(classify(val, rq.vmin, rq.inv_range, rq.M, s_tf), Cr, Cg, Cb, T);
          if (1.f - T >= ba.tau) break;
        }
      }
      rq.out[(int64_t)v * rq.cam.W + u] = make_float4(Cr, Cg, Cb, 1.f - T);
    }
  }
}

}  // namespace

hipError_t launch_batch(const BatchArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, a.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = sizeof(float4) * (size_t)a.max_M * 4;
  hipLaunchKernelGGL(k_batch, dim3(blocks), dim3(256), lds, s, a);
  return hipGetLastError();
}

}  // namespace vr
