// render.hip -- forward ray-casting and over-composite kernels for gfx950.
//
// March (paper Sec. 2 and 2.4): one lane per pixel ray of a brick's
// rendering rectangle, wavefronts own TW x TH pixel tiles.  Each lane does
// the ray setup in double precision (whole-volume box test, lattice count,
// the brick's share [k0, k1) of the lattice), then marches its share in
// single precision with brick-local coordinates: trilinear reconstruction from
// four dword-pair loads, normalisation, a transfer-function lookup from LDS,
// front-to-back emission-absorption and the early-termination test.  The
// wavefront keeps issuing while any of its lanes is still marching.
//
// Composite (paper Sec. 2.5): one lane per output pixel walks the brick
// images front to back and applies the over operator where its pixel lies
// inside a brick's rectangle (the element-wise maximum for maximum intensity
// projection, which needs no order).
//
// Maximum intensity projection (paper Sec. 2.4): the march keeps the largest
// normalised sample value M of the ray and stops once M reaches 1; pixels are
// (M, M, M, M).
#include "sample.h"
#include "vr_internal.h"

namespace vr {

namespace {

typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));
typedef const float __attribute__((address_space(1))) gfloat;

// two adjacent voxels with one 8-byte global load (dword alignment suffices)
__device__ __forceinline__ f2u ld_pair(gfloat* p) {
  return *reinterpret_cast<const f2u __attribute__((address_space(1)))*>(p);
}

// Blocks of 256 lanes (4 wavefronts, 4 consecutive tiles).  Consecutive
// hardware block ids go round-robin over the 8 XCDs; remap them so each XCD
// receives one contiguous range of tiles (neighbouring tiles of the same brick
// then share that XCD's L2).
__device__ __forceinline__ int xcd_block(int nblk) {
  const int per = (nblk + 7) >> 3;
  return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

template <int TW, bool MIP, bool MASK>
__global__ __launch_bounds__(256) void k_march(MarchArgs a) {
  extern __shared__ float4 s_tf[];
  for (int i = threadIdx.x; i < a.M; i += 256) s_tf[i] = a.tf[i];
  __syncthreads();

  constexpr int TH = 64 / TW;
  const int nblk = (a.ntiles + 3) >> 2;
  const int lb = xcd_block(nblk);
  if (lb >= nblk) return;
  int tile = __builtin_amdgcn_readfirstlane(lb * 4 + (int)(threadIdx.x >> 6));
  if (tile >= a.ntiles) return;

  // brick owning this tile: last entry with tile_begin <= tile
  int lo = 0, hi = a.nbv - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (a.bv[mid].tile_begin <= tile) lo = mid;
    else hi = mid - 1;
  }
  const DevBrickView bvw = a.bv[lo];
  const DevBrick br = a.bricks[bvw.brick];
  const int t = tile - bvw.tile_begin;
  const int tx = t % bvw.tiles_x, ty = t / bvw.tiles_x;
  const int lane = threadIdx.x & 63;
  const int lx = tx * TW + (lane % TW), ly = ty * TH + (lane / TW);
  if (lx >= bvw.w || ly >= bvw.h) return;
  const int u = bvw.x0 + lx, v = bvw.y0 + ly;

  double o[3], d[3];
  pixel_ray(a.cam, u, v, o, d);
  float4* const dst = a.carry ? a.img + (int64_t)v * a.cam.W + u : a.img + bvw.img_off + (int64_t)ly * bvw.w + lx;
  float Cr = 0.f, Cg = 0.f, Cb = 0.f, T = 1.f, mx = 0.f;
  if (a.carry) {
    const float4 s0 = *dst;
    if (1.f - s0.w >= a.tau) return;  // the ray stopped in a brick in front
    Cr = s0.x;
    Cg = s0.y;
    Cb = s0.z;
    T = s0.w;
  }
  double tin;
  int64_t n;
  bool touched = false;  // the ray has samples in this brick
  if (ray_lattice(o, d, a.hi, a.step, tin, n)) {
    int64_t k0, k1;
    brick_krange(o, d, tin, a.step, n, br.lo, br.hi, br.closed, k0, k1);
    if (k1 > k0) {
      touched = true;
      const double t0 = tin + ((double)k0 + 0.5) * a.step;
      const float px = (float)(o[0] + t0 * d[0] - (double)br.lo[0]);
      const float py = (float)(o[1] + t0 * d[1] - (double)br.lo[1]);
      const float pz = (float)(o[2] + t0 * d[2] - (double)br.lo[2]);
      const float sx = (float)(a.step * d[0]), sy = (float)(a.step * d[1]), sz = (float)(a.step * d[2]);
      const int cnt = (int)(k1 - k0);
      gfloat* base = (gfloat*)br.base;
      const int ys = br.sy, zs = br.sz;
      for (int j = 0; j < cnt; ++j) {
        const Cell c = cell_of(sample_pos(j, px, py, pz, sx, sy, sz), br);
        gfloat* p = base + (c.iz * zs + c.iy * ys + c.ix);
        const f2u a00 = ld_pair(p), a01 = ld_pair(p + ys), a10 = ld_pair(p + zs), a11 = ld_pair(p + zs + ys);
        const float val = trilerp(a00.x, a00.y, a01.x, a01.y, a10.x, a10.y, a11.x, a11.y, c);
        if (MIP) {
          float s = norm_value(val, a.vmin, a.inv_range);
          if constexpr (MASK) s *= channel_weight(a.mask, a.mask_axis, br.lo[a.mask_axis], c);
          mx = fmaxf(mx, s);
          if (mx >= 1.f) break;
        } else {
          Classified k = classify(val, a.vmin, a.inv_range, a.M, s_tf);
          if constexpr (MASK) k.a *= channel_weight(a.mask, a.mask_axis, br.lo[a.mask_axis], c);
          accumulate(k, Cr, Cg, Cb, T);
          if (1.f - T >= a.tau) break;
        }
      }
    }
  }
  // carried state: only a ray with samples here owns its pixel in this wave
  // (another brick of the wave whose rectangle holds the pixel may update it)
  if (a.carry && !touched) return;
  *dst = MIP ? make_float4(mx, mx, mx, mx) : make_float4(Cr, Cg, Cb, a.carry ? T : 1.f - T);
}

// Carried state over the frame: (C, T) = (0, 1) before the first brick, and
// (C, 1 - T) once the last has been marched.
__global__ __launch_bounds__(256) void k_carry_init(float4* img, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) img[i] = make_float4(0.f, 0.f, 0.f, 1.f);
}
// Cleared pixels (brick images of footprint-cell marches).
__global__ __launch_bounds__(256) void k_zero(float4* img, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) img[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}
__global__ __launch_bounds__(256) void k_carry_final(float4* img, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const float4 s = img[i];
    img[i] = make_float4(s.x, s.y, s.z, 1.f - s.w);
  }
}

__global__ __launch_bounds__(256) void k_composite(CompArgs a) {
  const int x = blockIdx.x * 16 + (threadIdx.x & 15);
  const int y = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (x >= a.W || y >= a.H) return;
  float Cr = 0.f, Cg = 0.f, Cb = 0.f, A = 0.f;
  for (int i = 0; i < a.n; ++i) {
    const CompLayer L = a.layers[i];
    const unsigned lx = (unsigned)(x - L.x0), ly = (unsigned)(y - L.y0);
    if (lx < (unsigned)L.w && ly < (unsigned)L.h) {
      const float4 c = L.rgba[(int64_t)ly * L.w + lx];
      if (a.mip) {
        Cr = fmaxf(Cr, c.x);
        Cg = fmaxf(Cg, c.y);
        Cb = fmaxf(Cb, c.z);
        A = fmaxf(A, c.w);
      } else {
        const float t = 1.f - A;
        Cr = fmaf(t, c.x, Cr);
        Cg = fmaf(t, c.y, Cg);
        Cb = fmaf(t, c.z, Cb);
        A = fmaf(t, c.w, A);
      }
    }
  }
  a.out[(int64_t)y * a.W + x] = make_float4(Cr, Cg, Cb, A);
}

}  // namespace

hipError_t launch_carry(float4* img, int64_t n, bool final, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t grid = (n + 255) / 256;
  if (final) hipLaunchKernelGGL(k_carry_final, dim3((unsigned)grid), dim3(256), 0, s, img, n);
  else hipLaunchKernelGGL(k_carry_init, dim3((unsigned)grid), dim3(256), 0, s, img, n);
  return hipGetLastError();
}

hipError_t launch_zero(float4* img, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t grid = (n + 255) / 256;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)grid), dim3(256), 0, s, img, n);
  return hipGetLastError();
}

hipError_t launch_march(const MarchArgs& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  const int nblk = (a.ntiles + 3) / 4;
  const int grid = ((nblk + 7) / 8) * 8;
  const size_t lds = sizeof(float4) * (size_t)a.M;
#define VR_LAUNCH_GATHER(MIPV, MASKV)                                                                        \
  switch (a.tile_w) {                                                                                     \
    case 8: hipLaunchKernelGGL((k_march<8, MIPV, MASKV>), dim3(grid), dim3(256), lds, s, a); break;       \
    case 16: hipLaunchKernelGGL((k_march<16, MIPV, MASKV>), dim3(grid), dim3(256), lds, s, a); break;     \
    case 4: hipLaunchKernelGGL((k_march<4, MIPV, MASKV>), dim3(grid), dim3(256), lds, s, a); break;       \
    default: return hipErrorInvalidValue;                                                                 \
  }
  if (a.mask) {
    if (a.mip) VR_LAUNCH_GATHER(true, true)
    else VR_LAUNCH_GATHER(false, true)
  } else {
    if (a.mip) VR_LAUNCH_GATHER(true, false)
    else VR_LAUNCH_GATHER(false, false)
  }
#undef VR_LAUNCH_GATHER
  return hipGetLastError();
}

hipError_t launch_composite(const CompArgs& a, hipStream_t s) {
  dim3 grid((a.W + 15) / 16, (a.H + 15) / 16);
  hipLaunchKernelGGL(k_composite, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace vr
