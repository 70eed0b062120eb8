// volume.hip -- once-per-cube kernels: global (min, max) with a non-finite
// count (paper Sec. 2.2: each GPU reduces its portion, the results are
// combined into the global range), per-brick (min, max) over each brick's
// stored voxels, box copies (sub-cube upload, brick materialisation), and the
// macrocell (min, max) grid with its per-table classification used for
// empty-space skipping.
#include "vr_internal.h"

namespace vr {

namespace {

struct MinMaxPart {
  float mn, mx;
  uint32_t bad, pad;
};

__device__ __forceinline__ void acc(float v, float& mn, float& mx, uint32_t& bad) {
  if (!isfinite(v)) {
    bad++;
    return;
  }
  mn = fminf(mn, v);
  mx = fmaxf(mx, v);
}

__device__ __forceinline__ void block_reduce(float& mn, float& mx, uint32_t& bad) {
  for (int off = 32; off > 0; off >>= 1) {
    mn = fminf(mn, __shfl_xor(mn, off));
    mx = fmaxf(mx, __shfl_xor(mx, off));
    bad += __shfl_xor(bad, off);
  }
  __shared__ float smn[4], smx[4];
  __shared__ uint32_t sbad[4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    smn[w] = mn;
    smx[w] = mx;
    sbad[w] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); i++) {
      mn = fminf(mn, smn[i]);
      mx = fmaxf(mx, smx[i]);
      bad += sbad[i];
    }
  }
}

__global__ __launch_bounds__(256) void k_minmax(const float* __restrict__ x, int64_t n, MinMaxPart* part) {
  float mn = INFINITY, mx = -INFINITY;
  uint32_t bad = 0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  const bool al = ((uintptr_t)x & 15) == 0;
  if (al) {
    const int64_t n4 = n >> 2;
    const float4* x4 = reinterpret_cast<const float4*>(x);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
      const float4 v = x4[i];
      acc(v.x, mn, mx, bad);
      acc(v.y, mn, mx, bad);
      acc(v.z, mn, mx, bad);
      acc(v.w, mn, mx, bad);
    }
    for (int64_t i = (n4 << 2) + (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) acc(x[i], mn, mx, bad);
  } else {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) acc(x[i], mn, mx, bad);
  }
  block_reduce(mn, mx, bad);
  if (threadIdx.x == 0) part[blockIdx.x] = MinMaxPart{mn, mx, bad, 0};
}

__global__ __launch_bounds__(256) void k_minmax_final(const MinMaxPart* part, int nb, float* out3) {
  float mn = INFINITY, mx = -INFINITY;
  uint32_t bad = 0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    mn = fminf(mn, part[i].mn);
    mx = fmaxf(mx, part[i].mx);
    bad += part[i].bad;
  }
  block_reduce(mn, mx, bad);
  if (threadIdx.x == 0) {
    out3[0] = mn;
    out3[1] = mx;
    out3[2] = (float)bad;
  }
}

// One block per (brick, group of z-planes); partial (min, max) per block.
__global__ __launch_bounds__(256) void k_brick_minmax(const float* __restrict__ vol, int64_t n1, int64_t n2,
                                                      const int64_t* __restrict__ boxes, int zgroups,
                                                      int zper, float2* part) {
  const int b = blockIdx.x / zgroups, g = blockIdx.x % zgroups;
  const int64_t* bx = boxes + 6 * b;
  const int64_t x0 = bx[0], y0 = bx[1], z0 = bx[2], x1 = bx[3], y1 = bx[4], z1 = bx[5];
  const int64_t za = z0 + (int64_t)g * zper;
  const int64_t zb = min(z1, za + zper - 1);
  float mn = INFINITY, mx = -INFINITY;
  uint32_t bad = 0;
  const int64_t w = x1 - x0 + 1, h = y1 - y0 + 1;
  for (int64_t z = za; z <= zb; z++) {
    for (int64_t r = threadIdx.x / 64; r < h; r += 4) {
      const float* row = vol + (z * n2 + (y0 + r)) * n1 + x0;
      for (int64_t i = threadIdx.x & 63; i < w; i += 64) acc(row[i], mn, mx, bad);
    }
  }
  block_reduce(mn, mx, bad);
  if (threadIdx.x == 0) part[blockIdx.x] = make_float2(mn, mx);
}

__global__ void k_brick_minmax_final(const float2* part, int nb, int zgroups, float* out2) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  float mn = INFINITY, mx = -INFINITY;
  for (int g = 0; g < zgroups; g++) {
    const float2 p = part[b * zgroups + g];
    mn = fminf(mn, p.x);
    mx = fmaxf(mx, p.y);
  }
  out2[2 * b] = mn;
  out2[2 * b + 1] = mx;
}

// dst[z][y][x] = src[so3 + z][so2 + y][so1 + x] for the dst box dn.
__global__ __launch_bounds__(256) void k_copy_box(const float* __restrict__ src, int64_t s1, int64_t s2,
                                                  int64_t o1, int64_t o2, int64_t o3, float* __restrict__ dst,
                                                  int64_t d1, int64_t d2, int64_t d3) {
  const int64_t rows = d2 * d3;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const int64_t z = r / d2, y = r % d2;
    const float* srow = src + ((o3 + z) * s2 + (o2 + y)) * s1 + o1;
    float* drow = dst + r * d1;
    for (int64_t i = threadIdx.x; i < d1; i += 256) drow[i] = srow[i];
  }
}

// Macrocell (min, max).  A work unit is (run of `per` macrocells along axis 1,
// macrocell row m2, macrocell plane m3): its threads first reduce each voxel
// column x of the unit over the unit's (mc + 1)^2 rows (coalesced row reads)
// into LDS, then one thread per macrocell reduces its mc + 1 columns.
constexpr int kMcCols = 2049;  // per * mc + 1 with per = floor(2048 / mc)

__global__ __launch_bounds__(256) void k_mc_minmax(const float* __restrict__ vol, int64_t n1, int64_t n2, int64_t n3,
                                                   int mc, int per, int64_t c1, int64_t c2, int64_t c3,
                                                   float2* __restrict__ out) {
  __shared__ float s_mn[kMcCols], s_mx[kMcCols];
  const int64_t runs = (c1 + per - 1) / per;
  const int64_t units = runs * c2 * c3;
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const int64_t r = u % runs, m2 = (u / runs) % c2, m3 = u / (runs * c2);
    const int64_t m1 = r * per;
    const int64_t x0 = m1 * mc, x1 = min(x0 + (int64_t)per * mc, n1 - 1);
    const int64_t y0 = m2 * mc, y1 = min(y0 + mc, n2 - 1);
    const int64_t z0 = m3 * mc, z1 = min(z0 + mc, n3 - 1);
    const int ncol = (int)(x1 - x0 + 1);
    for (int c = threadIdx.x; c < ncol; c += 256) {
      float mn = INFINITY, mx = -INFINITY;
      bool bad = false;
      for (int64_t z = z0; z <= z1; z++) {
        const float* col = vol + (z * n2 + y0) * n1 + x0 + c;
#pragma unroll 4
        for (int64_t y = 0; y <= y1 - y0; y++) {
          const float v = col[y * n1];
          bad |= !isfinite(v);
          mn = fminf(mn, v);
          mx = fmaxf(mx, v);
        }
      }
      s_mn[c] = bad ? NAN : mn;
      s_mx[c] = mx;
    }
    __syncthreads();
    const int nm = (int)min((int64_t)per, c1 - m1);
    for (int m = threadIdx.x; m < nm; m += 256) {
      const int a = m * mc, b = min(a + mc, ncol - 1);
      float mn = INFINITY, mx = -INFINITY;
      bool bad = false;
      for (int c = a; c <= b; c++) {
        bad |= isnan(s_mn[c]);
        mn = fminf(mn, s_mn[c]);
        mx = fmaxf(mx, s_mx[c]);
      }
      out[(m3 * c2 + m2) * c1 + m1 + m] = make_float2(bad ? NAN : mn, mx);
    }
    __syncthreads();
  }
}

// Same rule as the host's brick test: entries floor(u(min)) - 1 .. ceil(u(max)) + 1
// (clamped to the table) must all have opacity 0; the one-entry margin covers
// the rounding of a single-precision trilinear value and table coordinate.
__global__ __launch_bounds__(256) void k_mc_classify(const float2* __restrict__ mm, int64_t count,
                                                     const int32_t* __restrict__ nz, int M, double vmin, double vmax,
                                                     uint8_t* __restrict__ clear, unsigned int* nclear) {
  unsigned int mine = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) {
    const float2 r = mm[i];
    uint8_t c = 0;
    if (isfinite(r.x) && isfinite(r.y)) {
      const double inv = vmax > vmin ? 1.0 / (vmax - vmin) : 0.0;
      const double s0 = fmin(1.0, fmax(0.0, ((double)r.x - vmin) * inv));
      const double s1 = fmin(1.0, fmax(0.0, ((double)r.y - vmin) * inv));
      const int64_t i0 = max((int64_t)0, (int64_t)floor(s0 * (double)(M - 1)) - 1);
      const int64_t i1 = min((int64_t)(M - 1), (int64_t)ceil(s1 * (double)(M - 1)) + 1);
      c = (nz[i1 + 1] - nz[i0]) == 0 ? 1 : 0;
    }
    clear[i] = c;
    mine += c;
  }
  for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(nclear, mine);
}

}  // namespace

hipError_t launch_minmax(const float* x, int64_t n, float* partial, int32_t nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_minmax, dim3(nblocks), dim3(256), 0, s, x, n, reinterpret_cast<MinMaxPart*>(partial));
  return hipGetLastError();
}

hipError_t launch_minmax_final(const float* partial, int32_t nblocks, float* out3, hipStream_t s) {
  hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(256), 0, s, reinterpret_cast<const MinMaxPart*>(partial),
                     nblocks, out3);
  return hipGetLastError();
}

// `boxes` is a device array of nb x (slo1, slo2, slo3, shi1, shi2, shi3);
// `out2` receives nb (min, max) pairs.  Uses out2-adjacent scratch: the
// partial buffer is allocated by the caller as `scratch` of nb*zgroups float2.
hipError_t launch_brick_minmax_parts(const float* vol, const int64_t n[3], const int64_t* boxes, int32_t nb,
                                     int zgroups, int zper, float* scratch, float* out2, hipStream_t s) {
  hipLaunchKernelGGL(k_brick_minmax, dim3(nb * zgroups), dim3(256), 0, s, vol, n[0], n[1], boxes, zgroups, zper,
                     reinterpret_cast<float2*>(scratch));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_brick_minmax_final, dim3((nb + 127) / 128), dim3(128), 0, s,
                     reinterpret_cast<const float2*>(scratch), nb, zgroups, out2);
  return hipGetLastError();
}

// Permuted copy for views along axis 1: dst[x][z][y] = src[z][y][x] (the
// copy's axes 1, 2, 3 are the source's axes 2, 3, 1).  32 x 32 tiles of each
// (y, x) plane go through LDS so that both the reads (rows along x) and the
// writes (rows along y) are whole 128-byte lines.
__global__ __launch_bounds__(256) void k_twin(const float* __restrict__ src, float* __restrict__ dst, int64_t n1,
                                              int64_t n2, int64_t n3) {
  __shared__ float tile[32][33];
  const int64_t ntx = (n1 + 31) / 32, nty = (n2 + 31) / 32, units = ntx * nty * n3;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const int64_t bx = u % ntx, by = (u / ntx) % nty, z = u / (ntx * nty);
    const int64_t x0 = bx * 32, y0 = by * 32;
    for (int r = ty; r < 32; r += 8) {
      const int64_t y = y0 + r, x = x0 + tx;
      if (y < n2 && x < n1) tile[r][tx] = src[(z * n2 + y) * n1 + x];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
      const int64_t x = x0 + r, y = y0 + tx;
      if (x < n1 && y < n2) dst[(x * n3 + z) * n2 + y] = tile[tx][r];
    }
    __syncthreads();
  }
}

hipError_t launch_twin(const float* src, const int64_t n[3], float* dst, hipStream_t s) {
  const int64_t units = ((n[0] + 31) / 32) * ((n[1] + 31) / 32) * n[2];
  const int grid = (int)(units < (1 << 20) ? units : (1 << 20));
  hipLaunchKernelGGL(k_twin, dim3(grid), dim3(256), 0, s, src, dst, n[0], n[1], n[2]);
  return hipGetLastError();
}

hipError_t launch_copy_box(const float* src, const int64_t sn[3], const int64_t so[3], float* dst,
                           const int64_t dn[3], hipStream_t s) {
  const int64_t rows = dn[1] * dn[2];
  const int grid = (int)(rows < 65536 ? rows : 65536);
  hipLaunchKernelGGL(k_copy_box, dim3(grid), dim3(256), 0, s, src, sn[0], sn[1], so[0], so[1], so[2], dst, dn[0],
                     dn[1], dn[2]);
  return hipGetLastError();
}

hipError_t launch_mc_minmax(const float* vol, const int64_t n[3], int mc, const int64_t c[3], float* out2,
                            hipStream_t s) {
  if (mc < 2 || mc > 1024) return hipErrorInvalidValue;
  const int per = 2048 / mc;
  const int64_t units = ((c[0] + per - 1) / per) * c[1] * c[2];
  const int grid = (int)(units < 65536 ? units : 65536);
  hipLaunchKernelGGL(k_mc_minmax, dim3(grid), dim3(256), 0, s, vol, n[0], n[1], n[2], mc, per, c[0], c[1], c[2],
                     reinterpret_cast<float2*>(out2));
  return hipGetLastError();
}

hipError_t launch_mc_classify(const float* mm2, int64_t count, const int32_t* nz, int M, double vmin, double vmax,
                              uint8_t* clear, unsigned int* nclear, hipStream_t s) {
  hipError_t e = hipMemsetAsync(nclear, 0, sizeof(unsigned int), s);
  if (e != hipSuccess) return e;
  const int64_t blocks = (count + 255) / 256;
  const int grid = (int)(blocks < 16384 ? blocks : 16384);
  hipLaunchKernelGGL(k_mc_classify, dim3(grid), dim3(256), 0, s, reinterpret_cast<const float2*>(mm2), count, nz, M,
                     vmin, vmax, clear, nclear);
  return hipGetLastError();
}

}  // namespace vr
