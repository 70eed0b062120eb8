// grad.hip -- differentiable rendering kernels (gfx950): a forward march that
// saves transmittance checkpoints, the adjoint march, and the reduction of
// the per-workgroup transfer-function gradients.
//
// Forward with checkpoints: the whole-volume march of render.hip, storing T
// before samples 0, K, 2K, ... and the number of samples applied (early
// termination freezes it).
//
// Adjoint, per ray, for L = sum(g . (C_r, C_g, C_b, A)):
//   dL/dc_k = g_rgb T_{k-1} a_k
//   dL/da_k = T_{k-1} [ g_rgb . (c_k - R_k) + g_A (1 - Q_k) ]
//   R_{k-1} = a_k c_k + (1 - a_k) R_k,  Q_{k-1} = a_k + (1 - a_k) Q_k,  R_n = Q_n = 0
// walked from the last sample to the first without any division.  Segments of
// K samples are visited last to first; each is first replayed forward from
// its checkpoint to put T_{k-1} for its samples in LDS, then walked backward.
// The adjoint evaluates samples, the recursion and the gradient algebra in
// double precision (MI355X runs FP64 vector code at half the FP32 rate).
// Table gradients go to double LDS accumulators (one set per workgroup,
// flushed to a partial buffer and reduced by k_tf_reduce); voxel gradients are
// scattered to the eight trilinear corners with hardware float atomics.
#include "sample.h"
#include "vr_internal.h"

namespace vr {

namespace {

typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));
typedef const float __attribute__((address_space(1))) gfloat;

constexpr int kSub = 32;  // transmittances kept in LDS per lane during a backward walk

__device__ __forceinline__ f2u ld_pair(gfloat* p) {
  return *reinterpret_cast<const f2u __attribute__((address_space(1)))*>(p);
}

struct TileLane {
  int tile, u, v;
  bool active;
};

// Same tile mapping as the forward march: 4 tiles per 256-lane block,
// XCD-contiguous block ranges.
__device__ __forceinline__ TileLane tile_lane(const MarchArgs& a) {
  TileLane t;
  const int nblk = (a.ntiles + 3) >> 2;
  const int per = (nblk + 7) >> 3;
  const int lb = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  t.tile = lb * 4 + (int)(threadIdx.x >> 6);
  t.active = lb < nblk && t.tile < a.ntiles;
  const DevBrickView& bv = a.bv[0];
  const int tile = t.active ? t.tile : 0;
  const int TW = a.tile_w, TH = a.tile_h;
  const int tx = tile % bv.tiles_x, ty = tile / bv.tiles_x;
  const int lane = threadIdx.x & 63;
  const int lx = tx * TW + (lane % TW), ly = ty * TH + (lane / TW);
  t.active = t.active && lx < bv.w && ly < bv.h;
  t.u = lx;
  t.v = ly;
  return t;
}

__global__ __launch_bounds__(256) void k_fwd_save(MarchArgs a, SaveArgs sa) {
  extern __shared__ float4 s_tf[];
  for (int i = threadIdx.x; i < a.M; i += 256) s_tf[i] = a.tf[i];
  __syncthreads();
  const TileLane tl = tile_lane(a);
  if (!tl.active) return;
  const DevBrick br = a.bricks[0];
  const int pix = tl.v * a.bv[0].w + tl.u;
  double o[3], d[3];
  pixel_ray(a.cam, tl.u, tl.v, o, d);
  float Cr = 0.f, Cg = 0.f, Cb = 0.f, T = 1.f;
  int used = 0;
  double tin;
  int64_t n;
  if (ray_lattice(o, d, a.hi, a.step, tin, n)) {
    const float px = (float)(o[0] + (tin + 0.5 * a.step) * d[0]);
    const float py = (float)(o[1] + (tin + 0.5 * a.step) * d[1]);
    const float pz = (float)(o[2] + (tin + 0.5 * a.step) * d[2]);
    const float sx = (float)(a.step * d[0]), sy = (float)(a.step * d[1]), sz = (float)(a.step * d[2]);
    const int cnt = (int)n;
    gfloat* base = (gfloat*)br.base;
    const int ys = br.sy, zs = br.sz;
    int kc = 0, seg = 0;
    for (int j = 0; j < cnt; ++j) {
      if (kc == 0) {
        sa.ckpt[(int64_t)seg * sa.npix + pix] = T;
        seg++;
        kc = sa.K;
      }
      kc--;
      const Cell c = cell_of(sample_pos(j, px, py, pz, sx, sy, sz), br);
      gfloat* p = base + (c.iz * zs + c.iy * ys + c.ix);
      const f2u a00 = ld_pair(p), a01 = ld_pair(p + ys), a10 = ld_pair(p + zs), a11 = ld_pair(p + zs + ys);
      const float val = trilerp(a00.x, a00.y, a01.x, a01.y, a10.x, a10.y, a11.x, a11.y, c);
      accumulate(classify(val, a.vmin, a.inv_range, a.M, s_tf), Cr, Cg, Cb, T);
      used = j + 1;
      if (1.f - T >= a.tau) break;
    }
  }
  sa.nused[pix] = used;
  a.img[a.bv[0].img_off + pix] = make_float4(Cr, Cg, Cb, 1.f - T);
}

// One sample evaluated in double precision for the adjoint: position, clamped
// base cell, trilinear weights, value and table lookup.  (The forward's FP32
// rounding is not replayed: the adjoint differentiates the exact definition.)
struct SampleD {
  int off;              // base-corner offset in the volume
  double wx, wy, wz;    // fractions
  double r, g, b, a;    // table colour and opacity
  int i;                // table interval
  double w;             // table weight
  double sraw;          // unclamped normalised value
};

__device__ __forceinline__ SampleD sample_d(int k, const double p0[3], const double sv[3], const DevBrick& br,
                                            gfloat* base, double vmin, double inv_range, int M, const float4* s_tf) {
  SampleD S;
  const double kk = (double)k;
  const double qx = fma(kk, sv[0], p0[0]), qy = fma(kk, sv[1], p0[1]), qz = fma(kk, sv[2], p0[2]);
  const int ix = min(max((int)floor(qx), br.clo[0]), br.chi[0]);
  const int iy = min(max((int)floor(qy), br.clo[1]), br.chi[1]);
  const int iz = min(max((int)floor(qz), br.clo[2]), br.chi[2]);
  S.wx = qx - (double)ix;
  S.wy = qy - (double)iy;
  S.wz = qz - (double)iz;
  S.off = iz * br.sz + iy * br.sy + ix;
  gfloat* p = base + S.off;
  const int ys = br.sy, zs = br.sz;
  const f2u a00 = ld_pair(p), a01 = ld_pair(p + ys), a10 = ld_pair(p + zs), a11 = ld_pair(p + zs + ys);
  const double c00 = fma(S.wx, (double)a00.y - (double)a00.x, (double)a00.x);
  const double c01 = fma(S.wx, (double)a01.y - (double)a01.x, (double)a01.x);
  const double c10 = fma(S.wx, (double)a10.y - (double)a10.x, (double)a10.x);
  const double c11 = fma(S.wx, (double)a11.y - (double)a11.x, (double)a11.x);
  const double c0 = fma(S.wy, c01 - c00, c00), c1 = fma(S.wy, c11 - c10, c10);
  const double val = fma(S.wz, c1 - c0, c0);
  S.sraw = (val - vmin) * inv_range;
  const double s = fmin(fmax(S.sraw, 0.0), 1.0);
  const double u = s * (double)(M - 1);
  S.i = min((int)u, M - 2);
  S.w = u - (double)S.i;
  const float4 e0 = s_tf[S.i], e1 = s_tf[S.i + 1];
  S.r = fma(S.w, (double)e1.x - (double)e0.x, (double)e0.x);
  S.g = fma(S.w, (double)e1.y - (double)e0.y, (double)e0.y);
  S.b = fma(S.w, (double)e1.z - (double)e0.z, (double)e0.z);
  S.a = fma(S.w, (double)e1.w - (double)e0.w, (double)e0.w);
  return S;
}

__global__ __launch_bounds__(256) void k_bwd(MarchArgs a, BwdArgs ba) {
  extern __shared__ double dsm[];
  double* s_gtf = dsm;                                                     // [M][4] double
  float4* s_tf = reinterpret_cast<float4*>(dsm + 4 * a.M);                 // [M]
  float* s_T = reinterpret_cast<float*>(s_tf + a.M);                       // [kSub][256]
  for (int i = threadIdx.x; i < a.M; i += 256) {
    s_tf[i] = a.tf[i];
    s_gtf[4 * i] = s_gtf[4 * i + 1] = s_gtf[4 * i + 2] = s_gtf[4 * i + 3] = 0.0;
  }
  __syncthreads();
  const TileLane tl = tile_lane(a);
  const int tid = threadIdx.x;
  if (tl.active) {
    const DevBrick br = a.bricks[0];
    const int pix = tl.v * a.bv[0].w + tl.u;
    const int used = ba.nused[pix];
    double o[3], d[3];
    pixel_ray(a.cam, tl.u, tl.v, o, d);
    double tin;
    int64_t n;
    if (used > 0 && ray_lattice(o, d, a.hi, a.step, tin, n)) {
      const float4 gf = ba.gout[pix];
      const double gx = gf.x, gy = gf.y, gz = gf.z, gw = gf.w;
      const double t0 = tin + 0.5 * a.step;
      const double p0[3] = {o[0] + t0 * d[0], o[1] + t0 * d[1], o[2] + t0 * d[2]};
      const double sv[3] = {a.step * d[0], a.step * d[1], a.step * d[2]};
      gfloat* base = (gfloat*)br.base;
      const int ys = br.sy, zs = br.sz;
      const double dvs = (double)(a.M - 1) * ba.inv_range;  // du/dv inside the window
      double R0 = 0.0, R1 = 0.0, R2 = 0.0, Q = 0.0;
      const int K = ba.K;
      for (int seg = (used - 1) / K; seg >= 0; --seg) {
        const int kb = seg * K, ke = min(used, kb + K);
        // LDS holds T for at most kSub samples: a longer segment is walked in
        // sub-segments, last to first, each replayed from the segment's checkpoint
        for (int sub = (ke - kb - 1) / kSub; sub >= 0; --sub) {
        const int sb = kb + sub * kSub, se = min(ke, sb + kSub);
        double T = (double)ba.ckpt[(int64_t)seg * ba.npix + pix];
        for (int k = kb; k < sb; ++k) T = fma(-T, sample_d(k, p0, sv, br, base, ba.vmin, ba.inv_range, a.M, s_tf).a, T);
        for (int k = sb; k < se; ++k) {
          const SampleD S = sample_d(k, p0, sv, br, base, ba.vmin, ba.inv_range, a.M, s_tf);
          s_T[(k - sb) * 256 + tid] = (float)T;
          T = fma(-T, S.a, T);
        }
        // walk the sub-segment backward
        for (int k = se - 1; k >= sb; --k) {
          const SampleD S = sample_d(k, p0, sv, br, base, ba.vmin, ba.inv_range, a.M, s_tf);
          const double Tp = (double)s_T[(k - sb) * 256 + tid];
          const double ta = Tp * S.a;
          const double gr = gx * ta, gg = gy * ta, gb = gz * ta;
          const double ga = Tp * (gx * (S.r - R0) + gy * (S.g - R1) + gz * (S.b - R2) + gw * (1.0 - Q));
          const double om = 1.0 - S.a;
          R0 = fma(S.a, S.r, om * R0);
          R1 = fma(S.a, S.g, om * R1);
          R2 = fma(S.a, S.b, om * R2);
          Q = fma(om, Q, S.a);
          const double w1 = S.w, w0 = 1.0 - S.w;
          double* e0 = s_gtf + 4 * S.i;
          atomicAdd(e0 + 0, w0 * gr);
          atomicAdd(e0 + 1, w0 * gg);
          atomicAdd(e0 + 2, w0 * gb);
          atomicAdd(e0 + 3, w0 * ga);
          atomicAdd(e0 + 4, w1 * gr);
          atomicAdd(e0 + 5, w1 * gg);
          atomicAdd(e0 + 6, w1 * gb);
          atomicAdd(e0 + 7, w1 * ga);
          if (ba.gvol && S.sraw > 0.0 && S.sraw < 1.0) {
            const float4 t0f = s_tf[S.i], t1f = s_tf[S.i + 1];
            const double du = gr * ((double)t1f.x - (double)t0f.x) + gg * ((double)t1f.y - (double)t0f.y) +
                              gb * ((double)t1f.z - (double)t0f.z) + ga * ((double)t1f.w - (double)t0f.w);
            const double gv = du * dvs;
            if (gv != 0.0) {
              const double x1 = S.wx, x0 = 1.0 - S.wx, y1 = S.wy, y0 = 1.0 - S.wy, z1 = S.wz, z0 = 1.0 - S.wz;
              float* q = ba.gvol + S.off;
              unsafeAtomicAdd(q, (float)(gv * x0 * y0 * z0));
              unsafeAtomicAdd(q + 1, (float)(gv * x1 * y0 * z0));
              unsafeAtomicAdd(q + ys, (float)(gv * x0 * y1 * z0));
              unsafeAtomicAdd(q + ys + 1, (float)(gv * x1 * y1 * z0));
              unsafeAtomicAdd(q + zs, (float)(gv * x0 * y0 * z1));
              unsafeAtomicAdd(q + zs + 1, (float)(gv * x1 * y0 * z1));
              unsafeAtomicAdd(q + zs + ys, (float)(gv * x0 * y1 * z1));
              unsafeAtomicAdd(q + zs + ys + 1, (float)(gv * x1 * y1 * z1));
            }
          }
        }
        }
      }
    }
  }
  __syncthreads();
  double* part = ba.tf_part + (int64_t)blockIdx.x * a.M * 4;
  for (int i = threadIdx.x; i < a.M * 4; i += 256) part[i] = s_gtf[i];
}

// grad_tf[e] (+)= sum over blocks of the partials, accumulated in double, in
// two passes with a fixed order (the same bits on every run): slice s sums
// blocks s, s + kSlices, ...; then each entry sums its slices in order.
constexpr int kSlices = 64;

__global__ __launch_bounds__(256) void k_tf_slices(const double* part, int nblocks, int n, double* sl) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  double acc = 0.0;
  for (int b = (int)blockIdx.y; b < nblocks; b += kSlices) acc += part[(int64_t)b * n + e];
  sl[(int64_t)blockIdx.y * n + e] = acc;
}

__global__ __launch_bounds__(256) void k_tf_reduce(const double* sl, int n, float* grad_tf) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  double acc = 0.0;
  for (int s = 0; s < kSlices; s++) acc += sl[(int64_t)s * n + e];
  grad_tf[e] = (float)((double)grad_tf[e] + acc);
}

__global__ __launch_bounds__(256) void k_fill(float* p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

}  // namespace

static int march_grid(const MarchArgs& a) {
  const int nblk = (a.ntiles + 3) / 4;
  return ((nblk + 7) / 8) * 8;
}

hipError_t launch_fwd_save(const MarchArgs& a, const SaveArgs& sa, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fwd_save, dim3(march_grid(a)), dim3(256), sizeof(float4) * (size_t)a.M, s, a, sa);
  return hipGetLastError();
}

int bwd_blocks(const MarchArgs& a) { return a.ntiles <= 0 ? 0 : march_grid(a); }

hipError_t launch_bwd(const MarchArgs& a, const BwdArgs& ba, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  const size_t lds = sizeof(double) * 4 * (size_t)a.M + sizeof(float4) * (size_t)a.M + sizeof(float) * 256 * kSub;
  hipLaunchKernelGGL(k_bwd, dim3(march_grid(a)), dim3(256), lds, s, a, ba);
  return hipGetLastError();
}

int tf_reduce_slices() { return kSlices; }

hipError_t launch_tf_reduce(const double* part, int nblocks, int n, float* grad_tf, double* slices, hipStream_t s) {
  hipLaunchKernelGGL(k_tf_slices, dim3((n + 255) / 256, kSlices), dim3(256), 0, s, part, nblocks, n, slices);
  hipLaunchKernelGGL(k_tf_reduce, dim3((n + 255) / 256), dim3(256), 0, s, slices, n, grad_tf);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t want = (n + 255) / 256;
  const int grid = (int)(want < 65536 ? want : 65536);
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace vr
