// march_lds.hip -- forward march with LDS-staged slabs (gfx950).
//
// Same samples, same arithmetic and the same order as the gather march in
// render.hip (paper Sec. 2.4: each ray is sampled between its entry and exit
// points and accumulated front to back with early termination); only the
// way voxels reach the lanes differs.  One wavefront owns a TW x TH tile of
// pixel rays inside one brick and walks the brick in slabs of T cell layers
// along a slab axis b (y or z, chosen per view on the host so that rows
// along x -- the contiguous storage axis -- stay long).  For each slab the
// wavefront
//   1. bounds the footprint of its ray bundle in the slab from the four
//      corner rays of the tile (8 plane intersections, a wave reduction),
//   2. copies that box of voxels from HBM into LDS with row-contiguous
//      16-byte loads (each voxel fetched once per slab, coalesced),
//   3. lets every lane consume its own samples whose cell layer along b lies
//      in the slab, reading the eight trilinear corners from LDS.
// Lanes carry their colour, transmittance and sample cursor from slab to
// slab, so the per-ray result is the sequential front-to-back chain.  A
// wavefront stops when all of its lanes have finished or terminated early.
#include "sample.h"
#include "vr_internal.h"

namespace vr {

namespace {

typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef const float __attribute__((address_space(1))) gfloat;

__device__ __forceinline__ float wave_min(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ int wave_imin(int v) {
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ int wave_imax(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float unif(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

template <int TW>
__global__ __launch_bounds__(64) void k_march_lds(MarchArgs a) {
  extern __shared__ float4 smem[];
  float4* s_tf = smem;
  float* s_reg = reinterpret_cast<float*>(smem + a.M);
  const int lane = threadIdx.x;
  for (int i = lane; i < a.M; i += 64) s_tf[i] = a.tf[i];
  __syncthreads();

  constexpr int TH = 64 / TW;
  const int nblk = a.ntiles;
  const int per = (nblk + 7) >> 3;
  const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (tile >= nblk) return;  // whole wavefront

  int lo = 0, hi = a.nbv - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.bv[mid].tile_begin <= tile) lo = mid;
    else hi = mid - 1;
  }
  const DevBrickView bvw = a.bv[lo];
  const DevBrick br = a.bricks[bvw.brick];
  const int t = tile - bvw.tile_begin;
  const int tx = t % bvw.tiles_x, ty = t / bvw.tiles_x;
  const int lx = tx * TW + (lane % TW), ly = ty * TH + (lane / TW);
  const bool valid = lx < bvw.w && ly < bvw.h;
  const int u = bvw.x0 + min(lx, bvw.w - 1), v = bvw.y0 + min(ly, bvw.h - 1);

  // ---- per-lane ray setup (double precision, shared with the gather march)
  const double* d = a.cam.e3;
  double o[3];
  pixel_origin(a.cam, u, v, o);
  int cnt = 0;
  float px = 0.f, py = 0.f, pz = 0.f;
  double tin;
  int64_t n;
  if (valid && ray_lattice(o, d, a.hi, a.step, tin, n)) {
    int64_t k0, k1;
    brick_krange(o, d, tin, a.step, n, br.lo, br.hi, br.closed, k0, k1);
    if (k1 > k0) {
      const double t0 = tin + ((double)k0 + 0.5) * a.step;
      px = (float)(o[0] + t0 * d[0] - (double)br.lo[0]);
      py = (float)(o[1] + t0 * d[1] - (double)br.lo[1]);
      pz = (float)(o[2] + t0 * d[2] - (double)br.lo[2]);
      cnt = (int)(k1 - k0);
    }
  }
  const float sx = (float)(a.step * d[0]), sy = (float)(a.step * d[1]), sz = (float)(a.step * d[2]);

  // ---- slab frame: b = slab axis (1 or 2), g = the other of axes 2/3, f = axis 1
  const int b = a.slab_axis;
  const bool by = b == 1;  // slab axis is axis 2 (else axis 3)
  const float pb = by ? py : pz, sb = by ? sy : sz;
  const int cloB = by ? br.clo[1] : br.clo[2], chiB = by ? br.chi[1] : br.chi[2];
  const int cloG = by ? br.clo[2] : br.clo[1], chiG = by ? br.chi[2] : br.chi[1];
  const double db = by ? d[1] : d[2], dg = by ? d[2] : d[1];
  const bool up = db > 0.0;

  // first and last cell layer (along b) of the lane's samples
  int c_first = up ? 0x7fffffff : -0x7fffffff, c_last = up ? -0x7fffffff : 0x7fffffff;
  if (cnt > 0) {
    c_first = min(max((int)floorf(pb), cloB), chiB);
    c_last = min(max((int)floorf(fmaf((float)(cnt - 1), sb, pb)), cloB), chiB);
  }
  int Lbeg, Lend;  // cell layers visited, in marching order
  if (up) {
    Lbeg = uni(wave_imin(c_first));
    Lend = uni(wave_imax(c_last));
  } else {
    Lbeg = uni(wave_imax(c_first));
    Lend = uni(wave_imin(c_last));
  }
  if (up ? Lbeg > Lend : Lbeg < Lend) {
    if (valid) a.img[bvw.img_off + (int64_t)ly * bvw.w + lx] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }

  // corner rays of the tile (lanes 0..7: corner lane&3 at the near/far plane)
  const int cx = bvw.x0 + tx * TW, cy = bvw.y0 + ty * TH;
  const int ex = min(cx + TW - 1, bvw.x0 + bvw.w - 1), ey = min(cy + TH - 1, bvw.y0 + bvw.h - 1);
  const int cc = lane & 3;
  double oc[3];
  pixel_origin(a.cam, (cc & 1) ? ex : cx, (cc & 2) ? ey : cy, oc);
  const float ocb = (float)((by ? oc[1] : oc[2]) - (double)(by ? br.lo[1] : br.lo[2]));
  const float ocf = (float)(oc[0] - (double)br.lo[0]);
  const float ocg = (float)((by ? oc[2] : oc[1]) - (double)(by ? br.lo[2] : br.lo[1]));
  const float rf = (float)(d[0] / db), rg = (float)(dg / db);

  const int ysl = br.sy, zsl = br.sz;
  const int strideB = by ? ysl : zsl, strideG = by ? zsl : ysl;
  gfloat* gbase = (gfloat*)br.base;

  float Cr = 0.f, Cg = 0.f, Cb = 0.f, T = 1.f;
  int j = 0;
  bool done = cnt == 0;
  const int step_l = up ? a.slab_T : -a.slab_T;

  for (int L = Lbeg;; L += step_l) {
    const int cl = up ? L : max(L - a.slab_T + 1, Lend);
    const int ch = up ? min(L + a.slab_T - 1, Lend) : L;
    // ---- footprint of the bundle over cell layers [cl, ch] (planes cl and ch+1)
    float fmn = INFINITY, fmx = -INFINITY, gmn = INFINITY, gmx = -INFINITY;
    if (lane < 8) {
      const float P = lane < 4 ? (float)cl : (float)(ch + 1);
      const float tt = P - ocb;
      const float qf = fmaf(tt, rf, ocf), qg = fmaf(tt, rg, ocg);
      fmn = fmx = qf;
      gmn = gmx = qg;
    }
    fmn = wave_min(fmn);
    fmx = wave_max(fmx);
    gmn = wave_min(gmn);
    gmx = wave_max(gmx);
    // cells floor(q) and floor(q) + 1 of every sample q in the footprint (+-0.05 voxel)
    const int f_lo = uni(max((int)floorf(unif(fmn) - 0.05f), br.clo[0]));
    const int f_hi = uni(min((int)floorf(unif(fmx) + 0.05f) + 1, br.chi[0] + 1));
    const int g_lo = uni(max((int)floorf(unif(gmn) - 0.05f), cloG));
    const int g_hi = uni(min((int)floorf(unif(gmx) + 0.05f) + 1, chiG + 1));
    const int b_lo = cl, b_hi = ch + 1;
    const int nf = f_hi - f_lo + 1, ng = g_hi - g_lo + 1, nl = b_hi - b_lo + 1;
    const int pitch = (nf + 3) & ~3;
    const int layer = pitch * ng;
    const bool staged = nf > 0 && ng > 0 && layer * nl <= a.lds_budget;

    if (staged) {
      // ---- copy the box into LDS: rows along f, 16-byte chunks
      const int nf4 = pitch >> 2;
      const int rows = ng * nl;
      const int chunks = rows * nf4;
      const float inv_nf4 = 1.0f / (float)nf4, inv_ng = 1.0f / (float)ng;
      for (int i = lane; i < chunks; i += 64) {
        const int row = (int)(((float)i + 0.5f) * inv_nf4);
        const int c4 = i - row * nf4;
        const int lb = (int)(((float)row + 0.5f) * inv_ng);
        const int lg = row - lb * ng;
        const int f0 = 4 * c4;
        gfloat* src = gbase + ((b_lo + lb) * strideB + (g_lo + lg) * strideG + (f_lo + f0));
        float* dst = s_reg + row * pitch + f0;
        if (f0 + 3 < nf) {
          const f4u q = *reinterpret_cast<const f4u __attribute__((address_space(1)))*>(src);
          *reinterpret_cast<float4*>(dst) = make_float4(q.x, q.y, q.z, q.w);
        } else {
          for (int e = 0; e < nf - f0; e++) dst[e] = src[e];
        }
      }
      __syncthreads();
    }
    // ---- consume the lane's samples whose cell layer along b is in [cl, ch]
    const int Sy = by ? layer : pitch, Sz = by ? pitch : layer;
    const int oy = by ? b_lo : g_lo, oz = by ? g_lo : b_lo;
    const int omax = layer * nl - 1 - (Sy + Sz + 1);
    while (!done) {
      const Cell c = cell_of(sample_pos(j, px, py, pz, sx, sy, sz), br);
      const int ib = by ? c.iy : c.iz;
      if (up ? ib > ch : ib < cl) break;
      float v000, v001, v010, v011, v100, v101, v110, v111;
      if (staged) {
        int oo = (c.ix - f_lo) + (c.iy - oy) * Sy + (c.iz - oz) * Sz;
        oo = min(max(oo, 0), omax);
        const float* p = s_reg + oo;
        v000 = p[0];
        v001 = p[1];
        v010 = p[Sy];
        v011 = p[Sy + 1];
        v100 = p[Sz];
        v101 = p[Sz + 1];
        v110 = p[Sz + Sy];
        v111 = p[Sz + Sy + 1];
      } else {
        gfloat* p = gbase + (c.iz * zsl + c.iy * ysl + c.ix);
        v000 = p[0];
        v001 = p[1];
        v010 = p[ysl];
        v011 = p[ysl + 1];
        v100 = p[zsl];
        v101 = p[zsl + 1];
        v110 = p[zsl + ysl];
        v111 = p[zsl + ysl + 1];
      }
      const float val = trilerp(v000, v001, v010, v011, v100, v101, v110, v111, c);
      accumulate(classify(val, a.vmin, a.inv_range, a.M, s_tf), Cr, Cg, Cb, T);
      ++j;
      if (j >= cnt || 1.f - T >= a.tau) done = true;
    }
    if (up ? ch >= Lend : cl <= Lend) break;
    if (__all(done)) break;
    __syncthreads();
  }
  if (valid) a.img[bvw.img_off + (int64_t)ly * bvw.w + lx] = make_float4(Cr, Cg, Cb, 1.f - T);
}

}  // namespace

hipError_t launch_march_lds(const MarchArgs& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  const int grid = ((a.ntiles + 7) / 8) * 8;
  const size_t lds = sizeof(float4) * (size_t)a.M + sizeof(float) * (size_t)a.lds_budget;
  switch (a.tile_w) {
    case 8: hipLaunchKernelGGL(k_march_lds<8>, dim3(grid), dim3(64), lds, s, a); break;
    case 16: hipLaunchKernelGGL(k_march_lds<16>, dim3(grid), dim3(64), lds, s, a); break;
    case 4: hipLaunchKernelGGL(k_march_lds<4>, dim3(grid), dim3(64), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace vr
