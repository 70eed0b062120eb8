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
//      16-byte loads (each voxel fetched once per slab, coalesced); the loads
//      of slab s+1 are issued into registers before slab s is sampled, so
//      their latency overlaps the sampling (a two-stage software pipeline),
//   3. lets every lane consume its own samples whose cell layer along b lies
//      in the slab, reading the eight trilinear corners from LDS.
// With macrocells (empty-space skipping), a slab whose box touches only
// macrocells of zero opacity is neither loaded nor sampled: its samples would
// add nothing, so the lanes only advance their cursors past it.
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

// Voxel box of one slab in LDS: rows along axis 1 (f), `pitch` floats apart
// (a multiple of 4), ng rows per layer along the in-plane axis g, nl layers
// along the slab axis b.  Chunk i (16 bytes) of the box sits at LDS float 4i.
struct Region {
  int f_lo, g_lo, b_lo;
  int nf, ng, nl;
  int pitch, layer, chunks;
  int cl, ch;  // cell layers of the slab along b
  bool staged;
  bool skip;   // every macrocell holding a cell of the box has opacity 0 over its range
};

// Row, chunk-in-row, layer and row-in-layer of chunk i (reciprocal products;
// exact because i < 2^13 and the quotients are at least 0.5/nf4 away from the
// next integer).
struct ChunkPos {
  int c4, lb, lg;
};

__device__ __forceinline__ ChunkPos chunk_pos(int i, int nf4, int ng, float inv_nf4, float inv_ng) {
  ChunkPos c;
  const int row = (int)(((float)i + 0.5f) * inv_nf4);
  c.c4 = i - row * nf4;
  c.lb = (int)(((float)row + 0.5f) * inv_ng);
  c.lg = row - c.lb * ng;
  return c;
}

// Issue the global loads of a region's chunks into registers (lane-contiguous
// chunks, so one instruction reads 1 KB of consecutive row segments).  Every
// chunk is a full 16-byte load: with slack after the storage the last chunk of
// a row simply reads past the row's end (the extra floats land in the row's
// LDS padding); without it the chunk starts at nf - 4 instead (store_region
// shifts it back).  No load result is consumed here, so no wait is needed
// until the LDS store.
template <int CH>
__device__ __forceinline__ void issue_loads(const Region& r, gfloat* gbase, int sB, int sG, int lane, bool slack,
                                            float4 (&buf)[CH]) {
  const int nf4 = r.pitch >> 2;
  const float inv_nf4 = 1.0f / (float)nf4, inv_ng = 1.0f / (float)r.ng;
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int i = lane + 64 * k;
    if (i < r.chunks) {
      const ChunkPos c = chunk_pos(i, nf4, r.ng, inv_nf4, inv_ng);
      const int f0 = slack ? 4 * c.c4 : min(4 * c.c4, r.nf - 4);
      gfloat* src = gbase + ((r.b_lo + c.lb) * sB + (r.g_lo + c.lg) * sG + (r.f_lo + f0));
      const f4u v = *reinterpret_cast<const f4u __attribute__((address_space(1)))*>(src);
      buf[k] = make_float4(v.x, v.y, v.z, v.w);
    }
  }
}

template <int CH>
__device__ __forceinline__ void store_region(const Region& r, float* s_reg, int lane, bool slack, const float4 (&buf)[CH]) {
  if (slack) {  // chunks were read at their own position: store as loaded
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int i = lane + 64 * k;
      if (i < r.chunks) reinterpret_cast<float4*>(s_reg)[i] = buf[k];
    }
    return;
  }
  const int nf4 = r.pitch >> 2;
  const float inv_nf4 = 1.0f / (float)nf4, inv_ng = 1.0f / (float)r.ng;
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int i = lane + 64 * k;
    if (i < r.chunks) {
      const ChunkPos c = chunk_pos(i, nf4, r.ng, inv_nf4, inv_ng);
      const int rem = r.nf - 4 * c.c4;  // valid floats of this chunk (the row's tail may be short)
      float4 v = buf[k];
      if (rem == 3) v = make_float4(v.y, v.z, v.w, 0.f);
      else if (rem == 2) v = make_float4(v.z, v.w, 0.f, 0.f);
      else if (rem == 1) v = make_float4(v.w, 0.f, 0.f, 0.f);
      reinterpret_cast<float4*>(s_reg)[i] = v;
    }
  }
}

template <int TW, int CH>
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
  const bool by = a.slab_axis == 1;  // slab axis is axis 2 (else axis 3)
  const float pb = by ? py : pz, sb = by ? sy : sz;
  const int cloB = by ? br.clo[1] : br.clo[2], chiB = by ? br.chi[1] : br.chi[2];
  const int cloG = by ? br.clo[2] : br.clo[1], chiG = by ? br.chi[2] : br.chi[1];
  const int loB = by ? br.lo[1] : br.lo[2], loG = by ? br.lo[2] : br.lo[1];
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
  const int capacity = 256 * CH;  // floats the register pipeline can carry

  // voxel box of the slab covering cell layers starting at L (marching order)
  auto region_of = [&](int L) {
    Region r;
    r.cl = up ? L : max(L - a.slab_T + 1, Lend);
    r.ch = up ? min(L + a.slab_T - 1, Lend) : L;
    float fmn = INFINITY, fmx = -INFINITY, gmn = INFINITY, gmx = -INFINITY;
    if (lane < 8) {
      const float P = lane < 4 ? (float)r.cl : (float)(r.ch + 1);
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
    r.f_lo = uni(max((int)floorf(unif(fmn) - 0.05f), br.clo[0]));
    const int f_hi = uni(min((int)floorf(unif(fmx) + 0.05f) + 1, br.chi[0] + 1));
    r.g_lo = uni(max((int)floorf(unif(gmn) - 0.05f), cloG));
    const int g_hi = uni(min((int)floorf(unif(gmx) + 0.05f) + 1, chiG + 1));
    r.b_lo = r.cl;
    r.nf = f_hi - r.f_lo + 1;
    r.ng = g_hi - r.g_lo + 1;
    r.nl = r.ch + 2 - r.cl;
    r.pitch = (max(r.nf, 1) + 3) & ~3;
    r.layer = r.pitch * r.ng;
    r.chunks = (r.pitch >> 2) * r.ng * r.nl;
    r.skip = false;
    if (a.mc > 0) {
      // macrocells of the cells (global lower-corner indices) the slab's samples can use
      const int mc = a.mc;
      const int mf0 = (r.f_lo + br.lo[0]) / mc, mf1 = (max(f_hi - 1, r.f_lo) + br.lo[0]) / mc;
      const int mg0 = (r.g_lo + loG) / mc, mg1 = (max(g_hi - 1, r.g_lo) + loG) / mc;
      const int mb0 = (r.cl + loB) / mc, mb1 = (r.ch + loB) / mc;
      const int nmf = mf1 - mf0 + 1, nmg = mg1 - mg0 + 1;
      const int tot = nmf * nmg * (mb1 - mb0 + 1);
      bool opaque = false;
      for (int i = lane; i < tot; i += 64) {
        const int qf = i % nmf, rest = i / nmf;
        const int mg = mg0 + rest % nmg, mb = mb0 + rest / nmg;
        const int my = by ? mb : mg, mz = by ? mg : mb;
        opaque |= a.mc_clear[((int64_t)mz * a.mcn[1] + my) * a.mcn[0] + (mf0 + qf)] == 0;
      }
      r.skip = !__any(opaque);
    }
    r.staged = !r.skip && r.nf >= 4 && r.ng > 0 && r.layer * r.nl <= min(a.lds_budget, capacity);
    return r;
  };

  float Cr = 0.f, Cg = 0.f, Cb = 0.f, T = 1.f;
  int j = 0;
  bool done = cnt == 0;
  const int step_l = up ? a.slab_T : -a.slab_T;

  float4 buf[CH];
  int L = Lbeg;
  Region nxt = region_of(L);
  const bool slack = br.slack != 0;
  if (nxt.staged) issue_loads<CH>(nxt, gbase, strideB, strideG, lane, slack, buf);
  for (;;) {
    const Region cur = nxt;
    if (cur.staged) {
      store_region<CH>(cur, s_reg, lane, slack, buf);
      __syncthreads();
    }
    // prefetch the next slab while this one is sampled
    const bool last = up ? cur.ch >= Lend : cur.cl <= Lend;
    if (!last) {
      L += step_l;
      nxt = region_of(L);
      if (nxt.staged) issue_loads<CH>(nxt, gbase, strideB, strideG, lane, slack, buf);
    }
    // ---- consume the lane's samples whose cell layer along b is in [cl, ch]
    const int Sy = by ? cur.layer : cur.pitch, Sz = by ? cur.pitch : cur.layer;
    const int oy = by ? cur.b_lo : cur.g_lo, oz = by ? cur.g_lo : cur.b_lo;
    const int obase = cur.f_lo + oy * Sy + oz * Sz;
    // Two separate loops: the LDS loop must not share a block with global
    // loads, or the wait for those would also wait for the prefetch above.
    // a sample is in the slab while its cell layer (signed by the march
    // direction) has not passed the slab's last layer
    const int lim = up ? cur.ch : -cur.cl;
    if (cur.skip) {
      // every sample in the slab has opacity 0 (adds nothing, leaves T as it
      // is, cannot trigger termination): only move the cursor past them, with
      // the same layer test as the sampling loops
      const float fclo = (float)cloB, fchi = (float)chiB;
      while (!done) {
        const int ib = (int)floorf(__builtin_amdgcn_fmed3f(fmaf((float)j, sb, pb), fclo, fchi));
        if ((up ? ib : -ib) > lim) break;
        ++j;
        if (j >= cnt) done = true;
      }
    } else if (cur.staged) {
      while (!done) {
        const Cell c = cell_of(sample_pos(j, px, py, pz, sx, sy, sz), br);
        const int ib = by ? c.iy : c.iz;
        if ((up ? ib : -ib) > lim) break;
        // the cell lies in the slab's box by construction (footprint + margins)
        const float* p = s_reg + (c.ix + c.iy * Sy + c.iz * Sz - obase);
        const float val = trilerp(p[0], p[1], p[Sy], p[Sy + 1], p[Sz], p[Sz + 1], p[Sz + Sy], p[Sz + Sy + 1], c);
        accumulate(classify(val, a.vmin, a.inv_range, a.M, s_tf), Cr, Cg, Cb, T);
        ++j;
        if (j >= cnt || 1.f - T >= a.tau) done = true;
      }
    } else {
      while (!done) {
        const Cell c = cell_of(sample_pos(j, px, py, pz, sx, sy, sz), br);
        const int ib = by ? c.iy : c.iz;
        if ((up ? ib : -ib) > lim) break;
        gfloat* p = gbase + (c.iz * zsl + c.iy * ysl + c.ix);
        const float val = trilerp(p[0], p[1], p[ysl], p[ysl + 1], p[zsl], p[zsl + 1], p[zsl + ysl], p[zsl + ysl + 1], c);
        accumulate(classify(val, a.vmin, a.inv_range, a.M, s_tf), Cr, Cg, Cb, T);
        ++j;
        if (j >= cnt || 1.f - T >= a.tau) done = true;
      }
    }
    if (last || __all(done)) break;
    __syncthreads();
  }
  if (valid) a.img[bvw.img_off + (int64_t)ly * bvw.w + lx] = make_float4(Cr, Cg, Cb, 1.f - T);
}

}  // namespace

hipError_t launch_march_lds(const MarchArgs& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  if (a.cam.persp || a.mip) return hipErrorInvalidValue;  // parallel rays, emission-absorption only
  const int grid = ((a.ntiles + 7) / 8) * 8;
  // register pipeline depth: 16-byte chunks per lane that carry one slab's box
  const int ch = a.lds_budget <= 2048 ? 8 : (a.lds_budget <= 4096 ? 16 : 32);
  const size_t lds = sizeof(float4) * (size_t)a.M + sizeof(float) * 256 * (size_t)ch;
#define VR_LAUNCH_LDS(TW, CH) hipLaunchKernelGGL((k_march_lds<TW, CH>), dim3(grid), dim3(64), lds, s, a)
  if (a.tile_w != 4 && a.tile_w != 8 && a.tile_w != 16) return hipErrorInvalidValue;
  if (ch == 8) {
    if (a.tile_w == 8) VR_LAUNCH_LDS(8, 8);
    else if (a.tile_w == 16) VR_LAUNCH_LDS(16, 8);
    else VR_LAUNCH_LDS(4, 8);
  } else if (ch == 16) {
    if (a.tile_w == 8) VR_LAUNCH_LDS(8, 16);
    else if (a.tile_w == 16) VR_LAUNCH_LDS(16, 16);
    else VR_LAUNCH_LDS(4, 16);
  } else {
    if (a.tile_w == 8) VR_LAUNCH_LDS(8, 32);
    else if (a.tile_w == 16) VR_LAUNCH_LDS(16, 32);
    else VR_LAUNCH_LDS(4, 32);
  }
#undef VR_LAUNCH_LDS
  return hipGetLastError();
}

}  // namespace vr
