// march_cells.hip -- forward march over footprint cells (parallel rays): a
// wavefront per cell (k_march_cells), or a workgroup per block of cells
// sharing one window per layer (k_march_block).
//
// Same samples, same per-sample arithmetic and the same order as every other
// march (paper Sec. 2.4: each ray is sampled between its entry and exit points
// and accumulated front to back with early termination); only the way the
// eight trilinear corners reach the lanes differs.
//
// A footprint cell is the set of pixels whose rays cross a brick's plane
// b = 0 (b = axis 2 or 3, the slab axis) inside one Tf x Tg rectangle of
// (f, g) = (axis 1, the other in-plane axis).  Its rays are parallel, so on
// the plane b = P they fill the same rectangle moved by P (rf, rg); the window
// of voxel layer V -- every voxel a sample of the cell between the planes
// V - 1 and V + 1 can touch -- is that rectangle over [V - 1, V + 1] plus the
// trilinear margin, rows along f (the contiguous storage axis).  Cell layer c
// is sampled from voxel layers c and c + 1.
//
// k_march_cells: two LDS slots per wavefront hold the two layers being
// sampled; the window of the layer after next is loaded into registers while
// a layer is sampled and written over the finished layer afterwards, so every
// wavefront keeps a layer in flight without a third slot.  Window loads are
// addressed from a uniform base (scalar registers) plus a per-lane offset
// fixed for the cell, and the slab axis is a template parameter, so the
// per-layer and per-sample bookkeeping stays small.
//
// k_march_block: the blk_f x blk_g wavefronts of a workgroup march the cells
// of one block (a wavefront per cell) together, one cell layer at a time, with
// one window per voxel layer for the whole block (each wavefront loads its
// share of rows through registers); per layer: sample; barrier; write V_{k+2}
// over V_k and start V_{k+3}; barrier.
#include <algorithm>

#include "ring_common.h"
#include "sample.h"
#include "vr_internal.h"

namespace vr {

namespace {

using namespace ring;

constexpr int kBlkMaxWaves = 8;
typedef float v4f __attribute__((ext_vector_type(4)));

// Per-lane ray of a footprint cell: the pixel, its place in the output, and
// the brick's share of its lattice as brick-local single-precision start and
// step (ray setup in double precision, as in every march).
struct CellRay {
  bool valid, wr_ok;
  float4* dst;
  float4 carried;
  int cnt;
  float px, py, pz, sx, sy, sz;
};

template <bool PERSP>
__device__ __forceinline__ CellRay cell_ray(const MarchArgs& a, const DevBrickView& bvw, const DevBrick& br,
                                            const FootRuns& fr, int lane) {
  CellRay r;
  int u, v;
  foot_pixel(fr, lane, u, v);
  r.valid = lane < fr.n;
  if (!r.valid) {
    u = 0;
    v = 0;
  }
  const int lx = u - bvw.x0, ly = v - bvw.y0;
  const bool inrect = lx >= 0 && lx < bvw.w && ly >= 0 && ly < bvw.h;
  double o[3], dl[3];
  const double* d = a.cam.e3;  // parallel rays: the view direction
  if constexpr (PERSP) {
    pixel_ray(a.cam, u, v, o, dl);
    d = dl;
  } else {
    pixel_origin(a.cam, u, v, o);
  }
  r.cnt = 0;
  r.px = r.py = r.pz = 0.f;
  r.dst = a.carry ? a.img + (int64_t)v * a.cam.W + u : a.img + bvw.img_off + (int64_t)ly * bvw.w + lx;
  r.wr_ok = a.carry || inrect;  // dst is this pixel's place
  r.carried = make_float4(0.f, 0.f, 0.f, 1.f);
  if (a.carry && r.valid) r.carried = *r.dst;
  const bool live = !a.carry || 1.f - r.carried.w < a.tau;
  double tin;
  int64_t n;
  if (r.valid && live && ray_lattice(o, d, a.hi, a.step, tin, n)) {
    int64_t k0, k1;
    brick_krange(o, d, tin, a.step, n, br.lo, br.hi, br.closed, k0, k1);
    if (k1 > k0) {
      const double t0 = tin + ((double)k0 + 0.5) * a.step;
      r.px = (float)(o[0] + t0 * d[0] - (double)br.lo[0]);
      r.py = (float)(o[1] + t0 * d[1] - (double)br.lo[1]);
      r.pz = (float)(o[2] + t0 * d[2] - (double)br.lo[2]);
      r.cnt = (int)(k1 - k0);
    }
  }
  r.sx = (float)(a.step * d[0]);
  r.sy = (float)(a.step * d[1]);
  r.sz = (float)(a.step * d[2]);
  return r;
}

// The samples of one lane that fall in cell layer c, read from the two LDS
// windows whose origins are wl (voxel layer c) and wu (layer c + 1).
template <bool MIP, bool BY>
__device__ __forceinline__ void sample_layer(const MarchArgs& a, const DevBrick& br, const CellRay& r,
                                             const float4* s_tf, const float* s_ring, int slot, int pitch, int c,
                                             const Window& wl, const Window& wu, int sl, int su, float fclo,
                                             float fchi, int& j, bool& done, float& Cr, float& Cg, float& Cb,
                                             float& T, float& mx) {
  const float* baseL = s_ring + (sl * slot - wl.g0 * pitch - wl.f0);
  const int dU = (su * slot - wu.g0 * pitch - wu.f0) - (sl * slot - wl.g0 * pitch - wl.f0);
  while (!done) {
    const SamplePos q = sample_pos(j, r.px, r.py, r.pz, r.sx, r.sy, r.sz);
    const int ib = (int)floorf(__builtin_amdgcn_fmed3f(BY ? q.y : q.z, fclo, fchi));
    if (ib != c) break;
    const Cell cl = cell_of(q, br);
    const int ig = BY ? cl.iz : cl.iy;
    const float* p = baseL + (__mul24(ig, pitch) + cl.ix);
    const float* pu = p + dU;
    // corners v[dz][dy][dx]: within a window rows run along g, layers along b
    const float l00 = p[0], l01 = p[1], l10 = p[pitch], l11 = p[pitch + 1];
    const float u00 = pu[0], u01 = pu[1], u10 = pu[pitch], u11 = pu[pitch + 1];
    const float val = BY ? trilerp(l00, l01, u00, u01, l10, l11, u10, u11, cl)
                         : trilerp(l00, l01, l10, l11, u00, u01, u10, u11, cl);
    ++j;
    if (MIP) {
      const float sv = norm_value(val, a.vmin, a.inv_range);
      mx = fmaxf(mx, sv);
      if (j >= r.cnt || mx >= 1.f) done = true;
    } else {
      const Classified kk = classify(val, a.vmin, a.inv_range, a.M, s_tf);
      accumulate(kk, Cr, Cg, Cb, T);
      if (j >= r.cnt || 1.f - T >= a.tau) done = true;
    }
  }
}

template <bool MIP, bool BY, bool PERSP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_march_cells(MarchArgs a) {
  extern __shared__ float4 smem[];
  float4* s_tf = smem;
  for (int i = threadIdx.x; i < a.M; i += blockDim.x) s_tf[i] = a.tf[i];
  __syncthreads();

  const int wpb = (int)(blockDim.x >> 6);
  const int wave = uni((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int slot = a.ring_slot;  // floats per slot (one voxel layer's window)
  float* s_ring = reinterpret_cast<float*>(smem + a.M) + (size_t)wave * 2 * slot;

  // XCD-aware order: workgroup b runs on XCD b % 8; each XCD takes one
  // contiguous range of cells (neighbouring cells share its L2)
  const int ngroups = (a.ntiles + wpb - 1) / wpb;
  const int per = (ngroups + 7) >> 3;
  const int tile = ((int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3)) * wpb + wave;
  if (tile >= a.ntiles) return;  // this wavefront only: no barrier follows

  const DevBrickView bvw = a.bv[find_bv(a, tile)];
  const DevBrick br = a.bricks[bvw.brick];
  int ci, cj;
  foot_cell(bvw, tile - bvw.tile_begin, ci, cj);
  const FootRuns fr = PERSP ? foot_runs_persp(a, bvw, br, ci, cj, lane) : foot_runs(a, bvw, ci, cj, lane);
  // pixels past the 64th of a cell are marched by k_march_ring_ovf afterwards
  if (fr.n > 64 && lane == 0) a.ovf_tiles[atomicAdd(a.ovf_count, 1u)] = tile * 8;
  const CellRay r = cell_ray<PERSP>(a, bvw, br, fr, lane);

  // ---- frame: b = slab axis (axis 2 if BY, else axis 3), g = the other, f = axis 1
  const float pb = BY ? r.py : r.pz, sb = BY ? r.sy : r.sz;
  const int cloB = BY ? br.clo[1] : br.clo[2], chiB = BY ? br.chi[1] : br.chi[2];
  const int cloG = BY ? br.clo[2] : br.clo[1], chiG = BY ? br.chi[2] : br.chi[1];
  const int cloF = br.clo[0], chiF = br.chi[0];
  const double db = BY ? a.cam.e3[1] : a.cam.e3[2], dg = BY ? a.cam.e3[2] : a.cam.e3[1];
  // perspective: the brick-local eye E; the rays run away from it along b
  const double Eb = PERSP ? a.cam.eye[BY ? 1 : 2] - (double)br.lo[BY ? 1 : 2] : 0.0;
  const bool up = PERSP ? Eb < 0.0 : db > 0.0;

  // cell layers (along b) of the lane's first and last samples
  int c_first = up ? 0x7fffffff : -0x7fffffff, c_last = up ? -0x7fffffff : 0x7fffffff;
  if (r.cnt > 0) {
    c_first = (int)floorf(__builtin_amdgcn_fmed3f(pb, (float)cloB, (float)chiB));
    c_last = (int)floorf(__builtin_amdgcn_fmed3f(fmaf((float)(r.cnt - 1), sb, pb), (float)cloB, (float)chiB));
  }
  const int Lbeg = uni(up ? wave_imin(c_first) : wave_imax(c_first));
  const int Lend = uni(up ? wave_imax(c_last) : wave_imin(c_last));
  if (up ? Lbeg > Lend : Lbeg < Lend) return;  // no samples (the frame or arena was cleared)
  const int nlay = up ? Lend - Lbeg + 1 : Lbeg - Lend + 1;  // cell layers

  // ---- window geometry: the cell's rectangle on the plane b = 0 moves by
  // (rf, rg) per layer; window of voxel layer V = that rectangle over the
  // planes [V - 1, V + 1], cells floor(q) .. floor(q) + 1, 0.05 margins
  const float rf = PERSP ? 0.f : (float)(a.cam.e3[0] / db), rg = PERSP ? 0.f : (float)(dg / db);
  const float arf = fabsf(rf), arg = fabsf(rg);
  const double Tf = PERSP ? bvw.pTf : a.foot_Tf, Tg = PERSP ? bvw.pTg : a.foot_Tg;
  const float Af_lo = (float)((double)ci * Tf), Ag_lo = (float)((double)cj * Tg);
  const float Af_hi = (float)((double)(ci + 1) * Tf), Ag_hi = (float)((double)(cj + 1) * Tg);
  // perspective: on the plane b = P the cell's rays fill its rectangle scaled
  // by s(P) = 1 - P / E_b about the eye's foot point (Ef, Eg)
  const float Ef = PERSP ? (float)(a.cam.eye[0] - (double)br.lo[0]) : 0.f;
  const float Eg = PERSP ? (float)(a.cam.eye[BY ? 2 : 1] - (double)br.lo[BY ? 2 : 1]) : 0.f;
  const float inv_Eb = PERSP ? (float)(1.0 / Eb) : 0.f;
  const int pitch = PERSP ? bvw.ppitch : (a.foot_nf + 3) & ~3;
  const int NG = min(PERSP ? bvw.png : a.foot_ng, chiG + 2 - cloG);
  const int sB = BY ? br.sy : br.sz, sG = BY ? br.sz : br.sy;
  gfloat* gbase = (gfloat*)br.base;
  auto window = [&](int V) {
    Window w;
    int flo, glo;
    if constexpr (PERSP) {
      const float s0 = fmaf(-(float)(V - 1), inv_Eb, 1.f), s1 = fmaf(-(float)(V + 1), inv_Eb, 1.f);
      const float f00 = fmaf(s0, Af_lo - Ef, Ef), f01 = fmaf(s0, Af_hi - Ef, Ef);
      const float f10 = fmaf(s1, Af_lo - Ef, Ef), f11 = fmaf(s1, Af_hi - Ef, Ef);
      const float g00 = fmaf(s0, Ag_lo - Eg, Eg), g01 = fmaf(s0, Ag_hi - Eg, Eg);
      const float g10 = fmaf(s1, Ag_lo - Eg, Eg), g11 = fmaf(s1, Ag_hi - Eg, Eg);
      flo = max((int)floorf(fminf(fminf(f00, f01), fminf(f10, f11)) - 0.05f), cloF);
      glo = max((int)floorf(fminf(fminf(g00, g01), fminf(g10, g11)) - 0.05f), cloG);
      // the window is sized for the brick's widest layer; this layer's samples
      // read columns and rows up to these (the trilinear neighbour included)
      w.fb = (int)floorf(fmaxf(fmaxf(f00, f01), fmaxf(f10, f11)) + 0.05f) + 1;
      w.gb = (int)floorf(fmaxf(fmaxf(g00, g01), fmaxf(g10, g11)) + 0.05f) + 1;
    } else {
      const float Pf = (float)V * rf, Pg = (float)V * rg;
      flo = max((int)floorf(Af_lo + Pf - arf - 0.05f), cloF);
      glo = max((int)floorf(Ag_lo + Pg - arg - 0.05f), cloG);
      w.fb = w.gb = 0;
    }
    w.f0 = uni(max(cloF, min(flo, chiF + 2 - pitch)));
    w.g0 = uni(max(cloG, min(glo, chiG + 2 - NG)));
    if constexpr (PERSP) {
      w.fb = uni(w.fb - w.f0);
      w.gb = uni(w.gb - w.g0);
    }
    return w;
  };

  // chunk (16 bytes) of lane l in load instruction i: row i R + l / (pitch / 4),
  // column 4 (l % (pitch / 4)); R = 64 / (pitch / 4) whole rows per instruction.
  // A lane's byte offset from the instruction's first row is fixed for the
  // cell; only the uniform base moves.
  const int nf4 = pitch >> 2;
  const int R = uni(64 / nf4);
  const int rl = lane / nf4, c4l = lane - rl * nf4;
  // instructions that carry a row of the window for this lane
  const int nmine = rl < R ? (NG - rl + R - 1) / R : 0;
  const unsigned row_off = (unsigned)(rl * sG) * 4u;
  const unsigned step_off = (unsigned)(R * sG) * 4u;
  v4f rr[kRingRegLoads];
  auto rload = [&](int V, const Window& w) {
    const char* gb = (const char*)unip(gbase + ((int64_t)V * sB + (int64_t)w.g0 * sG + w.f0));
    if constexpr (PERSP) {
      // the window is sized for the brick's widest layer: this layer's
      // columns and rows end earlier.  A lane past them reads the last chunk
      // or row the layer needs instead (lines fetched anyway; what it leaves
      // in LDS is never sampled), so the predicate stays the cell's and no
      // load waits on another.
      const int kc = min(c4l, uni(min(nf4 - 1, w.fb >> 2)));
      const unsigned col_off = (unsigned)kc * 16u;
      const unsigned last_off = (unsigned)(min(NG - 1, w.gb) * sG) * 4u;
#pragma unroll
      for (int i = 0; i < kRingRegLoads; ++i)
        if (i < nmine)
          rr[i] = *(const v4f __attribute__((address_space(1)))*)(gb + (min(row_off + (unsigned)i * step_off, last_off) +
                                                                          col_off));
    } else {
      const unsigned lane_off = row_off + (unsigned)c4l * 16u;
#pragma unroll
      for (int i = 0; i < kRingRegLoads; ++i)
        if (i < nmine) rr[i] = *(const v4f __attribute__((address_space(1)))*)(gb + (lane_off + (unsigned)i * step_off));
    }
  };
  auto rstore = [&](float* sdst) {
    v4f* l = (v4f*)(sdst + 4 * lane);
#pragma unroll
    for (int i = 0; i < kRingRegLoads; ++i)
      if (i < nmine) l[i * R * nf4] = rr[i];
  };

  // voxel layers in marching order: V_k = Lbeg + k (up) or Lbeg + 1 - k (down);
  // cell layer c_k = Lbeg +- k reads V_k and V_{k+1}
  const int vstep = up ? 1 : -1;
  const int V0 = up ? Lbeg : Lbeg + 1;
  const float fclo = (float)cloB, fchi = (float)chiB;
  float Cr = r.carried.x, Cg = r.carried.y, Cb = r.carried.z, T = r.carried.w, mx = 0.f;
  int j = 0;
  bool done = r.cnt == 0;

  Window w0 = window(V0), w1 = window(V0 + vstep), w2;
  rload(V0, w0);
  rstore(s_ring);
  rload(V0 + vstep, w1);
  rstore(s_ring + slot);
  if (nlay > 1) {
    w2 = window(V0 + 2 * vstep);
    rload(V0 + 2 * vstep, w2);
  }
  int s0 = 0;  // slot of V_k (V_{k+1} is in the other)
  for (int k = 0; k < nlay; ++k) {
    const int c = up ? Lbeg + k : Lbeg - k;
    const Window& wl = up ? w0 : w1;
    const Window& wu = up ? w1 : w0;
    sample_layer<MIP, BY>(a, br, r, s_tf, s_ring, slot, pitch, c, wl, wu, up ? s0 : s0 ^ 1, up ? s0 ^ 1 : s0,
                          fclo, fchi, j, done, Cr, Cg, Cb, T, mx);
    if (__all(done)) break;
    if (k + 1 < nlay) {
      rstore(s_ring + s0 * slot);  // V_{k+2} replaces V_k (same wavefront: LDS order holds)
      w0 = w1;
      w1 = w2;
      if (k + 2 < nlay) {
        w2 = window(V0 + (k + 3) * vstep);
        rload(V0 + (k + 3) * vstep, w2);
      }
    }
    s0 ^= 1;
  }
  if (r.valid && r.wr_ok && r.cnt > 0)
    *r.dst = MIP ? make_float4(mx, mx, mx, mx) : make_float4(Cr, Cg, Cb, a.carry ? T : 1.f - T);
}

template <bool MIP, bool BY>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_march_block(MarchArgs a) {
  extern __shared__ float4 smem[];
  __shared__ int s_lb[kBlkMaxWaves], s_le[kBlkMaxWaves], s_vote[2];
  float4* s_tf = smem;
  float* s_ring = reinterpret_cast<float*>(smem + a.M);
  const int nw = (int)(blockDim.x >> 6);
  const int wave = uni((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int slot = a.ring_slot;  // floats per slot (one voxel layer's window)

  // XCD-aware order: workgroup b runs on XCD b % 8; each XCD takes one
  // contiguous range of blocks
  const int per = (a.ntiles + 7) >> 3;
  const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (tile >= a.ntiles) return;  // the whole workgroup

  for (int i = threadIdx.x; i < a.M; i += blockDim.x) s_tf[i] = a.tf[i];
  if (threadIdx.x < 2) s_vote[threadIdx.x] = 0;

  const DevBrickView bvw = a.bv[find_bv(a, tile)];
  const DevBrick br = a.bricks[bvw.brick];
  const int t = tile - bvw.tile_begin;
  int ci, cj;
  block_cell(a, bvw, t, wave, ci, cj);
  const FootRuns fr = foot_runs(a, bvw, ci, cj, lane);
  if (fr.n > 64 && lane == 0) a.ovf_tiles[atomicAdd(a.ovf_count, 1u)] = tile * 8 + wave;
  const CellRay r = cell_ray<false>(a, bvw, br, fr, lane);

  const float pb = BY ? r.py : r.pz, sb = BY ? r.sy : r.sz;
  const int cloB = BY ? br.clo[1] : br.clo[2], chiB = BY ? br.chi[1] : br.chi[2];
  const int cloG = BY ? br.clo[2] : br.clo[1], chiG = BY ? br.chi[2] : br.chi[1];
  const int cloF = br.clo[0], chiF = br.chi[0];
  const double db = BY ? a.cam.e3[1] : a.cam.e3[2], dg = BY ? a.cam.e3[2] : a.cam.e3[1];
  const bool up = db > 0.0;

  // cell layers of the block: the union over its wavefronts
  int c_first = up ? 0x7fffffff : -0x7fffffff, c_last = up ? -0x7fffffff : 0x7fffffff;
  if (r.cnt > 0) {
    c_first = (int)floorf(__builtin_amdgcn_fmed3f(pb, (float)cloB, (float)chiB));
    c_last = (int)floorf(__builtin_amdgcn_fmed3f(fmaf((float)(r.cnt - 1), sb, pb), (float)cloB, (float)chiB));
  }
  const int wlb = up ? wave_imin(c_first) : wave_imax(c_first);
  const int wle = up ? wave_imax(c_last) : wave_imin(c_last);
  if (lane == 0) {
    s_lb[wave] = wlb;
    s_le[wave] = wle;
  }
  __syncthreads();
  int Lbeg = s_lb[0], Lend = s_le[0];
  for (int w = 1; w < nw; ++w) {
    Lbeg = up ? min(Lbeg, s_lb[w]) : max(Lbeg, s_lb[w]);
    Lend = up ? max(Lend, s_le[w]) : min(Lend, s_le[w]);
  }
  Lbeg = uni(Lbeg);
  Lend = uni(Lend);
  if (up ? Lbeg > Lend : Lbeg < Lend) return;  // no samples in the block (whole workgroup)
  const int nlay = up ? Lend - Lbeg + 1 : Lbeg - Lend + 1;

  const float rf = (float)(a.cam.e3[0] / db), rg = (float)(dg / db);
  const float arf = fabsf(rf), arg = fabsf(rg);
  const int bi0 = bvw.cf0 + (t % bvw.blocks_x) * a.blk_f, bj0 = bvw.cg0 + (t / bvw.blocks_x) * a.blk_g;
  const float Af_lo = (float)((double)bi0 * a.foot_Tf), Ag_lo = (float)((double)bj0 * a.foot_Tg);
  const int pitch = (a.foot_nf + 3) & ~3;
  const int NG = min(a.foot_ng, chiG + 2 - cloG);
  const int sB = BY ? br.sy : br.sz, sG = BY ? br.sz : br.sy;
  gfloat* gbase = (gfloat*)br.base;
  auto window = [&](int V) {
    Window w;
    const float Pf = (float)V * rf, Pg = (float)V * rg;
    const int flo = max((int)floorf(Af_lo + Pf - arf - 0.05f), cloF);
    const int glo = max((int)floorf(Ag_lo + Pg - arg - 0.05f), cloG);
    w.f0 = uni(max(cloF, min(flo, chiF + 2 - pitch)));
    w.g0 = uni(max(cloG, min(glo, chiG + 2 - NG)));
    w.fb = w.gb = 0;
    return w;
  };

  // load instruction m (over the workgroup) carries rows m R .. m R + R - 1;
  // wavefront w issues instructions w, w + nw, ...
  const int nf4 = pitch >> 2;
  const int R = uni(64 / nf4);
  const int rl = lane / nf4, c4l = lane - rl * nf4;
  const int nload = uni((NG + R - 1) / R);
  const int nmine_w = uni((nload - wave + nw - 1) / nw);  // this wavefront's instructions
  v4f rr[kRingRegLoads];
  auto row_of = [&](int i) { return (wave + i * nw) * R + rl; };
  auto rload = [&](int V, const Window& w) {
    gfloat* gb = gbase + ((int64_t)V * sB + (int64_t)w.g0 * sG + w.f0) + 4 * c4l;
#pragma unroll
    for (int i = 0; i < kRingRegLoads; ++i)
      if (i < nmine_w && rl < R && row_of(i) < NG)
        rr[i] = *(const v4f __attribute__((address_space(1)))*)(gb + (int64_t)row_of(i) * sG);
  };
  auto rstore = [&](float* sdst) {
#pragma unroll
    for (int i = 0; i < kRingRegLoads; ++i)
      if (i < nmine_w && rl < R && row_of(i) < NG) *(v4f*)(sdst + row_of(i) * pitch + 4 * c4l) = rr[i];
  };

  const int vstep = up ? 1 : -1;
  const int V0 = up ? Lbeg : Lbeg + 1;
  const float fclo = (float)cloB, fchi = (float)chiB;
  float Cr = r.carried.x, Cg = r.carried.y, Cb = r.carried.z, T = r.carried.w, mx = 0.f;
  int j = 0;
  bool done = r.cnt == 0;

  Window w0 = window(V0), w1 = window(V0 + vstep), w2;
  rload(V0, w0);
  rstore(s_ring);
  rload(V0 + vstep, w1);
  rstore(s_ring + slot);
  if (nlay > 1) {
    w2 = window(V0 + 2 * vstep);
    rload(V0 + 2 * vstep, w2);
  }
  __syncthreads();  // table and the first two layers are in LDS
  int s0 = 0;
  for (int k = 0; k < nlay; ++k) {
    const int c = up ? Lbeg + k : Lbeg - k;
    const Window& wl = up ? w0 : w1;
    const Window& wu = up ? w1 : w0;
    sample_layer<MIP, BY>(a, br, r, s_tf, s_ring, slot, pitch, c, wl, wu, up ? s0 : s0 ^ 1, up ? s0 ^ 1 : s0,
                          fclo, fchi, j, done, Cr, Cg, Cb, T, mx);
    // vote of the block (slot k & 1 is cleared for the next layer's vote
    // between the two barriers)
    const bool wave_live = __any(!done);  // over all lanes, before any branch on the lane
    if (lane == 0 && wave_live) s_vote[k & 1] = 1;
    __syncthreads();  // every wavefront is done with V_k
    const bool more = s_vote[k & 1] != 0;
    if (!more || k + 1 >= nlay) break;
    if (threadIdx.x == 0) s_vote[(k + 1) & 1] = 0;
    rstore(s_ring + s0 * slot);  // V_{k+2} replaces V_k
    w0 = w1;
    w1 = w2;
    if (k + 2 < nlay) {
      w2 = window(V0 + (k + 3) * vstep);
      rload(V0 + (k + 3) * vstep, w2);
    }
    __syncthreads();  // V_{k+2} is complete
    s0 ^= 1;
  }
  if (r.valid && r.wr_ok && r.cnt > 0)
    *r.dst = MIP ? make_float4(mx, mx, mx, mx) : make_float4(Cr, Cg, Cb, a.carry ? T : 1.f - T);
}

}  // namespace

size_t block_lds_bytes(const MarchArgs& a) {
  return sizeof(float4) * (size_t)a.M + sizeof(float) * 2 * (size_t)a.ring_slot;
}

size_t cells_lds_bytes(const MarchArgs& a, int wpb) {
  return sizeof(float4) * (size_t)a.M + sizeof(float) * 2 * (size_t)wpb * (size_t)a.ring_slot;
}

// checks shared by both launches: a window's rows and loads as the kernels
// assume them
static bool cells_args_ok(const MarchArgs& a, int waves_per_window) {
  const int64_t pitch = (a.foot_nf + 3) & ~3;
  if (a.mc != 0 || a.mask || !a.foot || a.ring_slot <= 0 || (a.ring_slot & 3) != 0 ||
      (a.slab_axis != 1 && a.slab_axis != 2))
    return false;
  // perspective: windows sized per brick, each checked against the slot and
  // the register loads when the launch was planned
  if (a.cam.persp) return waves_per_window == 1;
  if (pitch > 256 || pitch * a.foot_ng > a.ring_slot) return false;
  const int64_t R = 64 / (pitch / 4);
  const int64_t nload = (a.foot_ng + R - 1) / R;
  return (nload + waves_per_window - 1) / waves_per_window <= kRingRegLoads;
}

hipError_t launch_march_block(const MarchArgs& a, hipStream_t s) {
  const int nw = a.blk_f * a.blk_g;
  if (a.ntiles <= 0) return hipSuccess;
  if (a.blk_f < 1 || a.blk_g < 1 || nw > kBlkMaxWaves || !cells_args_ok(a, nw)) return hipErrorInvalidValue;
  const int grid = ((a.ntiles + 7) / 8) * 8;
  const dim3 g(grid), b(64 * nw);
  const size_t lds = block_lds_bytes(a);
  const bool by = a.slab_axis == 1;
  if (a.mip && by) hipLaunchKernelGGL((k_march_block<true, true>), g, b, lds, s, a);
  else if (a.mip) hipLaunchKernelGGL((k_march_block<true, false>), g, b, lds, s, a);
  else if (by) hipLaunchKernelGGL((k_march_block<false, true>), g, b, lds, s, a);
  else hipLaunchKernelGGL((k_march_block<false, false>), g, b, lds, s, a);
  return hipGetLastError();
}

hipError_t launch_march_cells(const MarchArgs& a, int wpb, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  if ((wpb != 1 && wpb != 2 && wpb != 4) || !cells_args_ok(a, 1)) return hipErrorInvalidValue;
  const int groups = (a.ntiles + wpb - 1) / wpb;
  const int grid = ((groups + 7) / 8) * 8;
  const dim3 g(grid), b(64 * wpb);
  const size_t lds = std::max(cells_lds_bytes(a, wpb), (size_t)std::max(0, a.lds_floor));
  const bool by = a.slab_axis == 1;
  if (a.cam.persp) {
    if (a.mip && by) hipLaunchKernelGGL((k_march_cells<true, true, true>), g, b, lds, s, a);
    else if (a.mip) hipLaunchKernelGGL((k_march_cells<true, false, true>), g, b, lds, s, a);
    else if (by) hipLaunchKernelGGL((k_march_cells<false, true, true>), g, b, lds, s, a);
    else hipLaunchKernelGGL((k_march_cells<false, false, true>), g, b, lds, s, a);
  } else {
    if (a.mip && by) hipLaunchKernelGGL((k_march_cells<true, true, false>), g, b, lds, s, a);
    else if (a.mip) hipLaunchKernelGGL((k_march_cells<true, false, false>), g, b, lds, s, a);
    else if (by) hipLaunchKernelGGL((k_march_cells<false, true, false>), g, b, lds, s, a);
    else hipLaunchKernelGGL((k_march_cells<false, false, false>), g, b, lds, s, a);
  }
  return hipGetLastError();
}

}  // namespace vr
