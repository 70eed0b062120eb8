// grad_ring.hip -- the adjoint march on the ring-window layout (gfx950).
//
// The differentiable forward (k_march_ring<false, true>) walks every 8 x 8 ray
// tile cell layer by cell layer along the slab axis b and stores, for every
// group of L consecutive cell layers of the tile (in marching order), each
// ray's transmittance and sample cursor at the group's start.  This kernel
// walks the groups from the last to the first.  For a group it
//   1. copies the L + 1 voxel windows the group's samples read into LDS
//      (the same windows as the forward: rows along axis 1, direct
//      global->LDS loads) and clears L + 1 gradient windows of the same shape;
//   2. replays each ray's samples of the group forward from the stored
//      transmittance, keeping T before each sample in LDS;
//   3. walks them backward with the division-free recursion
//        dL/dc_k = g_rgb T_{k-1} a_k,
//        dL/da_k = T_{k-1} [g_rgb . (c_k - R_k) + g_A (1 - Q_k)],
//        R_{k-1} = a_k c_k + (1 - a_k) R_k,  Q_{k-1} = a_k + (1 - a_k) Q_k,
//      carrying R and Q from group to group; table gradients go to double LDS
//      accumulators (one set per workgroup, reduced by k_tf_reduce), voxel
//      gradients to the gradient windows with LDS float atomics;
//   4. adds the gradient windows to the gradient volume with one float atomic
//      per non-zero window voxel, row after row (coalesced), instead of eight
//      scattered atomics per sample.
// Samples are evaluated at double-precision positions (start + j step, one
// rounding per axis; cell_d), with the trilinear value, the table lookup, the
// recursion and the gradient algebra in double precision.  A tile whose window would not
// fit reads its corners from global memory and adds its voxel gradients with
// global atomics directly (same groups, same arithmetic).
#include <algorithm>

#include "ring_common.h"
#include "sample.h"
#include "vr_internal.h"

namespace vr {

namespace {

using namespace ring;

struct Eval {
  double a, r, g, b;  // table opacity and colour
  double w;           // table weight
  double sraw;        // unclamped normalised value
  double wx, wy, wz;  // trilinear fractions
  int i;              // table interval
};

// A sample in double precision: position start + j step (one rounding per
// axis), base cell clamped to the stored range, fractions.  The adjoint
// differentiates the definition at these positions, not the forward's
// single-precision ones.
struct CellD {
  int ix, iy, iz;
  double wx, wy, wz;
};

__device__ __forceinline__ CellD cell_d(int j, const double (&p0)[3], const double (&sv)[3], const DevBrick& br) {
  CellD c;
  const double kk = (double)j;
  const double qx = fma(kk, sv[0], p0[0]), qy = fma(kk, sv[1], p0[1]), qz = fma(kk, sv[2], p0[2]);
  c.ix = min(max((int)floor(qx), br.clo[0]), br.chi[0]);
  c.iy = min(max((int)floor(qy), br.clo[1]), br.chi[1]);
  c.iz = min(max((int)floor(qz), br.clo[2]), br.chi[2]);
  c.wx = qx - (double)c.ix;
  c.wy = qy - (double)c.iy;
  c.wz = qz - (double)c.iz;
  return c;
}

// Trilinear value (lerp along 1, then 2, then 3) and table lookup in double
// precision from the eight corners v[dz][dy][dx].
__device__ __forceinline__ Eval eval_d(const float (&v)[8], const CellD& c, double vmin, double inv_range, int M,
                                       const float4* s_tf) {
  Eval e;
  e.wx = c.wx;
  e.wy = c.wy;
  e.wz = c.wz;
  const double c00 = fma(e.wx, (double)v[1] - (double)v[0], (double)v[0]);
  const double c01 = fma(e.wx, (double)v[3] - (double)v[2], (double)v[2]);
  const double c10 = fma(e.wx, (double)v[5] - (double)v[4], (double)v[4]);
  const double c11 = fma(e.wx, (double)v[7] - (double)v[6], (double)v[6]);
  const double c0 = fma(e.wy, c01 - c00, c00), c1 = fma(e.wy, c11 - c10, c10);
  const double val = fma(e.wz, c1 - c0, c0);
  e.sraw = (val - vmin) * inv_range;
  const double s = fmin(fmax(e.sraw, 0.0), 1.0);
  const double u = s * (double)(M - 1);
  e.i = min((int)u, M - 2);
  e.w = u - (double)e.i;
  const float4 t0 = s_tf[e.i], t1 = s_tf[e.i + 1];
  e.r = fma(e.w, (double)t1.x - (double)t0.x, (double)t0.x);
  e.g = fma(e.w, (double)t1.y - (double)t0.y, (double)t0.y);
  e.b = fma(e.w, (double)t1.z - (double)t0.z, (double)t0.z);
  e.a = fma(e.w, (double)t1.w - (double)t0.w, (double)t0.w);
  return e;
}

__global__ __launch_bounds__(256) void k_bwd_ring(MarchArgs a, BwdArgs ba) {
  extern __shared__ double dsm[];
  const int M = a.M, L = ba.K;
  double* s_gtf = dsm;                                      // [M][4]
  float4* s_tf = reinterpret_cast<float4*>(dsm + 4 * M);    // [M]
  const int wpb = (int)(blockDim.x >> 6);
  const int wave = uni((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int slot = a.ring_slot;
  const int smax = ba.smax;  // samples of one ray in one group, at most
  // per wavefront: L + 1 voxel windows, L + 1 gradient windows, the slot
  // offsets and T before each sample of the group, [smax][64]
  const size_t per_wave = (size_t)2 * (L + 1) * slot + 64 + (size_t)smax * 64;
  float* s_vox = reinterpret_cast<float*>(s_tf + M) + (size_t)wave * per_wave;
  float* s_grad = s_vox + (size_t)(L + 1) * slot;
  int* s_boff = reinterpret_cast<int*>(s_grad + (size_t)(L + 1) * slot);
  float* s_T = reinterpret_cast<float*>(s_boff + 64);
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    s_tf[i] = a.tf[i];
    s_gtf[4 * i] = s_gtf[4 * i + 1] = s_gtf[4 * i + 2] = s_gtf[4 * i + 3] = 0.0;
  }
  __syncthreads();

  // same tile order as the forward
  const int ngroups_b = (a.ntiles + wpb - 1) / wpb;
  int grp;
  if (ba.band[8] > 0) {
    const int x = (int)(blockIdx.x & 7), g = ba.band[x] + (int)(blockIdx.x >> 3);
    grp = g < ba.band[x + 1] ? g : ngroups_b;
  } else {
    grp = (int)(blockIdx.x & 7) * ((ngroups_b + 7) >> 3) + (int)(blockIdx.x >> 3);
  }
  const int tile = grp < ngroups_b ? grp * wpb + wave : a.ntiles;
  const bool tile_on = tile < a.ntiles;
  // every wavefront reaches the workgroup barrier at the end, so the work
  // sits inside `if (tile_on)` rather than behind an early return
  if (tile_on) {
    const DevBrickView bvw = a.bv[0];
    const DevBrick br = a.bricks[0];
    const int tx = tile % bvw.tiles_x, ty = tile / bvw.tiles_x;
    const int lx = tx * 8 + (lane & 7), ly = ty * 8 + (lane >> 3);
    const bool valid = lx < bvw.w && ly < bvw.h;
    const int u = bvw.x0 + min(lx, bvw.w - 1), v = bvw.y0 + min(ly, bvw.h - 1);
    const int pix = ly * bvw.w + lx;

    // ---- ray setup, frame and layer range: as the forward ring march
    const double* d = a.cam.e3;
    double o[3];
    pixel_origin(a.cam, u, v, o);
    int cnt = 0;
    float px = 0.f, py = 0.f, pz = 0.f;
    double p0[3] = {0.0, 0.0, 0.0};
    const double sv[3] = {a.step * d[0], a.step * d[1], a.step * d[2]};
    double tin;
    int64_t n;
    if (valid && ray_lattice(o, d, a.hi, a.step, tin, n)) {
      int64_t k0, k1;
      brick_krange(o, d, tin, a.step, n, br.lo, br.hi, br.closed, k0, k1);
      if (k1 > k0) {
        const double t0 = tin + ((double)k0 + 0.5) * a.step;
        for (int i = 0; i < 3; i++) p0[i] = o[i] + t0 * d[i] - (double)br.lo[i];
        px = (float)p0[0];
        py = (float)p0[1];
        pz = (float)p0[2];
        cnt = (int)(k1 - k0);
      }
    }
    const float sx = (float)(a.step * d[0]), sy = (float)(a.step * d[1]), sz = (float)(a.step * d[2]);
    const bool by = a.slab_axis == 1;
    const float pb = by ? py : pz, sb = by ? sy : sz;
    const int cloB = by ? br.clo[1] : br.clo[2], chiB = by ? br.chi[1] : br.chi[2];
    const int cloG = by ? br.clo[2] : br.clo[1], chiG = by ? br.chi[2] : br.chi[1];
    const int cloF = br.clo[0], chiF = br.chi[0];
    const double db = by ? d[1] : d[2], dg = by ? d[2] : d[1];
    const bool up = db > 0.0;
    int c_first = up ? 0x7fffffff : -0x7fffffff, c_last = up ? -0x7fffffff : 0x7fffffff;
    if (cnt > 0) {
      c_first = (int)floorf(__builtin_amdgcn_fmed3f(pb, (float)cloB, (float)chiB));
      c_last = (int)floorf(__builtin_amdgcn_fmed3f(fmaf((float)(cnt - 1), sb, pb), (float)cloB, (float)chiB));
    }
    int Lbeg, Lend;
    if (up) {
      Lbeg = uni(wave_imin(c_first));
      Lend = uni(wave_imax(c_last));
    } else {
      Lbeg = uni(wave_imax(c_first));
      Lend = uni(wave_imin(c_last));
    }
    if (!(up ? Lbeg > Lend : Lbeg < Lend)) {
      const int nlay = up ? Lend - Lbeg + 1 : Lbeg - Lend + 1;
      const int vstep = up ? 1 : -1;
      const int V0 = up ? Lbeg : Lbeg + 1;  // voxel layer V_k = V0 + k vstep
      // window geometry from the tile's corner rays (lanes 0..3)
      const double rfd = d[0] / db, rgd = dg / db;
      const float rf = (float)rfd, rg = (float)rgd;
      float Af, Ag;
      {
        const int cx = bvw.x0 + tx * 8, cy = bvw.y0 + ty * 8;
        const int ex = min(cx + 7, bvw.x0 + bvw.w - 1), ey = min(cy + 7, bvw.y0 + bvw.h - 1);
        const int cc = lane & 3;
        double oc[3];
        pixel_origin(a.cam, (cc & 1) ? ex : cx, (cc & 2) ? ey : cy, oc);
        const double ob = (by ? oc[1] : oc[2]) - (double)(by ? br.lo[1] : br.lo[2]);
        Af = (float)(oc[0] - (double)br.lo[0] - ob * rfd);
        Ag = (float)((by ? oc[2] : oc[1]) - (double)(by ? br.lo[2] : br.lo[1]) - ob * rgd);
      }
      const float Af_lo = unif(wmin4(Af)), Af_hi = unif(wmax4(Af));
      const float Ag_lo = unif(wmin4(Ag)), Ag_hi = unif(wmax4(Ag));
      const float arf = fabsf(rf), arg = fabsf(rg);
      const int NF = uni((int)floorf(Af_hi - Af_lo + 2.f * arf + 0.2f) + 3);
      const int pitch = (NF + 3) & ~3;
      int NG = uni((int)floorf(Ag_hi - Ag_lo + 2.f * arg + 0.2f) + 3);
      NG = min(NG, chiG + 2 - cloG);
      const int ysl = br.sy, zsl = br.sz;
      const int sB = by ? ysl : zsl, sG = by ? zsl : ysl;
      gfloat* gbase = (gfloat*)br.base;
      float* gvol = ba.gvol;  // whole volume: brick-local == global
      const bool inl = !(pitch > chiF + 2 - cloF || pitch * NG > slot || pitch > 256 ||
                         ((int64_t)(64 / (pitch >> 2)) * sG + pitch) * 4 >= ((int64_t)1 << 32));
      auto window = [&](int V) {
        Window w;
        const float Pf = (float)V * rf, Pg = (float)V * rg;
        const int flo = max((int)floorf(Af_lo + Pf - arf - 0.05f), cloF);
        const int glo = max((int)floorf(Ag_lo + Pg - arg - 0.05f), cloG);
        w.f0 = uni(max(cloF, min(flo, chiF + 2 - pitch)));
        w.g0 = uni(max(cloG, min(glo, chiG + 2 - NG)));
        return w;
      };
      const int nf4 = pitch >> 2;
      const int R = uni(64 / max(nf4, 1));
      const int rl = lane / max(nf4, 1), c4l = lane - rl * nf4;
      const bool lane_on = rl < R;
      const int nload = uni((NG + R - 1) / max(R, 1));
      const unsigned voff = (unsigned)(rl * sG + 4 * c4l) * 4u;
      const int64_t gstep = (int64_t)R * sG;
      const unsigned lstep = (unsigned)(R * pitch) * 4u;
      auto issue = [&](int V, const Window& w, float* sdst) {
        gfloat* gb = gbase + ((int64_t)V * sB + (int64_t)w.g0 * sG + w.f0);
        const unsigned l0 = uni(lds_addr(sdst));
        for (int k = 0; k < nload; ++k)
          if (lane_on && k * R + rl < NG) lds_dma16(unip(gb + k * gstep), voff, l0 + (unsigned)k * lstep);
      };

      // per-ray state of the backward walk
      const int used = valid ? ba.nused[pix] : 0;
      const float4 gf = valid ? ba.gout[pix] : make_float4(0.f, 0.f, 0.f, 0.f);
      const double gx = gf.x, gy = gf.y, gz = gf.z, gw = gf.w;
      const double dvs = (double)(M - 1) * ba.inv_range;  // du/dv inside the window
      double R0 = 0.0, R1 = 0.0, R2 = 0.0, Q = 0.0;
      const int ngrp = (nlay + L - 1) / L;
      const int npix = ba.npix;
      // Consecutive samples of a ray mostly fall in the same table interval and
      // often in the same cell: their table- and voxel-gradient terms are summed
      // in registers and added to LDS once per run (far fewer atomics on the
      // few table entries every lane of the tile hits)
      int ti = -1;  // table interval of the pending sums
      float run_tf[8];  // a run is a few samples: float sums lose nothing the tolerance sees
      auto flush_tf = [&]() {
        if (ti >= 0) {
          double* e0 = s_gtf + 4 * ti;
          for (int q = 0; q < 8; ++q) atomicAdd(e0 + q, (double)run_tf[q]);
          ti = -1;
        }
      };
      int vl = -1, vu = -1;  // LDS offsets of the pending cell's lower and upper corner rows
      float va[8];
      auto flush_vox = [&]() {
        if (vl >= 0) {
          float* p = s_grad + vl;
          float* q = s_grad + vu;
          if (by) {  // dy selects the layer, dz the row
            atomicAdd(p, va[0]); atomicAdd(p + 1, va[1]); atomicAdd(q, va[2]); atomicAdd(q + 1, va[3]);
            atomicAdd(p + pitch, va[4]); atomicAdd(p + pitch + 1, va[5]);
            atomicAdd(q + pitch, va[6]); atomicAdd(q + pitch + 1, va[7]);
          } else {   // dz selects the layer, dy the row
            atomicAdd(p, va[0]); atomicAdd(p + 1, va[1]); atomicAdd(p + pitch, va[2]);
            atomicAdd(p + pitch + 1, va[3]); atomicAdd(q, va[4]); atomicAdd(q + 1, va[5]);
            atomicAdd(q + pitch, va[6]); atomicAdd(q + pitch + 1, va[7]);
          }
          vl = -1;
        }
      };

      // Voxel layer V_m lives in slot m % (L + 1) for every group, so the layer
      // two consecutive groups share (V_{k0} of a group, V_{k1} of the one
      // before it, which is taken next) keeps its voxel window and its gradient
      // window: it is neither reloaded nor cleared there, and flushed once,
      // with both groups' terms, by the group taken later.
      auto pslot = [&](int m) { return m % (L + 1); };
      for (int g = ngrp - 1; g >= 0; --g) {
        const int k0 = g * L, k1 = min(nlay, k0 + L);  // cell layers k0 .. k1 - 1
        const int nv = k1 - k0 + 1;                     // voxel layers V_{k0} .. V_{k1}
        const bool shared_top = g + 1 < ngrp;           // V_{k1} kept from group g + 1
        if (inl) {
          for (int i = 0; i < nv; ++i) {
            const Window w = window(V0 + (k0 + i) * vstep);
            const int ps = pslot(k0 + i);
            if (!(shared_top && i == nv - 1)) {
              issue(V0 + (k0 + i) * vstep, w, s_vox + ps * slot);
              for (int e = lane; e < slot; e += 64) s_grad[ps * slot + e] = 0.f;
            }
            if (lane == 0) s_boff[i] = ps * slot - w.g0 * pitch - w.f0;
          }
          wait_loads();  // also orders the clears and offsets above
        }
        // this ray's samples in the group: [js, je), at most `used`
        int js = 0, je = 0;
        double T = 1.0;
        if (valid) {
          js = ba.ckpt_j[(int64_t)g * npix + pix];
          je = g + 1 < ngrp ? ba.ckpt_j[(int64_t)(g + 1) * npix + pix] : cnt;
          je = min(je, used);
          T = (double)ba.ckpt[(int64_t)g * npix + pix];
          // the plan bounds a ray's samples in one group by smax (L layers
          // at one step each); a group beyond it is flagged, not clamped
          if (je - js > smax) {
            atomicOr(ba.flag, 1);
            je = js + smax;
          }
        }
        // cell of sample j and its eight corners, from the windows when both of
        // its voxel layers are in the group's slots (always, up to rounding at
        // a layer boundary), else from global memory; lofs/uofs: LDS offsets of
        // the lower and upper corner rows, -1 for global
        auto corners = [&](int j, CellD& c, float (&vv)[8], int& lofs, int& uofs) {
          c = cell_d(j, p0, sv, br);
          lofs = uofs = -1;
          if (inl) {
            const int ib = by ? c.iy : c.iz, ig = by ? c.iz : c.iy;
            const int kc = up ? ib - Lbeg : Lbeg - ib;  // cell layer index
            const int sl = (up ? kc : kc + 1) - k0, su = (up ? kc + 1 : kc) - k0;
            if (sl >= 0 && sl < nv && su >= 0 && su < nv) {
              lofs = s_boff[sl] + __mul24(ig, pitch) + c.ix;
              uofs = s_boff[su] + __mul24(ig, pitch) + c.ix;
              const float* p = s_vox + lofs;
              const float* q = s_vox + uofs;
              if (by) {  // rows along z inside a window, layers along y
                vv[0] = p[0]; vv[1] = p[1]; vv[2] = q[0]; vv[3] = q[1];
                vv[4] = p[pitch]; vv[5] = p[pitch + 1]; vv[6] = q[pitch]; vv[7] = q[pitch + 1];
              } else {   // rows along y, layers along z
                vv[0] = p[0]; vv[1] = p[1]; vv[2] = p[pitch]; vv[3] = p[pitch + 1];
                vv[4] = q[0]; vv[5] = q[1]; vv[6] = q[pitch]; vv[7] = q[pitch + 1];
              }
              return;
            }
          }
          gfloat* p = gbase + (c.iz * zsl + c.iy * ysl + c.ix);
          vv[0] = p[0]; vv[1] = p[1]; vv[2] = p[ysl]; vv[3] = p[ysl + 1];
          vv[4] = p[zsl]; vv[5] = p[zsl + 1]; vv[6] = p[zsl + ysl]; vv[7] = p[zsl + ysl + 1];
        };
        // replay: T before each sample of the group
        for (int j = js; j < je; ++j) {
          CellD c;
          float vv[8];
          int lofs, uofs;
          corners(j, c, vv, lofs, uofs);
          const Eval S = eval_d(vv, c, ba.vmin, ba.inv_range, M, s_tf);
          s_T[(j - js) * 64 + lane] = (float)T;
          T = fma(-T, S.a, T);
        }
        // backward walk
        for (int j = je - 1; j >= js; --j) {
          CellD c;
          float vv[8];
          int lofs, uofs;
          corners(j, c, vv, lofs, uofs);
          const Eval S = eval_d(vv, c, ba.vmin, ba.inv_range, M, s_tf);
          const double Tp = (double)s_T[(j - js) * 64 + lane];
          const double ta = Tp * S.a;
          const double gr = gx * ta, gg = gy * ta, gb = gz * ta;
          const double ga = Tp * (gx * (S.r - R0) + gy * (S.g - R1) + gz * (S.b - R2) + gw * (1.0 - Q));
          const double om = 1.0 - S.a;
          R0 = fma(S.a, S.r, om * R0);
          R1 = fma(S.a, S.g, om * R1);
          R2 = fma(S.a, S.b, om * R2);
          Q = fma(om, Q, S.a);
          const double w1 = S.w, w0 = 1.0 - S.w;
          if (S.i != ti) {
            flush_tf();
            ti = S.i;
            for (int q = 0; q < 8; ++q) run_tf[q] = 0.f;
          }
          run_tf[0] += (float)(w0 * gr);
          run_tf[1] += (float)(w0 * gg);
          run_tf[2] += (float)(w0 * gb);
          run_tf[3] += (float)(w0 * ga);
          run_tf[4] += (float)(w1 * gr);
          run_tf[5] += (float)(w1 * gg);
          run_tf[6] += (float)(w1 * gb);
          run_tf[7] += (float)(w1 * ga);
          if (gvol && S.sraw > 0.0 && S.sraw < 1.0) {
            const float4 t0f = s_tf[S.i], t1f = s_tf[S.i + 1];
            const double du = gr * ((double)t1f.x - (double)t0f.x) + gg * ((double)t1f.y - (double)t0f.y) +
                              gb * ((double)t1f.z - (double)t0f.z) + ga * ((double)t1f.w - (double)t0f.w);
            const double gv = du * dvs;
            if (gv != 0.0) {
              const double x1 = S.wx, x0 = 1.0 - S.wx, y1 = S.wy, y0 = 1.0 - S.wy, z1 = S.wz, z0 = 1.0 - S.wz;
              // corner weights in v[dz][dy][dx] order
              const float cw[8] = {(float)(gv * x0 * y0 * z0), (float)(gv * x1 * y0 * z0), (float)(gv * x0 * y1 * z0),
                                   (float)(gv * x1 * y1 * z0), (float)(gv * x0 * y0 * z1), (float)(gv * x1 * y0 * z1),
                                   (float)(gv * x0 * y1 * z1), (float)(gv * x1 * y1 * z1)};
              if (lofs >= 0) {
                if (lofs != vl) {
                  flush_vox();
                  vl = lofs;
                  vu = uofs;
                  for (int q = 0; q < 8; ++q) va[q] = 0.f;
                }
                for (int q = 0; q < 8; ++q) va[q] += cw[q];
              } else {
                float* q = gvol + (c.iz * zsl + c.iy * ysl + c.ix);
                unsafeAtomicAdd(q, cw[0]);
                unsafeAtomicAdd(q + 1, cw[1]);
                unsafeAtomicAdd(q + ysl, cw[2]);
                unsafeAtomicAdd(q + ysl + 1, cw[3]);
                unsafeAtomicAdd(q + zsl, cw[4]);
                unsafeAtomicAdd(q + zsl + 1, cw[5]);
                unsafeAtomicAdd(q + zsl + ysl, cw[6]);
                unsafeAtomicAdd(q + zsl + ysl + 1, cw[7]);
              }
            }
          }
        }
        flush_vox();
        // add the group's gradient windows to the volume: rows contiguous along axis 1
        if (inl && gvol) {
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
          const float inv_pitch = 1.0f / (float)pitch;
          for (int i = g > 0 ? 1 : 0; i < nv; ++i) {  // V_{k0} goes on into group g - 1
            const Window w = window(V0 + (k0 + i) * vstep);
            float* gl = gvol + ((int64_t)(V0 + (k0 + i) * vstep) * sB + (int64_t)w.g0 * sG + w.f0);
            const float* sg = s_grad + pslot(k0 + i) * slot;
            for (int e = lane; e < NG * pitch; e += 64) {
              const float val = sg[e];
              if (val != 0.f) {
                const int r = (int)(((float)e + 0.5f) * inv_pitch), col = e - r * pitch;
                unsafeAtomicAdd(gl + ((int64_t)r * sG + col), val);
              }
            }
          }
        }
        // the next group reuses the windows: every lane is done with them
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      }
      flush_tf();
    }
  }
  __syncthreads();
  double* part = ba.tf_part + (int64_t)blockIdx.x * M * 4;
  for (int i = threadIdx.x; i < M * 4; i += blockDim.x) part[i] = s_gtf[i];
}

}  // namespace

size_t bwd_ring_lds_bytes(const MarchArgs& a, const BwdArgs& ba, int wpb) {
  const size_t per_wave = (size_t)2 * (ba.K + 1) * a.ring_slot + 64 + (size_t)ba.smax * 64;
  return sizeof(double) * 4 * (size_t)a.M + sizeof(float4) * (size_t)a.M + sizeof(float) * wpb * per_wave;
}

int bwd_ring_blocks(const MarchArgs& a, const BwdArgs& ba, int wpb) {
  if (a.ntiles <= 0) return 0;
  if (ba.band[8] > 0) {
    int widest = 0;
    for (int x = 0; x < 8; x++) widest = std::max(widest, ba.band[x + 1] - ba.band[x]);
    return 8 * widest;
  }
  const int groups = (a.ntiles + wpb - 1) / wpb;
  return ((groups + 7) / 8) * 8;
}

hipError_t launch_bwd_ring(const MarchArgs& a, const BwdArgs& ba, int wpb, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  if (a.tile_w != 8 || a.ring_slot <= 0 || (a.ring_slot & 3) != 0 || (wpb != 1 && wpb != 2 && wpb != 4) ||
      a.cam.persp != 0 || ba.K < 1 || ba.smax < 1 || !ba.ckpt_j)
    return hipErrorInvalidValue;
  const size_t lds = bwd_ring_lds_bytes(a, ba, wpb);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  static bool attr_set = false;  // dynamic LDS beyond the default limit (up to 160 KB)
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bwd_ring),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_bwd_ring, dim3(bwd_ring_blocks(a, ba, wpb)), dim3(64 * wpb), lds, s, a, ba);
  return hipGetLastError();
}

}  // namespace vr
