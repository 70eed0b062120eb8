// ring_common.h -- device helpers shared by the ring-window kernels (the
// forward ring march and the ring adjoint): uniform-value helpers, wave
// reductions, the direct global->LDS load and its wait, and the window record.
#pragma once

#include "vr_internal.h"

namespace vr {
namespace ring {

typedef const float __attribute__((address_space(1))) gfloat;

__device__ __forceinline__ float wmin4(float v) {
  v = fminf(v, __shfl_xor(v, 1));
  return fminf(v, __shfl_xor(v, 2));
}
__device__ __forceinline__ float wmax4(float v) {
  v = fmaxf(v, __shfl_xor(v, 1));
  return fmaxf(v, __shfl_xor(v, 2));
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
// a pointer the compiler must treat as uniform (it lives in scalar registers)
__device__ __forceinline__ gfloat* unip(gfloat* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (gfloat*)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float unif(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
// wave vote known to the compiler as uniform
__device__ __forceinline__ bool wany(bool p) { return uni(__any(p) ? 1 : 0) != 0; }
// value of v in lane l (uniform)
__device__ __forceinline__ float lanef(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Wait until every global->LDS load this wavefront issued has landed (the
// memory clobber keeps LDS reads from moving above the wait).
__device__ __forceinline__ void wait_loads() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// 16 bytes per lane from global memory (base + voff bytes; base uniform, voff
// per lane) straight into LDS at lds_base + 16 lane (a byte address, uniform
// over the wavefront).  Written as inline assembly so that the compiler does
// not guard later LDS reads with waits for these loads: the code waits for
// them explicitly with wait_loads().  The kernel keeps no value of its own in
// M0 (it uses no instruction that reads M0 besides this one).
__device__ __forceinline__ void lds_dma16(gfloat* base, unsigned voff, unsigned lds_base) {
  asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1"
               :
               : "v"(voff), "s"(base), "s"(lds_base)
               : "memory", "m0");
}

__device__ __forceinline__ unsigned lds_addr(const float* p) {
  return (unsigned)(uintptr_t)(const __attribute__((address_space(3))) float*)p;
}

// Window of one voxel layer: rows along axis 1 (f), `pitch` floats each, NG rows
// along the in-plane axis g; origin (f0, g0) in brick-local voxel indices.
struct Window {
  int f0, g0;
  int fb, gb;  // perspective cells: last column and row (origin-relative) the layer's samples can read
};

// ---------------------------------------------------------------- footprint cells

// Pixels of footprint cell (ci, cj) of a brick: lane r holds the run of image
// row vrow0 + r that falls in the cell (first column u0, inclusive and
// exclusive counts over the rows before it); n = pixels in the cell.
struct FootRuns {
  int vrow0, u0, incl, excl, n;
};

__device__ inline FootRuns foot_runs(const MarchArgs& a, const DevBrickView& bvw, int ci, int cj, int lane) {
  FootRuns fr;
  const double au = a.fa_u, av = a.fa_v, bu = a.fb_u, bvv = a.fb_v;
  const double det = au * bvv - av * bu;
  // image rows the cell's corners span (one row of margin each side)
  double vmn = INFINITY, vmx = -INFINITY;
  for (int q = 0; q < 4; ++q) {
    const double ra = (double)(ci + (q & 1)) - bvw.fa0, rb = (double)(cj + (q >> 1)) - bvw.fb0;
    const double vq = (au * rb - bu * ra) / det;
    vmn = fmin(vmn, vq);
    vmx = fmax(vmx, vq);
  }
  fr.vrow0 = uni(max(0, (int)floor(vmn) - 1));
  const int vlast = uni(min(a.cam.H - 1, (int)ceil(vmx) + 1));
  const int vrow = fr.vrow0 + lane;
  int cnt_row = 0;
  fr.u0 = 0;
  if (vrow <= vlast) {
    // columns u in [0, W) of row vrow whose cell coordinate lies in
    // [cell, cell + 1): one run, the coordinate being monotone along the row
    auto run = [&](double c0, double su, double sv, int cell, int& lo_u, int& hi_u) {
      const int Wm = a.cam.W;
      if (su == 0.0) {
        const double x = foot_cell_coord(c0, su, sv, 0, vrow);
        const bool in = x >= (double)cell && x < (double)(cell + 1);
        lo_u = in ? 0 : 1;
        hi_u = in ? Wm - 1 : 0;
        return;
      }
      const bool inc = su > 0.0;
      int l = 0, h = Wm;  // first column past the cell's near edge
      while (l < h) {
        const int m = (l + h) >> 1;
        const double x = foot_cell_coord(c0, su, sv, m, vrow);
        if (inc ? x >= (double)cell : x < (double)(cell + 1)) h = m;
        else l = m + 1;
      }
      lo_u = l;
      l = 0;
      h = Wm;  // first column past the cell's far edge
      while (l < h) {
        const int m = (l + h) >> 1;
        const double x = foot_cell_coord(c0, su, sv, m, vrow);
        if (inc ? x >= (double)(cell + 1) : x < (double)cell) h = m;
        else l = m + 1;
      }
      hi_u = l - 1;
    };
    int fl, fh, gl, gh;
    run(bvw.fa0, au, av, ci, fl, fh);
    run(bvw.fb0, bu, bvv, cj, gl, gh);
    fr.u0 = max(fl, gl);
    cnt_row = max(0, min(fh, gh) - fr.u0 + 1);
  }
  fr.incl = cnt_row;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(fr.incl, off);
    if (lane >= off) fr.incl += y;
  }
  fr.excl = fr.incl - cnt_row;
  fr.n = uni(__builtin_amdgcn_readlane(fr.incl, 63));
  return fr;
}

// Perspective views: the pixels of cell (ci, cj) of a brick are those whose
// rays cross the brick-local plane b = 0 inside [ci Tf, (ci + 1) Tf) x
// [cj Tg, (cj + 1) Tg) (persp_plane_point).  Along an image row inside the
// brick's rectangle each plane coordinate is a monotone function of the
// column (a ratio of two linear functions whose denominator keeps its sign
// there), so the cell's pixels of a row are again one run, found by
// bisection; the rows are those of the cell's corners seen from the eye.
__device__ inline FootRuns foot_runs_persp(const MarchArgs& a, const DevBrickView& bvw, const DevBrick& br, int ci,
                                           int cj, int lane) {
  FootRuns fr;
  const int b = a.slab_axis == 1 ? 1 : 2, g = 3 - b;
  double E[3];
  for (int i = 0; i < 3; ++i) E[i] = a.cam.eye[i] - (double)br.lo[i];
  const double F0 = (double)ci * bvw.pTf, F1 = (double)(ci + 1) * bvw.pTf;
  const double G0 = (double)cj * bvw.pTg, G1 = (double)(cj + 1) * bvw.pTg;
  double vmn = INFINITY, vmx = -INFINITY;
  for (int q = 0; q < 4; ++q) {
    double r[3], uq, vq;
    r[0] = ((q & 1) ? F1 : F0) - E[0];
    r[g] = ((q & 2) ? G1 : G0) - E[g];
    r[b] = -E[b];
    persp_image_uv(a.cam, r, uq, vq);
    vmn = fmin(vmn, vq);
    vmx = fmax(vmx, vq);
  }
  // rows of the cell inside the brick's rectangle; at most 64 (the plan
  // bounds a cell's rows well below that)
  fr.vrow0 = uni(max(bvw.y0, (int)floor(vmn) - 1));
  const int vlast = uni(min(min(bvw.y0 + bvw.h - 1, (int)ceil(vmx) + 1), fr.vrow0 + 63));
  const int vrow = fr.vrow0 + lane;
  int cnt_row = 0;
  fr.u0 = 0;
  if (vrow <= vlast) {
    const int ul = bvw.x0, uh = bvw.x0 + bvw.w;  // columns [ul, uh)
    auto coord = [&](int u, bool along_f) {
      double pf, pg;
      persp_plane_point(a.cam, E, b, g, (double)u, (double)vrow, pf, pg);
      return along_f ? pf / bvw.pTf : pg / bvw.pTg;
    };
    auto run = [&](bool along_f, int cell, int& lo_u, int& hi_u) {
      const double x0 = coord(ul, along_f), x1 = coord(uh - 1, along_f);
      if (x1 == x0) {
        const bool in = x0 >= (double)cell && x0 < (double)(cell + 1);
        lo_u = in ? ul : uh;
        hi_u = in ? uh - 1 : ul - 1;
        return;
      }
      const bool inc = x1 > x0;
      int l = ul, h = uh;  // first column past the cell's near edge
      while (l < h) {
        const int m = (l + h) >> 1;
        const double x = coord(m, along_f);
        if (inc ? x >= (double)cell : x < (double)(cell + 1)) h = m;
        else l = m + 1;
      }
      lo_u = l;
      l = ul;
      h = uh;  // first column past the cell's far edge
      while (l < h) {
        const int m = (l + h) >> 1;
        const double x = coord(m, along_f);
        if (inc ? x >= (double)(cell + 1) : x < (double)cell) h = m;
        else l = m + 1;
      }
      hi_u = l - 1;
    };
    int fl, fh, gl, gh;
    run(true, ci, fl, fh);
    run(false, cj, gl, gh);
    fr.u0 = max(fl, gl);
    cnt_row = max(0, min(fh, gh) - fr.u0 + 1);
  }
  fr.incl = cnt_row;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(fr.incl, off);
    if (lane >= off) fr.incl += y;
  }
  fr.excl = fr.incl - cnt_row;
  fr.n = uni(__builtin_amdgcn_readlane(fr.incl, 63));
  return fr;
}

// Pixel k (0 <= k < n) of the cell: the row is the first whose inclusive count
// exceeds k.  Every lane takes part (cross-lane reads).
__device__ __forceinline__ void foot_pixel(const FootRuns& fr, int k, int& u, int& v) {
  int r = 0;
  for (int stp = 32; stp > 0; stp >>= 1)
    if (__shfl(fr.incl, r + stp - 1) <= k) r += stp;
  r = min(r, 63);
  u = __shfl(fr.u0, r) + (k - __shfl(fr.excl, r));
  v = fr.vrow0 + r;
}

// Footprint cell of work item t of a brick view.
__device__ __forceinline__ void foot_cell(const DevBrickView& bvw, int t, int& ci, int& cj) {
  ci = bvw.cf0 + t % bvw.tiles_x;
  cj = bvw.cg0 + t / bvw.tiles_x;
}

// Footprint cell of wavefront w of work item t when work items are blocks of
// blk_f x blk_g cells (wavefronts along f first).
__device__ __forceinline__ void block_cell(const MarchArgs& a, const DevBrickView& bvw, int t, int w, int& ci,
                                           int& cj) {
  const int bi = t % bvw.blocks_x, bj = t / bvw.blocks_x;
  ci = bvw.cf0 + bi * a.blk_f + w % a.blk_f;
  cj = bvw.cg0 + bj * a.blk_g + w / a.blk_f;
}

__device__ __forceinline__ int find_bv(const MarchArgs& a, int tile) {
  int lo = 0, hi = a.nbv - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.bv[mid].tile_begin <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace ring
}  // namespace vr
