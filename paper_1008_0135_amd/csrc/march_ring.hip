// march_ring.hip -- forward march with per-layer voxel windows kept in an LDS
// ring and filled by direct global->LDS loads (gfx950).
//
// Same samples, same per-sample arithmetic and the same order as the gather
// march (paper Sec. 2.4: each ray is sampled between its entry and exit points
// and accumulated front to back with early termination); only the way the
// eight trilinear corners reach the lanes differs.
//
// A wavefront owns an 8 x 8 tile of pixel rays inside one brick and walks the
// brick one cell layer at a time along a slab axis b (y or z, chosen per view
// on the host so that rows along x -- the contiguous storage axis -- stay
// long).  Cell layer c is sampled from voxel layers c and c + 1.  For every
// voxel layer V the wavefront loads a window of rows along x: the box that
// holds the cells of every sample of its 64 rays lying between the planes
// b = V - 1 and b = V + 1, bounded from the four corner rays of the tile (the
// rays are parallel, so the corners bound the bundle on any plane).  Windows
// go into a ring of three LDS slots: while cell layer c is sampled from the
// slots of V = c and c + 1, the window of the layer after next is already in
// flight (global_load_lds_dwordx4: 16 bytes per lane straight into LDS, no
// registers, no store instructions).  Every voxel layer is read once per
// tile, with no halo layer read twice.
//
// The layer index, the window origins and the slot addresses are uniform over
// the wavefront (scalar registers); lanes step through their own samples of
// the current layer (two to three on typical views).  Four wavefronts share a
// workgroup only to share the transfer-function table in LDS; after loading it
// each wavefront runs on its own, with no workgroup barrier.
//
// Carried state (a.carry, opacity tested over the whole ray): the image is the
// output frame holding each ray's (C, T) from the bricks in front of this
// one; a ray starts from it (and not at all once 1 - T >= tau) and leaves its
// new state there.
//
// Perspective views (PERSP): the tile's rays leave one eye, so their
// directions are positive combinations of the four corner directions; when
// the corner rays all move the same way along b, every ray of the tile meets
// a plane b = P inside the range the corner rays span there, and the window
// of layer V is the box of the four corner lines over [V - 1, V + 1] (its size
// grows with depth: the bound is taken at the tile's first and last layer,
// where the convex width is largest).  A tile whose corner rays disagree on
// the direction along b samples from global memory.
#include <cstring>

#include "ring_common.h"
#include "sample.h"
#include "vr_internal.h"

namespace vr {

namespace {

using namespace ring;

constexpr int kSlotsMax = 3;

// SAVE (differentiable forward, whole volume): also store, for every group of
// sa.K cell layers of the tile (in marching order), each ray's transmittance
// and sample cursor at the group's start, and the samples applied per ray.
// MIP: maximum intensity projection (no table, no skipping, no saving).
// REG (two slots, perspective views): the window of the layer after next is
// loaded into registers while the current cell layer is sampled and written
// over the finished layer afterwards, for tiles whose window takes at most
// kRingRegLoads loads per lane (the others load straight into LDS), so every
// wavefront keeps a layer in flight without a third slot.
template <bool ESS, bool SAVE, bool MIP, bool PERSP, bool TWO = false, bool MASK = false, bool REG = false>
__global__ __launch_bounds__(256) void k_march_ring(MarchArgs a, SaveArgs sa) {
  static_assert(!(PERSP && SAVE), "the checkpointing forward is orthographic");
  static_assert(!TWO || !(ESS || SAVE), "two slots: the plain march");
  static_assert(!(MASK && (SAVE || TWO)), "the channel mask: three-slot forward marches");
  static_assert(!REG || TWO, "registers stage the third layer of a two-slot ring");
  constexpr int kSlots = TWO ? 2 : 3;
  extern __shared__ float4 smem[];
  float4* s_tf = smem;
  for (int i = threadIdx.x; i < a.M; i += blockDim.x) s_tf[i] = a.tf[i];
  __syncthreads();

  const int wpb = (int)(blockDim.x >> 6);
  const int wave = uni((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int slot = a.ring_slot;  // floats per ring slot
  float* s_ring = reinterpret_cast<float*>(smem + a.M) + (size_t)wave * kSlots * slot;

  // XCD-aware order: workgroup b runs on XCD b % 8; give each XCD a
  // contiguous range of tiles so that neighbouring tiles share its L2
  const int ngroups = (a.ntiles + wpb - 1) / wpb;
  const int per = (ngroups + 7) >> 3;
  int grp = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (SAVE && sa.band[8] > 0) {
    // the checkpointing forward: bands of equal estimated work per XCD
    const int x = (int)(blockIdx.x & 7), g = sa.band[x] + (int)(blockIdx.x >> 3);
    grp = g < sa.band[x + 1] ? g : ngroups;
  }
  const int tile = grp * wpb + wave;
  if (tile >= a.ntiles) return;

  int lo = 0, hi = a.nbv - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.bv[mid].tile_begin <= tile) lo = mid;
    else hi = mid - 1;
  }
  const DevBrickView bvw = a.bv[lo];
  const DevBrick br = a.bricks[bvw.brick];
  const int t = tile - bvw.tile_begin;
  // Footprint cells (parallel rays): the wavefront's rays are the pixels whose
  // rays cross the brick-local plane b = 0 inside cell (ci, cj) of the
  // Tf x Tg grid in (f, g).  Each image row holds one run of them (the cell
  // coordinate is monotone along a row); lane r measures the run of row
  // vrow0 + r, and a wave scan numbers the cell's pixels row by row.  The
  // wavefront marches the cell's first 64 pixels.
  const bool foot = !PERSP && !SAVE && a.foot != 0;
  int ci = 0, cj = 0;
  FootRuns fr;
  int tx = 0, ty = 0;
  if (foot) {
    foot_cell(bvw, t, ci, cj);
    fr = foot_runs(a, bvw, ci, cj, lane);
    // cells of more than 64 pixels: the pixels past the 64th are marched by
    // k_march_ring_ovf after this launch
    if (fr.n > 64 && lane == 0) a.ovf_tiles[atomicAdd(a.ovf_count, 1u)] = tile * 8;
  } else {
    // tile numbering inside the brick's rectangle.  Tiles started together run
    // at about the same layer; the L2 keeps a line only a few microseconds, so
    // lines two windows share (the partial 128-byte ends of rows, the halo
    // rows) are fetched once only when the two tiles are close in this order.
    // Blocks of tiles put neighbours on both image axes close, whichever way
    // the view turns the image against the storage axes.
    if (a.tile_order == 1) {
      const int th = (bvw.h + 7) >> 3;
      tx = t / th;
      ty = t - tx * th;
    } else if (a.tile_order == 2) {
      // blocks of bw x bh tiles in row order (tiles in a block in row order),
      // then the tiles right of the last whole block column, then those below
      // the last whole block row
      const int tw = bvw.tiles_x, th = (bvw.h + 7) >> 3, bw = a.tile_bw, bh = a.tile_bh;
      const int fw = tw / bw, fh = th / bh, nfull = fw * fh * bw * bh;
      if (t < nfull) {
        const int q = t / (bw * bh), r = t - q * (bw * bh), qy = q / fw;
        const int ry = r / bw;
        tx = (q - qy * fw) * bw + (r - ry * bw);
        ty = qy * bh + ry;
      } else {
        int r = t - nfull;
        const int rw = tw - fw * bw;
        if (r < rw * th) {
          ty = r / rw;
          tx = fw * bw + (r - ty * rw);
        } else {
          r -= rw * th;
          const int lw = fw * bw;
          const int ry = r / lw;
          tx = r - ry * lw;
          ty = fh * bh + ry;
        }
      }
    } else {
      ty = t / bvw.tiles_x;
      tx = t - ty * bvw.tiles_x;
    }
  }
  // the march of the wavefront's 64 rays (a single pass: early exits leave it)
  do {
  int lx, ly, u, v;
  bool valid;
  if (foot) {
    int ur, vr;
    foot_pixel(fr, lane, ur, vr);
    valid = lane < fr.n;
    u = valid ? ur : 0;
    v = valid ? vr : 0;
    lx = u - bvw.x0;
    ly = v - bvw.y0;
  } else {
    lx = tx * 8 + (lane & 7);
    ly = ty * 8 + (lane >> 3);
    valid = lx < bvw.w && ly < bvw.h;
    u = bvw.x0 + min(lx, bvw.w - 1);
    v = bvw.y0 + min(ly, bvw.h - 1);
  }
  // a footprint cell's pixel lies in the brick's rectangle whenever its ray
  // has samples here; the image arena (or output) was cleared before the
  // march, so only pixels with samples are written
  const bool inrect = lx >= 0 && lx < bvw.w && ly >= 0 && ly < bvw.h;

  // ---- per-lane ray setup (double precision, shared with every march)
  double o[3], dl[3];
  const double* d;
  if constexpr (PERSP) {
    pixel_ray(a.cam, u, v, o, dl);
    d = dl;
  } else {
    d = a.cam.e3;
    pixel_origin(a.cam, u, v, o);
  }
  int cnt = 0;
  float px = 0.f, py = 0.f, pz = 0.f;
  float4* const dst =
      a.carry ? a.img + (int64_t)v * a.cam.W + u : a.img + bvw.img_off + (int64_t)ly * bvw.w + lx;
  const bool wr_ok = a.carry || !foot || inrect;  // dst is this pixel's place
  float4 carried = make_float4(0.f, 0.f, 0.f, 1.f);
  if (a.carry && valid) carried = *dst;
  const bool live = !a.carry || 1.f - carried.w < a.tau;
  double tin;
  int64_t n;
  if (valid && live && ray_lattice(o, d, a.hi, a.step, tin, n)) {
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

  // range of four lines x = A[c] + P r[c] over the planes [P0, P1] (P0 <= P1)
  auto crange = [](const float* A, const float* r, float P0, float P1, float& lo, float& hi) {
    lo = INFINITY;
    hi = -INFINITY;
    for (int c = 0; c < 4; ++c) {
      const float x0 = fmaf(P0, r[c], A[c]), x1 = fmaf(P1, r[c], A[c]);
      lo = fminf(lo, fminf(x0, x1));
      hi = fmaxf(hi, fmaxf(x0, x1));
    }
  };

  // ---- frame: b = slab axis (axis 2 or 3), g = the other of axes 2/3, f = axis 1
  // PERSP: the corner rays of the tile (lane l holds corner l & 3) pick the
  // axis per tile: of the axes along which all four move the same way, the one
  // whose window over the brick's layers is smaller (rays from an eye turn
  // across the image, so no one axis suits every tile)
  bool by = a.slab_axis == 1;
  bool force_gather = false;
  double oc[3] = {0.0, 0.0, 0.0}, dc[3] = {0.0, 0.0, 1.0};
  if constexpr (PERSP) {
    const int cx = bvw.x0 + tx * 8, cy = bvw.y0 + ty * 8;
    const int ex = min(cx + 7, bvw.x0 + bvw.w - 1), ey = min(cy + 7, bvw.y0 + bvw.h - 1);
    const int cc = lane & 3;
    pixel_ray(a.cam, (cc & 1) ? ex : cx, (cc & 2) ? ey : cy, oc, dc);
    int pick = 0;
    int best = 0x7fffffff;
    for (int bb = 1; bb <= 2; ++bb) {
      const double dcb = dc[bb];
      const bool upb = uni(dcb > 0.0 ? 1 : 0) != 0;
      if (wany(!(fabs(dcb) > 1e-6) || (dcb > 0.0) != upb)) continue;
      const int gg = 3 - bb;
      const double rfd = dc[0] / dcb, rgd = dc[gg] / dcb;
      const double ob = oc[bb] - (double)br.lo[bb];
      const float A_f = (float)(oc[0] - (double)br.lo[0] - ob * rfd);
      const float A_g = (float)(oc[gg] - (double)br.lo[gg] - ob * rgd);
      float qA[4], qr[4], qB[4], qs[4];
      for (int c = 0; c < 4; ++c) {
        qA[c] = lanef(A_f, c);
        qr[c] = lanef((float)rfd, c);
        qB[c] = lanef(A_g, c);
        qs[c] = lanef((float)rgd, c);
      }
      const float Va = (float)br.clo[bb], Vb = (float)(br.chi[bb] + 1);
      float l0, h0, l1, h1;
      crange(qA, qr, Va - 1.f, Va + 1.f, l0, h0);
      crange(qA, qr, Vb - 1.f, Vb + 1.f, l1, h1);
      const float wf = fmaxf(h0 - l0, h1 - l1);
      crange(qB, qs, Va - 1.f, Va + 1.f, l0, h0);
      crange(qB, qs, Vb - 1.f, Vb + 1.f, l1, h1);
      const float wg = fmaxf(h0 - l0, h1 - l1);
      if (!(wf < 4096.f && wg < 4096.f)) continue;
      const int nf = (((int)floorf(wf + 0.2f) + 3) + 3) & ~3;
      const int ng = min((int)floorf(wg + 0.2f) + 3, br.chi[gg] + 2 - br.clo[gg]);
      const int size = uni(nf * ng);
      if (size < best) {
        best = size;
        pick = bb;
      }
    }
    if (pick == 0) force_gather = true;
    else by = uni(pick) == 1;
  }
  const float pb = by ? py : pz, sb = by ? sy : sz;
  const int cloB = by ? br.clo[1] : br.clo[2], chiB = by ? br.chi[1] : br.chi[2];
  const int cloG = by ? br.clo[2] : br.clo[1], chiG = by ? br.chi[2] : br.chi[1];
  const int cloF = br.clo[0], chiF = br.chi[0];
  const double db = by ? d[1] : d[2], dg = by ? d[2] : d[1];
  // PERSP: the corner lines f = Afc + P rfc, g = Agc + P rgc on the planes
  // b = P bound the bundle
  float Afc = 0.f, Agc = 0.f, rfc = 0.f, rgc = 0.f;
  bool up;
  if constexpr (PERSP) {
    const double dcb = by ? dc[1] : dc[2], dcg = by ? dc[2] : dc[1];
    up = uni(dcb > 0.0 ? 1 : 0) != 0;
    if (!force_gather) {
      const double rfd = dc[0] / dcb, rgd = dcg / dcb;
      const double ob = (by ? oc[1] : oc[2]) - (double)(by ? br.lo[1] : br.lo[2]);
      Afc = (float)(oc[0] - (double)br.lo[0] - ob * rfd);
      Agc = (float)((by ? oc[2] : oc[1]) - (double)(by ? br.lo[2] : br.lo[1]) - ob * rgd);
      rfc = (float)rfd;
      rgc = (float)rgd;
    }
  } else {
    up = db > 0.0;
  }

  // cell layers (along b) of the lane's first and last samples
  int c_first = up ? 0x7fffffff : -0x7fffffff, c_last = up ? -0x7fffffff : 0x7fffffff;
  if (cnt > 0) {
    c_first = (int)floorf(__builtin_amdgcn_fmed3f(pb, (float)cloB, (float)chiB));
    c_last = (int)floorf(__builtin_amdgcn_fmed3f(fmaf((float)(cnt - 1), sb, pb), (float)cloB, (float)chiB));
  }
  int Lbeg, Lend;  // first and last cell layer in marching order
  if (up) {
    Lbeg = uni(wave_imin(c_first));
    Lend = uni(wave_imax(c_last));
  } else {
    Lbeg = uni(wave_imax(c_first));
    Lend = uni(wave_imin(c_last));
  }
  const int pix = ly * bvw.w + lx;  // SAVE: pixel of the whole-volume image
  if (!force_gather && (up ? Lbeg > Lend : Lbeg < Lend)) {
    if (valid && !a.carry && !foot) *dst = make_float4(0.f, 0.f, 0.f, 0.f);
    if (SAVE && valid) sa.nused[pix] = 0;
    continue;
  }
  const int nlay = up ? Lend - Lbeg + 1 : Lbeg - Lend + 1;  // cell layers
  // SAVE: state of the ray at the start of group g (cell layers gK .. gK + K - 1)
  auto save_group = [&](int g, float Tg, int jg) {
    if (valid) {
      sa.ckpt[(int64_t)g * sa.npix + pix] = Tg;
      sa.ckpt_j[(int64_t)g * sa.npix + pix] = jg;
    }
  };
  const int ngrp_tile = SAVE ? (nlay + sa.K - 1) / sa.K : 0;

  // ---- window geometry from the tile's corner rays (lanes 0..3)
  // A corner ray meets the plane b = P at f = Af + P rf, g = Ag + P rg.
  const double rfd = PERSP ? 0.0 : d[0] / db, rgd = PERSP ? 0.0 : dg / db;
  const float rf = (float)rfd, rg = (float)rgd;
  float Af = 0.f, Ag = 0.f;
  if (!PERSP && !foot) {
    const int cx = bvw.x0 + tx * 8, cy = bvw.y0 + ty * 8;
    const int ex = min(cx + 7, bvw.x0 + bvw.w - 1), ey = min(cy + 7, bvw.y0 + bvw.h - 1);
    const int cc = lane & 3;
    double oc[3];
    pixel_origin(a.cam, (cc & 1) ? ex : cx, (cc & 2) ? ey : cy, oc);
    const double ob = (by ? oc[1] : oc[2]) - (double)(by ? br.lo[1] : br.lo[2]);
    Af = (float)(oc[0] - (double)br.lo[0] - ob * rfd);
    Ag = (float)((by ? oc[2] : oc[1]) - (double)(by ? br.lo[2] : br.lo[1]) - ob * rgd);
  }
  float Af_lo = unif(wmin4(Af)), Af_hi = unif(wmax4(Af));
  float Ag_lo = unif(wmin4(Ag)), Ag_hi = unif(wmax4(Ag));
  if (foot) {  // the cell's rectangle on the plane b = 0
    Af_lo = (float)((double)ci * a.foot_Tf);
    Af_hi = (float)((double)(ci + 1) * a.foot_Tf);
    Ag_lo = (float)((double)cj * a.foot_Tg);
    Ag_hi = (float)((double)(cj + 1) * a.foot_Tg);
  }
  const float arf = fabsf(rf), arg = fabsf(rg);
  // PERSP: the four corner lines as uniform values
  float cAf[4], crf[4], cAg[4], crg[4];
  if constexpr (PERSP)
    for (int c = 0; c < 4; ++c) {
      cAf[c] = lanef(Afc, c);
      crf[c] = lanef(rfc, c);
      cAg[c] = lanef(Agc, c);
      crg[c] = lanef(rgc, c);
    }
  // window extents: f_hi - f_lo + 1 <= floor(span + 0.1) + 3 for the 0.05 margins
  int NF, NG;
  if constexpr (PERSP) {
    if (force_gather) {
      NF = 1 << 20;
      NG = 1;
    } else {
      // the span over [V - 1, V + 1] is convex in V: largest at the first or
      // last voxel layer the tile loads
      const float Va = (float)(up ? Lbeg : Lbeg + 1), Vb = (float)(up ? Lend + 1 : Lend);
      float l0, h0, l1, h1;
      crange(cAf, crf, Va - 1.f, Va + 1.f, l0, h0);
      crange(cAf, crf, Vb - 1.f, Vb + 1.f, l1, h1);
      NF = uni((int)floorf(fmaxf(h0 - l0, h1 - l1) + 0.2f) + 3);
      crange(cAg, crg, Va - 1.f, Va + 1.f, l0, h0);
      crange(cAg, crg, Vb - 1.f, Vb + 1.f, l1, h1);
      NG = uni((int)floorf(fmaxf(h0 - l0, h1 - l1) + 0.2f) + 3);
    }
  } else if (foot) {
    NF = a.foot_nf;
    NG = a.foot_ng;
  } else {
    NF = uni((int)floorf(Af_hi - Af_lo + 2.f * arf + 0.2f) + 3);
    NG = uni((int)floorf(Ag_hi - Ag_lo + 2.f * arg + 0.2f) + 3);
  }
  const int pitch = (NF + 3) & ~3;
  NG = min(NG, chiG + 2 - cloG);
  const int ysl = br.sy, zsl = br.sz;
  const int sB = by ? ysl : zsl, sG = by ? zsl : ysl;
  gfloat* gbase = (gfloat*)br.base;

  float Cr = carried.x, Cg = carried.y, Cb = carried.z, T = carried.w, mx = 0.f;
  int j = 0;
  bool done = cnt == 0;

  if (force_gather || pitch > chiF + 2 - cloF || pitch * NG > slot || pitch > 256 ||
      ((int64_t)(64 / (pitch >> 2)) * sG + pitch) * 4 >= ((int64_t)1 << 32)) {
    // the window does not fit: read the corners from global memory
    int gnext = 0;  // SAVE: next group whose start state is to be stored
    while (!done) {
      const Cell c = cell_of(sample_pos(j, px, py, pz, sx, sy, sz), br);
      if (SAVE) {
        const int ib = by ? c.iy : c.iz;
        const int gi = (up ? ib - Lbeg : Lbeg - ib) / sa.K;
        while (gnext <= gi) save_group(gnext++, T, j);
      }
      gfloat* p = gbase + (c.iz * zsl + c.iy * ysl + c.ix);
      const float val = trilerp(p[0], p[1], p[ysl], p[ysl + 1], p[zsl], p[zsl + 1], p[zsl + ysl], p[zsl + ysl + 1], c);
      ++j;
      if (MIP) {
        float s = norm_value(val, a.vmin, a.inv_range);
        if constexpr (MASK) s *= channel_weight(a.mask, a.mask_axis, br.lo[a.mask_axis], c);
        mx = fmaxf(mx, s);
        if (j >= cnt || mx >= 1.f) done = true;
      } else {
        Classified k = classify(val, a.vmin, a.inv_range, a.M, s_tf);
        if constexpr (MASK) k.a *= channel_weight(a.mask, a.mask_axis, br.lo[a.mask_axis], c);
        accumulate(k, Cr, Cg, Cb, T);
        if (j >= cnt || 1.f - T >= a.tau) done = true;
      }
    }
    if (SAVE) {
      while (gnext < ngrp_tile) save_group(gnext++, T, j);
      if (valid) sa.nused[pix] = j;
    }
    // carried state: only rays with samples here write (another brick of the
    // wave whose rectangle holds the pixel may update it)
    if (valid && cnt > 0 && wr_ok)
      *dst = MIP ? make_float4(mx, mx, mx, mx) : make_float4(Cr, Cg, Cb, a.carry ? T : 1.f - T);
    else if (valid && !a.carry && !foot)
      *dst = make_float4(0.f, 0.f, 0.f, 0.f);
    continue;
  }

  // window of voxel layer V (brick-local): rows [g0, g0 + NG), columns [f0, f0 + pitch)
  auto window = [&](int V) {
    Window w;
    int flo, glo;
    if constexpr (PERSP) {
      float lf, hf, lg, hg;
      crange(cAf, crf, (float)(V - 1), (float)(V + 1), lf, hf);
      crange(cAg, crg, (float)(V - 1), (float)(V + 1), lg, hg);
      flo = max((int)floorf(lf - 0.05f), cloF);
      glo = max((int)floorf(lg - 0.05f), cloG);
    } else {
      const float Pf = (float)V * rf, Pg = (float)V * rg;
      flo = max((int)floorf(Af_lo + Pf - arf - 0.05f), cloF);
      glo = max((int)floorf(Ag_lo + Pg - arg - 0.05f), cloG);
    }
    w.f0 = uni(max(cloF, min(flo, chiF + 2 - pitch)));
    w.g0 = uni(max(cloG, min(glo, chiG + 2 - NG)));
    return w;
  };
  // chunk (16 bytes) i of a window: row i / (pitch / 4), column 4 (i % (pitch / 4))
  // A load instruction carries R whole rows (R = 64 / (pitch / 4) lanes per
  // row group; the remaining lanes idle), so a lane's offset from the group's
  // first row is fixed for the tile and only the uniform group base moves.
  const int nf4 = pitch >> 2;
  const int R = uni(64 / nf4);
  const int rl = lane / nf4, c4l = lane - rl * nf4;
  const bool lane_on = rl < R;
  const int nload = uni((NG + R - 1) / R);  // load instructions per layer
  const unsigned voff = (unsigned)(rl * sG + 4 * c4l) * 4u;
  const int64_t gstep = (int64_t)R * sG;
  const unsigned lstep = (unsigned)(R * pitch) * 4u;
  auto issue = [&](int V, const Window& w, float* sdst) {
    gfloat* gb = gbase + ((int64_t)V * sB + (int64_t)w.g0 * sG + w.f0);
    const unsigned l0 = uni(lds_addr(sdst));
    for (int k = 0; k < nload; ++k)
      if (lane_on && k * R + rl < NG) lds_dma16(unip(gb + k * gstep), voff, (unsigned)uni((int)(l0 + (unsigned)k * lstep)));
  };

  // voxel layers in marching order: V_k = Lbeg + k (up) or Lbeg + 1 - k (down);
  // cell layer c_k = Lbeg +- k reads V_k and V_{k+1}
  const int vstep = up ? 1 : -1;
  const int V0 = up ? Lbeg : Lbeg + 1;
  if (REG && nload <= kRingRegLoads) {
    // two LDS slots; V_{k+2} waits in registers while c_k is sampled
    const float fclo = (float)cloB, fchi = (float)chiB;
    // every lane of a load instruction reads a row of the window (lanes past
    // the instruction's rows, and rows past the window, re-read its last row)
    // and only lanes holding a row of the window write it to LDS
    typedef float v4f __attribute__((ext_vector_type(4)));
    v4f rr[kRingRegLoads];
    const int rl_c = min(rl, R - 1), c4_c = lane_on ? c4l : 0;
    auto rload = [&](int V, const Window& w) {
      gfloat* gb = gbase + ((int64_t)V * sB + (int64_t)w.g0 * sG + w.f0) + 4 * c4_c;
#pragma unroll
      for (int i = 0; i < kRingRegLoads; ++i)
        if (i < nload)
          rr[i] = *(const v4f __attribute__((address_space(1)))*)(gb + (int64_t)min(i * R + rl_c, NG - 1) * sG);
    };
    auto rstore = [&](float* sdst) {
      v4f* l = (v4f*)(sdst + 4 * lane);
#pragma unroll
      for (int i = 0; i < kRingRegLoads; ++i)
        if (i < nload && lane_on && i * R + rl < NG) l[i * R * (pitch >> 2)] = rr[i];
    };
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
      const int sl = up ? s0 : s0 ^ 1, su = up ? s0 ^ 1 : s0;
      const float* baseL = s_ring + (sl * slot - wl.g0 * pitch - wl.f0);
      const int dU = (su * slot - wu.g0 * pitch - wu.f0) - (sl * slot - wl.g0 * pitch - wl.f0);
      while (!done) {
        const SamplePos q = sample_pos(j, px, py, pz, sx, sy, sz);
        const int ib = (int)floorf(__builtin_amdgcn_fmed3f(by ? q.y : q.z, fclo, fchi));
        if (ib != c) break;
        const Cell cl = cell_of(q, br);
        const int ig = by ? cl.iz : cl.iy;
        const float* p = baseL + (__mul24(ig, pitch) + cl.ix);
        const float* pu = p + dU;
        const float l00 = p[0], l01 = p[1], l10 = p[pitch], l11 = p[pitch + 1];
        const float u00 = pu[0], u01 = pu[1], u10 = pu[pitch], u11 = pu[pitch + 1];
        const float val = by ? trilerp(l00, l01, u00, u01, l10, l11, u10, u11, cl)
                             : trilerp(l00, l01, l10, l11, u00, u01, u10, u11, cl);
        ++j;
        if (MIP) {
          const float s = norm_value(val, a.vmin, a.inv_range);
          mx = fmaxf(mx, s);
          if (j >= cnt || mx >= 1.f) done = true;
        } else {
          const Classified kk = classify(val, a.vmin, a.inv_range, a.M, s_tf);
          accumulate(kk, Cr, Cg, Cb, T);
          if (j >= cnt || 1.f - T >= a.tau) done = true;
        }
      }
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
  } else if constexpr (!ESS) {
    const float fclo = (float)cloB, fchi = (float)chiB;
    Window w0 = window(V0), w1 = window(V0 + vstep);
    issue(V0, w0, s_ring);
    issue(V0 + vstep, w1, s_ring + slot);
    int s0 = 0;  // slot of V_k
    for (int k = 0; k < nlay; ++k) {
      if (SAVE && k % sa.K == 0) save_group(k / sa.K, T, j);
      wait_loads();  // V_k and V_{k+1} are in LDS
      // start V_{k+2} into the slot V_{k-1} used (cell layer c_{k-1} is finished);
      // with two slots, into the slot of V_k once c_k is finished
      const int s1 = s0 == kSlots - 1 ? 0 : s0 + 1;
      const int s2 = s1 == kSlots - 1 ? 0 : s1 + 1;
      Window w2;
      if (k + 1 < nlay) {
        const int V2 = V0 + (k + 2) * vstep;
        w2 = window(V2);
        if (!TWO) issue(V2, w2, s_ring + s2 * slot);
      }
      // lower and upper voxel layer of cell layer c_k
      const int c = up ? Lbeg + k : Lbeg - k;
      const Window& wl = up ? w0 : w1;
      const Window& wu = up ? w1 : w0;
      const int sl = up ? s0 : s1, su = up ? s1 : s0;
      const float* baseL = s_ring + (sl * slot - wl.g0 * pitch - wl.f0);
      const int dU = (su * slot - wu.g0 * pitch - wu.f0) - (sl * slot - wl.g0 * pitch - wl.f0);
      while (!done) {
        const SamplePos q = sample_pos(j, px, py, pz, sx, sy, sz);
        const int ib = (int)floorf(__builtin_amdgcn_fmed3f(by ? q.y : q.z, fclo, fchi));
        if (ib != c) break;
        const Cell cl = cell_of(q, br);
        const int ig = by ? cl.iz : cl.iy;
        const float* p = baseL + (__mul24(ig, pitch) + cl.ix);
        const float* pu = p + dU;
        // corners v[dz][dy][dx]: within a window rows run along g, layers along b
        const float l00 = p[0], l01 = p[1], l10 = p[pitch], l11 = p[pitch + 1];
        const float u00 = pu[0], u01 = pu[1], u10 = pu[pitch], u11 = pu[pitch + 1];
        const float val = by ? trilerp(l00, l01, u00, u01, l10, l11, u10, u11, cl)
                             : trilerp(l00, l01, l10, l11, u00, u01, u10, u11, cl);
        ++j;
        if (MIP) {
          float s = norm_value(val, a.vmin, a.inv_range);
          if constexpr (MASK) s *= channel_weight(a.mask, a.mask_axis, br.lo[a.mask_axis], cl);
          mx = fmaxf(mx, s);
          if (j >= cnt || mx >= 1.f) done = true;
        } else {
          Classified k = classify(val, a.vmin, a.inv_range, a.M, s_tf);
          if constexpr (MASK) k.a *= channel_weight(a.mask, a.mask_axis, br.lo[a.mask_axis], cl);
          accumulate(k, Cr, Cg, Cb, T);
          if (j >= cnt || 1.f - T >= a.tau) done = true;
        }
      }
      if (__all(done)) {
        if (SAVE)
          for (int g = k / sa.K + 1; g < ngrp_tile; ++g) save_group(g, T, j);
        break;
      }
      if (TWO && k + 1 < nlay) issue(V0 + (k + 2) * vstep, w2, s_ring + s0 * slot);
      s0 = s1;
      w0 = w1;
      w1 = w2;
    }
  } else {
    const float fclo = (float)cloB, fchi = (float)chiB;
    const int loB = by ? br.lo[1] : br.lo[2], loG = by ? br.lo[2] : br.lo[1];
    // Empty-space skipping: cell layers are taken in steps that end at macrocell
    // boundaries along b; a step whose cells all lie in macrocells with zero
    // opacity over their range is neither loaded nor sampled (its samples would
    // add nothing and leave T as it is), the lanes only move their cursors.
    auto step_clear = [&](int c, int c_end) {
      const int P0 = min(c, c_end), P1 = max(c, c_end) + 1;  // planes bounding the step
      int f0, f1, g0, g1;
      if constexpr (PERSP) {
        float lf, hf, lg, hg;
        crange(cAf, crf, (float)P0, (float)P1, lf, hf);
        crange(cAg, crg, (float)P0, (float)P1, lg, hg);
        f0 = max((int)floorf(lf - 0.05f), cloF);
        f1 = min((int)floorf(hf + 0.05f), chiF);
        g0 = max((int)floorf(lg - 0.05f), cloG);
        g1 = min((int)floorf(hg + 0.05f), chiG);
      } else {
        const float lo_f = fminf((float)P0 * rf, (float)P1 * rf), hi_f = fmaxf((float)P0 * rf, (float)P1 * rf);
        const float lo_g = fminf((float)P0 * rg, (float)P1 * rg), hi_g = fmaxf((float)P0 * rg, (float)P1 * rg);
        f0 = max((int)floorf(Af_lo + lo_f - 0.05f), cloF);
        f1 = min((int)floorf(Af_hi + hi_f + 0.05f), chiF);
        g0 = max((int)floorf(Ag_lo + lo_g - 0.05f), cloG);
        g1 = min((int)floorf(Ag_hi + hi_g + 0.05f), chiG);
      }
      const int mc = a.mc;
      const int mf0 = (f0 + br.lo[0]) / mc, mf1 = (max(f1, f0) + br.lo[0]) / mc;
      const int mg0 = (g0 + loG) / mc, mg1 = (max(g1, g0) + loG) / mc;
      const int mb = (c + loB) / mc;
      const int nmf = mf1 - mf0 + 1, tot = nmf * (mg1 - mg0 + 1);
      bool opaque = false;
#pragma nounroll
      for (int i = lane; i < tot; i += 64) {
        const int mf = mf0 + i % nmf, mg = mg0 + i / nmf;
        const int my = by ? mb : mg, mz = by ? mg : mb;
        opaque |= a.mc_clear[((int64_t)mz * a.mcn[1] + my) * a.mcn[0] + mf] == 0;
      }
      return !__any(opaque);
    };

    // voxel layer V_i lives in slot i % 3; `issued` counts the layers started
    auto start = [&](int i) {
      const int V = V0 + i * vstep;
      issue(V, window(V), s_ring + (i % kSlots) * slot);
    };
    int issued = 0;
    int next_check = 0;  // first layer of the next skipping step
    int k = 0;
    while (k < nlay) {
      const int c = up ? Lbeg + k : Lbeg - k;
      if (ESS && k >= next_check) {
        const int mb = (c + loB) / a.mc;
        const int c_end = up ? min(Lend, (mb + 1) * a.mc - 1 - loB) : max(Lend, mb * a.mc - loB);
        const int k_end = up ? c_end - Lbeg : Lbeg - c_end;
        if (step_clear(c, c_end)) {
#pragma nounroll
          while (!done) {
            const int ib = (int)floorf(__builtin_amdgcn_fmed3f(fmaf((float)j, sb, pb), fclo, fchi));
            if (up ? ib > c_end : ib < c_end) break;
            ++j;
            if (j >= cnt) done = true;
          }
          k = k_end + 1;
          next_check = k;
          if (__all(done)) break;
          continue;
        }
        next_check = k_end + 1;
        if (issued < k) {  // after a skipped step: restart the ring at V_k
          wait_loads();    // loads started before the step may still be landing
          issued = k;
        }
      }
#pragma nounroll
      while (issued <= k + 1) start(issued++);
      wait_loads();  // V_k and V_{k+1} are in LDS
      // start V_{k+2} into the slot V_{k-1} used (cell layer c_{k-1} is finished)
      if (k + 2 <= nlay) start(issued++);
      // lower and upper voxel layer of cell layer c_k
      const Window w0 = window(V0 + k * vstep), w1 = window(V0 + (k + 1) * vstep);
      const int s0 = k % kSlots, s1 = (k + 1) % kSlots;
      const Window& wl = up ? w0 : w1;
      const Window& wu = up ? w1 : w0;
      const int sl = up ? s0 : s1, su = up ? s1 : s0;
      const float* baseL = s_ring + (sl * slot - wl.g0 * pitch - wl.f0);
      const int dU = (su * slot - wu.g0 * pitch - wu.f0) - (sl * slot - wl.g0 * pitch - wl.f0);
      while (!done) {
        const SamplePos q = sample_pos(j, px, py, pz, sx, sy, sz);
        const int ib = (int)floorf(__builtin_amdgcn_fmed3f(by ? q.y : q.z, fclo, fchi));
        if (ib != c) break;
        const Cell cl = cell_of(q, br);
        const int ig = by ? cl.iz : cl.iy;
        const float* p = baseL + (__mul24(ig, pitch) + cl.ix);
        const float* pu = p + dU;
        // corners v[dz][dy][dx]: within a window rows run along g, layers along b
        const float l00 = p[0], l01 = p[1], l10 = p[pitch], l11 = p[pitch + 1];
        const float u00 = pu[0], u01 = pu[1], u10 = pu[pitch], u11 = pu[pitch + 1];
        const float val = by ? trilerp(l00, l01, u00, u01, l10, l11, u10, u11, cl)
                             : trilerp(l00, l01, l10, l11, u00, u01, u10, u11, cl);
        Classified k = classify(val, a.vmin, a.inv_range, a.M, s_tf);
        if constexpr (MASK) k.a *= channel_weight(a.mask, a.mask_axis, br.lo[a.mask_axis], cl);
        accumulate(k, Cr, Cg, Cb, T);
        ++j;
        if (j >= cnt || 1.f - T >= a.tau) done = true;
      }
      if (__all(done)) break;
      ++k;
    }
  }
  wait_loads();  // no load may still target LDS when the wavefront ends (or the next batch starts)
  if (SAVE && valid) sa.nused[pix] = j;
  if (valid && wr_ok && (cnt > 0 || (!a.carry && !foot)))
    *dst = MIP ? make_float4(mx, mx, mx, mx) : make_float4(Cr, Cg, Cb, a.carry ? T : 1.f - T);
  } while (false);

}

// Pixels past the 64th of footprint cells (listed by the march): one ray per
// lane, its corners read from global memory; the same samples, arithmetic and
// order as every march.  Wavefronts take listed cells in turn until the list
// is done.
template <bool MIP, bool MASK>
__global__ __launch_bounds__(256) void k_march_ring_ovf(MarchArgs a) {
  extern __shared__ float4 smem[];
  float4* s_tf = smem;
  for (int i = threadIdx.x; i < a.M; i += blockDim.x) s_tf[i] = a.tf[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int nw = (int)(gridDim.x * (blockDim.x >> 6));
  const int n_listed = (int)*a.ovf_count;
  for (int e = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)); e < n_listed; e += nw) {
    const int tile = a.ovf_tiles[e] >> 3, w = a.ovf_tiles[e] & 7;
    const DevBrickView bvw = a.bv[find_bv(a, tile)];
    const DevBrick br = a.bricks[bvw.brick];
    int ci, cj;
    if (a.blk_f > 0) block_cell(a, bvw, tile - bvw.tile_begin, w, ci, cj);
    else foot_cell(bvw, tile - bvw.tile_begin, ci, cj);
    const FootRuns fr = a.cam.persp ? foot_runs_persp(a, bvw, br, ci, cj, lane) : foot_runs(a, bvw, ci, cj, lane);
    gfloat* gb = (gfloat*)br.base;
    const int ys = br.sy, zs = br.sz;
    for (int k0 = 64; k0 < fr.n; k0 += 64) {
      int uu, vv;
      foot_pixel(fr, k0 + lane, uu, vv);
      if (k0 + lane >= fr.n) continue;
      const int lx = uu - bvw.x0, ly = vv - bvw.y0;
      const bool inr = lx >= 0 && lx < bvw.w && ly >= 0 && ly < bvw.h;
      float4* const dst =
          a.carry ? a.img + (int64_t)vv * a.cam.W + uu : a.img + bvw.img_off + (int64_t)ly * bvw.w + lx;
      float4 c0 = make_float4(0.f, 0.f, 0.f, 1.f);
      if (a.carry) c0 = *dst;
      if (a.carry && !(1.f - c0.w < a.tau)) continue;
      double o[3], d[3];
      pixel_ray(a.cam, uu, vv, o, d);  // parallel rays: the view direction
      double tin;
      int64_t n, k0b, k1b;
      if (!ray_lattice(o, d, a.hi, a.step, tin, n)) continue;
      brick_krange(o, d, tin, a.step, n, br.lo, br.hi, br.closed, k0b, k1b);
      if (k1b <= k0b) continue;
      const double t0 = tin + ((double)k0b + 0.5) * a.step;
      const float px = (float)(o[0] + t0 * d[0] - (double)br.lo[0]);
      const float py = (float)(o[1] + t0 * d[1] - (double)br.lo[1]);
      const float pz = (float)(o[2] + t0 * d[2] - (double)br.lo[2]);
      const float sx = (float)(a.step * d[0]), sy = (float)(a.step * d[1]), sz = (float)(a.step * d[2]);
      const int cnt = (int)(k1b - k0b);
      float Cr = c0.x, Cg = c0.y, Cb = c0.z, T = c0.w, mx = 0.f;
      for (int j = 0; j < cnt;) {
        const Cell c = cell_of(sample_pos(j, px, py, pz, sx, sy, sz), br);
        gfloat* p = gb + (c.iz * zs + c.iy * ys + c.ix);
        const float val = trilerp(p[0], p[1], p[ys], p[ys + 1], p[zs], p[zs + 1], p[zs + ys], p[zs + ys + 1], c);
        ++j;
        if (MIP) {
          float sv = norm_value(val, a.vmin, a.inv_range);
          if constexpr (MASK) sv *= channel_weight(a.mask, a.mask_axis, br.lo[a.mask_axis], c);
          mx = fmaxf(mx, sv);
          if (mx >= 1.f) break;
        } else {
          Classified k = classify(val, a.vmin, a.inv_range, a.M, s_tf);
          if constexpr (MASK) k.a *= channel_weight(a.mask, a.mask_axis, br.lo[a.mask_axis], c);
          accumulate(k, Cr, Cg, Cb, T);
          if (1.f - T >= a.tau) break;
        }
      }
      if (a.carry || inr)
        *dst = MIP ? make_float4(mx, mx, mx, mx) : make_float4(Cr, Cg, Cb, a.carry ? T : 1.f - T);
    }
  }
}

__global__ void k_ovf_reset(unsigned int* count) { *count = 0u; }

}  // namespace

size_t ring_lds_bytes(const MarchArgs& a, int wpb) {
  const int ns = a.ring_nslots == 2 ? 2 : kSlotsMax;
  return sizeof(float4) * (size_t)a.M + sizeof(float) * (size_t)wpb * ns * (size_t)a.ring_slot;
}

static hipError_t launch_march_ring_main(const MarchArgs& a, int wpb, hipStream_t s);

hipError_t launch_march_ring(const MarchArgs& a, int wpb, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  if (!a.foot) return launch_march_ring_main(a, wpb, s);
  // footprint cells: clear the overflow list, march, then the listed cells' pixels past the 64th
  // (perspective views: the register-staged cell march only)
  if ((a.cam.persp && (!a.ring_reg || a.blk_f > 0)) || !a.ovf_count || !a.ovf_tiles) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ovf_reset, dim3(1), dim3(1), 0, s, a.ovf_count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = a.blk_f > 0 ? launch_march_block(a, s)
                   : (a.ring_reg ? launch_march_cells(a, wpb, s) : launch_march_ring_main(a, wpb, s));
  if (e != hipSuccess) return e;
  const dim3 g(256), b(256);
  const size_t lds = sizeof(float4) * (size_t)a.M;
  if (a.mip && a.mask) hipLaunchKernelGGL((k_march_ring_ovf<true, true>), g, b, lds, s, a);
  else if (a.mip) hipLaunchKernelGGL((k_march_ring_ovf<true, false>), g, b, lds, s, a);
  else if (a.mask) hipLaunchKernelGGL((k_march_ring_ovf<false, true>), g, b, lds, s, a);
  else hipLaunchKernelGGL((k_march_ring_ovf<false, false>), g, b, lds, s, a);
  return hipGetLastError();
}

static hipError_t launch_march_ring_main(const MarchArgs& a, int wpb, hipStream_t s) {
  if (a.tile_w != 8 || a.ring_slot <= 0 || (a.ring_slot & 3) != 0 || (wpb != 1 && wpb != 2 && wpb != 4))
    return hipErrorInvalidValue;
  const int groups = (a.ntiles + wpb - 1) / wpb;
  const int grid = ((groups + 7) / 8) * 8;
  // macrocell skipping lives in its own instantiation: its bookkeeping costs
  // registers the plain march does not need
  SaveArgs none;
  std::memset(&none, 0, sizeof none);
  const dim3 g(grid), b(64 * wpb);
  const size_t lds = ring_lds_bytes(a, wpb);
  if (a.mip && a.mc > 0) return hipErrorInvalidValue;
  if (a.ring_nslots == 2 && a.mc > 0) return hipErrorInvalidValue;
  if (a.mask) {
    // the channel mask lives in instantiations of its own (three slots)
    if (a.ring_nslots == 2) return hipErrorInvalidValue;
    if (a.cam.persp) {
      if (a.mip) hipLaunchKernelGGL((k_march_ring<false, false, true, true, false, true>), g, b, lds, s, a, none);
      else if (a.mc > 0) hipLaunchKernelGGL((k_march_ring<true, false, false, true, false, true>), g, b, lds, s, a, none);
      else hipLaunchKernelGGL((k_march_ring<false, false, false, true, false, true>), g, b, lds, s, a, none);
    } else {
      if (a.mip) hipLaunchKernelGGL((k_march_ring<false, false, true, false, false, true>), g, b, lds, s, a, none);
      else if (a.mc > 0) hipLaunchKernelGGL((k_march_ring<true, false, false, false, false, true>), g, b, lds, s, a, none);
      else hipLaunchKernelGGL((k_march_ring<false, false, false, false, false, true>), g, b, lds, s, a, none);
    }
    return hipGetLastError();
  }
  if (a.cam.persp) {
    if (!a.mip && a.mc == 0 && a.ring_nslots == 2 && a.ring_reg)
      hipLaunchKernelGGL((k_march_ring<false, false, false, true, true, false, true>), g, b, lds, s, a, none);
    else if (a.mip && a.ring_nslots == 2) hipLaunchKernelGGL((k_march_ring<false, false, true, true, true>), g, b, lds, s, a, none);
    else if (a.mip) hipLaunchKernelGGL((k_march_ring<false, false, true, true>), g, b, lds, s, a, none);
    else if (a.mc > 0) hipLaunchKernelGGL((k_march_ring<true, false, false, true>), g, b, lds, s, a, none);
    else if (a.ring_nslots == 2) hipLaunchKernelGGL((k_march_ring<false, false, false, true, true>), g, b, lds, s, a, none);
    else hipLaunchKernelGGL((k_march_ring<false, false, false, true>), g, b, lds, s, a, none);
  } else {
    if (a.mip && a.ring_nslots == 2) hipLaunchKernelGGL((k_march_ring<false, false, true, false, true>), g, b, lds, s, a, none);
    else if (a.mip) hipLaunchKernelGGL((k_march_ring<false, false, true, false>), g, b, lds, s, a, none);
    else if (a.mc > 0) hipLaunchKernelGGL((k_march_ring<true, false, false, false>), g, b, lds, s, a, none);
    else if (a.ring_nslots == 2) hipLaunchKernelGGL((k_march_ring<false, false, false, false, true>), g, b, lds, s, a, none);
    else hipLaunchKernelGGL((k_march_ring<false, false, false, false>), g, b, lds, s, a, none);
  }
  return hipGetLastError();
}

hipError_t launch_march_ring_save(const MarchArgs& a, const SaveArgs& sa, int wpb, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  if (a.tile_w != 8 || a.ring_slot <= 0 || (a.ring_slot & 3) != 0 || (wpb != 1 && wpb != 2 && wpb != 4) ||
      a.mc != 0 || a.mip != 0 || a.cam.persp != 0 || a.ring_nslots == 2 || sa.K < 1 || !sa.ckpt_j)
    return hipErrorInvalidValue;
  const int groups = (a.ntiles + wpb - 1) / wpb;
  int grid = ((groups + 7) / 8) * 8;
  if (sa.band[8] > 0) {
    int widest = 0;
    for (int x = 0; x < 8; x++) widest = std::max(widest, sa.band[x + 1] - sa.band[x]);
    grid = 8 * widest;
  }
  hipLaunchKernelGGL((k_march_ring<false, true, false, false>), dim3(grid), dim3(64 * wpb), ring_lds_bytes(a, wpb), s, a, sa);
  return hipGetLastError();
}

}  // namespace vr
