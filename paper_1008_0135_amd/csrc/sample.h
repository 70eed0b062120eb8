// sample.h -- per-sample arithmetic shared by every march kernel (forward
// gather, forward LDS-staged, checkpointing forward and adjoint), so all of
// them evaluate a sample with the same single-precision operations in the
// same order (paper Sec. 2: trilinear value -> transfer function -> colour
// and opacity; Sec. 2.4: front-to-back accumulation).
#pragma once

#include "vr_internal.h"

namespace vr {

// Position of sample j of a lane: start + j * step (one rounding per axis).
struct SamplePos {
  float x, y, z;
};

__device__ __forceinline__ SamplePos sample_pos(int j, float px, float py, float pz, float sx, float sy, float sz) {
  const float fj = (float)j;
  return SamplePos{fmaf(fj, sx, px), fmaf(fj, sy, py), fmaf(fj, sz, pz)};
}

// Base cell (clamped to the brick's stored range) and fractions.
struct Cell {
  int ix, iy, iz;
  float wx, wy, wz;
};

// clamp(floor(q), lo, hi) == floor(clamp(q, lo, hi)) for integer bounds, and the
// clamp of q is one v_med3_f32; the fraction reuses the floored float.
__device__ __forceinline__ Cell cell_of(const SamplePos& q, const DevBrick& br) {
#pragma clang fp contract(off)
  Cell c;
  const float fx = floorf(__builtin_amdgcn_fmed3f(q.x, (float)br.clo[0], (float)br.chi[0]));
  const float fy = floorf(__builtin_amdgcn_fmed3f(q.y, (float)br.clo[1], (float)br.chi[1]));
  const float fz = floorf(__builtin_amdgcn_fmed3f(q.z, (float)br.clo[2], (float)br.chi[2]));
  c.ix = (int)fx;
  c.iy = (int)fy;
  c.iz = (int)fz;
  c.wx = q.x - fx;
  c.wy = q.y - fy;
  c.wz = q.z - fz;
  return c;
}

// Trilinear value from the eight corners v[dz][dy][dx] (lerp along 1, then 2, then 3).
__device__ __forceinline__ float trilerp(float v000, float v001, float v010, float v011, float v100, float v101,
                                         float v110, float v111, const Cell& c) {
  const float c00 = fmaf(c.wx, v001 - v000, v000), c01 = fmaf(c.wx, v011 - v010, v010);
  const float c10 = fmaf(c.wx, v101 - v100, v100), c11 = fmaf(c.wx, v111 - v110, v110);
  const float c0 = fmaf(c.wy, c01 - c00, c00), c1 = fmaf(c.wy, c11 - c10, c10);
  return fmaf(c.wz, c1 - c0, c0);
}

// Transfer-function lookup: value -> (r, g, b, a), plus the table interval i,
// the weight w and the unclamped normalised value (for the adjoint).
struct Classified {
  float r, g, b, a;
  int i;
  float w;
  float sraw;
};

__device__ __forceinline__ Classified classify(float val, float vmin, float inv_range, int M, const float4* s_tf) {
  // no contraction: every kernel (and every inlining context) must round the
  // table coordinate and weight alike, or the marches would differ in bits
#pragma clang fp contract(off)
  Classified k;
  k.sraw = (val - vmin) * inv_range;
  const float s = fminf(fmaxf(k.sraw, 0.f), 1.f);
  const float uu = s * (float)(M - 1);
  k.i = min((int)uu, M - 2);
  k.w = uu - (float)k.i;
  const float4 e0 = s_tf[k.i], e1 = s_tf[k.i + 1];
  k.a = fmaf(k.w, e1.w - e0.w, e0.w);
  k.r = fmaf(k.w, e1.x - e0.x, e0.x);
  k.g = fmaf(k.w, e1.y - e0.y, e0.y);
  k.b = fmaf(k.w, e1.z - e0.z, e0.z);
  return k;
}

// Normalised value clamped to [0, 1] (the table coordinate before scaling by
// M - 1): what maximum intensity projection keeps the largest of.
__device__ __forceinline__ float norm_value(float val, float vmin, float inv_range) {
#pragma clang fp contract(off)
  return fminf(fmaxf((val - vmin) * inv_range, 0.f), 1.f);
}

// Channel weight of a sample: the mask interpolated along its axis (2, or 1 in
// the permuted copy) with the sample's trilinear weight; 1 without a mask.
// lo: the brick's origin along that axis (cell indices are brick-local).
__device__ __forceinline__ float channel_weight(const float* mask, int axis, int lo, const Cell& c) {
#pragma clang fp contract(off)
  if (!mask) return 1.f;
  const int i = lo + (axis == 2 ? c.iz : c.iy);
  const float w = axis == 2 ? c.wz : c.wy;
  const float m0 = mask[i], m1 = mask[i + 1];
  return fmaf(w, m1 - m0, m0);
}

// One front-to-back emission-absorption step: C += T a rgb, T *= (1 - a).
__device__ __forceinline__ void accumulate(const Classified& k, float& Cr, float& Cg, float& Cb, float& T) {
#pragma clang fp contract(off)
  const float Ta = T * k.a;
  Cr = fmaf(Ta, k.r, Cr);
  Cg = fmaf(Ta, k.g, Cg);
  Cb = fmaf(Ta, k.b, Cb);
  T = fmaf(-T, k.a, T);
}

}  // namespace vr
