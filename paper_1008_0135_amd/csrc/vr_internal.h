// vr_internal.h -- internal types of libvr shared by the host runtime and the
// gfx950 kernels: camera and ray setup (double precision, used on both sides
// so the host plan and the device launch agree bit for bit), brick tables and
// POD kernel argument blocks.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "vr.h"

namespace vr {

// ---------------------------------------------------------------- camera
// Orthographic camera of one view (paper Sec. 2.2: a render request carries
// the transformation and projection).  Pixel pitch is S/W voxels on both axes.
struct Camera {
  double c[3];          // box centre
  double e1[3], e2[3];  // image axes
  double e3[3];         // viewing direction (the ray direction when orthographic)
  double S;             // image width in voxels
  double Sy;            // image height in voxels = S*H/W
  int32_t W, H;
  int32_t persp;        // 1: perspective from eye[], 0: orthographic
  int32_t pad;
  double D;             // eye distance from c (perspective)
  double eye[3];        // c - D e3 (perspective)
};

__host__ __device__ inline void make_camera(const vr_view& v, const int64_t n[3], Camera& cam) {
  double diag = 0.0;
  for (int i = 0; i < 3; i++) {
    cam.c[i] = 0.5 * (double)(n[i] - 1);
    diag += (double)(n[i] - 1) * (double)(n[i] - 1);
    cam.e1[i] = v.R[i];
    cam.e2[i] = v.R[3 + i];
    cam.e3[i] = v.R[6 + i];
  }
  cam.S = v.extent > 0.0 ? v.extent : sqrt(diag);
  cam.Sy = cam.S * (double)v.H / (double)v.W;
  cam.W = v.W;
  cam.H = v.H;
  cam.persp = v.eye_dist > 0.0 ? 1 : 0;
  cam.pad = 0;
  cam.D = cam.persp ? v.eye_dist : 0.0;
  for (int i = 0; i < 3; i++) cam.eye[i] = cam.c[i] - cam.D * cam.e3[i];
}

// Ray origin of pixel (u, v) of an orthographic camera; the direction is cam.e3.
__host__ __device__ inline void pixel_origin(const Camera& cam, int u, int v, double o[3]) {
#pragma clang fp contract(off)
  double x = (((double)u + 0.5) / (double)cam.W - 0.5) * cam.S;
  double y = (((double)v + 0.5) / (double)cam.H - 0.5) * cam.S * (double)cam.H / (double)cam.W;
  for (int i = 0; i < 3; i++) o[i] = cam.c[i] + x * cam.e1[i] + y * cam.e2[i] - cam.S * cam.e3[i];
}

// Ray of pixel (u, v), either projection: origin o and unit direction d.
// Perspective: from the eye through the pixel's point on the plane through
// the box centre normal to e3 (the pixel grid of the orthographic camera).
__host__ __device__ inline void pixel_ray(const Camera& cam, int u, int v, double o[3], double d[3]) {
#pragma clang fp contract(off)
  if (!cam.persp) {
    pixel_origin(cam, u, v, o);
    for (int i = 0; i < 3; i++) d[i] = cam.e3[i];
    return;
  }
  double x = (((double)u + 0.5) / (double)cam.W - 0.5) * cam.S;
  double y = (((double)v + 0.5) / (double)cam.H - 0.5) * cam.S * (double)cam.H / (double)cam.W;
  double w[3];
  for (int i = 0; i < 3; i++) {
    o[i] = cam.eye[i];
    w[i] = x * cam.e1[i] + y * cam.e2[i] + cam.D * cam.e3[i];
  }
  const double len = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  for (int i = 0; i < 3; i++) d[i] = w[i] / len;
}

// Perspective camera, footprint cells: where the ray of pixel (u, v) crosses
// the brick-local plane b = 0, with E = eye - lo (brick-local eye) and g the
// other of axes 2, 3: f = E_f - E_b w_f / w_b, g = E_g - E_b w_g / w_b for the
// unnormalised direction w = x e1 + y e2 + D e3 of pixel_ray.  One expression
// everywhere, so every evaluation puts a pixel in the same cell.
__host__ __device__ inline void persp_plane_point(const Camera& cam, const double E[3], int b, int g, double u,
                                                  double v, double& pf, double& pg) {
#pragma clang fp contract(off)
  const double x = ((u + 0.5) / (double)cam.W - 0.5) * cam.S;
  const double y = ((v + 0.5) / (double)cam.H - 0.5) * cam.S * (double)cam.H / (double)cam.W;
  const double wf = x * cam.e1[0] + y * cam.e2[0] + cam.D * cam.e3[0];
  const double wg = x * cam.e1[g] + y * cam.e2[g] + cam.D * cam.e3[g];
  const double wb = x * cam.e1[b] + y * cam.e2[b] + cam.D * cam.e3[b];
  const double t = -E[b] / wb;
  pf = E[0] + t * wf;
  pg = E[g] + t * wg;
}

// Image position (pixel units, centres at integers) of the point at offset r
// from the eye, for a perspective camera.
__host__ __device__ inline void persp_image_uv(const Camera& cam, const double r[3], double& u, double& v) {
  const double z = r[0] * cam.e3[0] + r[1] * cam.e3[1] + r[2] * cam.e3[2];
  const double x = cam.D * (r[0] * cam.e1[0] + r[1] * cam.e1[1] + r[2] * cam.e1[2]) / z;
  const double y = cam.D * (r[0] * cam.e2[0] + r[1] * cam.e2[1] + r[2] * cam.e2[2]) / z;
  u = (x / cam.S + 0.5) * (double)cam.W - 0.5;
  v = (y / (cam.S * (double)cam.H / (double)cam.W) + 0.5) * (double)cam.H - 0.5;
}

// Whole-volume ray/box test (slab method against the closed box [0, hi]) and
// lattice count n = max(0, ceil((t_out - t_in)/step - 1/2)): samples sit at
// t_k = t_in + (k + 1/2) step for k in [0, n) (paper Sec. 2.4: entry and exit
// points of the ray in the data's bounding box).  Returns false on a miss.
__host__ __device__ inline bool ray_lattice(const double o[3], const double d[3], const double hi[3],
                                            double step, double& tin, int64_t& n) {
#pragma clang fp contract(off)
  double a = -INFINITY, b = INFINITY;
  for (int i = 0; i < 3; i++) {
    if (d[i] == 0.0) {
      if (o[i] < 0.0 || o[i] > hi[i]) return false;
      continue;
    }
    double t1 = (0.0 - o[i]) / d[i], t2 = (hi[i] - o[i]) / d[i];
    double tn = t1 < t2 ? t1 : t2, tf = t1 < t2 ? t2 : t1;
    if (tn > a) a = tn;
    if (tf < b) b = tf;
  }
  if (!(a < b)) return false;
  tin = a;
  double X = (b - a) / step - 0.5;
  double c = ceil(X);
  n = c > 0.0 ? (int64_t)c : 0;
  return n > 0;
}

// Lattice index at which the ray crosses the plane x_i = P, as a real number:
// sample k lies at or beyond the plane (in the direction of d_i > 0) iff
// k >= X.  Every brick that shares the plane evaluates this same expression,
// so the partition of the lattice between neighbours is exact.
__host__ __device__ inline double plane_index(double P, double o, double d, double tin, double step) {
#pragma clang fp contract(off)
  return ((P - o) / d - tin) / step - 0.5;
}

__host__ __device__ inline int64_t clamp_idx(double x, int64_t lo, int64_t hi) {
  // x is a real-valued index already rounded by ceil/floor; clamp before converting
  if (!(x > (double)lo)) return lo;
  if (!(x < (double)hi)) return hi;
  return (int64_t)x;
}

// Samples [k0, k1) of the whole-volume lattice owned by the box
// lo <= p < hi (p <= hi along closed axes).  n is the lattice count.
__host__ __device__ inline void brick_krange(const double o[3], const double d[3], double tin, double step,
                                             int64_t n, const int32_t lo[3], const int32_t hi[3], int closed,
                                             int64_t& k0, int64_t& k1) {
  int64_t a = 0, b = n;
  for (int i = 0; i < 3; i++) {
    bool cl = (closed >> i) & 1;
    if (d[i] == 0.0) {
      bool in = o[i] >= (double)lo[i] && (cl ? o[i] <= (double)hi[i] : o[i] < (double)hi[i]);
      if (!in) {
        k0 = k1 = 0;
        return;
      }
      continue;
    }
    double Xl = plane_index((double)lo[i], o[i], d[i], tin, step);
    double Xh = plane_index((double)hi[i], o[i], d[i], tin, step);
    int64_t s, e;  // this axis admits k in [s, e)
    if (d[i] > 0.0) {
      s = clamp_idx(ceil(Xl), -1, n + 1);
      e = cl ? clamp_idx(floor(Xh) + 1.0, -1, n + 1) : clamp_idx(ceil(Xh), -1, n + 1);
    } else {
      s = cl ? clamp_idx(ceil(Xh), -1, n + 1) : clamp_idx(floor(Xh) + 1.0, -1, n + 1);
      e = clamp_idx(floor(Xl) + 1.0, -1, n + 1);
    }
    if (s > a) a = s;
    if (e < b) b = e;
  }
  k0 = a;
  k1 = b > a ? b : a;
}

// ---------------------------------------------------------------- brick tables
// Static per-brick record (one per brick of the partition).
struct DevBrick {
  const float* base;      // storage address of voxel (lo1, lo2, lo3)
  int32_t sy, sz;         // storage strides (elements) along axes 2 and 3
  int32_t lo[3], hi[3];   // ownership box
  int32_t closed;         // bit i: closed along axis i
  int32_t clo[3], chi[3]; // clamps of the local cell index (global [0, n-2] shifted by -lo)
  float vmin, vmax;       // range of the stored voxels
  int32_t slack;          // 1: the storage is followed by >= 64 readable floats (row tails may be over-read)
};

// Per (view, rendered brick) record, in launch order.
struct DevBrickView {
  int32_t brick;       // index into the DevBrick table
  int32_t x0, y0, w, h;
  int32_t tiles_x;     // tiles along x of the rectangle (footprint cells: cells along f)
  int32_t tile_begin;  // first work-item (tile) index of this brick
  int32_t cf0;         // footprint cells: index of the first cell along f
  int64_t img_off;     // offset (in pixels) of the brick image in the image arena
  int32_t cg0;         // footprint cells: index of the first cell along g
  int32_t blocks_x;    // blocks of footprint cells: blocks along f
  double fa0, fb0;     // footprint cells: cell coordinates (f / Tf, g / Tg) of pixel (0, 0)'s ray on the
                       // brick-local plane b = 0
  // footprint cells of a perspective view (sized per brick: rays from the eye
  // are denser on near bricks): cell size on the plane b = 0 and the window
  // of one voxel layer (row floats, a multiple of 4, and rows)
  double pTf, pTg;
  int32_t ppitch, png;
};

// One layer of the over-composite, front to back.
struct CompLayer {
  int32_t x0, y0, w, h;
  const float4* rgba;
};

// ---------------------------------------------------------------- kernel arguments
struct MarchArgs {
  Camera cam;
  double hi[3];          // n - 1 per axis (whole-volume box)
  double step;
  float tau;             // ERT threshold (ert == 0: off)
  int32_t ert;
  float vmin, inv_range; // normalisation window (inv_range = 0 when vmax == vmin)
  int32_t M;             // table entries
  int32_t nbv;           // rendered bricks in this launch
  int32_t ntiles;        // total work items (tiles)
  int32_t tile_w, tile_h;
  int32_t slab_axis;     // LDS-staged march: slab axis (1 = axis 2, 2 = axis 3); 0 = gather march
  int32_t slab_T;        // cell layers per slab
  int32_t lds_budget;    // floats of LDS for one slab's voxel box
  int32_t ring_slot;     // ring march: floats per LDS ring slot (one voxel layer's window)
  int32_t mip;           // 1: maximum intensity projection (pixels (M, M, M, M)), 0: emission-absorption
  int32_t carry;         // 1: rays continue from the state (C, T) held in img, the output frame
                         // (rows of cam.W pixels), and leave theirs there
  const float4* tf;      // [M] RGBA
  const DevBrick* bricks;
  const DevBrickView* bv;
  float4* img;           // image arena (or the output frame)
  const uint8_t* mc_clear; // per macrocell [m3][m2][m1]: 1 = opacity 0 over its whole range
  int32_t mc;            // macrocell edge in cells; 0 = no macrocell skipping
  int32_t mcn[3];        // macrocells per axis
  int32_t ring_nslots;   // ring march: LDS slots per wavefront, 3 (one layer in flight while sampling) or 2
  int32_t lds_floor;     // cells march: LDS bytes reserved per workgroup at least (caps how many
                         // workgroups share a compute unit); 0 = what the windows need
  int32_t ring_reg;      // footprint cells, two slots: 1 = the layer after next travels through
                         // registers while a layer is sampled (k_march_cells; at most
                         // kRingRegLoads loads per lane per layer)
  int32_t mask_axis;     // axis of the channel mask (2, or 1 in the permuted copy)
  const float* mask;     // channel weights along mask_axis (global indices), or null
  int32_t tile_order;    // ring march: tiles of a brick numbered along rows (0), down columns (1),
                         // or in blocks of tile_bw x tile_bh tiles (2)
  int32_t tile_bw, tile_bh;
  // ring march, parallel rays: work items are footprint cells instead of 8 x 8
  // pixel tiles (foot = 1).  A cell is the set of pixels whose rays cross the
  // brick-local plane b = 0 inside [i Tf, (i + 1) Tf) x [j Tg, (j + 1) Tg)
  // (f = axis 1, g = the other in-plane axis), taken through foot_cell_coord;
  // its windows are the rectangle moved along the rays plus the trilinear
  // margin, foot_nf x foot_ng floats
  int32_t foot;
  int32_t foot_nf, foot_ng;
  int32_t foot_pad;
  double foot_Tf, foot_Tg;
  double fa_u, fa_v, fb_u, fb_v;  // cell coordinates per pixel step along u and v
  unsigned int* ovf_count;        // cells of more than 64 pixels: count and entries 8 t + w (work
  int32_t* ovf_tiles;             // item t, wavefront w of a block; room for every cell of the launch)
  // blocks of footprint cells: a workgroup of blk_f x blk_g wavefronts marches
  // one block (a wavefront per cell) with one window per voxel layer; 0 = off
  int32_t blk_f, blk_g;
};

// Cell coordinate (f / Tf or g / Tg) of pixel (u, v)'s ray on a brick's plane
// b = 0: an affine function of (u, v) evaluated with two fused multiply-adds,
// which makes it exactly monotone along u within an image row (so the pixels
// of a row that fall in one cell form one run).
__host__ __device__ inline double foot_cell_coord(double c0, double su, double sv, int u, int v) {
  return fma((double)u, su, fma((double)v, sv, c0));
}

struct CompArgs {
  const CompLayer* layers;
  int32_t n;
  int32_t W, H;
  int32_t mip;        // 1: element-wise maximum instead of the over operator
  float4* out;
};

// Differentiable path (whole volume).  Checkpoints are stored [segment][pixel].
struct SaveArgs {
  float* ckpt;        // sample segments: T before samples 0, K, 2K, ... [segment][pixel];
                      // layer groups: T at the start of each group [group][pixel]
  int32_t* ckpt_j;    // layer groups: sample cursor at the start of each group [group][pixel]
  int32_t* nused;     // samples applied per ray (early termination included)
  int32_t K;          // samples per segment, or cell layers per group
  int32_t npix;       // W * H
  int32_t band[9];    // ring march: tile groups per XCD, as BwdArgs::band (band[8] == 0: equal counts)
};

struct BwdArgs {
  const float* ckpt;
  const int32_t* ckpt_j;  // layer groups: sample cursor at each group start (null for sample segments)
  const int32_t* nused;
  const float4* gout; // dL/d(image) of this view, [H][W]
  float* gvol;        // dL/d(voxels), [n3][n2][n1], or null
  double* tf_part;    // per-workgroup table gradients, [blocks][M][4]
  double vmin, inv_range;  // normalisation window in double precision
  int32_t K;          // samples per segment, or cell layers per group
  int32_t npix;
  int32_t smax;       // layer groups: samples of one ray in one group, at most
  // ring adjoint: tile groups of XCD x (workgroup b runs on XCD b % 8 and takes
  // group band[x] + b / 8 while below band[x + 1]); contiguous bands of equal
  // estimated work.  band[8] == 0: equal counts of groups
  int32_t band[9];
  int32_t* flag;      // set to 1 when a ray's group held more than smax samples
};

// Batched rendering: one descriptor per request (whole volume, own view,
// table, window and output), work items numbered request by request.
struct BatchReq {
  Camera cam;
  DevBrick br;           // the request's volume as one brick
  double hi[3];          // n - 1 per axis
  float vmin, inv_range;
  const float4* tf;
  float4* out;
  int32_t M, tiles_x, ntiles, item_begin;
  int32_t tile_shift;    // tile width 2^tile_shift pixels (4, 8, 16 or 32), height 64 / width
  int32_t pad_[3];
};

// Allocation-free batched entry point: its device scratch holds the
// descriptor table of at most kNoAllocMaxReq requests, then the work counter.
// register-staged ring march: 16-byte loads per lane for one voxel layer's window
constexpr int kRingRegLoads = 8;
constexpr int kNoAllocMaxReq = 512;
constexpr size_t kNoAllocBytes = sizeof(BatchReq) * kNoAllocMaxReq + 256;
constexpr int kMaxDevices = 64;

struct BatchArgs {
  const BatchReq* reqs;
  unsigned int* counter;  // next work item
  int32_t nreq, total_items, max_M, pad;
  double step;
  float tau;
  int32_t pad2;
};

// Launchers (defined in the .hip files); all asynchronous on `s`.
hipError_t launch_march(const MarchArgs& a, hipStream_t s);
// (C, T) = (0, 1) over a frame of n pixels (final = false), or (C, T) -> (C, 1 - T) (final = true)
hipError_t launch_carry(float4* img, int64_t n, bool final, hipStream_t s);
// (0, 0, 0, 0) over n pixels (a fill kernel, not a memset)
hipError_t launch_zero(float4* img, int64_t n, hipStream_t s);
// Ring march (march_ring.hip): 8 x 8 tiles, a.ring_slot floats per window slot,
// `wpb` wavefronts per workgroup (1, 2 or 4).
hipError_t launch_march_ring(const MarchArgs& a, int wpb, hipStream_t s);
size_t ring_lds_bytes(const MarchArgs& a, int wpb);
// footprint cells: a wavefront per cell, windows staged through registers
// (the host keeps a lane's offset inside a window's rows below 4 GiB), or
// blocks of a.blk_f x a.blk_g cells per workgroup
hipError_t launch_march_cells(const MarchArgs& a, int wpb, hipStream_t s);
size_t cells_lds_bytes(const MarchArgs& a, int wpb);
hipError_t launch_march_block(const MarchArgs& a, hipStream_t s);
size_t block_lds_bytes(const MarchArgs& a);
// Differentiable forward on the ring layout (whole volume): also stores the
// per-group checkpoints of sa (layer groups of sa.K cell layers).
hipError_t launch_march_ring_save(const MarchArgs& a, const SaveArgs& sa, int wpb, hipStream_t s);
// Adjoint on the ring layout (grad_ring.hip): layer groups of ba.K cell layers.
hipError_t launch_bwd_ring(const MarchArgs& a, const BwdArgs& ba, int wpb, hipStream_t s);
size_t bwd_ring_lds_bytes(const MarchArgs& a, const BwdArgs& ba, int wpb);
int bwd_ring_blocks(const MarchArgs& a, const BwdArgs& ba, int wpb);
hipError_t launch_march_lds(const MarchArgs& a, hipStream_t s);
hipError_t launch_composite(const CompArgs& a, hipStream_t s);
hipError_t launch_minmax(const float* x, int64_t n, float* partial, int32_t nblocks, hipStream_t s);
hipError_t launch_minmax_final(const float* partial, int32_t nblocks, float* out3, hipStream_t s);
// Per-brick (min, max) over stored voxel boxes: boxes is a device array of
// nb x (slo1, slo2, slo3, shi1, shi2, shi3); each brick's z range is split into
// zgroups groups of zper planes; scratch holds nb*zgroups float2 partials.
hipError_t launch_brick_minmax_parts(const float* vol, const int64_t n[3], const int64_t* boxes, int32_t nb,
                                     int zgroups, int zper, float* scratch, float* out2, hipStream_t s);
hipError_t launch_fwd_save(const MarchArgs& a, const SaveArgs& sa, hipStream_t s);
hipError_t launch_bwd(const MarchArgs& a, const BwdArgs& ba, hipStream_t s);
int bwd_blocks(const MarchArgs& a);
// slices: tf_reduce_slices() x n doubles of scratch
int tf_reduce_slices();
hipError_t launch_tf_reduce(const double* part, int nblocks, int n, float* grad_tf, double* slices, hipStream_t s);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_batch(const BatchArgs& a, int blocks, hipStream_t s);
hipError_t launch_copy_box(const float* src, const int64_t sn[3], const int64_t so[3], float* dst,
                           const int64_t dn[3], hipStream_t s);
// dst[x][z][y] = src[z][y][x] for a volume of dims n (dst holds n[0] n[1] n[2] floats)
hipError_t launch_twin(const float* src, const int64_t n[3], float* dst, hipStream_t s);
// Macrocell (min, max) pairs [c3][c2][c1] of edge `mc` over the volume (mc in [2, 1024]).
hipError_t launch_mc_minmax(const float* vol, const int64_t n[3], int mc, const int64_t c[3], float* out2,
                            hipStream_t s);
// clear[i] = 1 when the table's opacity is 0 over every entry macrocell i can reach
// (nz: [M + 1] prefix count of entries with opacity != 0); *nclear = number of such cells.
hipError_t launch_mc_classify(const float* mm2, int64_t count, const int32_t* nz, int M, double vmin, double vmax,
                              uint8_t* clear, unsigned int* nclear, hipStream_t s);

}  // namespace vr
