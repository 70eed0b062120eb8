// plan.h -- host-side planning of libvr (no GPU calls): sub-volume
// partitions (regular grid and longest-axis split, paper Sec. 2.3), rendering
// rectangles and depth order per view (paper Sec. 2.4, 2.5), empty-space
// classification of bricks and nominal sample counts.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "vr_internal.h"

namespace vr {

struct Box {
  int64_t lo[3], hi[3];  // ownership [lo, hi) per axis, [lo, hi] where closed
  int32_t closed[3];
};

struct KdNode {
  int32_t axis;   // split axis (internal nodes)
  int64_t plane;  // split plane (low child owns < plane)
  int32_t left, right;
  int32_t leaf;   // brick index for leaves, -1 for internal nodes
};

struct Partition {
  int32_t mode = VR_BRICK_GRID;
  int64_t gsize[3] = {0, 0, 0};
  int32_t gcount[3] = {0, 0, 0};
  std::vector<Box> boxes;
  std::vector<KdNode> nodes;  // longest-axis split tree (root = 0)
};

struct Rect {
  int32_t x0, y0, w, h;  // w == 0 or h == 0: empty
};

// Regular grid: brick j along an axis owns [j*size, (j+1)*size); the last one
// is closed at n-1; count = ceil((n-1)/size).  Box order: axis 1 fastest.
bool make_grid(const int64_t n[3], const int64_t size[3], Partition& out, std::string& err);

// Longest-axis recursive split into nparts boxes (leaves in depth-first, low
// side first order).
bool make_kd(const int64_t n[3], int32_t nparts, Partition& out, std::string& err);

// Stored voxel range of a box: ownership box plus a 1-voxel ghost layer,
// clipped to the volume.
void stored_box(const Box& b, const int64_t n[3], int64_t slo[3], int64_t shi[3]);

// Conservative pixel rectangle of the box's projection (corner bounding box
// padded by one pixel, clipped to the image).
Rect brick_rect(const Camera& cam, const Box& b);

// The partition of the permuted copy whose axes 1, 2, 3 are axes 2, 3, 1 of
// the partition's volume: the same boxes, axes permuted (grid: in the copy's
// grid order; longest-axis split: the same tree).
void permute_partition(const Partition& p, const int64_t n_twin[3], Partition& out);

// Front-to-back order of all boxes for ray direction d.
void depth_order(const Partition& p, const Camera& cam, std::vector<int32_t>& order);

// Front-to-back waves: wave[b] for every box such that no ray meets two boxes
// of one wave and every ray meets its boxes in increasing wave order (grid:
// the sum over axes of the box's slab distance from the rays' start, exact;
// longest-axis split: one past the largest wave of any earlier box in depth
// order whose rectangle overlaps).  Returns the number of waves.
int32_t brick_waves(const Partition& p, const Camera& cam, std::vector<int32_t>& wave);

// True when every sample a brick with stored range [bmin, bmax] can produce
// has zero opacity: all table alphas in [floor(u(bmin)) - 1, ceil(u(bmax)) + 1]
// (clipped to [0, M-1]) are zero.  Skipping such a brick is bit-exact.
bool brick_transparent(float bmin, float bmax, const float* tf_rgba, int32_t M, double vmin, double vmax);

// Slab parameters of the LDS-staged march for one view: the slab axis
// (1 = axis 2, 2 = axis 3; axis 1 is the contiguous storage axis and is never
// the slab axis) and the number of cell layers per slab, the largest for
// which a conservative bound of the voxel box that one tw x th tile of rays
// touches in a slab fits `budget` floats.  Among the two axes, the one that
// loads the fewest voxels per sample wins.  Returns false when no slab of one
// layer fits (rays nearly parallel to axis 1, or pixels much larger than
// voxels): the gather march is used then.
bool choose_slab(const Camera& cam, int32_t tw, int32_t th, int32_t budget, int32_t& axis, int32_t& T);

// Wavefronts per workgroup (1, 2 or 4) for a ring launch: the choice that fits
// the most wavefronts per compute unit into 160 KB of LDS (M-entry table per
// workgroup, three slots per wavefront), at most `max_waves` per unit.
int ring_waves_per_block(int32_t slot, int32_t M, int32_t max_waves, int32_t* waves_per_cu, int32_t nslots = 3);

// Ring march for one view (8 x 8 tiles).  For each slab axis (as above) the
// per-layer window bound -- the box of voxels that the samples of one tile
// between the planes b = V - 1 and b = V + 1 can touch, rows rounded up to
// whole 16-byte chunks -- and the wavefronts per compute unit that its LDS
// slots allow; picks the axis with the fewest window voxels per sample,
// weighted by how far occupancy falls below `want_waves`.  Needs a bound of
// at most `cap` floats and at least `min_waves` wavefronts per unit.
bool choose_ring(const Camera& cam, int32_t cap, int32_t M, int32_t max_waves, int32_t want_waves,
                 int32_t min_waves, int32_t& axis, int32_t& slot, int32_t& wpb, int32_t nslots = 3,
                 int32_t* waves_per_cu = nullptr);

// Perspective ring march: the window of a tile depends on its rays' directions
// and depth, and the kernel picks the slab axis per tile.  From a few sample
// tiles of every rendered region (box + pixel rectangle) the host sizes the
// slot to hold the windows of about 95 % of the tiles (the rest read global
// memory).  False when too few tiles would fit.
struct TileRegion {
  int64_t lo[3], hi[3];
  int32_t x0, y0, w, h;
};
// Window floats of the worst of five sampled 8 x 8 tiles of region r (its
// corners and centre) for the perspective ring march.
double persp_region_window(const Camera& cam, const TileRegion& r);
bool choose_ring_persp(const Camera& cam, const std::vector<TileRegion>& regs, int32_t cap, int32_t M,
                       int32_t max_waves, int32_t min_waves, int32_t& slot, int32_t& wpb, double fit = 0.95);

// Ring march with footprint cells (parallel rays): the work item of a
// wavefront is the set of pixels whose rays cross a brick's plane b = 0 in one
// Tf x Tg cell of (f, g) (f = axis 1, g = the other in-plane axis), so its
// window per voxel layer is the cell moved along the rays plus the rays'
// slant over two layers and the trilinear margin: rows along the storage axis
// of nf floats, ng rows, whatever the view's roll (8 x 8 pixel tiles project
// to rotated parallelograms whose bounding box is up to twice their area).
struct FootShape {
  int32_t axis = 0;           // slab axis b (1 = axis 2, 2 = axis 3)
  double Tf = 0.0, Tg = 0.0;  // cell size on the plane, voxels
  int32_t nf = 0, ng = 0;     // window extents (before rows are rounded to 16 bytes)
  int32_t slot = 0;           // floats per window slot (rows rounded up)
  int32_t wpb = 4, nslots = 3, waves = 0;
  int32_t reg = 0;            // 1: two slots, the layer after next staged in registers
  int32_t blk_f = 0, blk_g = 0;  // blocks of cells marched by one workgroup (0: a wavefront per cell)
  int32_t blk_nf = 0, blk_ng = 0, blk_slot = 0, blk_waves = 0;  // the block's window and occupancy
  double rf = 0.0, rg = 0.0;  // ray slope along f and g per unit of b
  double fa_u = 0.0, fa_v = 0.0, fb_u = 0.0, fb_v = 0.0;  // cell coordinates per pixel step
  double rays = 0.0;          // mean pixels per cell
};
// Picks b and (Tf, Tg) for one view: cells of about `rays` pixels whose rows
// of window span about whole multiples of 32 floats, at most 64 image rows and
// `cap` floats per slot; the choice with the fewest 128-byte lines per ray and
// unit of ray length, weighted by how far occupancy falls below want_waves.
// nslots_rule: 3, 2, or 0 = two slots wherever they fit more wavefronts than
// three (the plain march).  reg_waves > 0: the plain march stages the layer
// after next in registers wherever a layer's window takes at most reg_loads
// 16-byte loads per lane; two slots then, and at most reg_waves wavefronts
// per compute unit (the registers it takes).  max_px: the cell sizing keeps
// the pixels of a cell at most this (0: 64, or 128 for more than 64 rays; the
// pixels past a wavefront's 64 are marched by gathers).  False when no axis
// suits.
bool choose_foot(const Camera& cam, int32_t cap, int32_t M, int32_t max_waves, int32_t want_waves, double rays,
                 int32_t nslots_rule, FootShape& out, int32_t pad = 0, int32_t kmax = 4, int32_t reg_waves = 0,
                 int32_t reg_loads = 0, int32_t max_px = 0);
// Blocks of footprint cells for the chosen cell shape: blk_f x blk_g cells
// (at most 8) marched by one workgroup with one window per voxel layer, the
// choice with the fewest 128-byte lines per ray and layer, counting the cells
// a typical brick (edges `ext`) leaves empty in its blocks, weighted by the
// occupancy shortfall below want_waves.  force_f / force_g > 0 fix the block.
// False (fs unchanged) when a wavefront per cell is cheaper.
bool choose_foot_block(const Camera& cam, FootShape& fs, const int64_t ext[3], int32_t M, int32_t max_waves,
                       int32_t want_waves, int32_t reg_loads, int32_t force_f = 0, int32_t force_g = 0);
// 16-byte loads per lane that one window of pitch x ng floats takes (a load
// instruction carries 64 / (pitch / 4) whole rows)
int32_t window_loads(int32_t pitch, int32_t ng);
// Cells of one brick: the range of cells that rays crossing its ownership box
// fall in, and the cell coordinates of pixel (0, 0)'s ray on its plane b = 0.
void foot_cells(const Camera& cam, const FootShape& fs, const Box& box, int32_t& cf0, int32_t& cg0, int32_t& ncf,
                int32_t& ncg, double& fa0, double& fb0);

// Footprint cells of one brick of a perspective view, slab axis b (1 = axis 2,
// 2 = axis 3): the pixels whose rays (from the eye) cross the brick-local
// plane b = 0 inside one Tf x Tg rectangle.  On the plane b = V the rays of a
// cell fill that rectangle scaled about the eye's foot point by
// s(V) = 1 - V / E_b (E = eye - lo), so the window of voxel layer V is the
// scaled rectangle over [V - 1, V + 1] plus the trilinear margin.  Cells of
// about `rays` pixels (at most 64 where the pixels are densest), rows of at
// most kmax 128-byte lines, windows of at most reg_loads 16-byte loads per
// lane and cap floats.  False when the eye lies within the brick's slab along
// b, when a ray of the brick's rectangle runs the other way along b, or when
// no cell shape fits.
struct PerspCells {
  double Tf = 0.0, Tg = 0.0;
  int32_t cf0 = 0, cg0 = 0, ncf = 0, ncg = 0;
  int32_t pitch = 0, ng = 0;  // window of one voxel layer: row floats (multiple of 4), rows
  double rays = 0.0;          // mean pixels per cell where they are densest
};
bool persp_cells(const Camera& cam, int b, const Box& box, const Rect& rect, double rays, int32_t kmax,
                 int32_t cap, int32_t reg_loads, PerspCells& out, int32_t max_px = 64);

// Bytes the window loads of the footprint-cell march request over one brick
// (a model from the plan: every cell marches every layer its rays cross
// inside the brick's ownership box, windows placed and clamped as the kernel
// places them).  The terms separate what the design costs beyond the
// brick's own voxels: ghost layers and halo beyond the brick (union), halo
// shared by neighbouring cells (window), and 128-byte lines that a window
// row only partly uses (line).
struct FootTraffic {
  double own = 0.0;     // the ownership box's voxels x 4
  double uni = 0.0;     // 128-byte lines any window touches (per voxel layer and row) x 128
  double win = 0.0;     // sum over cells and loaded voxel layers of rows x pitch x 4
  double line = 0.0;    // the same rows counted in whole 128-byte lines
  double seg = 0.0;     // ... in 64-byte segments
  double cells = 0.0;   // cells with at least one layer
  double layers = 0.0;  // voxel layers loaded, summed over cells
};
void foot_traffic(const Camera& cam, const FootShape& fs, const Box& box, const int64_t n[3], FootTraffic& t);

// Sum over pixels of the whole-volume lattice count (no ERT, no skipping).
int64_t count_samples(const Camera& cam, const int64_t n[3], double step);

}  // namespace vr
