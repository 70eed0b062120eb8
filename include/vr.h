/*
 * vr.h -- C ABI of libvr: bricked GPU ray casting of a scalar spectral cube
 * with sort-last "over" compositing, for AMD Instinct MI355X (gfx950).
 *
 * Method: Hassan, Fluke & Barnes, "Interactive Visualization of the Largest
 * Radioastronomy Cubes" (arXiv:1008.0135).  The renderer casts one ray per
 * pixel through a float32 cube (Sec. 2), tests each ray against the box of
 * the data portion, samples it between entry and exit with a fixed step,
 * maps every sample through a transfer function to colour and opacity,
 * accumulates front to back and stops early once opacity reaches a threshold
 * (Sec. 2.4).  The cube is split into sub-volumes ("bricks", Sec. 2.3), each
 * rendered into its own rendering rectangle (Sec. 2.4), and the brick images
 * are combined in depth order with the over operator (Sec. 2.5).
 *
 * Conventions (all entry points):
 *  - Every function returns an int status: VR_OK (0) or a negative VR_E*
 *    code.  vr_last_error() returns a thread-local description of the most
 *    recent failure on the calling thread.  No C++ exception crosses the ABI.
 *  - Output handles (vr_ctx**, vr_volume**, ...) are written only on success.
 *    Every *_destroy(NULL) is a no-op returning VR_OK.
 *  - `stream` is a hipStream_t passed as uintptr_t (0 = the null stream).
 *    GPU work is enqueued asynchronously on it; functions that must read a
 *    GPU result on the host (noted below) synchronise that stream.
 *  - The library owns contexts, volumes (unless wrapped), brick storage,
 *    saved forward state, batch caches and internal scratch.  The caller owns
 *    every output buffer and every wrapped input; pointers documented as
 *    "device" must be device (HBM) allocations on the context's device.
 *  - Volumes are C-ordered [n3][n2][n1] float32 arrays (axis 1 fastest, axis 3
 *    spectral; FITS axis order).  Images are [H][W][4] float32, RGBA with
 *    premultiplied colour, row 0 = most negative image y, background (0,0,0,0).
 *  - Coordinates are in voxel units with voxel centres at integers; the
 *    volume's domain box is [0,n1-1] x [0,n2-1] x [0,n3-1].
 */
#ifndef VR_H
#define VR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
enum {
  VR_OK = 0,
  VR_EINVAL = -1,       /* invalid argument (NULL where required, bad size, bad range) */
  VR_ENOMEM = -2,       /* device or host allocation failed */
  VR_EHIP = -3,         /* a HIP runtime call failed (message names it) */
  VR_ENONFINITE = -4,   /* the cube holds NaN or Inf voxels */
  VR_ESTATE = -5,       /* call out of order, or saved state does not match */
  VR_EUNSUPPORTED = -6  /* valid request this build does not implement */
};

/* Description of the last failure on this thread ("" if none). */
const char *vr_last_error(void);

/* Library ABI version (increments when a struct or signature changes). */
int vr_version(void);

/* ------------------------------------------------------------------ types */
typedef struct vr_ctx vr_ctx;
typedef struct vr_volume vr_volume;
typedef struct vr_state vr_state;
typedef struct vr_batch vr_batch;

/*
 * Render request view (paper Sec. 2.2: a render request carries the
 * transformation and the projection, orthographic or perspective; Sec. 3
 * measures both).  Rows of R are the view axes in volume coordinates:
 * e1 = R[0..2] (image x), e2 = R[3..5] (image y), e3 = R[6..8] (viewing
 * direction).  Pixel (u,v) has x = ((u+1/2)/W - 1/2) S and
 * y = ((v+1/2)/H - 1/2) S H/W (c = box centre).
 *   Orthographic (eye_dist == 0): the ray starts at c + x e1 + y e2 - S e3 and
 *   runs along e3.
 *   Perspective (eye_dist = D > 0): the eye sits at c - D e3; the pixel grid
 *   lies on the plane through c normal to e3, and the ray of (u,v) starts at
 *   the eye and runs along the unit vector of x e1 + y e2 + D e3.  D must
 *   exceed half the box diagonal (the whole box then lies in front of the eye).
 * In both, samples are the step apart along the ray.  R = identity looks along
 * +axis 3 with image x = axis 1 and image y = axis 2.
 */
typedef struct {
  double R[9];     /* row-major rotation (orthonormal rows expected, not enforced) */
  int32_t W, H;    /* image size in pixels, each in [1, 16384] */
  double extent;   /* S: image width in voxels; <= 0 selects the box diagonal */
  double eye_dist; /* 0: orthographic; > 0: perspective, eye at this distance from the box centre */
} vr_view;

/* Early termination scope (Sec. 2.4; the sort-last split of Sec. 2.3/2.5):
 * VR_ERT_LOCAL: each brick accumulates from T = 1 and stops on its own (the
 *   paper's independent GPUs); brick images are then over-composited.
 * VR_ERT_GLOBAL: one opacity test over the whole ray: bricks are marched in
 *   front-to-back waves (no ray meets two bricks of one wave) straight into
 *   the frame, every ray continuing from the colour and transmittance the
 *   bricks in front left; the image equals the unbricked render.  No brick
 *   images exist (vr_render_bricks rejects it); unbricked volumes and
 *   VR_MODE_MIP are unaffected by the scope. */
enum { VR_ERT_LOCAL = 0, VR_ERT_GLOBAL = 1 };
/* VR_MODE_DVR: emission-absorption accumulated front to back, sub-volume
 * images over-composited in depth order.  VR_MODE_MIP: maximum intensity
 * projection (paper Sec. 2.4: the kernel's output is the maximum scalar value
 * recorded along each ray, and a ray stops once that value reaches its
 * maximum): M = max over the ray's samples of s = clamp((v - vmin)/(vmax -
 * vmin), 0, 1) (M = 0 without samples), stored as (M, M, M, M); sub-volume
 * images combine with the element-wise maximum; the table is not used, and
 * neither empty-space skipping nor tau applies (a ray stops when M reaches 1,
 * which leaves M unchanged). */
enum { VR_MODE_DVR = 0, VR_MODE_MIP = 1 };

/* Per-render parameters (paper Sec. 2.4: sampling distance, early termination). */
typedef struct {
  double step;       /* sample spacing along the ray in voxels, > 0 (0.5 typical) */
  double tau;        /* stop a ray after the sample where 1 - T >= tau; tau >= 1 disables */
  int32_t ess;       /* 1: empty-space skipping: skip bricks, and slabs of macrocells (when the
                        volume has them), whose transfer-function opacity is 0 over their range */
  int32_t ert_scope; /* VR_ERT_LOCAL or VR_ERT_GLOBAL */
  int32_t mode;      /* VR_MODE_DVR or VR_MODE_MIP */
  int32_t ckpt_K;    /* adjoint: longest transmittance checkpoint interval in samples (1..64; 32 typical) */
  int32_t tile;      /* pixel tile edge of one wavefront: 0 = autotuned/default (8) */
  int32_t reserved;
} vr_params;

/* Fill *p with the defaults: step 0.5, tau 0.99, ess 1, LOCAL, DVR, K 32, tile 0. */
void vr_params_default(vr_params *p);

/* ------------------------------------------------------------------ context */
/*
 * Create a context on HIP device `device` (>= 0): a transfer-function slot,
 * scratch arenas, a table-upload ring and the autotune cache.
 * Errors: VR_EINVAL (out NULL), VR_EHIP (no such device / HIP failure).
 */
int vr_create(int device, vr_ctx **out);
int vr_destroy(vr_ctx *ctx);

/* 1: record per-stage GPU times of later calls (see vr_stage_times); 0: off. */
int vr_set_profiling(vr_ctx *ctx, int on);

enum { VR_STAGE_SETUP = 0, VR_STAGE_MARCH = 1, VR_STAGE_COMPOSITE = 2, VR_STAGE_BACKWARD = 3,
       VR_STAGE_BATCH = 4, VR_NSTAGES = 5 };
/*
 * Per-stage GPU time (ms, summed over the stage's launches) of the most
 * recent profiled call, plus its launch count.  Synchronises the stream of
 * that call.  ms and launches are arrays of VR_NSTAGES (either may be NULL).
 */
int vr_stage_times(vr_ctx *ctx, double *ms, int32_t *launches);

/* ------------------------------------------------------------------ volumes */
/*
 * Upload a cube or a sub-cube (paper Sec. 2.2: the user loads the entire cube
 * or a selected sub-cube; min and max come from metadata or are recomputed
 * by the GPUs).  `src` is a [n3][n2][n1] float32 array on the host
 * (src_on_device = 0, pageable or pinned) or on the device (1).  If
 * sub_origin/sub_extent are non-NULL the volume is the box
 * [origin, origin+extent) of the source (each extent >= 2).  The data are
 * copied into library storage, scanned for non-finite values and reduced to
 * the global (min, max).  Synchronises `stream`.
 * Errors: VR_EINVAL (NULL, a dimension < 2, a sub-cube outside the source),
 * VR_ENOMEM, VR_ENONFINITE (NaN or Inf anywhere in the volume), VR_EHIP.
 */
int vr_volume_create(vr_ctx *ctx, const float *src, int src_on_device, int64_t n1, int64_t n2,
                     int64_t n3, const int64_t *sub_origin, const int64_t *sub_extent,
                     uintptr_t stream, vr_volume **out);

/*
 * Borrow a device array [n3][n2][n1] without copying (the differentiable
 * path: the caller's tensor is read directly).  The caller keeps it alive
 * and unchanged while the volume is used.  The range is computed on demand
 * (vr_volume_minmax); no non-finite scan is made.
 * Errors: VR_EINVAL, VR_EHIP.
 */
int vr_volume_wrap(vr_ctx *ctx, float *dev_ptr, int64_t n1, int64_t n2, int64_t n3, uintptr_t stream,
                   vr_volume **out);
int vr_volume_destroy(vr_volume *vol);

/* Global (min, max) over all voxels (paper Sec. 2.2).  Synchronises. */
int vr_volume_minmax(vr_volume *vol, float *vmin, float *vmax);

/* Dimensions of the volume (n[0] = n1, n[1] = n2, n[2] = n3). */
int vr_volume_dims(const vr_volume *vol, int64_t n[3]);

/* Sub-volume partitioning (paper Sec. 2.3). */
enum { VR_BRICK_GRID = 0, VR_BRICK_LONGEST_AXIS = 1 };
typedef struct {
  int32_t mode;        /* VR_BRICK_GRID or VR_BRICK_LONGEST_AXIS */
  int32_t nparts;      /* LONGEST_AXIS: number of sub-volumes, in [1, 4096] */
  int64_t size[3];     /* GRID: brick edge in cells per axis, each >= 1 */
  int32_t ghost;       /* ghost layer width: must be 1 */
  int32_t macrocell;   /* macrocell edge in cells for empty-space skipping: 0 = none, else in [2, 1024] */
  int32_t materialize; /* 1: copy each brick and its ghost layer into its own storage */
  int32_t twin;        /* 1: also keep a permuted copy of the volume (axes 1, 2, 3 = axes 2, 3, 1;
                          one more volume's worth of device memory), bricked with the same
                          sub-volumes, from which views looking mostly along axis 1 are
                          rendered (same image up to rounding).  The copy is taken now: a
                          wrapped volume whose data change needs vr_volume_brick again. */
} vr_brick_spec;

/*
 * Partition the volume into bricks.  GRID: brick j along an axis owns
 * [j*size, (j+1)*size), the last is closed at n-1 (count = ceil((n-1)/size)).
 * LONGEST_AXIS: recursive split of the longest extent (first axis on ties)
 * into floor(p/2) and p - floor(p/2) parts at the integer plane nearest the
 * proportional position (paper Sec. 2.3, equal weights).  Computes per-brick
 * (min, max) over each brick's stored voxels (ownership box plus a 1-voxel
 * ghost layer, clipped to the volume) and, with materialize = 1, copies the
 * bricks.  With macrocell = e > 0 it also computes a grid of macrocells over
 * the whole volume: macrocell (m1, m2, m3) holds the cells whose lower corner
 * index lies in [m_i e, (m_i + 1) e) on every axis, ceil((n_i - 1) / e) per
 * axis, and its (min, max) is taken over the voxels [m_i e, min((m_i + 1) e,
 * n_i - 1)] (every voxel a trilinear sample in those cells reads; NaN min
 * when one of them is not finite).  Rendering with ess = 1 then skips the
 * samples of any slab whose macrocells all have zero opacity over their range
 * (the result is unchanged: such samples add nothing and leave T as it is).
 * Re-bricking replaces the previous partition and macrocells.  Synchronises.
 * Errors: VR_EINVAL (spec NULL, size < 1, nparts out of range, ghost != 1,
 * macrocell outside {0} U [2, 1024], more than 65536 bricks), VR_ENOMEM, VR_EHIP.
 */
int vr_volume_brick(vr_volume *vol, const vr_brick_spec *spec, uintptr_t stream);

typedef struct {
  int64_t lo[3], hi[3];   /* ownership box: [lo, hi) per axis, [lo, hi] where closed */
  int32_t closed[3];
  int32_t reserved;
  int64_t slo[3], shi[3]; /* stored voxel range, inclusive (ghost included) */
  float vmin, vmax;       /* range over the stored voxels */
} vr_brick_desc;

/*
 * Number of bricks (*nb; 0 when not bricked) and, if out is non-NULL, their
 * descriptions (out must hold *nb entries on input when non-NULL: pass the
 * capacity in *nb).  Errors: VR_EINVAL (NULL nb, capacity too small).
 */
int vr_volume_brick_info(const vr_volume *vol, int32_t *nb, vr_brick_desc *out);

/*
 * Macrocell grid of the last vr_volume_brick call: *edge (0 when none),
 * count[3] macrocells per axis and, if minmax is non-NULL, their (min, max)
 * pairs copied to host memory as [count3][count2][count1][2] float32 (the
 * caller provides 2 * count1 * count2 * count3 floats; call first with
 * minmax = NULL to learn the counts).  Synchronises.
 * Errors: VR_EINVAL (NULL vol, edge or count), VR_EHIP.
 */
int vr_volume_macrocell_info(const vr_volume *vol, int32_t *edge, int64_t count[3], float *minmax);

/* ------------------------------------------------------------------ transfer function */
/*
 * Set the context's colour map (paper Sec. 2.2: generated once the global
 * range is known, sent to the renderers, and changed interactively).  `rgba`
 * is [m][4] float32 non-premultiplied, every value in [0,1], m in [2, 4096]; on the host
 * (src_on_device = 0, copied before return) or the device (1, copied on
 * `stream`; values are validated on the host and the copy synchronises).
 * The normalisation window maps v to s = clamp((v - vmin)/(vmax - vmin), 0, 1)
 * (s = 0 when vmax == vmin); vmin = vmax = 0 selects each volume's global range.
 * Lookup: u = s (m-1), i = min(floor(u), m-2), linear between entries i, i+1.
 * Errors: VR_EINVAL (m < 2 or > 4096, a value outside [0,1] or non-finite,
 * vmax < vmin, non-finite window), VR_EHIP.
 */
int vr_tf_set(vr_ctx *ctx, const float *rgba, int32_t m, double vmin, double vmax, int src_on_device,
              uintptr_t stream);

/*
 * Spectral-channel mask (paper Sec. 2.2: the user enables or disables spectral
 * channels).  `mask` is [n] float32 weights in [0, 1], one per index along
 * axis 3 (the spectral axis; 0 disables a channel), on the host
 * (src_on_device = 0) or the device (1, copied on `stream`, then validated on
 * the host).  Every sample's opacity (under VR_MODE_MIP its normalised value)
 * is multiplied by the mask interpolated linearly along axis 3 with the
 * sample's own trilinear weight: (1 - f3) mask[i3] + f3 mask[i3 + 1].  mask =
 * NULL or n = 0 removes it.  A render with a mask needs n equal to the volume's
 * axis-3 size (else VR_EINVAL); the adjoint and the batched launch do not take
 * a mask (VR_EUNSUPPORTED while one is set).
 * Errors: VR_EINVAL (n < 0, n in {1} or > 2^20, a weight outside [0, 1] or non-finite),
 * VR_EHIP.
 */
int vr_mask_set(vr_ctx *ctx, const float *mask, int32_t n, int src_on_device, uintptr_t stream);

/* ------------------------------------------------------------------ rendering */
/*
 * Render `nviews` views into out ([nviews][H][W][4] float32, device; all views
 * must share W and H).  Unbricked volume: one accumulation chain per ray
 * through the whole volume (at most 2^31 - 1 voxels).  Bricked volume: every
 * non-culled brick is rendered into its rendering rectangle with its own
 * accumulation and local early termination, then the brick images are
 * over-composited in depth order (paper Sec. 2.4, 2.5).  Sample lattice per
 * ray: t_k = t_in + (k + 1/2) step while t_k < t_out, anchored at the entry
 * into the whole volume; a sample belongs to the brick whose ownership box
 * holds it.  If save is non-NULL (unbricked volumes only), forward state for
 * vr_render_backward is kept and returned (library-owned; free it with
 * vr_state_destroy).
 * p->mode selects emission-absorption or maximum intensity projection (see
 * VR_MODE_MIP above).
 * Errors: VR_EINVAL (NULL, nviews < 1, W/H out of range or differing, bad
 * params), VR_ESTATE (no transfer function set), VR_EUNSUPPORTED (save with a
 * bricked volume or with VR_MODE_MIP; an unbricked volume of 2^31 voxels or
 * more), VR_ENOMEM, VR_EHIP.
 */
int vr_render(vr_ctx *ctx, const vr_volume *vol, const vr_view *views, int32_t nviews,
              const vr_params *p, float *out, uintptr_t stream, vr_state **save);

/* One brick image: rectangle [x0, x0+w) x [y0, y0+h) of the frame, premultiplied RGBA. */
typedef struct {
  int32_t brick, x0, y0, w, h, reserved;
  float *rgba; /* device, [h][w][4]; library arena memory (vr_render_bricks) or caller's */
} vr_brick_image;

/*
 * Sort-last first half: render the bricks of a bricked volume for one view
 * (paper Sec. 2.4: each renderer fills its rendering rectangle).  On input
 * *nimg is the capacity of imgs and order; on output the number of images.
 * order receives the front-to-back order as indices into imgs.  Image memory
 * is library arena storage valid until the next render call on this context.
 * Errors: VR_EINVAL, VR_ESTATE (not bricked, no transfer function), VR_EUNSUPPORTED
 * (VR_ERT_GLOBAL), VR_ENOMEM, VR_EHIP.
 */
int vr_render_bricks(vr_ctx *ctx, const vr_volume *vol, const vr_view *view, const vr_params *p,
                     vr_brick_image *imgs, int32_t *nimg, int32_t *order, uintptr_t stream);

/*
 * Sort-last second half: over-composite n brick images front to back into out
 * ([H][W][4] float32, device, fully written) (paper Sec. 2.5).  order lists
 * indices into imgs, front first (NULL: array order).  (Images of VR_MODE_MIP
 * renders combine with the element-wise maximum instead; vr_render does that
 * itself.)
 * Errors: VR_EINVAL (a rectangle outside W x H, an index out of range), VR_EHIP.
 */
int vr_composite(vr_ctx *ctx, const vr_brick_image *imgs, int32_t n, const int32_t *order, int32_t W,
                 int32_t H, float *out, uintptr_t stream);

/* ------------------------------------------------------------------ adjoint */
/*
 * Gradient of sum(grad_out * image) with respect to the transfer-function
 * table and the voxel values, for the views of a vr_render call made with
 * save.  grad_out: [nviews][H][W][4] float32 device.  grad_tf: [m][4] float32
 * device.  grad_vol: [n3][n2][n1] float32 device or NULL.  accumulate = 0
 * overwrites the outputs, 1 adds to them.  The normalisation window is a
 * constant.  Each ray is walked back to front, recomputing each stretch
 * forward from its saved transmittance checkpoint.  ckpt_K bounds a stretch:
 * on the ring-window layout (the default where its windows fit) a stretch is
 * a group of L cell layers of the ray's 8 x 8 tile, L = round(ckpt_K step
 * |d_b|) capped at 3 layers (the environment variable VR_BWD_LAYERS sets the
 * cap, 1 to 16: longer groups need more LDS per wavefront), so a checkpoint
 * falls every min(ckpt_K, about 3 / (step |d_b|)) samples (vr_state_info
 * reports it per view); otherwise a stretch is a segment of exactly ckpt_K
 * samples.  Views run side by side on the library's side streams (forked from
 * and joined back to `stream`; VR_BWD_SIDE=0 runs them one after another).
 * Synchronises with `stream` at the end (it checks the adjoint's
 * per-group sample bound).
 * Errors: VR_EINVAL, VR_ESTATE (state from another volume, or the transfer
 * function changed since the forward), VR_EHIP (also a group beyond its
 * sample bound).
 */
int vr_render_backward(vr_ctx *ctx, const vr_volume *vol, const vr_state *st, const float *grad_out,
                       float *grad_tf, float *grad_vol, int accumulate, uintptr_t stream);
int vr_state_destroy(vr_state *st);

/*
 * How the forward state of one view checkpoints the transmittance (the
 * interval the adjoint recomputes from): ring = 1 when the view uses the
 * ring-window layout, whose checkpoints sit at the start of each group of
 * layers_per_group cell layers of a ray's 8 x 8 tile, i.e. every
 * samples_per_group = layers_per_group / (step |d_b|) samples along the ray
 * (d_b: the view direction's component along the slab axis); ring = 0: every
 * ckpt_K samples (layers_per_group = 0).  Any output pointer may be NULL.  No
 * GPU use.  Errors: VR_EINVAL.
 */
int vr_state_info(const vr_state *st, int32_t view, int32_t *ring, int32_t *layers_per_group,
                  double *samples_per_group);

/* ------------------------------------------------------------------ batched */
/* One request of a batch: its own volume (unbricked), view, table, window and output. */
typedef struct {
  const vr_volume *vol;
  vr_view view;
  const float *tf; /* device [m][4], values in [0,1] */
  int32_t m;
  int32_t reserved;
  double vmin, vmax; /* window; vmin = vmax = 0 selects the volume's range */
  float *out;        /* device [view.H][view.W][4] */
} vr_request;

/*
 * Render n requests in one persistent launch: (request, pixel tile) work
 * items, ordered by estimated cost, are pulled from an atomic counter by a
 * grid sized to the device.  The launch sequence is captured once into a HIP
 * graph held in *cache (created when *cache is NULL) and replayed while the
 * request shapes (count, volumes, image sizes, table sizes) match; otherwise
 * it is rebuilt.  Table values, views, windows and output pointers may change
 * between calls.  Errors: VR_EINVAL, VR_EUNSUPPORTED (p->mode other than
 * VR_MODE_DVR), VR_ENOMEM, VR_EHIP.
 */
int vr_render_batch(vr_ctx *ctx, const vr_request *reqs, int32_t n, const vr_params *p, vr_batch **cache,
                    uintptr_t stream);
int vr_batch_destroy(vr_batch *b);

/*
 * Allocation-free variant of vr_render_batch, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The same persistent kernel and the same
 * images, launched directly (no graph); its descriptor table and work counter
 * live in a fixed device array of the library (at most 512 requests, about 160 KiB
 * per device, held by each device the library runs on until the process
 * ends); the descriptors travel through pinned staging made by vr_create.
 * The call allocates nothing.  Windows must be given, or the volume's range
 * already known (vr_volume_create computes it).  Every call on one device
 * shares that device's array: calls on one context are ordered, but calls
 * through different contexts of one device must not overlap in time (they
 * would race on the array).  Errors: VR_EINVAL (n outside [1, 512], bad
 * request), VR_ESTATE (a volume range not known yet), VR_EUNSUPPORTED
 * (p->mode other than VR_MODE_DVR, a channel mask set), VR_EHIP.
 */
int vr_render_batch_noalloc(vr_ctx *ctx, const vr_request *reqs, int32_t n, const vr_params *p,
                            uintptr_t stream);

/* ------------------------------------------------------------------ autotuning */
typedef struct {
  int32_t tile;          /* chosen wavefront tile edge (pixels) */
  int32_t waves_per_cu;  /* chosen persistent-grid occupancy (batched path) */
  double ms;             /* best measured time */
  double ms_default;     /* time with the defaults */
  int32_t lds_budget;    /* chosen LDS floats per slab box (LDS-staged march) */
  int32_t march_mode;    /* 0: LDS-staged slabs where they fit, 1: gathers */
} vr_tune_result;

/*
 * Time candidate launch shapes for rendering `view` of `vol` -- wavefront
 * tile (4x16, 8x8, 16x4 pixels), LDS budget of the slab-staged march, or the
 * gather march -- and store the fastest in the context's cache, keyed by the
 * volume's size class (floor(log2) per axis), bricked or not, and the image
 * size; later renders with p->tile = 0 on that key use it.  The cache is read
 * from and written to the file named by the environment variable
 * VR_TUNE_CACHE when set.  Synchronises.
 * Errors: VR_EINVAL, VR_ESTATE (no transfer function), VR_ENOMEM, VR_EHIP.
 */
int vr_autotune(vr_ctx *ctx, const vr_volume *vol, const vr_view *view, const vr_params *p,
                vr_tune_result *out, uintptr_t stream);

/*
 * Autotune the batched launch of these requests (a training-system pattern,
 * not in the paper).  First the tile shape per size class: requests are
 * grouped by volume size class (floor(log2 voxels) / 3) and image class
 * (floor(log2 pixels) / 2); the requests of each class are rendered as a
 * batch of their own with 8 x 8, 16 x 4, 4 x 16 and 32 x 2 pixel tiles, and
 * the fastest is kept per class.  Then the persistent grid: 2, 4, 8, 16 and
 * 32 wavefronts per compute unit over the whole batch with the tuned tiles.
 * Both choices apply to later batched calls on this context (and are written
 * to VR_TUNE_CACHE); *cache is left holding the graph of the chosen shapes.
 * out->tile is the tile chosen for most classes.  Synchronises.
 * Errors: as vr_render_batch.
 */
int vr_autotune_batch(vr_ctx *ctx, const vr_request *reqs, int32_t n, const vr_params *p, vr_batch **cache,
                      vr_tune_result *out, uintptr_t stream);

/*
 * Tile width (4, 8, 16 or 32 pixels; the tile is 64 pixels) each request of a
 * batch would run with: the autotuner's choice for its size class, else 8.
 * tiles: [n] host.  No GPU use.  Errors: VR_EINVAL.
 */
int vr_batch_tiles(const vr_ctx *ctx, const vr_request *reqs, int32_t n, int32_t *tiles);

/* ------------------------------------------------------------------ host-only helpers */
/*
 * Rendering rectangles, depth order and front-to-back waves for a brick
 * partition of a volume of size dims and one view (paper Sec. 2.4: the
 * rectangle bounds the projection of the brick; it never changes the image).
 * No GPU use.  rects: [nb][4] (x0, y0, w, h; w = 0 for an empty rectangle),
 * order: [nb] brick indices front to back, waves: [nb] wave of each brick
 * under VR_ERT_GLOBAL (no ray meets two bricks of one wave; every ray meets
 * its bricks in increasing wave order).  Each output may be NULL.  *nb is the
 * capacity on input, the brick count on output.  Errors: VR_EINVAL.
 */
int vr_plan_view(const int64_t dims[3], const vr_brick_spec *spec, const vr_view *view, int32_t *nb,
                 int32_t *rects, int32_t *order, int32_t *waves);

/*
 * The partition vr_volume_brick would make for a volume of size dims, without
 * a GPU: ownership boxes and stored (ghost) ranges; vmin/vmax are left 0.
 * *nb is the capacity of out on input (out may be NULL to query the count),
 * the brick count on output.  Errors: VR_EINVAL.
 */
int vr_partition(const int64_t dims[3], const vr_brick_spec *spec, int32_t *nb, vr_brick_desc *out);

/*
 * Nominal sample count of a view: the sum over pixel rays of the lattice
 * count inside the whole-volume box (no early termination, no skipping).
 * No GPU use.  Errors: VR_EINVAL.
 */
int vr_count_samples(const int64_t dims[3], const vr_view *view, double step, int64_t *nominal);

/*
 * Window traffic of the footprint-cell march for one parallel view (a model
 * from the plan, no GPU use).  The march of Sec. 2.4 reads every voxel of a
 * rendered brick once at best (own_bytes); the cell march loads, per cell
 * and voxel layer, a window of rows along axis 1 that its rays' samples
 * between two neighbouring layers can touch.  Every cell is taken to march
 * every layer its rays cross inside the brick (no early termination), with
 * the windows placed and clamped as the kernel places them.  The terms:
 *   union_bytes   128-byte lines that any window of a brick touches, per
 *                 voxel layer and row (the brick with its ghost layers and the
 *                 halo beyond its sides: what perfect reuse would fetch);
 *   window_bytes  sum over cells and loaded layers of rows x row floats x 4
 *                 (adds the halo that neighbouring cells share);
 *   line_bytes    the same rows counted in whole 128-byte lines (adds the
 *                 partly used lines at the rows' ends): the traffic with no
 *                 reuse between cells.
 * rays: mean pixels per cell (0: the library's default), kmax: window rows of
 * at most this many 128-byte lines (0: default), tf_entries: table entries
 * (they share the compute unit's LDS with the windows; 0: 256).  Bricks are
 * those of spec over a volume of size dims, every brick with a non-empty
 * rectangle counted (no transfer-function culling); with spec->twin set, a
 * view looking mostly along axis 1 is planned on the permuted copy, as it is
 * rendered.  Errors: VR_EINVAL (bad arguments, or a perspective view), and
 * VR_EUNSUPPORTED when the view has no slab axis for the cell march.
 */
typedef struct {
  double own_bytes, union_bytes, window_bytes, line_bytes;
  double segment_bytes;          /* the rows of line_bytes counted in 64-byte segments */
  double cells, cell_layers;     /* cells with samples; voxel layers loaded over all cells */
  double rays_per_cell;          /* mean pixels per cell of the chosen shape */
  double Tf, Tg;                 /* cell size on the slab plane, voxels */
  int32_t axis;                  /* slab axis (2 or 3, of the volume rendered: the copy's for a permuted view) */
  int32_t row_floats, rows;      /* window row length (floats, a multiple of 4) and rows per window */
  int32_t twin;                  /* 1: planned on the permuted copy */
} vr_cell_traffic;

int vr_plan_cells(const int64_t dims[3], const vr_brick_spec *spec, const vr_view *view, double rays, int32_t kmax,
                  int32_t tf_entries, vr_cell_traffic *out);

#ifdef __cplusplus
}
#endif

#endif /* VR_H */
