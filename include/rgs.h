/*
 * rgs.h -- C ABI of librgs.so, the MI355X (gfx950) partitioned 3D Gaussian
 * splatting rasterizer of RetinaGS (arXiv 2406.11836).
 *
 * The method (Sec. 3.2-3.4 of the paper): the scene is cut into K = 2^L
 * convex cells by a KD tree over the Gaussian centres (Sec. 3.3); for every
 * pixel ray, each cell k blends, front to back, the Gaussians whose ray
 * crossing point lies inside it (Eq. 3, Eq. 4 with the indicator of Eq. 6)
 * into a partial colour C_k and transmittance T_k; the partials are merged in
 * the order the ray visits the cells (Eq. 5), which reproduces the
 * single-worker render (Eq. 2) exactly.  Here all K cells live on one GPU and
 * the merge is an on-device pass; the backward sends the loss gradient
 * through the merge to every cell (Sec. 3.4).
 *
 * Conventions (all entry points):
 *   - Pointers are device memory unless marked [host].  The caller owns every
 *     buffer, including workspaces sized by the *_workspace() queries; the
 *     library never allocates and keeps no state between calls, so calls on
 *     different streams with disjoint buffers may run concurrently.
 *     Workspaces must be 256-byte aligned (any hipMalloc'd pointer is).
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = default stream) and
 *     the call returns without waiting, except rgs_bin_sort, which copies one
 *     counter to the host (the instance count) and therefore waits once
 *     (rgs_bin_sort_async does not).
 *   - Argument errors are reported synchronously (RGS_E_ARG) and enqueue
 *     nothing.  They include an output buffer that overlaps an input or
 *     another output (byte ranges from the sizes each call implies).  A failed kernel launch returns RGS_E_HIP and records the HIP
 *     error code (rgs_last_hip_error, per thread).  Faults inside kernels
 *     surface at the caller's next synchronisation.
 *   - Degenerate data is not an error: Gaussians behind z_near, with a zero
 *     quaternion, opacity below 1/255 or an empty footprint are culled (no
 *     instances, zero gradient); N = 0 renders the background with T = 1.
 *   - Gradient outputs are overwritten, never accumulated.
 *
 * Layouts (float32, structure of arrays):
 *   means [3][N], log_scales [3][N], quats [4][N] (w, x, y, z),
 *   opacity [N] (logit; alpha = sigmoid), sh [3 (D+1)^2][N] with row
 *   3 j + channel for the real SH index j = l^2 + l + m, D = sh_degree <= 3.
 *   A view's image is [3][H][W]; several views are concatenated in order.
 *   "src" numbers a (view, Gaussian) pair: src = view * N + gid.
 */
#ifndef RGS_H
#define RGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RGS_ABI_VERSION 7
#define RGS_TILE 16       /* screen tiles are 16 x 16 pixels */
#define RGS_MAX_L 6       /* K = 2^L <= 64 cells */
#define RGS_MAX_VIEWS 16  /* views per call */
#define RGS_REC_FLOATS 16 /* floats per projected render record (64 bytes, one aligned line) */
#define RGS_T_FLOOR 0x1p-100f /* a pixel always stops in a cell once T_k < max(eps_T, RGS_T_FLOOR) */

/* How rgs_kd_partition places each node's cut (Sec. 3.3; Sec. 4.2, Table 2). */
enum {
    RGS_SPLIT_MEDIAN = 0,   /* the paper's KD tree: equal-count bisection */
    RGS_SPLIT_MIDPOINT = 1  /* the fixed-size partition it is compared with: a uniform grid */
};

/* Which Gaussians each cell renders (rgs_project_sh). */
enum {
    RGS_CELLS_EXACT = 0,          /* every cell its footprint's ray crossing points can reach
                                     (Eq. 6): the merged image equals the single-worker render */
    RGS_CELLS_PAPER_SUBSETS = 1,  /* only cells k whose subset N_k (centre within the leaf box
                                     inflated by D_i, Sec. 3.3) holds the Gaussian: contributions
                                     whose crossing point lies elsewhere are lost ("escapes") */
    RGS_CELLS_EXCLUSIVE = 2       /* the cell of the centre only, without the indicator of Eq. 6:
                                     the cell-based methods the paper contrasts with (Sec. 2,
                                     Sec. 4.2), whose borders leak */
};

typedef int32_t rgs_status;
enum {
    RGS_OK = 0,
    RGS_E_ARG = -1,         /* invalid argument; nothing enqueued */
    RGS_E_CAPACITY = -2,    /* caller buffers too small; see *n_required */
    RGS_E_HIP = -3,         /* a HIP call failed; see rgs_last_hip_error() */
    RGS_E_UNSUPPORTED = -4  /* size outside what the library supports */
};

typedef void *rgs_stream; /* hipStream_t */

int32_t rgs_abi_version(void);
const char *rgs_status_string(rgs_status status);
int32_t rgs_last_hip_error(void);

/* Gaussian parameters (Sec. 3.1: centre mu, covariance from scale and
 * rotation, opacity alpha, SH colour). */
typedef struct {
    int64_t n;
    int32_t sh_degree;
    const float *means;
    const float *log_scales;
    const float *quats;
    const float *opacity;
    const float *sh;
} rgs_gaussians;

/* Gradients w.r.t. the parameters, same layouts (written, not accumulated). */
typedef struct {
    float *means;
    float *log_scales;
    float *quats;
    float *opacity;
    float *sh;
} rgs_gaussians_grad;

/* [host] Pinhole camera, OpenCV axes (x right, y down, z forward):
 * p_cam = R p_world + t, R row-major; campos is the camera centre o of the
 * paper's rays l(t) = o + t d (Sec. 3.2).  Pixel (x, y) samples image point
 * (x + 0.5, y + 0.5).  bg is added once, after the merge. */
typedef struct {
    float R[9];
    float t[3];
    float campos[3];
    float fx, fy, cx, cy;
    int32_t width, height;
    float z_near;
    float bg[3];
} rgs_camera;

/* KD tree of depth L over the Gaussian centres (Sec. 3.3). */
typedef struct {
    int32_t L;
    float *split;          /* [max(K-1,1)] split values, heap order; axis of a node = depth mod 3 */
    float *box_lo;         /* [3][K] leaf boxes, half-open [lo, hi), +-inf outer faces */
    float *box_hi;         /* [3][K] */
    int32_t *center_cell;  /* [N] leaf containing each centre (output of rgs_kd_partition) */
    int32_t *counts;       /* [K] centres per leaf */
    uint32_t *own_mask;    /* [N][ceil(K/32)] the paper's subsets N_k, or NULL to skip */
    float *cell_bounds;    /* [8][K] per cell: min x, y, z and max x, y, z of its centres (empty
                              cell: +inf / -inf), the largest scale exp(log_scale) of its Gaussians
                              (0 if empty), and 0; or NULL to skip.  rgs_cell_visibility reads a
                              host copy; rgs_group_by_cell the device one. */
} rgs_kdtree;

/* Per-(view, Gaussian) projection output.  Where count is 0 (culled) only
   count is written: rec, bin and depth hold whatever the buffers held. */
typedef struct {
    float *rec;         /* [V*N][16]: mx, my, ca, k | e, alpha, tau, z | r, g, b, flags |
                           (footprint d^2 = ca (dx + k dy)^2 + e dy^2, i.e. the conic
                           ca, cb = k ca, cc = e + k cb, with dx = x + 0.5 - mx) |
                           rect as two uint32 (x_lo | x_hi << 16, y_lo | y_hi << 16), then
                           the row-span descriptor as two uint32 (low word first): for a
                           rectangle of <= 8 tile rows and <= 15 tile columns, byte k =
                           (tiles of row k) << 4 | (its first column - the rectangle's
                           first tile column), else all ones;
                           64-byte aligned: the render kernels fetch one line per instance */
    uint32_t *bin;      /* [V*N][8] words, 32-byte aligned: the binning record of a pair, which
                           the instance emission reads as one line: words 0-1 the rect (as in
                           rec), words 2-3 the row-span descriptor (as in rec), words 4-5 the
                           cell mask (low word first; bit k = cell k: the cells the footprint
                           can reach), word 6 the instance count, word 7 the tiles per cell */
    uint32_t *count;    /* [V*N]: instances = |cell mask| * tiles of the rectangle that the
                           footprint's ellipse can reach (per tile row, the span of columns
                           holding a pixel centre of the padded ellipse); 0 = culled */
    float *depth;       /* [V*N]: camera depth z (the same value as in rec): the key of the
                           depth order, read densely by binning */
} rgs_projected;

/* Tile/cell instance lists and slots (one slot per non-empty (tile, cell)). */
typedef struct {
    int64_t capacity;       /* instance capacity of keys and vals */
    int64_t slot_capacity;  /* slot capacity: >= min(instances, total_tiles * K) */
    uint32_t *keys;         /* [capacity] sorted keys (global_tile << L) | rank of cell in view order */
    uint64_t *vals;         /* [capacity] sorted (src << 32) | position in emission order */
    uint32_t *pair_src;     /* [V*N] visible pairs in (view, depth, gid) order */
    uint32_t *pair_off;     /* [V*N+1] first instance of each ordered pair */
    int32_t *pair_rank;     /* [V*N] position of src in pair_src (valid where count > 0) */
    uint32_t *slot_key;     /* [slot_capacity] key of each slot */
    uint32_t *slot_range;   /* [slot_capacity][2] begin, end into keys/vals */
    uint32_t *tile_slot;    /* [total_tiles+1] first slot of each global tile (slots of a tile are in view order) */
    uint32_t *slot_order;   /* [slot_capacity] slots by decreasing size class of their instance count (the
                               backward launches its slots by the instances it visits instead, ordered in its
                               workspace from the forward's `last`) */
    uint32_t *tile_order;   /* [total_tiles] tiles by decreasing size class of their instance count (the forward's
                               launch order) */
    uint32_t *counters;     /* [4]: pairs, instances, slots, required instances if over capacity (async; else 0);
                               all four written by every bin_sort call */
    int64_t n_instances;    /* [out, host] */
} rgs_bins;

/* Per-slot partial maps (Eq. 3, Eq. 4): 256 pixels of the slot's tile. */
typedef struct {
    float *C;        /* [slot_capacity][3][256] partial colour C_k */
    float *T;        /* [slot_capacity][256]    partial transmittance T_k */
    uint32_t *last;  /* [slot_capacity][256]    1 + index in the slot of the last processed instance */
} rgs_partials;

typedef struct {
    float *dC;       /* [slot_capacity][3][256] dL/dC_k */
    float *dT;       /* [slot_capacity][256]    dL/dT_k */
} rgs_partials_grad;

/* ------------------------------------------------------------------ */
/* Views                                                               */
/* ------------------------------------------------------------------ */
/* Size of the device view table. */
size_t rgs_views_bytes(void);
/* Writes the device view table for n_views cameras (<= RGS_MAX_VIEWS) and the
 * per-view cell order ([host] rank_of[v][K]: rank of cell k in view v's merge
 * order, from rgs_cell_order).  Copies from host memory on `stream`; the
 * host arrays may be reused when the call returns.  Global tiles of view v
 * follow those of views 0..v-1 (16 x 16 tiles, row-major).  Returns
 * RGS_E_UNSUPPORTED if the views hold 2^32 pixels or more in all, or if
 * (total tiles << L) reaches 2^31 (pixel offsets and tile keys are 32-bit). */
/* cell_visible ([host] n_views masks, or NULL = every cell): bit k clear
 * promises that no Gaussian whose centre lies in cell k (kd->center_cell) can
 * reach view v; rgs_project_sh then culls those Gaussians without reading
 * their parameters.  rgs_cell_visibility computes such masks; a caller that
 * clears bits by other means must be as conservative (a wrong mask changes
 * the image). */
rgs_status rgs_views_upload(const rgs_camera *cams, int32_t n_views, int32_t L,
                            const int32_t *rank_of, const uint64_t *cell_visible, void *views_dev,
                            rgs_stream stream);
/* [host] The same table written to host memory (views_host: rgs_views_bytes()
 * bytes), for a caller that copies it to the device itself, e.g. from pinned
 * memory without waiting (rgs_views_upload waits for its stream so that its
 * stack copy has been consumed). */
rgs_status rgs_views_pack(const rgs_camera *cams, int32_t n_views, int32_t L, const int32_t *rank_of,
                          const uint64_t *cell_visible, void *views_host);
/* [host] total 16x16 tiles over the views. */
int64_t rgs_total_tiles(const rgs_camera *cams, int32_t n_views);

/* ------------------------------------------------------------------ */
/* KD partition (Sec. 3.3)                                             */
/* ------------------------------------------------------------------ */
/* Depth-L tree: at depth l the axis is l mod 3 (X, Y, Z in turn) and, with
 * rule RGS_SPLIT_MEDIAN, the split is the floor(n/2)-th smallest coordinate
 * (0-based, IEEE total order) of the node's centres; centres below the split
 * go left, the rest right; an empty node splits at the midpoint of its finite
 * bounds (one finite bound: that bound; none: 0).  With RGS_SPLIT_MIDPOINT
 * every node splits at 0.5f * (lo + hi) of its extent inside the bounding box
 * of all centres (0 if there are none): a uniform grid of 2^ceil(L/3) x
 * 2^ceil((L-1)/3) x 2^floor(L/3) blocks.  Leaves are numbered by their path bits (left 0,
 * right 1), first level most significant.  own_mask, if not NULL, marks
 * N_k = { i : centre in the leaf box inflated by D_i on every face },
 * D_i = d_factor * max_a exp(log_scale_a) (the paper uses three times the
 * major axis).  Writes split, box_lo/hi, center_cell, counts, own_mask and
 * cell_bounds (the box of N_k's inflated centres: what a view must see for
 * cell k to matter, used for cell culling). */
size_t rgs_kd_partition_workspace(int64_t n, int32_t L);
rgs_status rgs_kd_partition(const rgs_gaussians *g, int32_t L, float d_factor, int32_t rule,
                            const rgs_kdtree *kd, void *ws, size_t ws_bytes, rgs_stream stream);

/* A copy of the Gaussians grouped by cell (Sec. 3.3: sub-model k holds the
 * Gaussians of its cell): out[j] = in[perm[j]], cells ascending, and inside
 * a cell along a Morton curve over the cell's bounds (8 bits per axis),
 * ties in gid order.  kd must come from rgs_kd_partition on `in` with
 * cell_bounds set; `out` has the same n and sh_degree and shares no buffer
 * with `in`; perm ([N] int32, device) may be NULL.  Running rgs_kd_partition
 * on `out` gives the same splits, boxes and counts (the tree depends only on
 * the set of centres).  Views that cannot see a cell then skip a contiguous
 * range of Gaussians, whose parameters projection never reads. */
size_t rgs_group_by_cell_workspace(int64_t n);
rgs_status rgs_group_by_cell(const rgs_gaussians *in, const rgs_kdtree *kd, int32_t L, const rgs_gaussians *out,
                             int32_t *perm, void *ws, size_t ws_bytes, rgs_stream stream);

/* [host] Cell culling for a batch of views (Sec. 3.4: the manager hands a
 * render request only to the sub-models it concerns).  cell_bounds_host:
 * [8][K] as written by rgs_kd_partition; any number of views (not limited
 * to RGS_MAX_VIEWS); visible: [n_views] masks, bit k set
 * unless no Gaussian of cell k can reach view v.  Conservative: a cell is
 * dropped only if, for every centre in its box and the cell's largest scale,
 * the centre lies behind z_near or the footprint's rectangle misses the
 * image on one side.  The bound covers the EWA linearisation at the clamped
 * Jacobian (the footprint of an off-axis Gaussian reaches up to (1 + guard)
 * times the 3-sigma radius), the 0.3 px^2 low-pass, tau <= 9 and the
 * rectangle's rounding pads, so passing the masks to rgs_views_upload /
 * rgs_views_pack changes no output.  Empty cells are dropped; cells with
 * non-finite bounds are kept. */
rgs_status rgs_cell_visibility(const rgs_camera *cams, int32_t n_views, int32_t L, const float *cell_bounds_host,
                               uint64_t *visible);

/* [host] The order in which any ray from campos visits the cells (Eq. 5's
 * permutation o_l): in-order traversal, near child first, near = left iff
 * campos[axis] < split.  order[r] = cell at rank r; rank_of[k] = rank of k. */
rgs_status rgs_cell_order(int32_t L, const float *split_host, const float campos[3], int32_t *order,
                          int32_t *rank_of);

/* ------------------------------------------------------------------ */
/* Projection and SH colour (Sec. 3.1)                                  */
/* ------------------------------------------------------------------ */
/* Per (view, Gaussian): activations, EWA screen covariance with a 0.3 px^2
 * low-pass and the Jacobian at the guarded camera-space centre, its inverse
 * (conic), screen mean, cut threshold tau = min(9, 2 ln(255 alpha))
 * (contribution iff d^2 <= tau), SH colour 0.5 + sum f Y clamped at 0,
 * sample-pixel rectangle, the cell set (KD leaves met by the padded box of
 * the footprint's ray crossing points), the instance count and the camera
 * depth (also dense in out->depth, the key of binning's depth order).
 * rec[11] holds flag bits (bit 0: the footprint lies in one cell). */
/* cells (RGS_CELLS_*) restricts which cells a Gaussian is listed in:
 * PAPER_SUBSETS needs kd->own_mask; EXCLUSIVE needs kd->center_cell and sets
 * flag bit 0 (no indicator test).  If the views carry cell visibility masks,
 * kd->center_cell must be set. */
rgs_status rgs_project_sh(const rgs_gaussians *g, const rgs_camera *cams, int32_t n_views,
                          const void *views_dev, const rgs_kdtree *kd, int32_t cells,
                          const rgs_projected *out, rgs_stream stream);

/* ------------------------------------------------------------------ */
/* Binning and sorting                                                  */
/* ------------------------------------------------------------------ */
/* Orders the visible (view, Gaussian) pairs by (view, depth z, gid), emits one
 * instance per (pair, cell in its cell set, tile in its rectangle), sorts the
 * instances stably by (global tile, rank of the cell in the view's order) with
 * an LSD radix sort, and builds the slot table.  Copies the instance count to
 * host (*n_required, bins->n_instances); if it exceeds bins->capacity, or the
 * slot bound exceeds bins->slot_capacity, returns RGS_E_CAPACITY having
 * written only the pair arrays; the caller grows the buffers and calls again. */
size_t rgs_bin_sort_workspace(int64_t n, int32_t n_views, int64_t total_tiles, int32_t L, int64_t capacity);
rgs_status rgs_bin_sort(const rgs_projected *proj, int64_t n, const rgs_camera *cams, int32_t n_views,
                        const void *views_dev, int32_t L, rgs_bins *bins, int64_t *n_required,
                        void *ws, size_t ws_bytes, rgs_stream stream);

/* The same without waiting on the host (for a pass whose buffers were sized by
 * an earlier one, e.g. a training step): the instance count stays on the
 * device and grids are sized by the capacities, so the host can enqueue the
 * rest of the pass at once.  Requires bins->slot_capacity >=
 * min(bins->capacity, total_tiles << L).  If the instances exceed
 * bins->capacity, counters[3] receives the required count and counters[0..2]
 * are zeroed: every later call of the pass finds no work and writes no more
 * than the background, and the caller must grow the buffers and redo the
 * pass.  counters[3] == 0 means the pass is valid.  Sets bins->n_instances to
 * -1 (unknown on the host). */
rgs_status rgs_bin_sort_async(const rgs_projected *proj, int64_t n, const rgs_camera *cams, int32_t n_views,
                              const void *views_dev, int32_t L, rgs_bins *bins, void *ws, size_t ws_bytes,
                              rgs_stream stream);

/* ------------------------------------------------------------------ */
/* Partial render (Eq. 3, Eq. 4, Eq. 6)                                 */
/* ------------------------------------------------------------------ */
/* For every slot (tile t, cell k) and pixel p of t, front to back over the
 * slot's instances: the instance contributes iff d^2 <= tau and its crossing
 * point x = campos + z D(p) lies in cell k's box; sigma = min(0.99,
 * alpha exp(-d^2/2)); C_k += T_k sigma c; T_k *= 1 - sigma.  The slots of a
 * tile are walked in the view's merge order, so P_k T_k (P_k = product of
 * the T_m of the tile's earlier slots at p) is the merged render's
 * transmittance: a pixel stops after the contribution that takes P_k T_k
 * below max(eps_T, RGS_T_FLOOR), and every later slot of its tile keeps
 * C = 0, T = 1, last = 0 at that pixel.  With the exact cell sets this is
 * the plain render's early termination (eps_T = 0: at the floor only; what
 * lies behind it weighs less than 2^-100).  eps_T must lie in [0, 1). */
/* stats, if not NULL, must point to two device uint64 counters that are
 * incremented by the number of (pixel, instance) pairs the method must test
 * (pixel inside the Gaussian's rectangle and not yet stopped) and of pairs
 * that contributed. */
rgs_status rgs_render_partial(const rgs_projected *proj, int64_t n, const rgs_bins *bins,
                              const rgs_camera *cams, int32_t n_views, const void *views_dev,
                              const rgs_kdtree *kd, float eps_T, const rgs_partials *out,
                              uint64_t *stats, rgs_stream stream);

/* The partial render and the merge of Eq. 5 in one launch, for a caller
 * that renders every cell of a tile itself (one GPU): writes the same
 * partials as rgs_render_partial, and image / T_final exactly as
 * rgs_merge_partials would write them from those partials (the render block
 * folds each slot into the merged pixel in the same order and arithmetic as
 * the merge, so the results are bit-identical; the merge's second read of
 * the partials is saved).  image: concatenated [3][H][W] per view; T_final:
 * concatenated [H][W]; both device memory owned by the caller, disjoint from
 * every other buffer of the call (RGS_E_ARG otherwise).  Other arguments,
 * stats and errors as rgs_render_partial. */
rgs_status rgs_render_partial_merged(const rgs_projected *proj, int64_t n, const rgs_bins *bins,
                                     const rgs_camera *cams, int32_t n_views, const void *views_dev,
                                     const rgs_kdtree *kd, float eps_T, const rgs_partials *out,
                                     float *image, float *T_final, uint64_t *stats, rgs_stream stream);

/* ------------------------------------------------------------------ */
/* Merge (Eq. 5)                                                        */
/* ------------------------------------------------------------------ */
/* Per pixel: fold (C, T) <- (C + T C_k, T T_k) over the tile's slots in the
 * view's cell order starting from (0, 1); image = C + T bg, T_final = T.
 * image: concatenated [3][H][W] per view; T_final: concatenated [H][W]. */
rgs_status rgs_merge_partials(const rgs_partials *parts, const rgs_bins *bins, const rgs_camera *cams,
                              int32_t n_views, const void *views_dev, float *image, float *T_final,
                              rgs_stream stream);

/* ------------------------------------------------------------------ */
/* Loss (L1 + w (1 - SSIM))                                             */
/* ------------------------------------------------------------------ */
/* One view, [3][H][W] in [0,1]: L1 = mean |x - y|; SSIM with an 11x11
 * Gaussian window (std 1.5), zero padding, C1 = 1e-4, C2 = 9e-4, mean over
 * 3HW.  Writes the scalar loss (device) and d loss / d image. */
size_t rgs_loss_workspace(int32_t H, int32_t W);
rgs_status rgs_loss_l1_ssim(const float *image, const float *target, int32_t H, int32_t W,
                            float ssim_weight, float *loss, float *d_image, void *ws, size_t ws_bytes,
                            rgs_stream stream);

/* The same loss for callers that cannot allocate (code under HIP graph
 * capture, serving loops, hosts that forbid allocation): no workspace
 * argument and no allocation of any kind.  The workspace is a fixed
 * RGS_LOSS_SCRATCH_BYTES array in device memory, one per device, which the
 * library holds until the process ends; its address is looked up once per
 * device on the first call there (the current device; the stream must belong
 * to it).  Returns RGS_E_CAPACITY, with nothing enqueued, when the view needs
 * more than the array (rgs_loss_workspace(H, W) > RGS_LOSS_SCRATCH_BYTES:
 * up to about 3.7 Mpx, e.g. 2560x1440; 3840x2160 does not fit).  Every call
 * on one device uses the same array: calls that overlap in time on one
 * device (other streams, other threads) race and give wrong results; calls
 * in one stream are ordered and safe.  Nothing in the array has to start at
 * zero: each call writes every word it reads.  Results equal those of
 * rgs_loss_l1_ssim. */
#define RGS_LOSS_SCRATCH_BYTES ((size_t)128 << 20)
rgs_status rgs_loss_l1_ssim_noalloc(const float *image, const float *target, int32_t H, int32_t W,
                                    float ssim_weight, float *loss, float *d_image, rgs_stream stream);

/* ------------------------------------------------------------------ */
/* Backward                                                             */
/* ------------------------------------------------------------------ */
/* Merge backward (the manager's gradient to every sub-model, Sec. 3.4):
 * dC_k = P_k g, dT_k = P_k (<g, R_k> + gT Q_k) with P_k the transmittance
 * before k, R_k the merged colour (with background) after k and Q_k the
 * transmittance after k.  d_T_final may be NULL (zero). */
rgs_status rgs_merge_partials_bwd(const float *d_image, const float *d_T_final, const rgs_partials *parts,
                                  const rgs_bins *bins, const rgs_camera *cams, int32_t n_views,
                                  const void *views_dev, const rgs_partials_grad *out, rgs_stream stream);

/* Partial-render backward plus the per-pair reduction: back to front from
 * each pixel's `last`, recovering the transmittance before each contribution
 * by division, giving per-instance gradients of (screen mean, conic, alpha,
 * colour) summed over the tile's pixels, then summed over each pair's
 * instances in a fixed order (no atomics).  d_proj: [9][V*N] rows
 * d mx, d my, d ca, d cb, d cc, d alpha, d r, d g, d b (zero for culled
 * pairs; cb is the off-diagonal conic entry). */
size_t rgs_render_bwd_workspace(int64_t capacity);
rgs_status rgs_render_partial_bwd(const rgs_partials_grad *dparts, const rgs_partials *parts,
                                  const rgs_bins *bins, const rgs_projected *proj, int64_t n,
                                  const rgs_camera *cams, int32_t n_views, const void *views_dev,
                                  const rgs_kdtree *kd, float *d_proj, void *ws, size_t ws_bytes,
                                  rgs_stream stream);

/* The same in two calls (the backward's blend and its reduction, Sec. 3.4),
 * so that each can be timed on its own.  rgs_render_partial_bwd_records
 * writes the per-instance records into ws (same workspace and arguments as
 * above, minus d_proj): a record for each instance that some pixel of its
 * slot reaches at or before its last contributor, marked in a bitmask by
 * emission position in the same ws (the others count as zero); stats, if
 * not NULL, points to two device uint64 counters incremented by the
 * (pixel, instance) pairs tested (pixel inside
 * the rectangle, at or before its last contributor) and the contributing
 * pairs.  Its blocks are launched by decreasing size class of the instances
 * each slot is walked over (the largest `last` of its pixels; slots without
 * a contribution are not launched), an order it builds in ws from
 * parts->last.  rgs_pair_reduce then sums each pair's records from the same
 * ws into d_proj ([9][V*N], as above), with the per-64-instance pair lookup
 * the records call also left there (so it must follow a records call on the
 * same bins and ws). */
rgs_status rgs_render_partial_bwd_records(const rgs_partials_grad *dparts, const rgs_partials *parts,
                                          const rgs_bins *bins, const rgs_projected *proj, int64_t n,
                                          const rgs_camera *cams, int32_t n_views, const void *views_dev,
                                          const rgs_kdtree *kd, void *ws, size_t ws_bytes, uint64_t *stats,
                                          rgs_stream stream);
rgs_status rgs_pair_reduce(const rgs_bins *bins, const rgs_projected *proj, int64_t n, int32_t n_views,
                           float *d_proj, void *ws, size_t ws_bytes, rgs_stream stream);

/* Projection backward: chain rule from d_proj to the parameters, summed over
 * the views.  Exact derivative: zero through the colour clamp, the clamp of
 * the projected x/z, y/z (where the clamped value is proportional to z) and
 * for culled pairs. */
rgs_status rgs_project_sh_bwd(const float *d_proj, const rgs_gaussians *g, const rgs_projected *proj,
                              const rgs_camera *cams, int32_t n_views, const void *views_dev,
                              const rgs_gaussians_grad *out, rgs_stream stream);

/* ------------------------------------------------------------------ */
/* Training: parameter update and re-partition reorder (Sec. 3.4, Sec. 4) */
/* ------------------------------------------------------------------ */
/* Adam with fp32 states and one learning rate per parameter group (the
 * 3DGS optimiser the paper trains with; the position rate decays
 * exponentially, which the caller passes per step in lr_means).  Per
 * element: m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t = step >= 1.
 * The SH rows of degree 0 (rows 0..2) use lr_sh_dc, the others lr_sh_rest.
 * params, m and v are read and written in place (layouts as rgs_gaussians),
 * grads is read; the four must not overlap. */
typedef struct {
    float lr_means, lr_log_scales, lr_quats, lr_opacity, lr_sh_dc, lr_sh_rest;
    double beta1, beta2, eps; /* 1 - b1, 1 - b2 and the bias corrections are formed in fp64 and rounded once */
    int32_t step;
} rgs_adam_params;
rgs_status rgs_adam_step(const rgs_gaussians_grad *params, const rgs_gaussians_grad *grads,
                         const rgs_gaussians_grad *m, const rgs_gaussians_grad *v, int64_t n, int32_t sh_degree,
                         const rgs_adam_params *hp, rgs_stream stream);

/* out row j = in row perm[j] for every parameter array (the same layouts;
 * out must not overlap in or perm).  With perm from rgs_group_by_cell it
 * carries per-Gaussian state (Adam's m and v) along when a re-partition
 * regroups the parameters by cell.  perm entries outside [0, n) leave the
 * row untouched. */
rgs_status rgs_permute_gaussians(const rgs_gaussians *in, const int32_t *perm, const rgs_gaussians_grad *out,
                                 rgs_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* RGS_H */
