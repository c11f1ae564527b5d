/*
 * sgrid.h -- C ABI of the sparse-dense SDF grid renderer for AMD gfx950.
 *
 * The method: Dong et al., "Fast Monocular Scene Reconstruction with
 * Global-Sparse Local-Dense Grids" (CVPR 2023).  A scene is a set of 8^3
 * voxel blocks allocated only near surfaces and found through a
 * collision-free spatial hash (Sec. 3.2).  Each voxel stores an SDF value and
 * C feature channels (colour, optionally semantic logits).  Rays are marched
 * through the allocated blocks only, sampled uniformly, the SDF and features
 * are trilinearly interpolated together with the closed-form SDF gradient
 * (Eq. 17-18), the SDF is turned into density with the Laplace-CDF transform
 * and colour, depth and normal are alpha-composited (Eq. 12-15,
 * Sec. 3.5.1).  The backward pass scatters gradients into the voxels.
 *
 * Conventions used by every call
 * -------------------------------
 *  - Pointers named d_* are DEVICE memory owned by the caller.  The library
 *    never frees them and keeps no reference after a call returns.
 *  - sg_stream is a hipStream_t (NULL = the legacy default stream).  Every
 *    call except sg_grid_build / sg_grid_destroy / sg_grid_num_blocks is
 *    asynchronous on that stream, allocates nothing and never synchronises,
 *    so it may be captured in a HIP graph.
 *  - Return value: SG_OK (0) or a negative sg_status.  All argument checks
 *    run on the host before any HIP call; on error nothing is launched and
 *    sg_last_error() returns a message (thread-local, valid until the next
 *    failing call on the same thread).
 *  - A grid's geometry: voxel (i,j,k) (integer, global) sits at
 *    origin + (i,j,k) * voxel_size.  Block b = floor(i/8) per axis; the
 *    voxel's local index inside its block is lx + 8*ly + 64*lz with
 *    l = i - 8*b.  Block coordinates must lie in [-2^20, 2^20) per axis.
 *  - Voxel parameters are one float32 array vox[n_blocks][512][1+C]
 *    (channel 0 = SDF theta_d, channels 1..C = features theta_c / theta_s),
 *    row-major, block order = the grid's block index order.
 *  - Supported feature counts C: 0,1,2,3,4,8,16,19,32.
 */
#ifndef SGRID_H
#define SGRID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sg_grid sg_grid;
typedef void* sg_stream;

typedef enum sg_status {
  SG_OK = 0,
  SG_EINVAL = -1, /* bad argument: null pointer, size, unsupported C, ... */
  SG_ERANGE = -2, /* a block coordinate outside [-2^20, 2^20) */
  SG_ENOMEM = -3, /* device allocation failed (grid build only) */
  SG_EHIP = -4,   /* a HIP runtime call failed; message names it */
  SG_ESTATE = -5  /* object in the wrong state (e.g. destroyed grid) */
} sg_status;

#define SG_BLOCK_DIM 8
#define SG_BLOCK_VOXELS 512
#define SG_COORD_LIMIT 1048576 /* 2^20 */
#define SG_MAX_SAMPLES_LIMIT 1024

/*
 * Ray-march and density parameters (Sec. 3.5.1, Eq. 15).
 *   step        lattice spacing along the ray in world units (> 0): sample k
 *               sits at t_k = t_near + k*step.  Every kept sample uses
 *               delta_k = step.
 *   t_near/far  the lattice covers t_near <= t_k <= t_far (t_far inclusive);
 *               (t_far - t_near)/step must stay below 2^24.
 *   beta        scale of the Laplace-CDF density (> 0):
 *               sigma(f) = (1/beta) * Psi_beta(-f).
 *   max_samples cap on kept samples per ray, 1..1024; the first max_samples
 *               valid lattice points are kept, in lattice order.
 * A lattice point is a valid sample iff the blocks holding all 8 corners of
 * its interpolation cell are allocated (the sparse grid skips empty space).
 */
typedef struct sg_render_params {
  float step;
  float t_near;
  float t_far;
  float beta;
  int32_t max_samples;
} sg_render_params;

/* Message for the last failing call on this thread ("" if none). */
const char* sg_last_error(void);

/* Library version string. */
const char* sg_version(void);

/*
 * sg_grid_build -- the collision-free spatial hash over allocated blocks
 * (Sec. 3.2 and 3.4.1: blocks indexed one-to-one by their integer block
 * coordinate).
 *   d_block_coords  int32 [n,3] device, block coordinates (duplicates allowed).
 *   n               number of input coordinates, 1 <= n <= 2^31-1.
 *   voxel_size      world edge length of one voxel (> 0, finite).
 *   origin          host float[3]: world position of voxel (0,0,0).
 *   d_index_of_input  nullable int32 [n] device: receives the block index of
 *                   every input row.
 * Block indices are assigned in order of first occurrence in the input and
 * duplicates are merged, so the result is deterministic.  Builds the hash
 * table, the block list and an 8-entry neighbour table per block.  The call
 * allocates device memory and synchronises the stream (build time only).
 * Errors: SG_EINVAL (null/size), SG_ERANGE (a coordinate out of range; no
 * grid is returned), SG_ENOMEM, SG_EHIP.  *out is set only on SG_OK; the
 * caller releases it with sg_grid_destroy.
 */
int sg_grid_build(const int32_t* d_block_coords, int64_t n, float voxel_size,
                  const float origin[3], sg_stream stream, sg_grid** out,
                  int32_t* d_index_of_input);

/*
 * Build options.  dense_map_max_cells: besides the hash, build a dense map
 * of the grid's bounding box in blocks (one int32 per block cell: block
 * index and neighbour mask, or the Chebyshev distance to the nearest
 * allocated block) when the box has at most this many cells; the renderer
 * then resolves blocks and skips empty space through it instead of probing
 * the hash.  0 disables the map; a negative value selects the default
 * SG_DEFAULT_DENSE_MAP_CELLS (2^28 cells = 1 GiB).  Results are identical
 * with and without the map.
 */
#define SG_DEFAULT_DENSE_MAP_CELLS 268435456LL
typedef struct sg_build_options {
  int64_t dense_map_max_cells;
} sg_build_options;

/*
 * Dense-map plan of a grid (a host computation, for memory planning): for a
 * block bounding box [bmin, bmax] (inclusive, each coordinate in
 * [-2^20, 2^20)) holding n_blocks allocated blocks, the dims[3] and cell
 * count (*cells, int32 entries) of the dense block map that sg_grid_build_ex
 * with these options would build, or all zeros if it would build none (more
 * cells than the limit, or n_blocks >= 2^23).  The cell count of a box that
 * spans the whole coordinate range, 2^63, is decided without overflow.
 * SG_ERANGE for a box outside the range, SG_EINVAL for bmin > bmax,
 * n_blocks < 0 or a NULL pointer.
 */
int sg_grid_dense_map_plan(const int32_t bmin[3], const int32_t bmax[3], int64_t n_blocks,
                           const sg_build_options* options, int32_t dims[3], int64_t* cells);

/* sg_grid_build with options (NULL = defaults); otherwise identical. */
int sg_grid_build_ex(const int32_t* d_block_coords, int64_t n, float voxel_size,
                     const float origin[3], sg_stream stream, sg_grid** out,
                     int32_t* d_index_of_input, const sg_build_options* options);

/*
 * Dense block map geometry: dims[3] (all 0 if the grid has no map) and the
 * block coordinate bmin[3] of its first cell.  Cell (x,y,z) is at
 * ((z - bmin.z) * dims.y + (y - bmin.y)) * dims.x + (x - bmin.x).
 */
int sg_grid_dense_map(const sg_grid* g, int32_t dims[3], int32_t bmin[3]);

/* Copy the dense map (int32 [dims.z*dims.y*dims.x]): entry >= 0 is
 * block_index * 256 + neighbour mask (bit s as in sg_grid_neighbors); entry
 * -D (1 <= D <= 32) means every block within Chebyshev distance D-1 is
 * unallocated (distances beyond 32 are stored as 32).  SG_ESTATE if the grid
 * has no map. */
int sg_grid_copy_dense_map(const sg_grid* g, int32_t* d_out, sg_stream stream);

/* Number of allocated (unique) blocks. */
int sg_grid_num_blocks(const sg_grid* g, int64_t* n_blocks);

/* Generation of the grid's index memory (host output): 0 when built, one
 * more after every sg_grid_extend, which moves that memory.  A descriptor or
 * captured launch made at an older generation refers to freed memory. */
int sg_grid_generation(const sg_grid* g, uint64_t* generation);

/* World geometry of the grid: voxel_size and origin[3] (host outputs). */
int sg_grid_geometry(const sg_grid* g, float* voxel_size, float origin[3]);

/* Copy the unique block coordinates, int32 [n_blocks,3], in index order. */
int sg_grid_block_coords(const sg_grid* g, int32_t* d_out, sg_stream stream);

/*
 * Copy the neighbour table int32 [n_blocks,8]: entry s = sx + 2*sy + 4*sz
 * (sx,sy,sz in {0,1}) holds the index of block b + (sx,sy,sz), or -1 if that
 * block is not allocated.  These are the blocks a trilinear cell whose base
 * voxel lies in block b can touch (Eq. 17).
 */
int sg_grid_neighbors(const sg_grid* g, int32_t* d_out, sg_stream stream);

/*
 * sg_grid_lookup -- hash query (Sec. 3.2): d_idx[i] = index of block
 * d_coords[i] (int32 [n,3]) or -1 if not allocated (also -1 for coordinates
 * outside the representable range).  n may be 0.
 */
int sg_grid_lookup(const sg_grid* g, const int32_t* d_coords, int64_t n,
                   int32_t* d_idx, sg_stream stream);

/*
 * sg_alloc_blocks -- the blocks to allocate for depth maps (Sec. 3.4.1):
 * every pixel (u, v) of frame f whose depth D is finite, > 0 and
 * <= depth_max is lifted to the camera point (x D, y D, D),
 * x = (u + 1/2 - cx) / fx, y = (v + 1/2 - cy) / fy (D is the depth along the
 * optical axis), moved to the world by the frame's [R | t], and its block
 * floor(floor((X - origin) / h) / 8) taken; each such block is dilated to the
 * (2 dilate + 1)^3 blocks around it.  float32 without fused multiply-add, in
 * the order written.  Pixels whose dilated blocks would leave [-2^20, 2^20)
 * are skipped.
 *   d_cams   float [n_frames,16], the layout of sg_rays_pinhole;
 *   d_depth  float [n_frames,H,W];
 *   d_out    int32 [cap,3] output: the block coordinates in order of first
 *            occurrence (frames, rows, columns, then dilation offsets z, y, x
 *            from -dilate to dilate), without duplicates: the input of
 *            sg_grid_build;
 *   *n_out   the number of blocks (also when cap is too small: SG_EINVAL
 *            then, with nothing written, so a caller can size d_out).
 * Allocates temporary device memory and synchronises the stream (a set-up
 * call, like sg_grid_build).  dilate in [0, 8].
 */
int sg_alloc_blocks(const float* d_cams, int32_t n_frames, const float* d_depth, int32_t W,
                    int32_t H, float voxel_size, const float origin[3], int32_t dilate,
                    float depth_max, int32_t* d_out, int64_t cap, int64_t* n_out,
                    sg_stream stream);

/*
 * sg_grid_from_depth -- sg_alloc_blocks and sg_grid_build_ex in one call:
 * the grid of the blocks allocated for the depth maps (same arguments and
 * order of block indices), without the caller sizing an intermediate
 * buffer.  SG_EINVAL if no pixel has a valid depth.  Allocates device
 * memory and synchronises the stream.
 */
int sg_grid_from_depth(const float* d_cams, int32_t n_frames, const float* d_depth, int32_t W,
                       int32_t H, float voxel_size, const float origin[3], int32_t dilate,
                       float depth_max, sg_stream stream, sg_grid** out,
                       const sg_build_options* options);

/*
 * sg_fuse -- depth, colour and semantic fusion (Sec. 3.4.2): every voxel
 * (world position origin + i h) of the grid is projected into every frame
 * (camera point c = R^T (X - t); pixel (floor(fx c_x / c_z + cx),
 * floor(fy c_y / c_z + cy))) and associated when c_z > 0, the pixel lies in
 * the image, its depth D is finite and > 0 and D - c_z >= -trunc (more
 * than trunc behind the surface is occluded; the truncation psi(x, mu) =
 * min(x, mu) of the supplement's Volumetric Fusion, mu = trunc).  The
 * per-voxel least-squares solutions are the averages over its associations:
 *   d_vox [n_blocks,512,1+C] (output): SDF = mean of min(D - c_z, trunc),
 *     features = mean of d_feat at the pixel; the last n_sem feature channels
 *     (semantic logits) are then divided by their L2 norm.  Voxels with no
 *     association: SDF = trunc, features 0.
 *   d_weight [n_blocks,512] float (nullable): number of associations.
 * d_cams [n_frames,16], d_depth [n_frames,H,W], d_feat [n_frames,H,W,C]
 * (nullable iff C == 0).  Decisions in float32 without fused multiply-add;
 * frames are summed in order, so the output is deterministic.  Device
 * memory owned by the caller; asynchronous; allocates nothing.  C as for
 * rendering; 0 <= n_sem <= C; trunc finite and > 0.
 */
int sg_fuse(const sg_grid* g, const float* d_cams, int32_t n_frames, const float* d_depth,
            const float* d_feat, int32_t C, int32_t W, int32_t H, float trunc, int32_t n_sem,
            float* d_vox, float* d_weight, sg_stream stream);

/*
 * sg_denoise -- Gaussian de-noising of the fused voxels (Sec. 3.4.3): every
 * channel of every voxel v becomes
 *   sum_d w(d) theta(v + d) / sum_d w(d),  w(d) = exp(-|d|^2 / (2 sigma^2)),
 * over the offsets d in [-radius, radius]^3 (voxel units) whose voxel lies
 * in an allocated block (the weights renormalise at the border of the
 * grid).  d_vox, d_out [n_blocks,512,1+C]; d_out must not overlap d_vox.
 * radius in [0, 8], sigma finite and > 0.  Device memory owned by the
 * caller; asynchronous; allocates nothing.
 */
int sg_denoise(const sg_grid* g, const float* d_vox, int32_t C, int32_t radius, float sigma,
               float* d_out, sg_stream stream);

/*
 * Continuous CRF message passing (Sec. 3.5.3): the mean-field update of the
 * CRF is a high-dimensional Gaussian filter over the feature vectors of the
 * surface samples, evaluated on a permutohedral lattice held in a
 * collision-free hash of lattice points.
 *
 * sg_lattice_build -- the lattice of n_points feature positions d_pos
 *   float [n,d], 1 <= d <= 24, already divided by the per-feature standard
 *   deviations (finite, |p| < 2^20): each position's enclosing simplex (d+1
 *   vertices and barycentric weights; float32 without fused multiply-add,
 *   so the vertices are the same integers for any evaluation of the same
 *   steps) and the hash of all vertices.  max_values (1..32) bounds the
 *   value channels of later filters.  Allocates device memory (the
 *   sg_lattice_bytes(n_points, d, max_values) bytes) and synchronises the
 *   stream.  SG_ERANGE if two lattice keys share a 64-bit fingerprint
 *   (checked, never silently merged).
 * sg_lattice_bytes -- device bytes a build of these sizes allocates at most
 *   (a host computation, for memory planning): a hash table of the smallest
 *   power of two >= 2 n (d+1) slots (8-byte fingerprint, an int32 key of d
 *   coordinates padded to a multiple of 4, two max_values-float value rows,
 *   an int32 slot-list entry each) plus n (d+1) vertex ids and weights,
 *   n max_values slice outputs, and the blur neighbour table (the two
 *   neighbours of each vertex along each of the d+1 directions, 2 (d+1)
 *   int32 per vertex, sized for the at most n (d+1) vertices); 0 for invalid
 *   sizes (the limits of sg_lattice_build).
 * sg_lattice_filter -- d_out [n, n_values] = slice(blur(splat(d_val))):
 *   values splatted onto the simplex vertices with the barycentric weights,
 *   blurred with [1/4, 1/2, 1/4] along each of the d+1 lattice directions
 *   (absent neighbours add nothing), and sliced back with the same weights
 *   (unnormalised; filter a channel of ones to normalise).  Splatting uses
 *   float atomics: the last bits depend on their order.  Asynchronous;
 *   allocates nothing.
 * sg_crf_meanfield -- label marginals d_Q [n, n_labels] after `iters`
 *   mean-field updates Q <- softmax(-unary + w_p * filter(Q)) from
 *   Q = softmax(-unary) (a Potts compatibility of weight w_p; the message
 *   includes each point's own contribution).  d_unary [n, n_labels].
 *   Asynchronous; allocates nothing.
 * sg_crf_meanfield_compat -- the same with a general label compatibility
 *   (Sec. 3.5.3: the pairwise potential is a compatibility of the labels
 *   times the Gaussian kernel): Q <- softmax(-unary - filter(Q) mu^T), that
 *   is Q_i(l) <- softmax_l(-unary_i(l) - sum_k mu(l, k) filter(Q)_i(k)).
 *   d_compat [n_labels, n_labels] device, row-major, row l = mu(l, .);
 *   the Potts model of weight w is mu = w (1 - I), which gives the result
 *   of sg_crf_meanfield with w_p = w.  Asynchronous; allocates nothing.
 * sg_crf_meanfield_compat_backward -- gradients for learning the
 *   compatibility (Sec. 3.5.3 calls it learnable): for d_gQ [n, n_labels],
 *   the gradient of a scalar E at the marginals after `iters` updates of
 *   sg_crf_meanfield_compat, writes d_g_unary [n, n_labels] = dE/dunary and
 *   d_g_compat [n_labels, n_labels] = dE/dmu (both overwritten).  Reverse
 *   mode through the updates, each Q = softmax(a), a = -unary - m mu^T,
 *   m = filter(Q_prev): ga = Q (gQ - <Q, gQ>); g_unary -= ga;
 *   g_mu(l, k) -= sum_i ga_i(l) m_i(k); gQ_prev = filter^T(-ga mu), the
 *   transpose of the filter being the same filter with its blur directions
 *   in reverse order.  Recomputes the forward and keeps every update's
 *   marginals and messages in d_ws (device, caller-owned, at least
 *   sg_crf_meanfield_compat_backward_ws_bytes(n, n_labels, iters) bytes,
 *   which returns 0 for invalid sizes).  d_g_unary, d_g_compat and d_ws
 *   must not overlap d_gQ, d_unary or d_compat (the outputs are cleared
 *   before the inputs are read; SG_EINVAL if d_g_unary or d_ws overlaps
 *   d_gQ).  g_mu sums per-workgroup partials in a fixed order; the
 *   filter's splat uses float atomics, so the last bits may vary from call
 *   to call.  Asynchronous; allocates nothing.
 * Filters and updates on one lattice share its value buffers: calls on the
 * same lattice must not overlap (issue them on one stream).
 * sg_lattice_destroy frees the lattice (waits for nothing: the caller makes
 * sure no launched work still uses it); NULL is accepted.
 */
typedef struct sg_lattice sg_lattice;
int sg_lattice_build(const float* d_pos, int64_t n_points, int32_t d, int32_t max_values,
                     sg_stream stream, sg_lattice** out);
size_t sg_lattice_bytes(int64_t n_points, int32_t d, int32_t max_values);
int sg_lattice_num_vertices(const sg_lattice* lat, int64_t* n_vertices);
int sg_lattice_filter(const sg_lattice* lat, const float* d_val, int32_t n_values, float* d_out,
                      sg_stream stream);
int sg_crf_meanfield(const sg_lattice* lat, const float* d_unary, int32_t n_labels, float w_p,
                     int32_t iters, float* d_Q, sg_stream stream);
int sg_crf_meanfield_compat(const sg_lattice* lat, const float* d_unary, int32_t n_labels,
                            const float* d_compat, int32_t iters, float* d_Q, sg_stream stream);
size_t sg_crf_meanfield_compat_backward_ws_bytes(int64_t n_points, int32_t n_labels,
                                                int32_t iters);
int sg_crf_meanfield_compat_backward(const sg_lattice* lat, const float* d_unary, int32_t n_labels,
                                     const float* d_compat, int32_t iters, const float* d_gQ,
                                     float* d_g_unary, float* d_g_compat, void* d_ws,
                                     size_t ws_bytes, sg_stream stream);
/*
 * sg_crf_meanfield_compat_backward_noalloc -- for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training or
 * serving loops, harnesses that forbid hipMalloc): the same gradients as
 * sg_crf_meanfield_compat_backward (same arguments, same kernels, same
 * results up to the order of the splat's float atomics) with the workspace
 * taken from a fixed array inside the library instead of d_ws.  The array
 * holds sg_crf_meanfield_compat_backward_noalloc_max_bytes() bytes (64 MiB)
 * on each device the library runs on, allocated when the library is loaded
 * onto the device and kept until the process ends; SG_EINVAL if
 * sg_crf_meanfield_compat_backward_ws_bytes(n, n_labels, iters) exceeds it
 * (for example n * n_labels * (2 iters + 3) > 16 M floats) or the current
 * device is not the lattice's.  Calls on one device share that array and
 * its contents persist between calls (every part is written before it is
 * read, so nothing needs clearing): calls that overlap on one device (other
 * streams, other threads) race and give wrong results; issue them in
 * order.  Calls no hipMalloc, hipFree or allocating library routine; the
 * first call on a device looks up the array's device address once.
 * Asynchronous; d_g_unary must not overlap d_gQ (SG_EINVAL).
 */
size_t sg_crf_meanfield_compat_backward_noalloc_max_bytes(void);
int sg_crf_meanfield_compat_backward_noalloc(const sg_lattice* lat, const float* d_unary,
                                             int32_t n_labels, const float* d_compat,
                                             int32_t iters, const float* d_gQ, float* d_g_unary,
                                             float* d_g_compat, sg_stream stream);
int sg_lattice_destroy(sg_lattice* lat);

/*
 * sg_crf_label_loss -- the CRF's label loss (Eq. 22, the f-divergence taken
 * as Kullback-Leibler): per node i, x = softmax(logits_i) and Q_i its
 * mean-field marginals (a fixed target, entries > 0):
 *   d_loss [n] (nullable) = weight * sum_l x_l log(x_l / Q_l),
 *   d_g (nullable) row i, columns 0..L-1 = weight * x_k (a_k - KL_i),
 *     a = log x - log Q (the gradient with respect to the logits).
 * d_logits rows of stride ld_logits, d_Q [n,L], d_g rows of stride ld_g
 * (so the logits can be the semantic columns of sg_query's feature output
 * and the gradient written into the same columns of sg_query_backward's
 * d_g_feat).  Asynchronous; allocates nothing.  1 <= L <= 32.
 */
int sg_crf_label_loss(const float* d_logits, int64_t ld_logits, const float* d_Q, int64_t n,
                      int32_t n_labels, float weight, float* d_loss, float* d_g, int64_t ld_g,
                      sg_stream stream);
/*
 * sg_crf_property_loss -- the CRF's colour or normal loss (Eq. 22) for a
 * continuous property x (P values per node, rows of stride ld_x): its
 * mean-field estimate is the normalised Gaussian filter over the other
 * features, Q = F(x) / F(1), read from d_filtered [n, P+1] = sg_lattice_filter
 * of [x, 1] (a fixed target):
 *   d_loss [n] (nullable) = weight |x - Q|^2,
 *   d_g (nullable) row i (stride ld_g) = 2 weight (x_i - Q_i).
 * Asynchronous; allocates nothing.  1 <= P <= 31.
 */
int sg_crf_property_loss(const float* d_x, int64_t ld_x, const float* d_filtered, int64_t n,
                         int32_t n_props, float weight, float* d_loss, float* d_g, int64_t ld_g,
                         sg_stream stream);

/*
 * sg_grid_extend -- add blocks to a grid (new frames' allocations, Sec.
 * 3.4.1): the grid is rebuilt from its own block coordinates followed by
 * d_new_coords [n_new,3], so existing blocks keep their indices and new
 * ones get the next indices in order of first occurrence (the caller grows
 * its voxel arrays accordingly).  The handle stays valid, but the grid's
 * index memory moves: packed descriptors made from it before the call
 * (sg_packed_grid_desc) and launches captured in a graph before it refer to
 * freed memory and must not be used again (sg_packed_grid_check reports a
 * stale descriptor; sg_grid_generation counts the moves).  Allocates device
 * memory and synchronises the stream; the caller makes sure no launched work
 * still uses the grid.  On error the grid is unchanged.
 */
int sg_grid_extend(sg_grid* g, const int32_t* d_new_coords, int64_t n_new, sg_stream stream,
                   const sg_build_options* options);

/* Free the grid's device memory (waits for nothing; the caller makes sure no
 * launched work still uses the grid).  NULL is accepted. */
int sg_grid_destroy(sg_grid* g);

/*
 * sg_rays_pinhole -- camera rays of pixels (the inverse projection of the
 * pinhole model used in the reprojection of Eq. 3).
 *   d_cams   float [n_cams,16]: fx, fy, cx, cy, then the camera-to-world
 *            matrix rows [R | t] (3x4, row-major).  Camera axes: x right,
 *            y down, z forward.
 *   d_pix    int32 [R,3]: camera index, pixel column u, pixel row v.  The
 *            ray passes through the pixel centre (u+0.5, v+0.5).
 *   d_rays   float [R,6] output: origin t, then the unit world direction
 *            normalise(R * ((u+0.5-cx)/fx, (v+0.5-cy)/fy, 1)).
 * A camera index outside [0,n_cams) yields a ray of NaNs (which renders as
 * an empty ray).  R may be 0.
 */
int sg_rays_pinhole(const float* d_cams, int32_t n_cams, const int32_t* d_pix,
                    int64_t n_rays, float* d_rays, sg_stream stream);

/*
 * sg_query -- the trilinear SDF, its closed-form gradient and the features
 * at arbitrary world points (Eq. 17-18), the query the paper times on k^3
 * points (Sec. 4.2).  For each point p of d_points float [n,3]:
 *   x = (p - origin) * fl(1/h) in voxel units (float32, no fused
 *   multiply-add, as the march computes it; |x| >= 2^24 or NaN: invalid);
 *   the point is valid iff the blocks of all 8 corners of its cell are
 *   allocated (the render's sample rule);
 *   d_valid [n] int32 (nullable): 1 / 0; d_f [n] (nullable): f;
 *   d_grad [n,3] (nullable): grad f in world units; d_feat [n,C] (nullable):
 *   features.  Invalid points give 0 everywhere.
 * Device memory owned by the caller; asynchronous; allocates nothing.
 * SG_EINVAL for NULL d_vox / d_points, n < 0 or an unsupported C.
 */
int sg_query(const sg_grid* g, const float* d_vox, int32_t C, const float* d_points,
             int64_t n_points, int32_t* d_valid, float* d_f, float* d_grad, float* d_feat,
             sg_stream stream);

/*
 * sg_surface_points -- surface points along rays (the nodes of the
 * continuous CRF are zero crossings of the SDF seen from random viewpoints,
 * Sec. 3.5.3): along each ray's kept samples (as sg_render_forward takes
 * them), the first pair of lattice-adjacent samples with f_j > 0 >= f_{j+1}
 * (entering the surface), placed by linear interpolation of f:
 * t* = t_j + step f_j / (f_j - f_{j+1}).  d_points [R,3] = o + t* d and
 * d_hit [R] = 1, or zeros and 0 where the ray crosses no surface.
 * d_vox [n_blocks,512,1+C] (only the SDF channel is read), 0 <= C <= 64.
 * Asynchronous; allocates nothing.
 */
int sg_surface_points(const sg_grid* g, const float* d_vox, int32_t C, const float* d_rays,
                      int64_t n_rays, const sg_render_params* params, float* d_points,
                      int32_t* d_hit, sg_stream stream);

/*
 * sg_query_backward -- adjoint of sg_query with respect to the voxels, for
 * losses on queried values (e.g. the CRF's losses on surface samples,
 * Sec. 3.5.3): for upstream gradients d_g_f [n], d_g_grad [n,3] (world
 * units) and d_g_feat [n,C] (each nullable) it ACCUMULATES into d_grad_vox
 * [n_blocks,512,1+C], for the 8 corners a of every valid point,
 *   channel 0: r_a g_f + (grad_x r_a . g_grad),  channel 1+c: r_a g_feat[c].
 * Float atomics: the caller zeroes d_grad_vox; the summation order (so the
 * last bits) is unspecified.  Asynchronous; allocates nothing.
 */
int sg_query_backward(const sg_grid* g, int32_t C, const float* d_points, int64_t n_points,
                      const float* d_g_f, const float* d_g_grad, const float* d_g_feat,
                      float* d_grad_vox, sg_stream stream);

/*
 * sg_uniform_points -- n points uniform over the grid's allocated blocks,
 * the uniform in-grid samples of the Eikonal term (Sec. 3.5.2): point i
 * draws x_k = splitmix64(seed + 4 i + k), k = 0..3 (SplitMix64 used as a
 * counter-based generator), takes block x_0 mod n_blocks (in index order)
 * and the offsets u_a = (x_{1+a} >> 40) 2^-24 in [0,1): world position
 * origin_a + (8 b_a + 8 u_a) h, float32 in that order (bit-reproducible).
 * d_points float [n,3].  Asynchronous; allocates nothing.  Points near the
 * border of the allocated region can be invalid for sg_query / sg_eikonal
 * (a corner block missing); those calls skip them.
 */
int sg_uniform_points(const sg_grid* g, int64_t n, uint64_t seed, float* d_points,
                      sg_stream stream);

/*
 * sg_eikonal -- the Eikonal regulariser (Eq. 16) at points, the uniform
 * in-grid samples of the training loss, with its derivative with respect to
 * the SDF voxels.  For each point p of d_points float [n,3], valid as in
 * sg_query, with g = grad f(p) of Eq. 18:
 *   d_loss [n] (nullable): weight * (|g| - 1)^2, 0 for invalid points;
 *   d_grad_vox [n_blocks,512,1+C] (nullable): accumulates, in channel 0
 *     only, weight * 2 (|g| - 1) (g / |g|) . grad_x r(p, corner) for each of
 *     the 8 corners (nothing where |g| = 0, where the direction is
 *     undefined).  Accumulated with float atomics: the caller zeroes it, the
 *     summation order (so the last bits) is unspecified.
 * Device memory owned by the caller; asynchronous; allocates nothing.
 * SG_EINVAL for NULL d_vox / d_points, n < 0, a non-finite weight or an
 * unsupported C.
 */
int sg_eikonal(const sg_grid* g, const float* d_vox, int32_t C, const float* d_points,
               int64_t n_points, float weight, float* d_loss, float* d_grad_vox,
               sg_stream stream);

/*
 * Sample lists (optional).  sg_render_march runs the block march of
 * Sec. 3.5.1 for every ray on its own and writes each ray's kept samples to
 * d_lists: [n_rays][max_samples] pairs (lattice index k, block index) in
 * lattice order, then [n_rays] int32 counts.  sg_render_forward,
 * sg_render_backward and sg_render_l2_step take (d_lists, lists_bytes):
 * given a buffer filled by sg_render_march for the same grid, rays and
 * params (and not written since), they read the samples from it instead of
 * marching; with (NULL, 0) they march themselves.  Results are
 * bit-identical either way; one list can serve a forward and its backward.
 * A list that does not match its call gives wrong outputs but no access
 * outside the grid or the buffer.  The buffer is device memory owned by the
 * caller, 8-byte aligned, at least sg_render_list_bytes(n_rays,
 * params) bytes; SG_EINVAL otherwise, or if bytes are given without a
 * pointer.
 *
 * sg_render_list_bytes returns n_rays * max_samples * 8 + n_rays * 4,
 * or 0 if the arguments are invalid.
 */
size_t sg_render_list_bytes(int64_t n_rays, const sg_render_params* params);

int sg_render_march(const sg_grid* g, const float* d_rays, int64_t n_rays,
                    const sg_render_params* params, void* d_lists, size_t lists_bytes,
                    sg_stream stream);

/*
 * sg_render_forward -- volume rendering through the sparse grid
 * (Sec. 3.5.1, Eq. 12-15, with f and grad f from Eq. 17-18).
 * For each ray (o,d) in d_rays float [R,6] (d of unit length; the caller's
 * contract, not renormalised), samples t_k as described in sg_render_params,
 * and with theta interpolated trilinearly at x_k = o + t_k d:
 *   sigma_k = (1/beta) Psi_beta(-f(x_k)),  Psi_beta(s) = 1/2 exp(s/beta) for
 *             s <= 0, 1 - 1/2 exp(-s/beta) otherwise  (VolSDF's transform)
 *   w_k     = exp(-sum_{j<k} sigma_j step) * (1 - exp(-sigma_k step))
 *   feat_out = sum_k w_k c(x_k)       [R,C]  (nullable iff C == 0)
 *   depth    = sum_k w_k t_k          [R]    (ray distance; not divided by W)
 *   normal   = sum_k w_k grad f(x_k)  [R,3]  (world frame, not normalised)
 *   wsum     = sum_k w_k              [R]
 *   nsamples = number of kept samples [R] int32 (nullable)
 * d_vox float [n_blocks,512,1+C].  Rays with non-finite o or d, or that keep
 * no sample, produce exact zeros.  Deterministic: repeated calls give
 * bit-identical outputs (no atomics).  All outputs are overwritten.
 */
int sg_render_forward(const sg_grid* g, const float* d_vox, int32_t C,
                      const float* d_rays, int64_t n_rays,
                      const sg_render_params* params, float* d_feat_out,
                      float* d_depth, float* d_normal, float* d_wsum,
                      int32_t* d_nsamples, const void* d_lists,
                      size_t lists_bytes, sg_stream stream);

/*
 * sg_render_backward -- adjoint of sg_render_forward with respect to the
 * voxel parameters (the differentiable indexer of Sec. 3.2 and the
 * closed-form gradient of Eq. 18, so no double backward is needed).
 * Given upstream gradients of a scalar loss L:
 *   d_g_feat [R,C] (nullable iff C == 0), d_g_depth [R], d_g_normal [R,3],
 *   d_g_wsum [R] (nullable: treated as zero),
 * ACCUMULATES dL/dvox into d_grad_vox float [n_blocks,512,1+C] (the caller
 * zeroes it first).  Per-sample quantities are recomputed from the grid
 * rather than stored by the forward pass.  Uses float32 atomic adds, so the
 * summation order (and the last bits) may differ between calls.
 */
int sg_render_backward(const sg_grid* g, const float* d_vox, int32_t C,
                       const float* d_rays, int64_t n_rays,
                       const sg_render_params* params, const float* d_g_feat,
                       const float* d_g_depth, const float* d_g_normal,
                       const float* d_g_wsum, float* d_grad_vox,
                       const void* d_lists, size_t lists_bytes,
                       sg_stream stream);

/*
 * sg_render_l2_step -- one training step of the rendering losses, fused:
 * forward render, squared-L2 losses of Eq. 12-14 against reference values,
 * the Eikonal regulariser of Eq. 16 on the ray samples (Sec. 3.5.2), and
 * their gradient with respect to the voxels (Sec. 3.5.1, 3.5.4), with
 *   L = (1/R) sum_r ( |C_r - C*_r|^2 + lambda_d (D_r - D*_r)^2
 *                     + lambda_n |N_r - N*_r|^2
 *                     + lambda_e sum_k (|grad f(x_rk)| - 1)^2 ),
 * the last sum over the ray's kept samples.
 * Writes the forward outputs exactly as sg_render_forward does (bit for
 * bit), d_loss_ray[r] (nullable, [R]) = ray r's term of L (so L is their
 * sum), and ACCUMULATES dL/dvox into d_grad_vox [n_blocks,512,1+C] as
 * sg_l2_loss_grad followed by sg_render_backward would, plus, for
 * lambda_e != 0, the gradient of the Eikonal term as sg_eikonal gives it at
 * each sample (up to rounding and the order of the float32 atomic adds).
 * Each ray is marched and its corners gathered once.  d_ref_feat [R,C]
 * (nullable iff C == 0), d_ref_depth [R], d_ref_normal [R,3].  SG_EINVAL
 * also for a non-finite lambda.
 */
int sg_render_l2_step(const sg_grid* g, const float* d_vox, int32_t C, const float* d_rays,
                      int64_t n_rays, const sg_render_params* params, const float* d_ref_feat,
                      const float* d_ref_depth, const float* d_ref_normal, float lambda_d,
                      float lambda_n, float lambda_e, float* d_feat_out, float* d_depth,
                      float* d_normal, float* d_wsum, int32_t* d_nsamples, float* d_loss_ray,
                      float* d_grad_vox, const void* d_lists, size_t lists_bytes,
                      sg_stream stream);

/*
 * Packed multi-grid rendering for a render server.  A launch renders the
 * pixel ranges ("slots") of several requests over several resident grids;
 * every pixel's result is bit-identical to sg_rays_pinhole +
 * sg_render_forward on that pixel alone, whatever else is packed with it.
 *
 * sg_packed_grid: opaque device-copyable descriptor of one grid + its
 * voxels + march parameters, filled on the host by sg_packed_grid_desc; the
 * caller copies an array of them to device memory (the grid and d_vox must
 * outlive every launch that uses the descriptor).
 */
typedef struct sg_packed_grid {
  unsigned char opaque[512];
} sg_packed_grid;

int sg_packed_grid_desc(const sg_grid* g, const float* d_vox, int32_t C,
                        const sg_render_params* params, sg_packed_grid* out);

/* SG_OK if desc (host copy) was made by sg_packed_grid_desc from grid g at
 * its current generation; SG_ESTATE if it was made from another grid or
 * before an sg_grid_extend of g moved the grid's memory (the descriptor then
 * refers to freed memory); SG_EINVAL for a NULL pointer. */
int sg_packed_grid_check(const sg_grid* g, const sg_packed_grid* desc);

/*
 * One slot: pixels [pixel_begin, pixel_begin + count) (row-major linear
 * index, u = pixel % width, v = pixel / width) of a request rendered on grid
 * `grid` with pinhole camera `cam` (layout as in sg_rays_pinhole).  Outputs
 * are written at the pixel's index: feat [.,C], depth [.], normal [.,3],
 * wsum [.], nsamples [.] (nullable); the caller sizes them for every pixel
 * its slots name.  ray_base = sum of count over the slots before this one.
 */
typedef struct sg_render_slot {
  int32_t grid;
  int32_t width;
  int64_t pixel_begin;
  int64_t count;
  int64_t ray_base;
  float cam[16];
  float* feat;
  float* depth;
  float* normal;
  float* wsum;
  int32_t* nsamples;
} sg_render_slot;

/*
 * Render the first min(*d_n_slots, max_slots) slots of d_slots (device
 * memory; *d_n_slots is read on the device, so a captured launch can be
 * replayed after the tables change).  All grids used must have feature
 * count C and max_samples <= max_samples_cap; slots naming another grid are
 * skipped.  d_grids is an array of n_grids descriptors (512 bytes each,
 * 8-byte aligned; SG_EINVAL otherwise).  launch_rays sizes the launch
 * (waves loop over however many rays the slots hold).  Asynchronous,
 * allocates nothing, graph-capturable.
 */
int sg_render_forward_packed(const sg_packed_grid* d_grids, int32_t n_grids,
                             const sg_render_slot* d_slots, const int32_t* d_n_slots,
                             int32_t max_slots, int32_t C, int32_t max_samples_cap,
                             int64_t launch_rays, sg_stream stream);

/*
 * The same over one resident grid known on the host: every slot among the
 * first min(*d_n_slots, max_slots) is rendered on grid g with voxels d_vox
 * and params (the slots' `grid` field is ignored).  Each pixel's result is
 * bit-identical to sg_rays_pinhole + sg_render_forward on that pixel.  With
 * the grid fixed per launch the kernel keeps its view in registers, which
 * makes it as fast per ray as sg_render_forward; a server captures one
 * launch per resident grid.  Asynchronous, allocates nothing,
 * graph-capturable.  SG_EINVAL for a NULL pointer, an unsupported C or
 * max_slots / launch_rays < 1.
 */
int sg_render_forward_slots(const sg_grid* g, const float* d_vox, int32_t C,
                            const sg_render_params* params, const sg_render_slot* d_slots,
                            const int32_t* d_n_slots, int32_t max_slots, int64_t launch_rays,
                            sg_stream stream);

/*
 * sg_render_footprint -- memory-traffic accounting of the render (integer,
 * exact).  For each ray writes d_counts int32 [R,3] = (S, U, K): kept
 * samples, distinct voxels read by their interpolation cells, distinct
 * blocks holding those voxels.  If d_touched (uint8 [n_blocks*512],
 * nullable) is given, sets d_touched[voxel] = 1 for every voxel read by any
 * ray (entries never read are left unchanged; the caller zeroes it).
 */
int sg_render_footprint(const sg_grid* g, const float* d_rays, int64_t n_rays,
                        const sg_render_params* params, int32_t* d_counts,
                        uint8_t* d_touched, sg_stream stream);

/*
 * sg_l2_loss_grad -- the rendering losses of Eq. 12-14 in squared-L2 form,
 * averaged over rays:
 *   L = (1/R) sum_r ( |C_r - C*_r|^2 + lambda_d (D_r - D*_r)^2
 *                     + lambda_n |N_r - N*_r|^2 )
 * Inputs: d_feat/d_feat_ref [R,C], d_depth/d_depth_ref [R],
 * d_normal/d_normal_ref [R,3].  Writes dL/d(feat, depth, normal) into
 * d_g_feat [R,C], d_g_depth [R], d_g_normal [R,3] and, if d_loss (float[1])
 * is non-null, the loss value (deterministic two-level reduction).
 * lambda_d or lambda_n may be 0 (that term's gradient is then zero).
 */
int sg_l2_loss_grad(const float* d_feat, const float* d_feat_ref,
                    const float* d_depth, const float* d_depth_ref,
                    const float* d_normal, const float* d_normal_ref,
                    int64_t n_rays, int32_t C, float lambda_d, float lambda_n,
                    float* d_g_feat, float* d_g_depth, float* d_g_normal,
                    float* d_loss, sg_stream stream);

/*
 * sg_optim_step -- one in-place optimiser step on float32 parameters
 * (Sec. 3.5.4 optimises the voxel parameters directly).
 *   kind 0: Adam  (m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *                  p -= lr * (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps))
 *   kind 1: RMSProp (v = b2 v + (1-b2) g^2;  p -= lr * g / (sqrt(v) + eps));
 *           d_m is unused and may be NULL, b1 is ignored.
 *   t is the 1-based step count (Adam bias correction).  n may be 0.
 */
int sg_optim_step(int32_t kind, float* d_param, const float* d_grad,
                  float* d_m, float* d_v, int64_t n, float lr, float b1,
                  float b2, float eps, int32_t t, sg_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* SGRID_H */
