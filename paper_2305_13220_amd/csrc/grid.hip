// Collision-free spatial hash over allocated 8^3 blocks (Sec. 3.2, 3.4.1):
// build with first-occurrence indexing, neighbour table, lookup.
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"

namespace sg {

// ---------------------------------------------------------------------------
// Errors.
static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(SG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int check_grid(const sg_grid* g) {
  if (!g) return fail(SG_EINVAL, "grid is NULL");
  if (g->magic != kGridMagic) return fail(SG_ESTATE, "grid handle is not a live grid");
  return SG_OK;
}

GridView view_of(const sg_grid* g) {
  GridView v;
  v.slots = g->d_slots;
  v.mask = g->capacity - 1;
  v.nbr = g->d_nbr;
  v.n_blocks = g->n_blocks;
  for (int a = 0; a < 3; ++a) {
    v.bmin[a] = g->bmin[a];
    v.bmax[a] = g->bmax[a];
    v.org[a] = g->org[a];
  }
  v.h = g->h;
  v.inv_h = 1.0f / g->h;  // one correctly rounded float32 division
  v.map = g->d_map;
  for (int a = 0; a < 3; ++a) v.mdim[a] = g->mdim[a];
  return v;
}

// ---------------------------------------------------------------------------
// Build kernels.
struct alignas(16) BuildSlot {
  uint64_t key;
  int32_t first;  // smallest input position holding this key
  int32_t idx;    // assigned block index
};

__global__ void k_pack(const int32_t* __restrict__ coords, int64_t n, uint64_t* __restrict__ keys,
                       int* __restrict__ bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t x = coords[3 * i], y = coords[3 * i + 1], z = coords[3 * i + 2];
  if (!in_range(x, y, z)) {
    atomicOr(bad, 1);
    keys[i] = kEmptyKey;
    return;
  }
  keys[i] = pack_key(x, y, z);
}

__global__ void k_fill_build(BuildSlot* __restrict__ s, uint64_t cap) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap) return;
  s[i].key = kEmptyKey;
  s[i].first = INT_MAX;
  s[i].idx = -1;
}

__global__ void k_fill_slots(Slot* __restrict__ s, uint64_t cap) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap) return;
  s[i].key = kEmptyKey;
  s[i].idx = -1;
  s[i].nmask = 0;
}

__device__ inline uint64_t find_build(const BuildSlot* s, uint64_t mask, uint64_t key) {
  uint64_t p = mix64(key) & mask;
  while (s[p].key != key) p = (p + 1) & mask;  // key is known to be present
  return p;
}

__global__ void k_insert_first(const uint64_t* __restrict__ keys, int64_t n, BuildSlot* s,
                               uint64_t mask) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t key = keys[i];
  if (key == kEmptyKey) return;  // a masked-out entry
  // An entry equal to its predecessor is not a first occurrence: skipping
  // it leaves the minimum unchanged and spares the contended slot (runs of
  // equal keys are common, e.g. neighbouring pixels in one block).
  if (i > 0 && keys[i - 1] == key) return;
  uint64_t p = mix64(key) & mask;
  for (;;) {
    unsigned long long prev =
        atomicCAS((unsigned long long*)&s[p].key, (unsigned long long)kEmptyKey,
                  (unsigned long long)key);
    if (prev == kEmptyKey || prev == key) {
      atomicMin(&s[p].first, (int32_t)i);
      return;
    }
    p = (p + 1) & mask;
  }
}

__global__ void k_mark_first(const uint64_t* __restrict__ keys, int64_t n, const BuildSlot* s,
                             uint64_t mask, int32_t* __restrict__ flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flags[i] = (keys[i] != kEmptyKey && s[find_build(s, mask, keys[i])].first == (int32_t)i) ? 1 : 0;
}

__global__ void k_assign(const uint64_t* __restrict__ keys, const int32_t* __restrict__ coords,
                         int64_t n, BuildSlot* s, uint64_t mask, const int32_t* __restrict__ flags,
                         const int32_t* __restrict__ offs, int32_t* __restrict__ out_coords) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flags[i]) return;
  const int32_t idx = offs[i];
  s[find_build(s, mask, keys[i])].idx = idx;
  out_coords[3 * idx] = coords[3 * i];
  out_coords[3 * idx + 1] = coords[3 * i + 1];
  out_coords[3 * idx + 2] = coords[3 * i + 2];
}

__global__ void k_index_of_input(const uint64_t* __restrict__ keys, int64_t n, const BuildSlot* s,
                                 uint64_t mask, int32_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = s[find_build(s, mask, keys[i])].idx;
}

__global__ void k_insert_unique(const int32_t* __restrict__ coords, int64_t n, Slot* s,
                                uint64_t mask) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t key = pack_key(coords[3 * i], coords[3 * i + 1], coords[3 * i + 2]);
  uint64_t p = mix64(key) & mask;
  for (;;) {
    unsigned long long prev =
        atomicCAS((unsigned long long*)&s[p].key, (unsigned long long)kEmptyKey,
                  (unsigned long long)key);
    if (prev == kEmptyKey) {
      s[p].idx = (int32_t)i;
      return;
    }
    p = (p + 1) & mask;
  }
}

// Neighbour table, neighbour mask in the block's own slot, bounding box.
__global__ void k_neighbors(const int32_t* __restrict__ coords, int64_t n, Slot* s, uint64_t mask,
                            int32_t* __restrict__ nbr, int32_t* __restrict__ bbox) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t x = coords[3 * i], y = coords[3 * i + 1], z = coords[3 * i + 2];
  GridView v;
  v.slots = s;
  v.mask = mask;
  int32_t nm = 0;
  for (int q = 0; q < 8; ++q) {
    int32_t idx, unused;
    probe(v, x + (q & 1), y + ((q >> 1) & 1), z + ((q >> 2) & 1), idx, unused);
    nbr[8 * i + q] = idx;
    if (idx >= 0) nm |= 1 << q;
  }
  const uint64_t key = pack_key(x, y, z);
  uint64_t p = mix64(key) & mask;
  while (s[p].key != key) p = (p + 1) & mask;
  s[p].nmask = nm;
  atomicMin(&bbox[0], x);
  atomicMin(&bbox[1], y);
  atomicMin(&bbox[2], z);
  atomicMax(&bbox[3], x);
  atomicMax(&bbox[4], y);
  atomicMax(&bbox[5], z);
}

__global__ void k_init_bbox(int32_t* bbox) {
  if (threadIdx.x < 3) bbox[threadIdx.x] = INT_MAX;
  else if (threadIdx.x < 6) bbox[threadIdx.x] = INT_MIN;
}

// ---------------------------------------------------------------------------
// Exclusive prefix sum of int32 flags (build time only).
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline int wave_inclusive_sum_int(int v) {
  const int l = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int o = shfl(v, l - off < 0 ? l : l - off);
    if (l >= off) v += o;
  }
  return v;
}

// Exclusive scan of kScanThreads values held one per thread; returns the
// exclusive prefix of this thread and the block total.
__device__ inline int block_exclusive_scan(int v, int& total) {
  __shared__ int wave_tot[kScanThreads / kWave];
  const int l = lane_id(), w = threadIdx.x / kWave;
  int inc = wave_inclusive_sum_int(v);
  if (l == kWave - 1) wave_tot[w] = inc;
  __syncthreads();
  int before = 0;
  total = 0;
  for (int j = 0; j < kScanThreads / kWave; ++j) {
    if (j < w) before += wave_tot[j];
    total += wave_tot[j];
  }
  __syncthreads();
  return before + inc - v;
}

__global__ void k_scan_tiles(const int32_t* __restrict__ in, int64_t n, int32_t* __restrict__ out,
                             int32_t* __restrict__ tile_sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int vals[kScanItems];
  int s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    vals[j] = (base + j < n) ? in[base + j] : 0;
    s += vals[j];
  }
  int total;
  int pre = block_exclusive_scan(s, total);
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = pre;
    pre += vals[j];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_sums(int32_t* sums, int64_t m) {
  int carry = 0;
  for (int64_t start = 0; start < m; start += kScanThreads) {
    int64_t i = start + threadIdx.x;
    int v = (i < m) ? sums[i] : 0;
    int total;
    int pre = block_exclusive_scan(v, total);
    if (i < m) sums[i] = carry + pre;
    carry += total;
  }
}

__global__ void k_scan_add(int32_t* __restrict__ out, int64_t n, const int32_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int add = sums[blockIdx.x];
  for (int j = threadIdx.x; j < kScanTile; j += kScanThreads)
    if (base + j < n) out[base + j] += add;
}

// Dense block map: allocated blocks first, then Chebyshev distances by
// repeated 26-neighbour dilation (in place: a cell labelled in round r is
// never mistaken for one of round r-1).
__global__ void k_map_fill(int32_t* __restrict__ map, int64_t cells) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cells) map[i] = -kMapMaxDist;
}

__global__ void k_map_blocks(const int32_t* __restrict__ coords, const int32_t* __restrict__ nbr,
                             int64_t n, int32_t bx0, int32_t by0, int32_t bz0, int32_t dx,
                             int32_t dy, int32_t* __restrict__ map) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int nm = 0;
  for (int q = 0; q < 8; ++q)
    if (nbr[8 * i + q] >= 0) nm |= 1 << q;
  const int64_t cell = ((int64_t)(coords[3 * i + 2] - bz0) * dy + (coords[3 * i + 1] - by0)) * dx +
                       (coords[3 * i] - bx0);
  map[cell] = (int32_t)(i * 256 + nm);
}

__global__ void k_map_dilate(int32_t* map, int32_t dx, int32_t dy, int32_t dz, int32_t r) {
  const int64_t cells = (int64_t)dx * dy * dz;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cells || map[i] != -kMapMaxDist) return;
  const int32_t x = (int32_t)(i % dx), y = (int32_t)((i / dx) % dy), z = (int32_t)(i / ((int64_t)dx * dy));
  for (int oz = -1; oz <= 1; ++oz)
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox) {
        const int32_t X = x + ox, Y = y + oy, Z = z + oz;
        if (X < 0 || Y < 0 || Z < 0 || X >= dx || Y >= dy || Z >= dz) continue;
        const int32_t e = map[((int64_t)Z * dy + Y) * dx + X];
        if ((r == 1 && e >= 0) || (r > 1 && e == -(r - 1))) {
          map[i] = -r;
          return;
        }
      }
}

__global__ void k_lookup(GridView g, const int32_t* __restrict__ q, int64_t n,
                         int32_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t idx, nm;
  probe(g, q[3 * i], q[3 * i + 1], q[3 * i + 2], idx, nm);
  out[i] = idx;
}

static unsigned grid1d(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

static uint64_t pow2_at_least(uint64_t x) {
  uint64_t c = 64;
  while (c < x) c <<= 1;
  return c;
}

// Frees every device pointer it holds on scope exit.
struct DevFree {
  std::vector<void*> ptrs;
  ~DevFree() {
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
  }
  template <class T>
  hipError_t alloc(T** p, size_t bytes) {
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, bytes ? bytes : 16);
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
  void release(void* p) {
    for (auto& q : ptrs)
      if (q == p) q = nullptr;
  }
};

#define SG_ALLOC(holder, ptr, bytes)                                              \
  do {                                                                            \
    hipError_t _e = (holder).alloc(&(ptr), (bytes));                              \
    if (_e != hipSuccess) {                                                       \
      (void)hipGetLastError();                                                    \
      return fail(SG_ENOMEM, std::string("device allocation of ") +               \
                                 std::to_string((size_t)(bytes)) + " bytes failed"); \
    }                                                                             \
  } while (0)


// ---------------------------------------------------------------------------
// Block allocation from depth maps (Sec. 3.4.1).

// Key and block of pixel p of a frame: the pixel is lifted to the camera
// point (x D, y D, D) with x = (u + 1/2 - cx) / fx, y = (v + 1/2 - cy) / fy,
// moved to the world by [R | t], and its block taken through the voxel
// floor((X - origin) / h).  float32, no fused multiply-add, in this order.
// kEmptyKey for an invalid depth or a block (dilated by r) out of range.
__global__ void k_unproject(const float* __restrict__ cams, const float* __restrict__ depth,
                            int32_t W, int32_t H, int64_t P, float inv_h, float ox, float oy,
                            float oz, int32_t r, float depth_max, uint64_t* __restrict__ keys,
                            int32_t* __restrict__ coords) {
#pragma clang fp contract(off)
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int64_t f = p / ((int64_t)W * H);
  const int32_t rem = (int32_t)(p - f * (int64_t)W * H);
  const int32_t v = rem / W, u = rem - v * W;
  const float* K = cams + 16 * f;
  const float D = depth[p];
  uint64_t key = kEmptyKey;
  int32_t b[3] = {0, 0, 0};
  if (isfinite(D) && D > 0.0f && D <= depth_max) {
    const float x = ((float)u + 0.5f - K[2]) / K[0];
    const float y = ((float)v + 0.5f - K[3]) / K[1];
    const float xc[3] = {x * D, y * D, D};
    const float org[3] = {ox, oy, oz};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float* M = K + 4 + 4 * a;
      const float p0 = M[0] * xc[0];
      const float p1 = M[1] * xc[1];
      const float p2 = M[2] * xc[2];
      const float X = ((p0 + p1) + p2) + M[3];
      const float xv = (X - org[a]) * inv_h;
      const bool fin = fabsf(xv) < 16777216.0f;
      ok = ok && fin;
      b[a] = ((int32_t)floorf(fin ? xv : 0.0f)) >> 3;  // arithmetic shift: floor division
      ok = ok && b[a] - r >= -kCoordLimit && b[a] + r < kCoordLimit;
    }
    if (ok) key = pack_key(b[0], b[1], b[2]);
  }
  keys[p] = key;
  coords[3 * p] = b[0];
  coords[3 * p + 1] = b[1];
  coords[3 * p + 2] = b[2];
}

// The (2r+1)^3 blocks around each block, offsets z, y, x from -r to r.
__global__ void k_dilate(const int32_t* __restrict__ in, int64_t n, int32_t r,
                         int32_t* __restrict__ out, uint64_t* __restrict__ keys) {
  const int64_t side = 2 * r + 1, per = side * side * side;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * per) return;
  const int64_t src = i / per;
  const int32_t o = (int32_t)(i - src * per);
  const int32_t dz = o / (int32_t)(side * side), dy = (o / (int32_t)side) % (int32_t)side,
                dx = o % (int32_t)side;
  const int32_t c[3] = {in[3 * src] + dx - r, in[3 * src + 1] + dy - r, in[3 * src + 2] + dz - r};
  out[3 * i] = c[0];
  out[3 * i + 1] = c[1];
  out[3 * i + 2] = c[2];
  keys[i] = pack_key(c[0], c[1], c[2]);
}

}  // namespace sg

using namespace sg;

// First occurrence of every valid key (kEmptyKey entries skipped), in input
// order: coords of the kept entries to out (capacity n), their count to nu.
static int unique_first(const uint64_t* d_keys, const int32_t* d_coords, int64_t n,
                        int32_t* d_out, int64_t& nu, hipStream_t s) {
  nu = 0;
  if (n == 0) return SG_OK;
  DevFree tmp;
  int32_t *d_flags, *d_offs, *d_sums;
  BuildSlot* d_bslots;
  const uint64_t cap = pow2_at_least(2 * (uint64_t)n);
  const int64_t n_tiles = (n + kScanTile - 1) / kScanTile;
  SG_ALLOC(tmp, d_flags, sizeof(int32_t) * n);
  SG_ALLOC(tmp, d_offs, sizeof(int32_t) * n);
  SG_ALLOC(tmp, d_sums, sizeof(int32_t) * n_tiles);
  SG_ALLOC(tmp, d_bslots, sizeof(BuildSlot) * cap);
  const int T = 256;
  k_fill_build<<<grid1d((int64_t)cap, T), T, 0, s>>>(d_bslots, cap);
  k_insert_first<<<grid1d(n, T), T, 0, s>>>(d_keys, n, d_bslots, cap - 1);
  k_mark_first<<<grid1d(n, T), T, 0, s>>>(d_keys, n, d_bslots, cap - 1, d_flags);
  k_scan_tiles<<<(unsigned)n_tiles, kScanThreads, 0, s>>>(d_flags, n, d_offs, d_sums);
  k_scan_sums<<<1, kScanThreads, 0, s>>>(d_sums, n_tiles);
  k_scan_add<<<(unsigned)n_tiles, kScanThreads, 0, s>>>(d_offs, n, d_sums);
  k_assign<<<grid1d(n, T), T, 0, s>>>(d_keys, d_coords, n, d_bslots, cap - 1, d_flags, d_offs,
                                      d_out);
  int32_t last_off = 0, last_flag = 0;
  SG_HIP_CHECK(hipMemcpyAsync(&last_off, d_offs + (n - 1), sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
  SG_HIP_CHECK(hipMemcpyAsync(&last_flag, d_flags + (n - 1), sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
  SG_HIP_CHECK(hipGetLastError());
  SG_HIP_CHECK(hipStreamSynchronize(s));
  nu = (int64_t)last_off + last_flag;
  return SG_OK;
}

// Uniform samples in the allocated blocks (the Eikonal term's uniform
// in-grid samples): point i draws x_k = splitmix64(seed + 4 i + k) (the
// counter-based form of Steele, Lea and Flood's SplitMix64), block
// x_0 mod n, and offsets (x_{1+a} >> 40) 2^-24 inside it; float32 in the
// order written, so the points are the same bits on any device.
__device__ inline uint64_t splitmix64(uint64_t c) {
  uint64_t z = c + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void k_uniform_points(const int32_t* __restrict__ coords, int64_t n_blocks, float h,
                                 float ox, float oy, float oz, int64_t n, uint64_t seed,
                                 float* __restrict__ out) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t base = seed + 4ull * (uint64_t)i;
  const int64_t b = (int64_t)(splitmix64(base) % (uint64_t)n_blocks);
  const float org[3] = {ox, oy, oz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float u = (float)(splitmix64(base + 1 + a) >> 40) * 5.9604644775390625e-8f;  // 2^-24
    const float v0 = (float)(8 * coords[3 * b + a]);
    const float v = v0 + 8.0f * u;
    const float d = v * h;
    out[3 * i + a] = org[a] + d;
  }
}

// The allocated block coordinates for depth maps (shared by sg_alloc_blocks
// and sg_grid_from_depth), in first-occurrence order, in device memory
// owned by `keep`; synchronises the stream.
static int alloc_blocks_dev(const float* d_cams, int32_t n_frames, const float* d_depth,
                            int32_t W, int32_t H, float voxel_size, const float origin[3],
                            int32_t dilate, float depth_max, hipStream_t s, DevFree& keep,
                            int32_t*& d_res, int64_t& no) {
  no = 0;
  d_res = nullptr;
  if (n_frames < 0 || W < 0 || H < 0) return fail(SG_EINVAL, "sizes must be >= 0");
  if (dilate < 0 || dilate > 8) return fail(SG_EINVAL, "dilate must be in [0, 8]");
  if (!(voxel_size > 0.0f) || !std::isfinite(voxel_size))
    return fail(SG_EINVAL, "voxel_size must be finite and > 0");
  if (!origin) return fail(SG_EINVAL, "origin is NULL");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(origin[a])) return fail(SG_EINVAL, "origin must be finite");
  if (std::isnan(depth_max)) return fail(SG_EINVAL, "depth_max is NaN");
  const int64_t P = (int64_t)n_frames * W * H;
  if (P > (int64_t)INT_MAX) return fail(SG_EINVAL, "more than 2^31-1 pixels in one call");
  if (P == 0) return SG_OK;
  if (!d_cams || !d_depth) return fail(SG_EINVAL, "a required pointer is NULL");
  DevFree tmp;
  uint64_t* d_keys;
  int32_t *d_coords, *d_unique;
  SG_ALLOC(tmp, d_keys, sizeof(uint64_t) * P);
  SG_ALLOC(tmp, d_coords, sizeof(int32_t) * 3 * P);
  SG_ALLOC(tmp, d_unique, sizeof(int32_t) * 3 * P);
  const int T = 256;
  k_unproject<<<grid1d(P, T), T, 0, s>>>(d_cams, d_depth, W, H, P, 1.0f / voxel_size, origin[0],
                                         origin[1], origin[2], dilate, depth_max, d_keys,
                                         d_coords);
  int64_t nu = 0;
  int rc = unique_first(d_keys, d_coords, P, d_unique, nu, s);
  if (rc) return rc;
  const int64_t side = 2 * (int64_t)dilate + 1, nd = nu * side * side * side;
  if (nd > (int64_t)INT_MAX) return fail(SG_EINVAL, "too many dilated blocks");
  if (nd == 0) return SG_OK;
  uint64_t* d_dkeys;
  int32_t* d_dil;
  SG_ALLOC(tmp, d_dkeys, sizeof(uint64_t) * nd);
  SG_ALLOC(tmp, d_dil, sizeof(int32_t) * 3 * nd);
  SG_ALLOC(keep, d_res, sizeof(int32_t) * 3 * nd);
  k_dilate<<<grid1d(nd, T), T, 0, s>>>(d_unique, nu, dilate, d_dil, d_dkeys);
  return unique_first(d_dkeys, d_dil, nd, d_res, no, s);  // synchronises the stream
}

extern "C" {

const char* sg_last_error(void) { return g_last_error.c_str(); }

const char* sg_version(void) { return "sgrid 0.1 (gfx950)"; }

int sg_grid_build(const int32_t* d_block_coords, int64_t n, float voxel_size,
                  const float origin[3], sg_stream stream, sg_grid** out,
                  int32_t* d_index_of_input) {
  return sg_grid_build_ex(d_block_coords, n, voxel_size, origin, stream, out, d_index_of_input,
                          nullptr);
}

// Dense block map of a bounding box [bmin, bmax] (block coordinates, each in
// [-2^20, 2^20)) for n_blocks allocated blocks: dims and cell count when the
// box has at most `limit` cells and n_blocks < 2^23 (the map packs a block
// index into 23 bits), else dims = 0 and cells = 0.  The box may span up to
// 2^21 blocks per axis, whose product (2^63) overflows int64: the decision
// is taken in floating point before the (then small) integer count is
// formed.  Returns false for an invalid box.
static bool map_plan(const int32_t bmin[3], const int32_t bmax[3], int64_t n_blocks, int64_t limit,
                     int32_t dims[3], int64_t& cells) {
  dims[0] = dims[1] = dims[2] = 0;
  cells = 0;
  double cells_d = 1.0;
  for (int a = 0; a < 3; ++a) {
    if (bmin[a] > bmax[a] || bmin[a] < -kCoordLimit || bmax[a] >= kCoordLimit) return false;
    cells_d *= (double)bmax[a] - (double)bmin[a] + 1.0;
  }
  if (n_blocks < 0) return false;
  if (limit < 0) limit = SG_DEFAULT_DENSE_MAP_CELLS;
  if (!(cells_d <= (double)limit) || n_blocks >= (int64_t(1) << 23)) return true;
  for (int a = 0; a < 3; ++a) dims[a] = bmax[a] - bmin[a] + 1;
  cells = (int64_t)dims[0] * dims[1] * dims[2];
  return true;
}

int sg_grid_build_ex(const int32_t* d_block_coords, int64_t n, float voxel_size,
                     const float origin[3], sg_stream stream, sg_grid** out,
                     int32_t* d_index_of_input, const sg_build_options* options) {
  int64_t map_limit = SG_DEFAULT_DENSE_MAP_CELLS;
  if (options && options->dense_map_max_cells >= 0) map_limit = options->dense_map_max_cells;
  if (!out) return fail(SG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d_block_coords) return fail(SG_EINVAL, "d_block_coords is NULL");
  if (n < 1 || n > (int64_t)INT_MAX) return fail(SG_EINVAL, "n must be in [1, 2^31-1]");
  if (!(voxel_size > 0.0f) || !std::isfinite(voxel_size))
    return fail(SG_EINVAL, "voxel_size must be finite and > 0");
  if (!origin) return fail(SG_EINVAL, "origin is NULL");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(origin[a])) return fail(SG_EINVAL, "origin must be finite");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  SG_HIP_CHECK(hipGetDevice(&dev));

  DevFree tmp;
  uint64_t* d_keys;
  int* d_bad;
  int32_t *d_flags, *d_offs, *d_sums, *d_tmp_coords;
  BuildSlot* d_bslots;
  const uint64_t cap1 = pow2_at_least(2 * (uint64_t)n);
  const int64_t n_tiles = (n + kScanTile - 1) / kScanTile;
  SG_ALLOC(tmp, d_keys, sizeof(uint64_t) * n);
  SG_ALLOC(tmp, d_bad, sizeof(int));
  SG_ALLOC(tmp, d_flags, sizeof(int32_t) * n);
  SG_ALLOC(tmp, d_offs, sizeof(int32_t) * n);
  SG_ALLOC(tmp, d_sums, sizeof(int32_t) * n_tiles);
  SG_ALLOC(tmp, d_tmp_coords, sizeof(int32_t) * 3 * n);
  SG_ALLOC(tmp, d_bslots, sizeof(BuildSlot) * cap1);

  const int T = 256;
  SG_HIP_CHECK(hipMemsetAsync(d_bad, 0, sizeof(int), s));
  k_pack<<<grid1d(n, T), T, 0, s>>>(d_block_coords, n, d_keys, d_bad);
  int bad = 0;
  SG_HIP_CHECK(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
  SG_HIP_CHECK(hipStreamSynchronize(s));
  if (bad) return fail(SG_ERANGE, "a block coordinate lies outside [-2^20, 2^20)");

  k_fill_build<<<grid1d((int64_t)cap1, T), T, 0, s>>>(d_bslots, cap1);
  k_insert_first<<<grid1d(n, T), T, 0, s>>>(d_keys, n, d_bslots, cap1 - 1);
  k_mark_first<<<grid1d(n, T), T, 0, s>>>(d_keys, n, d_bslots, cap1 - 1, d_flags);
  k_scan_tiles<<<(unsigned)n_tiles, kScanThreads, 0, s>>>(d_flags, n, d_offs, d_sums);
  k_scan_sums<<<1, kScanThreads, 0, s>>>(d_sums, n_tiles);
  k_scan_add<<<(unsigned)n_tiles, kScanThreads, 0, s>>>(d_offs, n, d_sums);
  int32_t last_off = 0, last_flag = 0;
  SG_HIP_CHECK(hipMemcpyAsync(&last_off, d_offs + (n - 1), sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
  SG_HIP_CHECK(hipMemcpyAsync(&last_flag, d_flags + (n - 1), sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
  SG_HIP_CHECK(hipStreamSynchronize(s));
  const int64_t nu = (int64_t)last_off + last_flag;
  k_assign<<<grid1d(n, T), T, 0, s>>>(d_keys, d_block_coords, n, d_bslots, cap1 - 1, d_flags,
                                      d_offs, d_tmp_coords);
  if (d_index_of_input)
    k_index_of_input<<<grid1d(n, T), T, 0, s>>>(d_keys, n, d_bslots, cap1 - 1, d_index_of_input);

  DevFree keep;
  sg_grid* g = new sg_grid();
  g->magic = 0;
  g->device = dev;
  g->n_blocks = nu;
  g->h = voxel_size;
  for (int a = 0; a < 3; ++a) g->org[a] = origin[a];
  g->capacity = pow2_at_least(2 * (uint64_t)nu);
  struct Guard {
    sg_grid* g;
    ~Guard() { delete g; }
  } guard{g};
  int32_t* d_bbox;
  SG_ALLOC(keep, g->d_coords, sizeof(int32_t) * 3 * nu);
  SG_ALLOC(keep, g->d_slots, sizeof(Slot) * g->capacity);
  SG_ALLOC(keep, g->d_nbr, sizeof(int32_t) * 8 * nu);
  SG_ALLOC(tmp, d_bbox, sizeof(int32_t) * 6);
  SG_HIP_CHECK(hipMemcpyAsync(g->d_coords, d_tmp_coords, sizeof(int32_t) * 3 * nu,
                              hipMemcpyDeviceToDevice, s));
  k_fill_slots<<<grid1d((int64_t)g->capacity, T), T, 0, s>>>(g->d_slots, g->capacity);
  k_insert_unique<<<grid1d(nu, T), T, 0, s>>>(g->d_coords, nu, g->d_slots, g->capacity - 1);
  k_init_bbox<<<1, 64, 0, s>>>(d_bbox);
  k_neighbors<<<grid1d(nu, T), T, 0, s>>>(g->d_coords, nu, g->d_slots, g->capacity - 1, g->d_nbr,
                                          d_bbox);
  int32_t bbox[6];
  SG_HIP_CHECK(hipMemcpyAsync(bbox, d_bbox, sizeof(bbox), hipMemcpyDeviceToHost, s));
  SG_HIP_CHECK(hipGetLastError());
  SG_HIP_CHECK(hipStreamSynchronize(s));
  for (int a = 0; a < 3; ++a) {
    g->bmin[a] = bbox[a];
    g->bmax[a] = bbox[3 + a];
  }
  g->d_map = nullptr;
  g->mdim[0] = g->mdim[1] = g->mdim[2] = 0;
  int64_t cells = 0;
  if (map_plan(g->bmin, g->bmax, nu, map_limit, g->mdim, cells) && cells > 0) {
    SG_ALLOC(keep, g->d_map, sizeof(int32_t) * cells);
    k_map_fill<<<grid1d(cells, T), T, 0, s>>>(g->d_map, cells);
    k_map_blocks<<<grid1d(nu, T), T, 0, s>>>(g->d_coords, g->d_nbr, nu, g->bmin[0], g->bmin[1],
                                            g->bmin[2], g->mdim[0], g->mdim[1], g->d_map);
    for (int r = 1; r < kMapMaxDist; ++r)
      k_map_dilate<<<grid1d(cells, T), T, 0, s>>>(g->d_map, g->mdim[0], g->mdim[1], g->mdim[2], r);
    SG_HIP_CHECK(hipGetLastError());
    SG_HIP_CHECK(hipStreamSynchronize(s));
  }
  g->magic = kGridMagic;
  keep.ptrs.clear();  // ownership moves to the grid
  guard.g = nullptr;
  *out = g;
  return SG_OK;
}

int sg_alloc_blocks(const float* d_cams, int32_t n_frames, const float* d_depth, int32_t W,
                    int32_t H, float voxel_size, const float origin[3], int32_t dilate,
                    float depth_max, int32_t* d_out, int64_t cap, int64_t* n_out,
                    sg_stream stream) {
  if (!n_out) return fail(SG_EINVAL, "n_out is NULL");
  *n_out = 0;
  if (cap < 0) return fail(SG_EINVAL, "cap must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  DevFree keep;
  int32_t* d_res = nullptr;
  int64_t no = 0;
  int rc = alloc_blocks_dev(d_cams, n_frames, d_depth, W, H, voxel_size, origin, dilate, depth_max,
                            s, keep, d_res, no);
  if (rc) return rc;
  *n_out = no;
  if (no == 0) return SG_OK;
  if (no > cap) return fail(SG_EINVAL, "cap is smaller than the number of blocks (in *n_out)");
  if (!d_out) return fail(SG_EINVAL, "d_out is NULL");
  SG_HIP_CHECK(hipMemcpyAsync(d_out, d_res, sizeof(int32_t) * 3 * no, hipMemcpyDeviceToDevice, s));
  SG_HIP_CHECK(hipStreamSynchronize(s));
  return SG_OK;
}

int sg_grid_from_depth(const float* d_cams, int32_t n_frames, const float* d_depth, int32_t W,
                       int32_t H, float voxel_size, const float origin[3], int32_t dilate,
                       float depth_max, sg_stream stream, sg_grid** out,
                       const sg_build_options* options) {
  if (!out) return fail(SG_EINVAL, "out is NULL");
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  DevFree keep;
  int32_t* d_res = nullptr;
  int64_t no = 0;
  int rc = alloc_blocks_dev(d_cams, n_frames, d_depth, W, H, voxel_size, origin, dilate, depth_max,
                            s, keep, d_res, no);
  if (rc) return rc;
  if (no == 0) return fail(SG_EINVAL, "no pixel has a valid depth: nothing to allocate");
  return sg_grid_build_ex(d_res, no, voxel_size, origin, stream, out, nullptr, options);
}


int sg_grid_extend(sg_grid* grid, const int32_t* d_new_coords, int64_t n_new, sg_stream stream,
                   const sg_build_options* options) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (n_new < 0) return fail(SG_EINVAL, "n_new must be >= 0");
  if (n_new == 0) return SG_OK;
  if (!d_new_coords) return fail(SG_EINVAL, "d_new_coords is NULL");
  const int64_t n = grid->n_blocks + n_new;
  if (n > (int64_t)INT_MAX) return fail(SG_EINVAL, "more than 2^31-1 blocks");
  hipStream_t s = (hipStream_t)stream;
  DevFree tmp;
  int32_t* d_all;
  SG_ALLOC(tmp, d_all, sizeof(int32_t) * 3 * n);
  // existing blocks first, so they keep their indices; new ones follow in
  // order of first occurrence
  SG_HIP_CHECK(hipMemcpyAsync(d_all, grid->d_coords, sizeof(int32_t) * 3 * grid->n_blocks,
                              hipMemcpyDeviceToDevice, s));
  SG_HIP_CHECK(hipMemcpyAsync(d_all + 3 * grid->n_blocks, d_new_coords, sizeof(int32_t) * 3 * n_new,
                              hipMemcpyDeviceToDevice, s));
  sg_grid* fresh = nullptr;
  const float org[3] = {grid->org[0], grid->org[1], grid->org[2]};
  if ((rc = sg_grid_build_ex(d_all, n, grid->h, org, stream, &fresh, nullptr, options))) return rc;
  // the handle stays valid: its contents move to the new structure, and the
  // generation tells descriptors made before the move from current ones
  (void)hipFree(grid->d_slots);
  (void)hipFree(grid->d_nbr);
  (void)hipFree(grid->d_coords);
  if (grid->d_map) (void)hipFree(grid->d_map);
  const uint64_t gen = grid->generation + 1;
  *grid = *fresh;
  grid->generation = gen;
  fresh->magic = 0;
  delete fresh;
  return SG_OK;
}

int sg_uniform_points(const sg_grid* grid, int64_t n, uint64_t seed, float* d_points,
                      sg_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (n < 0) return fail(SG_EINVAL, "n must be >= 0");
  if (n == 0) return SG_OK;
  if (!d_points) return fail(SG_EINVAL, "d_points is NULL");
  if ((n + 255) / 256 > INT_MAX) return fail(SG_EINVAL, "too many points for one launch");
  k_uniform_points<<<grid1d(n, 256), 256, 0, (hipStream_t)stream>>>(
      grid->d_coords, grid->n_blocks, grid->h, grid->org[0], grid->org[1], grid->org[2], n, seed,
      d_points);
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_grid_num_blocks(const sg_grid* g, int64_t* n_blocks) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!n_blocks) return fail(SG_EINVAL, "n_blocks is NULL");
  *n_blocks = g->n_blocks;
  return SG_OK;
}

int sg_grid_dense_map(const sg_grid* g, int32_t dims[3], int32_t bmin[3]) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!dims || !bmin) return fail(SG_EINVAL, "output pointer is NULL");
  for (int a = 0; a < 3; ++a) {
    dims[a] = g->mdim[a];
    bmin[a] = g->bmin[a];
  }
  return SG_OK;
}

int sg_grid_copy_dense_map(const sg_grid* g, int32_t* d_out, sg_stream stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!g->d_map) return fail(SG_ESTATE, "grid has no dense block map");
  if (!d_out) return fail(SG_EINVAL, "d_out is NULL");
  SG_HIP_CHECK(hipMemcpyAsync(d_out, g->d_map,
                              sizeof(int32_t) * (size_t)g->mdim[0] * g->mdim[1] * g->mdim[2],
                              hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return SG_OK;
}

int sg_grid_dense_map_plan(const int32_t bmin[3], const int32_t bmax[3], int64_t n_blocks,
                           const sg_build_options* options, int32_t dims[3], int64_t* cells) {
  if (!bmin || !bmax || !dims || !cells) return fail(SG_EINVAL, "a required pointer is NULL");
  int64_t c = 0;
  int32_t d[3];
  const int64_t limit = options ? options->dense_map_max_cells : -1;
  if (!map_plan(bmin, bmax, n_blocks, limit, d, c)) {
    dims[0] = dims[1] = dims[2] = 0;
    *cells = 0;
    for (int a = 0; a < 3; ++a)
      if (bmin[a] < -kCoordLimit || bmax[a] >= kCoordLimit)
        return fail(SG_ERANGE, "box outside [-2^20, 2^20)");
    return fail(SG_EINVAL, "bmin must not exceed bmax and n_blocks must be >= 0");
  }
  for (int a = 0; a < 3; ++a) dims[a] = d[a];
  *cells = c;
  return SG_OK;
}

int sg_grid_generation(const sg_grid* g, uint64_t* generation) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!generation) return fail(SG_EINVAL, "generation is NULL");
  *generation = g->generation;
  return SG_OK;
}

int sg_grid_geometry(const sg_grid* g, float* voxel_size, float origin[3]) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!voxel_size || !origin) return fail(SG_EINVAL, "output pointer is NULL");
  *voxel_size = g->h;
  for (int a = 0; a < 3; ++a) origin[a] = g->org[a];
  return SG_OK;
}

int sg_grid_block_coords(const sg_grid* g, int32_t* d_out, sg_stream stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!d_out) return fail(SG_EINVAL, "d_out is NULL");
  SG_HIP_CHECK(hipMemcpyAsync(d_out, g->d_coords, sizeof(int32_t) * 3 * g->n_blocks,
                              hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return SG_OK;
}

int sg_grid_neighbors(const sg_grid* g, int32_t* d_out, sg_stream stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!d_out) return fail(SG_EINVAL, "d_out is NULL");
  SG_HIP_CHECK(hipMemcpyAsync(d_out, g->d_nbr, sizeof(int32_t) * 8 * g->n_blocks,
                              hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return SG_OK;
}

int sg_grid_lookup(const sg_grid* g, const int32_t* d_coords, int64_t n, int32_t* d_idx,
                   sg_stream stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (n < 0) return fail(SG_EINVAL, "n must be >= 0");
  if (n == 0) return SG_OK;
  if (!d_coords || !d_idx) return fail(SG_EINVAL, "d_coords / d_idx is NULL");
  k_lookup<<<grid1d(n, 256), 256, 0, (hipStream_t)stream>>>(view_of(g), d_coords, n, d_idx);
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_grid_destroy(sg_grid* g) {
  if (!g) return SG_OK;
  if (g->magic != kGridMagic) return fail(SG_ESTATE, "grid handle is not a live grid");
  g->magic = 0;
  (void)hipFree(g->d_slots);
  (void)hipFree(g->d_nbr);
  (void)hipFree(g->d_coords);
  if (g->d_map) (void)hipFree(g->d_map);
  delete g;
  return SG_OK;
}

}  // extern "C"
