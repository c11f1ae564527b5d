// Internals shared by the HIP translation units of libsgrid (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "sgrid.h"

namespace sg {

constexpr int kWave = 64;
constexpr uint64_t kEmptyKey = ~0ull;
constexpr int32_t kCoordLimit = SG_COORD_LIMIT;

// ---------------------------------------------------------------------------
// Error reporting (host).
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define SG_HIP_CHECK(expr)                              \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return ::sg::hip_fail(_e, #expr); \
  } while (0)

// ---------------------------------------------------------------------------
// Hash table of allocated blocks: open addressing, linear probing, 16-byte
// slots so one load returns the key, the block index and the neighbour mask.
struct alignas(16) Slot {
  uint64_t key;   // packed block coordinate, kEmptyKey if free
  int32_t idx;    // block index
  int32_t nmask;  // bit s set iff block + (s&1, s>>1&1, s>>2&1) is allocated
};

// 21 bits per axis, offset by 2^20; callers check the range first.
__host__ __device__ inline uint64_t pack_key(int32_t x, int32_t y, int32_t z) {
  return ((uint64_t)(uint32_t)(x + kCoordLimit) << 42) |
         ((uint64_t)(uint32_t)(y + kCoordLimit) << 21) |
         (uint64_t)(uint32_t)(z + kCoordLimit);
}

__host__ __device__ inline bool in_range(int32_t x, int32_t y, int32_t z) {
  return x >= -kCoordLimit && x < kCoordLimit && y >= -kCoordLimit && y < kCoordLimit &&
         z >= -kCoordLimit && z < kCoordLimit;
}

// 64-bit finaliser (MurmurHash3 fmix64): spreads neighbouring coordinates.
__host__ __device__ inline uint64_t mix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// Device view of a built grid.
struct GridView {
  const Slot* slots;
  uint64_t mask;        // capacity - 1 (power of two)
  const int32_t* nbr;   // [n,8]
  int64_t n_blocks;
  int32_t bmin[3], bmax[3];  // bounding box of allocated block coordinates
  float h, inv_h;
  float org[3];
  // Dense block map over the bounding box (nullptr: use the hash).  Entry
  // of block b, at ((bz-bmin.z)*dim.y + by-bmin.y)*dim.x + bx-bmin.x:
  //   >= 0: idx * 256 + neighbour mask of the allocated block
  //   <  0: -D, every block within Chebyshev distance D-1 of b is empty
  const int32_t* map;
  int32_t mdim[3];
};

constexpr int kMapMaxDist = 32;  // distances are capped (a conservative bound)

// Probe for block (x,y,z); returns the slot contents (idx = -1 if absent).
__device__ inline void probe(const GridView& g, int32_t x, int32_t y, int32_t z, int32_t& idx,
                             int32_t& nmask) {
  idx = -1;
  nmask = 0;
  if (!in_range(x, y, z)) return;
  const uint64_t key = pack_key(x, y, z);
  uint64_t s = mix64(key) & g.mask;
  for (;;) {
    const Slot e = g.slots[s];
    if (e.key == key) {
      idx = e.idx;
      nmask = e.nmask;
      return;
    }
    if (e.key == kEmptyKey) return;
    s = (s + 1) & g.mask;
  }
}

// Allocation state of block (x,y,z): idx (-1 if absent), neighbour mask,
// and for an absent block a Chebyshev radius D >= 1 of emptiness around it.
__device__ inline void block_state(const GridView& g, int32_t x, int32_t y, int32_t z,
                                   int32_t& idx, int32_t& nmask, int32_t& dist) {
  dist = 1;
  if (g.map) {
    idx = -1;
    nmask = 0;
    const int32_t rx = x - g.bmin[0], ry = y - g.bmin[1], rz = z - g.bmin[2];
    if ((uint32_t)rx >= (uint32_t)g.mdim[0] || (uint32_t)ry >= (uint32_t)g.mdim[1] ||
        (uint32_t)rz >= (uint32_t)g.mdim[2])
      return;
    const int32_t e = g.map[((int64_t)rz * g.mdim[1] + ry) * g.mdim[0] + rx];
    if (e >= 0) {
      idx = e >> 8;
      nmask = e & 255;
    } else {
      dist = -e;
    }
    return;
  }
  probe(g, x, y, z, idx, nmask);
}

// Camera ray through the centre of pixel (u, v) of a pinhole camera
// K = [fx, fy, cx, cy, R|t (3x4 row-major, camera-to-world)], camera axes x
// right, y down, z forward: origin t, direction normalise(R ((u + 0.5 - cx) /
// fx, (v + 0.5 - cy) / fy, 1)).  No operation is fused, so every kernel that
// calls this produces the same bits.
__device__ inline void pinhole_ray(const float* __restrict__ K, int32_t u, int32_t v, float out[6]) {
#pragma clang fp contract(off)
  const float x = ((float)u + 0.5f - K[2]) / K[0];
  const float y = ((float)v + 0.5f - K[3]) / K[1];
  float d[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float p0 = K[4 + 4 * a] * x;
    const float p1 = K[5 + 4 * a] * y;
    d[a] = (p0 + p1) + K[6 + 4 * a];
  }
  const float s0 = d[0] * d[0], s1 = d[1] * d[1], s2 = d[2] * d[2];
  const float inv = 1.0f / sqrtf((s0 + s1) + s2);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    out[a] = K[7 + 4 * a];
    out[3 + a] = d[a] * inv;
  }
}

// ---------------------------------------------------------------------------
// Wave helpers.
__device__ inline int lane_id() { return __builtin_amdgcn_mbcnt_hi(-1, __builtin_amdgcn_mbcnt_lo(-1, 0)); }

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Number of set bits of m strictly below this lane.
__device__ inline int rank_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

__device__ inline float shfl(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
__device__ inline int shfl(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }

// DPP moves (data-parallel primitives of the GFX9 vector ALU): the source
// lane is read through the instruction's operand path, with no LDS round
// trip.  Lanes whose source does not exist (or whose row is masked off)
// read 0.
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, kRowMask, 0xf, true));
}
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143, kWaveShr1 = 0x138;

// Inclusive prefix sum over the 64 lanes (lane order): a Hillis-Steele scan
// inside each 16-lane row, then the row totals are carried upwards with row
// broadcasts.  Fixed order, so the result is deterministic.
__device__ inline float wave_inclusive_sum(float v) {
  // the adds are kept apart from whatever produced v (no contraction), so a
  // value reduces to the same bits whichever kernel computed it
#pragma clang fp contract(off)
  v += dpp<kRowShr1>(v);
  v += dpp<kRowShr2>(v);
  v += dpp<kRowShr4>(v);
  v += dpp<kRowShr8>(v);
  v += dpp<kRowBcast15, 0xa>(v);  // row 0 -> row 1, row 2 -> row 3
  v += dpp<kRowBcast31, 0xc>(v);  // rows 0-1 -> rows 2-3
  return v;
}

// Value of lane l-1 (0 in lane 0): turns an inclusive scan into an exclusive one.
__device__ inline float wave_shift_up(float v) { return dpp<kWaveShr1>(v); }

// Sum over all 64 lanes, in every lane (deterministic).
__device__ inline float wave_sum(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_inclusive_sum(v)), kWave - 1));
}

__device__ inline int wave_sum_int(int v) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m);
  return v;
}

}  // namespace sg

// Host-side grid object behind the opaque sg_grid handle.
struct sg_grid {
  uint32_t magic;
  int device;
  sg::Slot* d_slots;
  uint64_t capacity;
  int32_t* d_nbr;          // [n,8]
  int32_t* d_coords;       // [n,3]
  int64_t n_blocks;
  int32_t bmin[3], bmax[3];
  float h;
  float org[3];
  int32_t* d_map;          // dense block map over the bounding box, or nullptr
  int32_t mdim[3];
  uint64_t generation;     // 0 when built, +1 per sg_grid_extend (its memory moves)
};

namespace sg {
constexpr uint32_t kGridMagic = 0x53475244u;  // "SGRD"
int check_grid(const sg_grid* g);
GridView view_of(const sg_grid* g);
}  // namespace sg
