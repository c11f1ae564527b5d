// Differentiable volume rendering through the sparse-dense grid
// (Sec. 3.5.1, Eq. 12-15 with the trilinear value and gradient of Eq. 17-18).
//
// Waves are persistent over a strided set of rays (the next ray's origin and
// direction are fetched while the current one is processed); each ray is
// handled by one wavefront.
//   March: the 64 lanes test 64 consecutive lattice points t_k = t_near +
//   k*step at a time -- float32 position, floor, block, block state (dense
//   map or hash), neighbour mask -- and the kept (k, block) pairs are
//   compacted in lattice order into the wave's LDS list.  Runs of lattice
//   points inside empty regions of the dense map are skipped exactly.
//   Shade: lanes take 64 kept samples at a time, gather the 8 corners,
//   interpolate, convert SDF to density and composite with a DPP prefix sum
//   of sigma*step.
//   Backward: a recompute pass stores per-sample (w, dL/dw, T_{k+1}, f) in
//   LDS; the reverse pass maps samples to lanes in reverse order so that the
//   suffix sums of the adjoint are prefix sums over lanes, stages the
//   per-corner terms in LDS, merges runs of samples in one cell and scatters
//   them with float32 atomic adds laid out as (cell, corner, channel).
#include <climits>
#include <cmath>
#include <cstring>

#include <cstddef>

#include "common.h"

namespace sg {

struct Params {
  float step, t_near, t_far, beta, inv_beta;
  int32_t max_samples;
  int32_t k_max;     // last lattice index with t_k <= t_far (-1: none)
  float inv_step;    // 1 / step (rounded; used only for conservative estimates)
};

struct March {
  float ov[3], dv[3];  // voxel-space origin and direction (float32, as rounded)
  int32_t k_lo, k_hi;  // lattice indices to examine, inclusive
};

// t_k and x_k exactly as float32 with one rounding per operation: these
// values decide integers (voxel, block) and must not be contracted.
__host__ __device__ __forceinline__ float lattice_t(float t_near, float step, int32_t k) {
#pragma clang fp contract(off)
  const float kf = (float)k;
  const float ks = kf * step;
  return t_near + ks;
}

__device__ __forceinline__ float lattice_t(const Params& p, int32_t k) {
  return lattice_t(p.t_near, p.step, k);
}

__device__ __forceinline__ float lattice_x(float ov, float dv, float t) {
#pragma clang fp contract(off)
  const float td = t * dv;
  return ov + td;
}

__device__ __forceinline__ float to_voxel(float x, float org, float inv_h) {
#pragma clang fp contract(off)
  const float d = x - org;
  return d * inv_h;
}

constexpr float kPosLimit = 16777216.0f;  // 2^24 voxels: no block beyond
constexpr int32_t kKMax = 1 << 24;

__device__ __forceinline__ void ray_to_voxel(const GridView& g, const float r[6], March& m) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    m.ov[a] = to_voxel(r[a], g.org[a], g.inv_h);
    m.dv[a] = r[3 + a] * g.inv_h;
  }
}

// Ray set-up: voxel-space ray and the lattice range clipped to the grid's
// bounding box.  The clip is computed in float32 with an approximate
// reciprocal and is conservative: the box is widened by 2 voxels plus 1e-5
// of every magnitude involved (float32 lattice positions, the box corners
// and this computation are off by far less), the t interval by 1e-5 of its
// ends, and the index range by 2 plus 1e-5 of its ends.  Lattice points
// outside the range therefore cannot lie in an allocated block.
__device__ bool march_setup(const GridView& g, const float r[6], const Params& p, March& m) {
#pragma unroll
  for (int a = 0; a < 6; ++a)
    if (!isfinite(r[a])) return false;
  if (p.k_max < 0) return false;
  ray_to_voxel(g, r, m);
  float maxo = 0.0f, maxd = 0.0f, maxb = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    maxo = fmaxf(maxo, fabsf(m.ov[a]));
    maxd = fmaxf(maxd, fabsf(m.dv[a]));
    maxb = fmaxf(maxb, fmaxf(fabsf(8.0f * (float)g.bmin[a]), fabsf(8.0f * (float)(g.bmax[a] + 1))));
  }
  const float tabs = fmaxf(fabsf(p.t_near), fabsf(p.t_far));
  const float margin = 2.0f + 1e-5f * (maxo + maxb + tabs * maxd);
  float t0 = -INFINITY, t1 = INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float lo = 8.0f * (float)g.bmin[a] - margin;
    const float hi = 8.0f * (float)(g.bmax[a] + 1) + margin;
    const float o = m.ov[a], d = m.dv[a];
    if (d == 0.0f) {
      if (o < lo || o > hi) return false;
    } else {
      // fmaxf / fminf drop a NaN operand (0 * inf), which only widens
      const float inv = __builtin_amdgcn_rcpf(d);
      const float ta = (lo - o) * inv, tb = (hi - o) * inv;
      t0 = fmaxf(t0, fminf(ta, tb));
      t1 = fminf(t1, fmaxf(ta, tb));
    }
  }
  t0 -= 1e-5f * fabsf(t0);
  t1 += 1e-5f * fabsf(t1);
  if (!(t0 <= t1)) return false;
  const float fl = (t0 - p.t_near) * p.inv_step, fu = (t1 - p.t_near) * p.inv_step;
  const float kl = floorf(fl - 1e-5f * fabsf(fl)) - 2.0f;
  const float ku = ceilf(fu + 1e-5f * fabsf(fu)) + 2.0f;
  if (!(ku >= 0.0f) || !(kl <= (float)p.k_max)) return false;
  m.k_lo = kl <= 0.0f ? 0 : (int32_t)kl;
  m.k_hi = ku >= (float)p.k_max ? p.k_max : (int32_t)ku;
  return m.k_lo <= m.k_hi;
}

// Bits s = sx + 2 sy + 4 sz of the neighbour blocks a cell with local base
// voxel l touches: sx may be 1 only if l.x == 7, etc.
__device__ __forceinline__ int need_mask(int lx, int ly, int lz) {
  int need = 1;
  if (lx == 7) need |= need << 1;
  if (ly == 7) need |= need << 2;
  if (lz == 7) need |= need << 4;
  return need;
}

// True iff lattice point k lies (as float32) in a block within Chebyshev
// distance r of block c.
__device__ __forceinline__ bool in_block_cube(const March& m, const Params& p, int32_t k,
                                              const int32_t c[3], int32_t r) {
  const float t = lattice_t(p, k);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float x = lattice_x(m.ov[a], m.dv[a], t);
    if (!(fabsf(x) < kPosLimit)) return false;
    const int32_t b = ((int32_t)floorf(x)) >> 3;
    if (b < c[a] - r || b > c[a] + r) return false;
  }
  return true;
}

// Lattice point kk lies in the empty block c whose Chebyshev ball of radius
// D-1 holds no allocated block.  Returns (in every lane) a lattice index
// j >= kk such that every point of [kk, j] lies in that ball.  Each
// coordinate of the float32 position is monotone in k, so the lattice points
// in the ball form one run: if kk and j both lie in it, every point between
// them does too and can be skipped.  The ray's exit from the ball's box gives
// an estimate of the run's end; the 64 lanes test the 64 points at and below
// one past it at once, so membership is decided exactly and the estimate only
// places the window.  Called by all lanes with uniform arguments.
__device__ int32_t empty_run_end(const March& m, const Params& p, int32_t kk, const int32_t c[3],
                                 int32_t D, int32_t k_hi) {
  float t_exit = 3.0e38f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float d = m.dv[a], o = m.ov[a];
    const float inv = __builtin_amdgcn_rcpf(d);  // an estimate is all that is needed here
    if (d > 0.0f) t_exit = fminf(t_exit, (8.0f * (float)(c[a] + D) - o) * inv);
    else if (d < 0.0f) t_exit = fminf(t_exit, (8.0f * (float)(c[a] - D + 1) - o) * inv);
  }
  const float top_f = floorf((t_exit - p.t_near) * p.inv_step) + 1.0f;
  // NaN (0 * inf from the reciprocal of a tiny d) falls back to kk: the
  // window top is always in [kk, k_hi].
  const int32_t top =
      !(top_f > (float)kk) ? kk : (top_f >= (float)k_hi ? k_hi : (int32_t)top_f);
  const int32_t j = top - lane_id();
  const bool in = j <= kk || in_block_cube(m, p, j, c, D - 1);
  // the inside points of the window are its lanes from the first set one on
  const uint64_t bal = __ballot(in);
  return bal ? top - (int32_t)__builtin_ctzll(bal) : kk;
}

// The next first lattice point of a march after the 64 points from k0: past
// the empty run when the last of them lies in an empty block at distance >= 2
// from every allocated block.
__device__ __forceinline__ int32_t march_next(const March& m, const Params& p, int32_t k0,
                                              int32_t idx, int32_t dist, const int32_t b[3]) {
  const int32_t D = __builtin_amdgcn_readlane(idx < 0 ? dist : 0, kWave - 1);
  if (D < 2) return k0 + kWave;
  const int32_t c[3] = {__builtin_amdgcn_readlane(b[0], kWave - 1),
                        __builtin_amdgcn_readlane(b[1], kWave - 1),
                        __builtin_amdgcn_readlane(b[2], kWave - 1)};
  return empty_run_end(m, p, k0 + kWave - 1, c, D, m.k_hi) + 1;
}

// One lattice point against the dense block map, without branches: every
// lane loads a map entry (index clamped into the map), and out-of-range
// points read as empty with distance 1.  Returns whether the point is in
// range with a representable position (then b is its block).
__device__ __forceinline__ bool map_point(const GridView& g, const March& m, const Params& p,
                                          int32_t k, bool in_range, bool& valid, int32_t& idx,
                                          int32_t& dist, int32_t b[3]) {
  const float t = lattice_t(p, k);
  int32_t i[3];
  bool ok = in_range;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float x = lattice_x(m.ov[a], m.dv[a], t);
    ok = ok && (fabsf(x) < kPosLimit);
    i[a] = (int32_t)floorf(fabsf(x) < kPosLimit ? x : 0.0f);
    b[a] = i[a] >> 3;
  }
  const uint32_t rx = (uint32_t)(b[0] - g.bmin[0]), ry = (uint32_t)(b[1] - g.bmin[1]),
                 rz = (uint32_t)(b[2] - g.bmin[2]);
  const bool inb = ok && rx < (uint32_t)g.mdim[0] && ry < (uint32_t)g.mdim[1] &&
                   rz < (uint32_t)g.mdim[2];
  // at most 2^28 cells: the index fits 32 bits
  const int32_t cell = inb ? (int32_t)((rz * (uint32_t)g.mdim[1] + ry) * (uint32_t)g.mdim[0] + rx) : 0;
  int32_t e = g.map[cell];
  e = inb ? e : -1;
  idx = e >= 0 ? (e >> 8) : -1;
  dist = e >= 0 ? 0 : -e;
  const int need = need_mask(i[0] & 7, i[1] & 7, i[2] & 7);
  valid = e >= 0 && ((e & 255) & need) == need;
  return ok;
}

// Lattice points per segment of the coarse pass of the dense-map march.
constexpr int kSeg = 8;

// March: kept samples of the ray, in lattice order, into q[0..n) (n <= M).
//
// Dense map: two passes per 8 * 64 lattice points.  The coarse pass gives
// each lane a segment of 8 consecutive points and proves it empty when its
// first point lies in an empty block at Chebyshev distance D >= 1 from every
// allocated block and its last point lies in the ball of radius D-1 around
// that block: each coordinate of the float32 position is monotone in k, so
// every point between lies in the ball too, in blocks that hold no voxel.
// The fine pass then tests the points of the other segments one per lane,
// eight segments per batch, in lattice order.
//
// Hash lookups (no map): 64 points per batch; when the last of them lies in
// an empty block with empty surroundings, the run of points inside that
// empty region is skipped.
__device__ int march_collect(const GridView& g, const March& m, const Params& p, int2* q) {
  const int lane = lane_id();
  int n = 0;
  int32_t k0 = m.k_lo;
  if (g.map) {
    constexpr int32_t kSpan = kSeg * kWave;
    const int seg = lane >> 3, sub = lane & (kSeg - 1);
    while (k0 <= m.k_hi && n < p.max_samples) {
      bool need;
      {
        const bool in = lane <= (m.k_hi - k0) / kSeg;  // first point <= k_hi, no overflow
        const int32_t ks = in ? k0 + kSeg * lane : k0;
        bool valid;
        int32_t idx, dist, b[3];
        const bool ok = map_point(g, m, p, ks, in, valid, idx, dist, b);
        const int32_t ke = in ? min(m.k_hi - ks, kSeg - 1) + ks : ks;
        need = in && !(ok && idx < 0 && in_block_cube(m, p, ke, b, dist - 1));
      }
      uint64_t mask = __ballot(need);
      while (mask && n < p.max_samples) {
        // this lane's segment: the seg-th set bit of the mask
        const int cnt = (int)__popcll(mask);
        int32_t pos = 0;
#pragma unroll
        for (int i = 0; i < kWave / kSeg; ++i) {
          const int32_t pi = mask ? (int32_t)__builtin_ctzll(mask) : 0;
          pos = seg == i ? pi : pos;
          mask &= mask - 1;
        }
        const int32_t k = k0 + kSeg * pos + sub;
        const bool in = seg < cnt && kSeg * pos + sub <= m.k_hi - k0;
        bool valid;
        int32_t idx, dist, b[3];
        map_point(g, m, p, k, in, valid, idx, dist, b);
        const uint64_t bal = __ballot(valid);
        const int r = rank_below(bal);
        if (valid && n + r < p.max_samples) q[n + r] = make_int2(k, idx);
        n = min(p.max_samples, n + (int)__popcll(bal));
      }
      if (m.k_hi - k0 < kSpan) break;
      k0 += kSpan;
    }
    wave_sync();
    return n;
  }
  while (k0 <= m.k_hi && n < p.max_samples) {
    const int32_t k = k0 + lane;
    bool valid = false;
    int32_t idx = -1, dist = 0;
    int32_t b[3] = {0, 0, 0};
    if (k <= m.k_hi) {
      const float t = lattice_t(p, k);
      float x[3];
      bool ok = true;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        x[a] = lattice_x(m.ov[a], m.dv[a], t);
        ok = ok && (fabsf(x[a]) < kPosLimit);
      }
      if (ok) {
        const int32_t ix = (int32_t)floorf(x[0]), iy = (int32_t)floorf(x[1]),
                      iz = (int32_t)floorf(x[2]);
        b[0] = ix >> 3;
        b[1] = iy >> 3;
        b[2] = iz >> 3;
        dist = 1;
        if (b[0] >= g.bmin[0] && b[0] <= g.bmax[0] && b[1] >= g.bmin[1] && b[1] <= g.bmax[1] &&
            b[2] >= g.bmin[2] && b[2] <= g.bmax[2]) {
          int32_t nm;
          block_state(g, b[0], b[1], b[2], idx, nm, dist);
          const int need = need_mask(ix & 7, iy & 7, iz & 7);
          valid = idx >= 0 && (nm & need) == need;
        }
      }
    }
    const uint64_t bal = __ballot(valid);
    const int r = rank_below(bal);
    if (valid && n + r < p.max_samples) q[n + r] = make_int2(k, idx);
    n = min(p.max_samples, n + (int)__popcll(bal));
    k0 = march_next(m, p, k0, idx, dist, b);
  }
  wave_sync();
  return n;
}

// The interpolation cell of a kept sample: t, fraction u, and the element
// offset (block * 512 + local) of each of the 8 corners a = ax + 2 ay + 4 az.
struct Cell {
  float t;
  float u[3];
  int32_t off[8];
};

// Cell of the voxel-space point x in block bi (the block of its base voxel).
__device__ __forceinline__ void cell_at(const GridView& g, const float x[3], int32_t block,
                                        Cell& c) {
  int32_t i[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float fl = floorf(x[a]);
    i[a] = (int32_t)fl;
    c.u[a] = x[a] - fl;
  }
  // Block indices come from a march, a lookup or a caller's list buffer;
  // clamping keeps a stale list from addressing outside the grid (it then
  // renders wrong values, never faults).
  const int64_t bi = min(max((int64_t)block, (int64_t)0), g.n_blocks - 1);
  const int4* row = reinterpret_cast<const int4*>(g.nbr + 8 * bi);
  const int4 n0 = row[0], n1 = row[1];
  int32_t nb[8] = {n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, n1.z, n1.w};
  const int lx = i[0] & 7, ly = i[1] & 7, lz = i[2] & 7;
  // Corner a lies in neighbour block a & o, o = the axes along which the
  // cell crosses its block's upper face (local coordinate 7): one select
  // stage per axis, in place, instead of an 8-way choice per corner.
  const bool ox = lx == 7, oy = ly == 7, oz = lz == 7;
#pragma unroll
  for (int a = 1; a < 8; a += 2) nb[a] = ox ? nb[a] : nb[a - 1];
#pragma unroll
  for (int a = 2; a < 8; a += (a & 1) ? 3 : 1) nb[a] = oy ? nb[a] : nb[a - 2];
#pragma unroll
  for (int a = 4; a < 8; ++a) nb[a] = oz ? nb[a] : nb[a - 4];
  const int px[2] = {lx, (lx + 1) & 7}, py[2] = {8 * ly, 8 * ((ly + 1) & 7)},
            pz[2] = {64 * lz, 64 * ((lz + 1) & 7)};
#pragma unroll
  for (int a = 0; a < 8; ++a)
    c.off[a] = max(nb[a], 0) * SG_BLOCK_VOXELS + px[a & 1] + py[(a >> 1) & 1] + pz[a >> 2];
}

__device__ __forceinline__ void locate(const GridView& g, const March& m, const Params& p, int2 e,
                                       Cell& c) {
  c.t = lattice_t(p, e.x);
  float x[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] = lattice_x(m.ov[a], m.dv[a], c.t);
  cell_at(g, x, e.y, c);
}

// Load the 1 + C parameters of one voxel.
template <int C>
__device__ __forceinline__ void load_voxel(const float* __restrict__ vox, int32_t off, float th[1 + C]) {
  constexpr int V = 1 + C;
  const float* src = vox + (int64_t)off * V;
  if constexpr (V % 4 == 0) {
#pragma unroll
    for (int j = 0; j < V / 4; ++j) {
      const float4 v = reinterpret_cast<const float4*>(src)[j];
      th[4 * j] = v.x;
      th[4 * j + 1] = v.y;
      th[4 * j + 2] = v.z;
      th[4 * j + 3] = v.w;
    }
  } else if constexpr (V % 2 == 0) {
#pragma unroll
    for (int j = 0; j < V / 2; ++j) {
      const float2 v = reinterpret_cast<const float2*>(src)[j];
      th[2 * j] = v.x;
      th[2 * j + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j) th[j] = src[j];
  }
}

// f, grad f (world units) and features at a located cell.  Each gradient
// component is a positive-weighted sum of raw differences of neighbouring
// SDF values, e.g. d/du_x = sum_{y,z} w_y w_z (theta_{1yz} - theta_{0yz}):
// the same polynomial as sum_a (dr_a/du) theta_a, evaluated without the
// cancellation between corners (and exactly zero where the SDF is flat).
template <int C>
__device__ __forceinline__ void interpolate(const float* __restrict__ vox, const Cell& c, float inv_h,
                                            float& f, float grad[3], float feat[C > 0 ? C : 1]) {
  const float wx[2] = {1.0f - c.u[0], c.u[0]}, wy[2] = {1.0f - c.u[1], c.u[1]},
              wz[2] = {1.0f - c.u[2], c.u[2]};
  float sdf[8];
  f = 0.0f;
#pragma unroll
  for (int ch = 0; ch < C; ++ch) feat[ch] = 0.0f;
  // Records of up to four floats: the eight loads are written before any
  // use, so that they are in flight together (the compiler otherwise may
  // wait on each before the next where registers are tight); longer records
  // are consumed corner by corner.
  constexpr int kAhead = 1 + C <= 4 ? 8 : 1;
  float th[kAhead][1 + C];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    if (kAhead == 8) {
      if (a == 0) {
#pragma unroll
        for (int b = 0; b < 8; ++b) load_voxel<C>(vox, c.off[b], th[b % kAhead]);
      }
    } else {
      load_voxel<C>(vox, c.off[a], th[0]);
    }
    const float* t = th[a % kAhead];
    const float r = wx[a & 1] * wy[(a >> 1) & 1] * wz[(a >> 2) & 1];
    sdf[a] = t[0];
    f += r * t[0];
#pragma unroll
    for (int ch = 0; ch < C; ++ch) feat[ch] += r * t[1 + ch];
  }
  float gx = 0.0f, gy = 0.0f, gz = 0.0f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int lo = q & 1, hi = q >> 1;  // the two coordinates held fixed
    const int c0x = 2 * lo + 4 * hi;    // corner (0, lo, hi)
    const int c0y = lo + 4 * hi;        // corner (lo, 0, hi)
    const int c0z = lo + 2 * hi;        // corner (lo, hi, 0)
    gx += wy[lo] * wz[hi] * (sdf[c0x | 1] - sdf[c0x]);
    gy += wx[lo] * wz[hi] * (sdf[c0y | 2] - sdf[c0y]);
    gz += wx[lo] * wy[hi] * (sdf[c0z | 4] - sdf[c0z]);
  }
  grad[0] = gx * inv_h;
  grad[1] = gy * inv_h;
  grad[2] = gz * inv_h;
}

// Laplace-CDF density sigma = Psi_beta(-f)/beta; e = exp(-|f|/beta)/2.
__device__ __forceinline__ float density(float f, const Params& p, float& e) {
  e = 0.5f * expf(-fabsf(f) * p.inv_beta);
  const float psi = (f >= 0.0f) ? e : 1.0f - e;
  return psi * p.inv_beta;
}

// Weight w = T (1 - exp(-sigma delta)) of a sample (Eq. 12-13), rounded once
// and accumulated with explicit fused multiply-adds: every kernel that forms
// a ray's outputs gets the same bits, whatever else the compiler fuses.
__device__ __forceinline__ float sample_weight(float T, float sd) {
  return __fmul_rn(T, -expm1f(-sd));
}

// Rays of one wave: r, r + stride, ...; the next ray is loaded (scalar
// loads: the index is wave-uniform) while the current one is processed.
struct RayStream {
  int64_t r, stride, R;
  float cur[6], nxt[6];
  __device__ RayStream(const float* __restrict__ rays, int64_t first, int64_t stride_, int64_t R_)
      : r(first), stride(stride_), R(R_) {
    if (r < R)
      for (int a = 0; a < 6; ++a) nxt[a] = rays[6 * r + a];
  }
  __device__ bool next(const float* __restrict__ rays) {
    if (r >= R) return false;
#pragma unroll
    for (int a = 0; a < 6; ++a) cur[a] = nxt[a];
    const int64_t rn = r + stride;
    if (rn < R)
      for (int a = 0; a < 6; ++a) nxt[a] = rays[6 * rn + a];
    return true;
  }
  __device__ void advance() { r += stride; }
};

// The same sequence of rays (first, first + stride, ...), set up in batches
// of up to kWave: lane i loads ray i of the batch and runs march_setup on it
// (one pass for the whole batch instead of one wave-wide pass per ray);
// ray i is then read from lane i.
struct BatchRays {
  int64_t stride, R, base, r;
  int i = 0, nb = 0;
  float ray_l[6];
  March m_l;
  uint64_t okm = 0;
  __device__ BatchRays(int64_t first, int64_t stride_, int64_t R_)
      : stride(stride_), R(R_), base(first - (int64_t)kWave * stride_), r(first) {}
  template <bool SETUP>
  __device__ bool next(const float* __restrict__ rays, const GridView& g, const Params& p) {
    if (++i >= nb) {
      base += (int64_t)kWave * stride;
      i = 0;
      if (base >= R) return false;
      nb = (int)min((int64_t)kWave, (R - base + stride - 1) / stride);
      const int64_t rl = base + (int64_t)lane_id() * stride;
      bool ok = false;
#pragma unroll
      for (int a = 0; a < 6; ++a) ray_l[a] = 0.0f;
      if (rl < R) {
#pragma unroll
        for (int a = 0; a < 6; ++a) ray_l[a] = rays[6 * rl + a];
        if (SETUP) ok = march_setup(g, ray_l, p, m_l);
      }
      okm = __ballot(ok);
    }
    r = base + (int64_t)i * stride;
    return true;
  }
  // march set-up of the current ray; false if it has no lattice range
  __device__ bool march_of(March& m) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      m.ov[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m_l.ov[a]), i));
      m.dv[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m_l.dv[a]), i));
    }
    m.k_lo = __builtin_amdgcn_readlane(m_l.k_lo, i);
    m.k_hi = __builtin_amdgcn_readlane(m_l.k_hi, i);
    return (okm >> i) & 1;
  }
  __device__ void ray_of(float out[6]) const {
#pragma unroll
    for (int a = 0; a < 6; ++a)
      out[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ray_l[a]), i));
  }
};

// ---------------------------------------------------------------------------
// Sample lists.  With a caller workspace the march runs as its own light
// kernel (few registers, so many waves per SIMD hide the dependent block
// lookups) and writes each ray's kept samples (lattice index, block index)
// to list[r * max_samples + i], i < counts[r]; the shading kernels then read
// the list instead of marching.  Without a workspace they march themselves.
// Both give the same samples in the same order, so the results are
// bit-identical.
struct SampleList {
  int2* q;          // [R][max_samples]
  int32_t* counts;  // [R]
};

__global__ __launch_bounds__(256) void k_march(GridView g, const float* __restrict__ rays, int64_t R,
                                               Params p, SampleList L) {
  const int wpb = blockDim.x / kWave;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  BatchRays rs((int64_t)blockIdx.x * wpb + w, (int64_t)gridDim.x * wpb, R);
  while (rs.next<true>(rays, g, p)) {
    March m;
    int n = 0;
    if (rs.march_of(m)) n = march_collect(g, m, p, L.q + rs.r * p.max_samples);
    if (lane_id() == 0) L.counts[rs.r] = n;
  }
}

// List prefetch: the count and first 2 kWave entries of the wave's next ray
// are loaded while the current ray is processed; at the next ray they are
// copied into the wave's LDS queue, so the shading reads LDS as it does
// after an in-kernel march.
// The shading kernels take the lists as separate read-only restrict
// parameters, so the (wave-uniform) count is a scalar load whose wait is
// deferred to its first use.
struct ListPrefetch {
  int n = 0;
  int2 e0 = make_int2(0, 0), e1 = make_int2(0, 0);  // entries lane and kWave + lane
  __device__ void load(const int2* __restrict__ lq, const int32_t* __restrict__ lc, int M,
                       int64_t r, int64_t R) {
    if (r < R) {
      n = lc[r];
      const int lane = lane_id();
      if (lane < M) e0 = lq[r * M + lane];
      if (kWave + lane < M) e1 = lq[r * M + kWave + lane];
    }
  }
};

// The samples of ray r into the wave's LDS queue q: from the list if there
// is one (entries beyond the prefetched first kWave are read here), else
// marched.  m.ov / m.dv are set whenever n > 0.
template <bool LIST>
__device__ __forceinline__ int ray_samples(const GridView& g, const BatchRays& rs, const Params& p,
                                           const int2* __restrict__ lq,
                                           const int32_t* __restrict__ lc, ListPrefetch& pf,
                                           int64_t r, int64_t r_next, int64_t R, March& m,
                                           int2* q) {
  if constexpr (LIST) {
    const int M = p.max_samples;
    const int n = min(max(pf.n, 0), M);  // a stale list cannot overrun its row
    const int lane = lane_id();
    if (lane < M) q[lane] = pf.e0;
    if (kWave + lane < M) q[kWave + lane] = pf.e1;
    for (int j = 2 * kWave + lane; j < n; j += kWave) q[j] = lq[r * M + j];
    pf.load(lq, lc, M, r_next, R);
    wave_sync();
    if (n > 0) {
      float ray[6];
      rs.ray_of(ray);
      ray_to_voxel(g, ray, m);
    }
    return n;
  } else {
    return rs.march_of(m) ? march_collect(g, m, p, q) : 0;
  }
}

// ---------------------------------------------------------------------------
// Forward.

// One ray: march, shade, composite; lane 0 writes output row o.
template <int C>
__device__ __forceinline__ void shade_ray(const GridView& g, const float* __restrict__ vox,
                                          const Params& p, const March& m, int n, const int2* q,
                                          int64_t o, float* __restrict__ feat_out,
                                          float* __restrict__ depth, float* __restrict__ normal,
                                          float* __restrict__ wsum, int32_t* __restrict__ nsamples) {
  const int lane = lane_id();
  float accC[C > 0 ? C : 1], accD = 0.0f, accN[3] = {0.0f, 0.0f, 0.0f}, accW = 0.0f;
#pragma unroll
  for (int ch = 0; ch < C; ++ch) accC[ch] = 0.0f;
  float tau = 0.0f;
  for (int c0 = 0; c0 < n; c0 += kWave) {
    const int j = c0 + lane;
    const bool act = j < n;
    float sd = 0.0f, f = 0.0f, grad[3] = {0.0f, 0.0f, 0.0f}, col[C > 0 ? C : 1];
    Cell cell;
    cell.t = 0.0f;
    if (act) {
      locate(g, m, p, q[j], cell);
      interpolate<C>(vox, cell, g.inv_h, f, grad, col);
      float e;
      sd = density(f, p, e) * p.step;
    }
    const float incl = wave_inclusive_sum(sd);
    const float excl = wave_shift_up(incl);
    if (act) {
      const float wt = sample_weight(expf(-(tau + excl)), sd);
#pragma unroll
      for (int ch = 0; ch < C; ++ch) accC[ch] = fmaf(wt, col[ch], accC[ch]);
      accD = fmaf(wt, cell.t, accD);
      accN[0] = fmaf(wt, grad[0], accN[0]);
      accN[1] = fmaf(wt, grad[1], accN[1]);
      accN[2] = fmaf(wt, grad[2], accN[2]);
      accW += wt;
    }
    tau += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(incl), kWave - 1));
  }
#pragma unroll
  for (int ch = 0; ch < C; ++ch) accC[ch] = wave_sum(accC[ch]);
  accD = wave_sum(accD);
  accN[0] = wave_sum(accN[0]);
  accN[1] = wave_sum(accN[1]);
  accN[2] = wave_sum(accN[2]);
  accW = wave_sum(accW);
  if (lane == 0) {
#pragma unroll
    for (int ch = 0; ch < C; ++ch) feat_out[(int64_t)C * o + ch] = accC[ch];
    depth[o] = accD;
    normal[3 * o] = accN[0];
    normal[3 * o + 1] = accN[1];
    normal[3 * o + 2] = accN[2];
    wsum[o] = accW;
    if (nsamples) nsamples[o] = n;
  }
  wave_sync();  // q is reused by the next ray of this wave
}

template <int C, bool LIST>
__global__ __launch_bounds__(256) void k_render_fwd(GridView g, const float* __restrict__ vox,
                                                    const float* __restrict__ rays, int64_t R,
                                                    Params p, const int2* __restrict__ lq,
                                                    const int32_t* __restrict__ lc,
                                                    float* __restrict__ feat_out,
                                                    float* __restrict__ depth,
                                                    float* __restrict__ normal,
                                                    float* __restrict__ wsum,
                                                    int32_t* __restrict__ nsamples) {
  extern __shared__ int2 lds_q[];
  const int wpb = blockDim.x / kWave;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  int2* const q = lds_q + (int64_t)w * p.max_samples;
  BatchRays rs((int64_t)blockIdx.x * wpb + w, (int64_t)gridDim.x * wpb, R);
  ListPrefetch pf;
  if (LIST) pf.load(lq, lc, p.max_samples, rs.r, R);
  while (rs.next<!LIST>(rays, g, p)) {
    March m;
    const int n = ray_samples<LIST>(g, rs, p, lq, lc, pf, rs.r, rs.r + rs.stride, R, m, q);
    shade_ray<C>(g, vox, p, m, n, q, rs.r, feat_out, depth, normal, wsum, nsamples);
  }
}

// Surface points (the nodes of the continuous CRF are zero crossings of the
// SDF seen from random viewpoints): along the kept samples of each ray, the
// first pair of lattice-adjacent samples with f_j > 0 >= f_{j+1}, placed by
// linear interpolation of f, t* = t_j + step f_j / (f_j - f_{j+1}), at
// o + t* d.  Lanes test consecutive pairs of a chunk; the lowest candidate
// writes the ray's point.
__device__ __forceinline__ float sdf_at(const float* __restrict__ vox, const Cell& c, int V) {
  const float wx[2] = {1.0f - c.u[0], c.u[0]}, wy[2] = {1.0f - c.u[1], c.u[1]},
              wz[2] = {1.0f - c.u[2], c.u[2]};
  float f = 0.0f;
#pragma unroll
  for (int a = 0; a < 8; ++a)
    f += wx[a & 1] * wy[(a >> 1) & 1] * wz[(a >> 2) & 1] * vox[(int64_t)c.off[a] * V];
  return f;
}

__global__ __launch_bounds__(256) void k_surface(GridView g, const float* __restrict__ vox, int V,
                                                 const float* __restrict__ rays, int64_t R,
                                                 Params p, float* __restrict__ points,
                                                 int32_t* __restrict__ hit) {
  extern __shared__ int2 lds_q[];
  const int wpb = blockDim.x / kWave, lane = lane_id();
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  int2* const q = lds_q + (int64_t)w * p.max_samples;
  BatchRays rs((int64_t)blockIdx.x * wpb + w, (int64_t)gridDim.x * wpb, R);
  ListPrefetch pf;
  while (rs.next<true>(rays, g, p)) {
    const int64_t r = rs.r;
    March m;
    const int n = ray_samples<false>(g, rs, p, nullptr, nullptr, pf, r, r + rs.stride, R, m, q);
    bool found = false;
    for (int c0 = 0; c0 + 1 < n && !found; c0 += kWave) {
      const int j = c0 + lane;
      bool cand = false;
      float fj = 0.0f, fn = 0.0f, tj = 0.0f;
      if (j + 1 < n && q[j + 1].x == q[j].x + 1) {
        Cell a, b;
        locate(g, m, p, q[j], a);
        locate(g, m, p, q[j + 1], b);
        fj = sdf_at(vox, a, V);
        fn = sdf_at(vox, b, V);
        tj = a.t;
        cand = fj > 0.0f && fn <= 0.0f;
      }
      const uint64_t bal = __ballot(cand);
      if (bal) {
        found = true;
        if (lane == __builtin_ctzll(bal)) {
          float ray[6];
          rs.ray_of(ray);
          const float ts = tj + p.step * (fj / (fj - fn));
#pragma unroll
          for (int a = 0; a < 3; ++a) points[3 * r + a] = ray[a] + ts * ray[3 + a];
          hit[r] = 1;
        }
      }
    }
    if (!found && lane == 0) {
      points[3 * r] = points[3 * r + 1] = points[3 * r + 2] = 0.0f;
      hit[r] = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Packed multi-grid render for serving: one launch renders the pixel ranges
// ("slots") of several requests over several resident grids.  Rays are made
// in the kernel from each slot's camera (the same pinhole function as
// sg_rays_pinhole) and rendered by the same per-ray code as
// sg_render_forward, so each pixel's result does not depend on what else is
// packed with it.  The slot count is read from device memory: the launch can
// be captured once in a graph and replayed with new tables.
struct PackedGrid {
  GridView view;
  const float* vox;
  Params params;
  int32_t C;
  const sg_grid* owner;  // host-side checks only (sg_packed_grid_check)
  uint64_t generation;
};
static_assert(sizeof(PackedGrid) <= sizeof(sg_packed_grid), "descriptor does not fit");

// The kernel reads the descriptors through these mirrors, whose pointers are
// typed global: a pointer loaded from memory is otherwise generic, and every
// access through it would be a flat instruction.
#define SG_GLOBAL __attribute__((address_space(1)))
struct GridViewG {
  const SG_GLOBAL Slot* slots;
  uint64_t mask;
  const SG_GLOBAL int32_t* nbr;
  int64_t n_blocks;
  int32_t bmin[3], bmax[3];
  float h, inv_h;
  float org[3];
  const SG_GLOBAL int32_t* map;
  int32_t mdim[3];
};
struct PackedGridG {
  GridViewG view;
  const SG_GLOBAL float* vox;
  Params params;
  int32_t C;
  const void* owner;
  uint64_t generation;
};
struct SlotG {
  int32_t grid, width;
  int64_t pixel_begin, count, ray_base;
  float cam[16];
  SG_GLOBAL float *feat, *depth, *normal, *wsum;
  SG_GLOBAL int32_t* nsamples;
};
static_assert(sizeof(GridViewG) == sizeof(GridView) && sizeof(PackedGridG) == sizeof(PackedGrid) &&
                  offsetof(PackedGridG, params) == offsetof(PackedGrid, params) &&
                  offsetof(GridViewG, map) == offsetof(GridView, map),
              "descriptor mirrors must match");
static_assert(sizeof(SlotG) == sizeof(sg_render_slot) &&
                  offsetof(SlotG, feat) == offsetof(sg_render_slot, feat) &&
                  offsetof(SlotG, nsamples) == offsetof(sg_render_slot, nsamples),
              "slot mirror must match");

__device__ __forceinline__ GridView view_of(const GridViewG& x) {
  GridView v;
  v.slots = (const Slot*)x.slots;
  v.mask = x.mask;
  v.nbr = (const int32_t*)x.nbr;
  v.n_blocks = x.n_blocks;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    v.bmin[a] = x.bmin[a];
    v.bmax[a] = x.bmax[a];
    v.org[a] = x.org[a];
    v.mdim[a] = x.mdim[a];
  }
  v.h = x.h;
  v.inv_h = x.inv_h;
  v.map = (const int32_t*)x.map;
  return v;
}

// Each wave sets up a batch of its rays lane-parallel (slot lookup, the
// slot's grid, pinhole ray and march clip for ray i in lane i, with that
// grid's box read per lane); the rays are then marched and shaded one by
// one with their grid's view in scalar registers, exactly as k_render_fwd
// does, so every pixel gets the same bits as alone.
template <int C>
__global__ __launch_bounds__(256) void k_render_packed(const sg_packed_grid* __restrict__ grids,
                                                       int32_t n_grids,
                                                       const sg_render_slot* __restrict__ slots,
                                                       const int32_t* __restrict__ d_n_slots,
                                                       int32_t max_slots, int32_t q_cap) {
  extern __shared__ int2 lds_q[];
  const int wpb = blockDim.x / kWave;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  int2* q = lds_q + (int64_t)w * q_cap;
  const int32_t ns = min(*d_n_slots, max_slots);
  if (ns <= 0) return;
  const SlotG* sl = reinterpret_cast<const SlotG*>(slots);
  const int64_t total = sl[ns - 1].ray_base + sl[ns - 1].count;
  const int64_t stride = (int64_t)gridDim.x * wpb;
  const int lane = lane_id();
  for (int64_t base = (int64_t)blockIdx.x * wpb + w; base < total; base += (int64_t)kWave * stride) {
    const int64_t rl = base + (int64_t)lane * stride;
    int32_t lo = 0, gi = 0;
    int64_t pix = 0;
    March ml;
    bool ok = false, use = false;
    if (rl < total) {
      int32_t hi = ns - 1;  // last slot with ray_base <= r
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (sl[mid].ray_base <= rl) lo = mid;
        else hi = mid - 1;
      }
      const SlotG& S = sl[lo];
      gi = S.grid;
      // slots whose ranges leave a gap: rays in the gap belong to no slot
      if (gi >= 0 && gi < n_grids && S.width > 0 && rl - S.ray_base < S.count) {
        // descriptors are sg_packed_grid-sized (512 B) records, not PackedGrid-sized
        const PackedGridG& G = *reinterpret_cast<const PackedGridG*>(grids + gi);
        if (G.C == C && G.params.max_samples <= q_cap) {
          use = true;
          pix = S.pixel_begin + (rl - S.ray_base);
          // a frame has fewer than 2^31 pixels: 32-bit division
          const uint32_t pu = (uint32_t)pix, wu = (uint32_t)S.width;
          const uint32_t row = pu / wu;
          float ray[6];
          pinhole_ray(S.cam, (int32_t)(pu - row * wu), (int32_t)row, ray);
          ok = march_setup(view_of(G.view), ray, G.params, ml);
        }
      }
    }
    const uint64_t use_m = __ballot(use), ok_m = __ballot(ok);
    const int nb = (int)min((int64_t)kWave, (total - base + stride - 1) / stride);
    for (int i = 0; i < nb; ++i) {
      if (!((use_m >> i) & 1)) continue;
      const SlotG& S = sl[__builtin_amdgcn_readlane(lo, i)];
      const PackedGridG& G =
          *reinterpret_cast<const PackedGridG*>(grids + __builtin_amdgcn_readlane(gi, i));
      const int64_t pi = ((int64_t)__builtin_amdgcn_readlane((int32_t)(pix >> 32), i) << 32) |
                         (uint32_t)__builtin_amdgcn_readlane((int32_t)pix, i);
      March m;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        m.ov[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ml.ov[a]), i));
        m.dv[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ml.dv[a]), i));
      }
      m.k_lo = __builtin_amdgcn_readlane(ml.k_lo, i);
      m.k_hi = __builtin_amdgcn_readlane(ml.k_hi, i);
      const GridView g = view_of(G.view);
      const int n = ((ok_m >> i) & 1) ? march_collect(g, m, G.params, q) : 0;
      shade_ray<C>(g, (const float*)G.vox, G.params, m, n, q, pi, (float*)S.feat, (float*)S.depth,
                   (float*)S.normal, (float*)S.wsum, (int32_t*)S.nsamples);
    }
  }
}

// Packed launch over one resident grid (the grid is a kernel argument, so
// its view lives in scalar registers as in k_render_fwd).  Each wave sets up
// a batch of its rays lane-parallel: slot lookup, pinhole ray and march
// clip for ray i in lane i; the rays are then marched and shaded one by one
// exactly as k_render_fwd does, so every pixel gets the same bits.
template <int C>
__global__ __launch_bounds__(256) void k_render_slots(GridView g, const float* __restrict__ vox,
                                                      Params p,
                                                      const sg_render_slot* __restrict__ slots,
                                                      const int32_t* __restrict__ d_n_slots,
                                                      int32_t max_slots) {
  extern __shared__ int2 lds_q[];
  const int wpb = blockDim.x / kWave;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  int2* q = lds_q + (int64_t)w * p.max_samples;
  const int32_t ns = min(*d_n_slots, max_slots);
  if (ns <= 0) return;
  const SlotG* sl = reinterpret_cast<const SlotG*>(slots);
  const int64_t total = sl[ns - 1].ray_base + sl[ns - 1].count;
  const int64_t stride = (int64_t)gridDim.x * wpb;
  const int lane = lane_id();
  for (int64_t base = (int64_t)blockIdx.x * wpb + w; base < total; base += (int64_t)kWave * stride) {
    const int64_t rl = base + (int64_t)lane * stride;
    int32_t lo = 0;
    int64_t pix = 0;
    March ml;
    bool ok = false, in_slot = false;
    if (rl < total) {
      int32_t hi = ns - 1;  // last slot with ray_base <= r
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (sl[mid].ray_base <= rl) lo = mid;
        else hi = mid - 1;
      }
      const SlotG& S = sl[lo];
      // slots whose ranges leave a gap: rays in the gap belong to no slot
      in_slot = S.width > 0 && rl - S.ray_base < S.count;
      if (in_slot) {
        pix = S.pixel_begin + (rl - S.ray_base);
        // a frame has fewer than 2^31 pixels: 32-bit division
        const uint32_t pu = (uint32_t)pix, wu = (uint32_t)S.width;
        const uint32_t row = pu / wu;
        float ray[6];
        pinhole_ray(S.cam, (int32_t)(pu - row * wu), (int32_t)row, ray);
        ok = march_setup(g, ray, p, ml);
      }
    }
    const uint64_t slot_m = __ballot(in_slot), ok_m = __ballot(ok);
    const int nb = (int)min((int64_t)kWave, (total - base + stride - 1) / stride);
    for (int i = 0; i < nb; ++i) {
      if (!((slot_m >> i) & 1)) continue;
      const SlotG& S = sl[__builtin_amdgcn_readlane(lo, i)];
      const int64_t pi = ((int64_t)__builtin_amdgcn_readlane((int32_t)(pix >> 32), i) << 32) |
                         (uint32_t)__builtin_amdgcn_readlane((int32_t)pix, i);
      March m;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        m.ov[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ml.ov[a]), i));
        m.dv[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ml.dv[a]), i));
      }
      m.k_lo = __builtin_amdgcn_readlane(ml.k_lo, i);
      m.k_hi = __builtin_amdgcn_readlane(ml.k_hi, i);
      const int n = ((ok_m >> i) & 1) ? march_collect(g, m, p, q) : 0;
      shade_ray<C>(g, vox, p, m, n, q, pi, (float*)S.feat, (float*)S.depth, (float*)S.normal,
                   (float*)S.wsum, (int32_t*)S.nsamples);
    }
  }
}

// ---------------------------------------------------------------------------
// Point query (Eq. 17-18 at arbitrary points): one lane per point.  The
// voxel-space position, its floor and the validity rule (all 8 corner
// blocks allocated) are the march's, so a query at a sample's position
// returns that sample's f, grad f and features.
__device__ __forceinline__ bool point_cell(const GridView& g, const float* __restrict__ p,
                                           Cell& cell) {
  float x[3];
  bool ok = true;
  int32_t i[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    x[a] = to_voxel(p[a], g.org[a], g.inv_h);
    ok = ok && (fabsf(x[a]) < kPosLimit);
    i[a] = (int32_t)floorf(fabsf(x[a]) < kPosLimit ? x[a] : 0.0f);
  }
  int32_t idx = -1, nm = 0, dist = 0;
  if (ok) {
    const int32_t bx = i[0] >> 3, by = i[1] >> 3, bz = i[2] >> 3;
    if (bx >= g.bmin[0] && bx <= g.bmax[0] && by >= g.bmin[1] && by <= g.bmax[1] &&
        bz >= g.bmin[2] && bz <= g.bmax[2])
      block_state(g, bx, by, bz, idx, nm, dist);
  }
  const int need = need_mask(i[0] & 7, i[1] & 7, i[2] & 7);
  const bool valid = ok && idx >= 0 && (nm & need) == need;
  if (valid) cell_at(g, x, idx, cell);
  return valid;
}

template <int C>
__global__ __launch_bounds__(256) void k_query(GridView g, const float* __restrict__ vox,
                                               const float* __restrict__ pts, int64_t m,
                                               int32_t* __restrict__ valid_out,
                                               float* __restrict__ f_out,
                                               float* __restrict__ grad_out,
                                               float* __restrict__ feat_out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  Cell cell;
  const bool valid = point_cell(g, pts + 3 * q, cell);
  float f = 0.0f, grad[3] = {0.0f, 0.0f, 0.0f}, col[C > 0 ? C : 1];
#pragma unroll
  for (int ch = 0; ch < C; ++ch) col[ch] = 0.0f;
  if (valid) interpolate<C>(vox, cell, g.inv_h, f, grad, col);
  if (valid_out) valid_out[q] = valid ? 1 : 0;
  if (f_out) f_out[q] = f;
  if (grad_out) {
    grad_out[3 * q] = grad[0];
    grad_out[3 * q + 1] = grad[1];
    grad_out[3 * q + 2] = grad[2];
  }
  if (feat_out) {
#pragma unroll
    for (int ch = 0; ch < C; ++ch) feat_out[(int64_t)C * q + ch] = col[ch];
  }
}

// Adjoint of the point query with respect to the voxels: for upstream
// gradients of f, grad f and the features at each valid point, corner a
// receives r_a g_f + (dr_a/du . g_grad) / h in the SDF channel and
// r_a g_feat[c] in feature channel c (float atomics).
// The atomics run with lanes laid out (point, channel) over the wave's 64
// points, corner by corner: consecutive lanes add consecutive channels of
// one voxel's record, so an instruction covers about three records of
// 4(1 + C) bytes instead of 64 scattered ones (float atomics on device
// memory are performed past the L2, one request per 64-byte piece an
// instruction touches).  Without feature gradients only the SDF channel is
// emitted, one lane per point.
template <int C>
__global__ __launch_bounds__(256) void k_query_backward(GridView g, const float* __restrict__ pts,
                                                        int64_t m, const float* __restrict__ g_f,
                                                        const float* __restrict__ g_grad,
                                                        const float* __restrict__ g_feat,
                                                        float* __restrict__ grad_vox) {
  constexpr int V = 1 + C;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = lane_id();
  Cell cell;
  const bool valid = q < m && point_cell(g, pts + 3 * q, cell);
  const uint64_t vmask = __ballot(valid);
  if (vmask == 0) return;  // wave-uniform
  float ra[8], v0[8];
  int32_t off[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    ra[a] = 0.0f;
    v0[a] = 0.0f;
    off[a] = 0;
  }
  if (valid) {
    const float wx[2] = {1.0f - cell.u[0], cell.u[0]}, wy[2] = {1.0f - cell.u[1], cell.u[1]},
                wz[2] = {1.0f - cell.u[2], cell.u[2]};
    const float gf = g_f ? g_f[q] : 0.0f;
    float gg[3] = {0.0f, 0.0f, 0.0f};
    if (g_grad) {
#pragma unroll
      for (int a = 0; a < 3; ++a) gg[a] = g_grad[3 * q + a] * g.inv_h;
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      ra[a] = wx[ax] * wy[ay] * wz[az];
      const float gn = (ax ? 1.0f : -1.0f) * wy[ay] * wz[az] * gg[0] +
                       (ay ? 1.0f : -1.0f) * wx[ax] * wz[az] * gg[1] +
                       (az ? 1.0f : -1.0f) * wx[ax] * wy[ay] * gg[2];
      v0[a] = ra[a] * gf + gn;
      off[a] = cell.off[a];
    }
  }
  const int64_t q0 = q - lane;  // the wave's first point
  const bool sdf_side = g_f || g_grad;
  const int VE = g_feat ? V : 1;  // channels emitted per voxel (uniform)
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    for (int f0 = 0; f0 < kWave * VE; f0 += kWave) {
      const int f = f0 + lane, i = f / VE, ch = f - i * VE;  // i < kWave
      const int32_t o = shfl(off[a], i);
      const float r = shfl(ra[a], i), s0 = shfl(v0[a], i);
      if ((vmask >> i) & 1) {
        if (ch == 0) {
          if (sdf_side) unsafeAtomicAdd(grad_vox + (int64_t)o * V, s0);
        } else if (g_feat) {
          unsafeAtomicAdd(grad_vox + (int64_t)o * V + ch, r * g_feat[(int64_t)C * (q0 + i) + ch - 1]);
        }
      }
    }
  }
}

// Eikonal regulariser (Eq. 16) at points: loss = weight (|g| - 1)^2 with g
// the closed-form gradient of Eq. 18, and its derivative with respect to the
// SDF of the 8 corners.  g is linear in the corner SDFs, one difference per
// cell edge, so its adjoint a = weight 2 (|g| - 1) g / |g| reaches the upper
// end of an x edge as + a_x w_y w_z / h and the lower end as the negative
// (likewise for y and z).  Where |g| = 0 the direction is undefined and
// nothing is scattered.  V = 1 + C floats per voxel; only the SDF channel is
// read and written.
// The scatter runs with lanes laid out (point, x corner): lanes 2j and
// 2j + 1 add the two x-neighbouring corners of one row of cell j of a half
// wave, so one atomic instruction covers the same row of 32 cells, which
// along a lattice or a batch of nearby points mostly share 64-byte pieces
// (float atomics on device memory are performed past the L2, one request
// per piece an instruction touches).
__global__ __launch_bounds__(256) void k_eikonal(GridView g, const float* __restrict__ vox,
                                                 int32_t V, const float* __restrict__ pts,
                                                 int64_t m, float weight,
                                                 float* __restrict__ loss_out,
                                                 float* __restrict__ grad_vox) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Cell cell;
  float l = 0.0f;
  float d[8];
  bool scatter = false;
#pragma unroll
  for (int a = 0; a < 8; ++a) d[a] = 0.0f;
  if (q < m && point_cell(g, pts + 3 * q, cell)) {
    const float wx[2] = {1.0f - cell.u[0], cell.u[0]}, wy[2] = {1.0f - cell.u[1], cell.u[1]},
                wz[2] = {1.0f - cell.u[2], cell.u[2]};
    float sdf[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) sdf[a] = vox[(int64_t)cell.off[a] * V];
    float gx = 0.0f, gy = 0.0f, gz = 0.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int lo = e & 1, hi = e >> 1;
      const int c0x = 2 * lo + 4 * hi, c0y = lo + 4 * hi, c0z = lo + 2 * hi;
      gx += wy[lo] * wz[hi] * (sdf[c0x | 1] - sdf[c0x]);
      gy += wx[lo] * wz[hi] * (sdf[c0y | 2] - sdf[c0y]);
      gz += wx[lo] * wy[hi] * (sdf[c0z | 4] - sdf[c0z]);
    }
    gx *= g.inv_h;
    gy *= g.inv_h;
    gz *= g.inv_h;
    const float n = sqrtf(gx * gx + gy * gy + gz * gz);
    l = weight * (n - 1.0f) * (n - 1.0f);
    if (grad_vox && n > 0.0f) {
      scatter = true;
      const float coef = weight * 2.0f * (n - 1.0f) / n * g.inv_h;
      const float ax = coef * gx, ay = coef * gy, az = coef * gz;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int lo = e & 1, hi = e >> 1;
        const int c0x = 2 * lo + 4 * hi, c0y = lo + 4 * hi, c0z = lo + 2 * hi;
        const float ex = ax * wy[lo] * wz[hi], ey = ay * wx[lo] * wz[hi], ez = az * wx[lo] * wy[hi];
        d[c0x | 1] += ex;
        d[c0x] -= ex;
        d[c0y | 2] += ey;
        d[c0y] -= ey;
        d[c0z | 4] += ez;
        d[c0z] -= ez;
      }
    }
  }
  if (q < m && loss_out) loss_out[q] = l;
  if (!grad_vox) return;  // uniform over the launch
  int32_t off[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) off[a] = scatter ? cell.off[a] : -1;
  const int lane = lane_id(), ax = lane & 1;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int src = half * (kWave / 2) + (lane >> 1);
#pragma unroll
    for (int row = 0; row < 4; ++row) {
      const float v0 = shfl(d[2 * row], src), v1 = shfl(d[2 * row + 1], src);
      const int o0 = shfl(off[2 * row], src), o1 = shfl(off[2 * row + 1], src);
      const int o = ax ? o1 : o0;
      if (o >= 0) unsafeAtomicAdd(grad_vox + (int64_t)o * V, ax ? v1 : v0);
    }
  }
}

// ---------------------------------------------------------------------------
// Backward.
struct SampleState {
  float w, s, tn, f;  // weight, dL/dw, T_{k+1}, SDF
};

// Scatter of the adjoint into grad_vox.  Float atomics on device memory are
// performed past the L2 (each XCD has its own L2), one request per 64-byte
// piece of memory that an instruction touches, so the corner terms of a
// chunk of samples are first summed per voxel and each voxel then gets one
// atomic add per channel, with lanes laid out (voxel, channel).
//
// Per voxel, without atomics in LDS: the samples of a chunk form a monotone
// path of cells (each coordinate of the base voxel is monotone along the
// ray), so the cells holding a voxel as a corner are consecutive lanes.  The
// first of them owns the voxel (it is not a corner of the previous lane's
// cell); the owners' (lane, corner) pairs are listed with a prefix sum, and
// each listed voxel is summed by one lane walking forward from its owner
// while the voxel stays a corner of the lane's cell.
//
// Per-wave LDS: 8 KiB, with the ray's upstream feature gradient added in
// LDS only when C > 4 (up to four channels it is selected from registers).
struct ScatCore {
  float2 val[8 * kWave];    // [a][lane]: (SDF term, w r_a) of corner a
  int32_t off[8 * kWave];   // [a][lane]: element offset of corner a
  int4 base[kWave];         // base voxel of the lane's cell; w = 1 if the lane holds a sample
  uint16_t pair[8 * kWave]; // owned (lane, corner) pairs, lane * 8 + a
};
template <int C, bool IN_LDS = (C > 4)>
struct Scat : ScatCore {
  float gC[C];
};
template <int C>
struct Scat<C, false> : ScatCore {};

// The feature gradient factor of channel ch (1..C) of a voxel's emission.
template <int C>
__device__ __forceinline__ float emit_gC(const Scat<C>* sc, const float gC[C > 0 ? C : 1], int ch) {
  if constexpr (C > 4) {
    return sc->gC[ch > 0 ? ch - 1 : 0];
  } else {
    float v = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) v = ch == c + 1 ? gC[c] : v;
    return v;
  }
}

// Bits a = ax + 2 ay + 4 az of the corners of a cell with base b that are
// also corners of the cell with base b - d: per axis, d = 0 shares both
// corners, d = 1 the lower, d = -1 the upper, anything else none.
__device__ __forceinline__ int shared_corners(int dx, int dy, int dz) {
  auto axis = [](int d, int lo, int hi) {
    return (d == 0 ? (lo | hi) : 0) | (d == 1 ? lo : 0) | (d == -1 ? hi : 0);
  };
  return axis(dx, 0x55, 0xAA) & axis(dy, 0x33, 0xCC) & axis(dz, 0x0F, 0xF0);
}

// Adjoint scatter of one chunk.  Lane holds a sample (act) with its cell,
// weight w, dL/df and gA = dL/d(grad f) of the sample (w g_N from the normal
// output, plus the Eikonal term where it is on); the per-corner terms
//   dL/dtheta_d[a] += r_a dL/df + (dr_a/du . gA) / h      (Eq. 17-18)
//   dL/dtheta_c[a] += w r_a g_C
// are summed per voxel and added to grad_vox.  The samples may be in ray
// order or in reverse order along the lanes.
template <int C>
__device__ __forceinline__ void scatter_chunk(Scat<C>* sc, bool act, const Cell& cell, float w,
                                              float df, const float gA[3],
                                              const float gC[C > 0 ? C : 1], float inv_h,
                                              const March& m, float* __restrict__ grad_vox) {
  constexpr int V = 1 + C;
  const int lane = lane_id();
  int bi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) bi[a] = (int32_t)floorf(lattice_x(m.ov[a], m.dv[a], cell.t));
  if (act) {
    const float wx[2] = {1.0f - cell.u[0], cell.u[0]}, wy[2] = {1.0f - cell.u[1], cell.u[1]},
                wz[2] = {1.0f - cell.u[2], cell.u[2]};
    const float gx = gA[0] * inv_h, gy = gA[1] * inv_h, gz = gA[2] * inv_h;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      const float ra = wx[ax] * wy[ay] * wz[az];
      const float vs = ra * df + (ax ? 1.0f : -1.0f) * wy[ay] * wz[az] * gx +
                       (ay ? 1.0f : -1.0f) * wx[ax] * wz[az] * gy +
                       (az ? 1.0f : -1.0f) * wx[ax] * wy[ay] * gz;
      sc->val[a * kWave + lane] = make_float2(vs, w * ra);
      sc->off[a * kWave + lane] = cell.off[a];
    }
  }
  sc->base[lane] = make_int4(bi[0], bi[1], bi[2], act ? 1 : 0);
  wave_sync();
  // owned corners: not corners of the previous lane's cell
  int owned = 0;
  if (act) {
    owned = 0xFF;
    if (lane > 0) {
      const int4 bp = sc->base[lane - 1];
      if (bp.w) owned &= ~shared_corners(bi[0] - bp.x, bi[1] - bp.y, bi[2] - bp.z);
    }
  }
  const int cnt = __popc(owned);
  const int incl = (int)wave_inclusive_sum((float)cnt);  // exact: at most 512
  const int n_own = __builtin_amdgcn_readlane(incl, kWave - 1);
  int at = incl - cnt;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    if ((owned >> a) & 1) sc->pair[at++] = (uint16_t)(lane * 8 + a);
  }
  wave_sync();
  for (int e0 = 0; e0 < n_own; e0 += kWave) {
    const int e = e0 + lane;
    int32_t e_off = 0;
    float e_vs = 0.0f, e_vw = 0.0f;
    if (e < n_own) {
      const int pr = sc->pair[e];
      const int j = pr >> 3, a = pr & 7;
      const int4 bj = sc->base[j];
      const int cx = bj.x + (a & 1), cy = bj.y + ((a >> 1) & 1), cz = bj.z + (a >> 2);
      float vs = 0.0f, vw = 0.0f;
      for (int k = j; k < kWave; ++k) {
        const int4 bk = sc->base[k];
        const unsigned dx = (unsigned)(cx - bk.x), dy = (unsigned)(cy - bk.y),
                       dz = (unsigned)(cz - bk.z);
        if (!bk.w || (dx | dy | dz) > 1u) break;
        const int ak = (int)(dx + 2 * dy + 4 * dz);
        const float2 v = sc->val[ak * kWave + k];
        vs += v.x;
        vw += v.y;
      }
      e_off = sc->off[a * kWave + j];
      e_vs = vs;
      e_vw = vw;
    }
    // emission: lanes laid out (voxel, channel), each voxel's sums read from
    // the lane that walked it (every lane active for the shuffles)
    const int n_e = min(kWave, n_own - e0);
    for (int f0 = 0; f0 < n_e * V; f0 += kWave) {
      const int f = f0 + lane;
      const int i = min(f / V, kWave - 1), ch = f - (f / V) * V;
      const int32_t o = shfl(e_off, i);
      const float vs = shfl(e_vs, i), vw = shfl(e_vw, i);
      if (f < n_e * V)
        unsafeAtomicAdd(grad_vox + (int64_t)o * V + ch, ch == 0 ? vs : vw * emit_gC<C>(sc, gC, ch));
    }
  }
  wave_sync();
}

// Sum over lanes m > l of v_m (lane order), without cancellation: the wave
// is reversed, prefix-summed and reversed back.
__device__ __forceinline__ float wave_exclusive_suffix_sum(float v) {
  const int lane = lane_id();
  const float rev = shfl(v, kWave - 1 - lane);
  const float ex = wave_shift_up(wave_inclusive_sum(rev));
  return shfl(ex, kWave - 1 - lane);
}

// Reference values of the squared-L2 rendering losses (Eq. 12-14) for the
// fused training step; L = (1/R) sum_r |C - C*|^2 + lambda_d (D - D*)^2 +
// lambda_n |N - N*|^2 + lambda_e sum_k (|grad f(x_k)| - 1)^2 (the Eikonal
// term of Eq. 16 on the ray's samples).
struct L2Ref {
  const float* feat;    // [R,C]
  const float* depth;   // [R]
  const float* normal;  // [R,3]
  float lambda_d, lambda_n, lambda_e;
  float* loss_ray;      // [R] nullable: each ray's term of L
};

// Eikonal term of one sample with gradient g: adds (|g| - 1)^2 to eik and
// returns the factor c of its adjoint, dL/dg = c g, for weight lam (0 where
// |g| = 0: the direction is undefined there).
__device__ __forceinline__ float eikonal_sample(const float g[3], float lam, float& eik) {
  const float n = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  eik += (n - 1.0f) * (n - 1.0f);
  return n > 0.0f ? lam * 2.0f * (n - 1.0f) / n : 0.0f;
}

// Upstream gradients g = dL/d(feat, depth, normal, wsum) of one ray.
template <int C>
struct Upstream {
  float gC[C > 0 ? C : 1];
  float gD, gN[3], gW;
};

// Per-ray inputs, loaded before the march so that their latency is hidden:
// the upstream gradients (backward) or the reference outputs (fused step).
template <int C, bool FUSED>
__device__ __forceinline__ void load_ray_inputs(int64_t r, const float* __restrict__ g_feat,
                                                const float* __restrict__ g_depth,
                                                const float* __restrict__ g_normal,
                                                const float* __restrict__ g_wsum, const L2Ref& ref,
                                                Upstream<C>& v) {
  const float* fc = FUSED ? ref.feat : g_feat;
  const float* fd = FUSED ? ref.depth : g_depth;
  const float* fn = FUSED ? ref.normal : g_normal;
#pragma unroll
  for (int ch = 0; ch < C; ++ch) v.gC[ch] = fc[(int64_t)C * r + ch];
  v.gD = fd[r];
  v.gN[0] = fn[3 * r];
  v.gN[1] = fn[3 * r + 1];
  v.gN[2] = fn[3 * r + 2];
  v.gW = (!FUSED && g_wsum) ? g_wsum[r] : 0.0f;
}

// Stage the ray's upstream feature gradient in LDS for the scatter
// (selects: a dynamic index into a register array would go to scratch).
template <int C>
__device__ __forceinline__ void stage_gC(const Upstream<C>& up, Scat<C>* sc) {
  if constexpr (C > 4) {
    const int lane = lane_id();
    float mine = 0.0f;
#pragma unroll
    for (int ch = 0; ch < C; ++ch) mine = lane == ch ? up.gC[ch] : mine;
    if (lane < C) sc->gC[lane] = mine;
  }
}

// Forward outputs of a ray are reduced over the wave and written by lane 0;
// the fused step then turns them into the upstream gradients of the L2 loss.
template <int C>
__device__ __forceinline__ void write_outputs_and_l2_grad(
    int64_t r, int64_t R, int n, float accC[C > 0 ? C : 1], float accD, float accN[3], float accW,
    float* __restrict__ feat_out, float* __restrict__ depth, float* __restrict__ normal,
    float* __restrict__ wsum, int32_t* __restrict__ nsamples, const L2Ref& ref,
    const Upstream<C>& refv, Upstream<C>& up, Scat<C>* sc, float eik) {
  const int lane = lane_id();
#pragma unroll
  for (int ch = 0; ch < C; ++ch) accC[ch] = wave_sum(accC[ch]);
  accD = wave_sum(accD);
  accN[0] = wave_sum(accN[0]);
  accN[1] = wave_sum(accN[1]);
  accN[2] = wave_sum(accN[2]);
  accW = wave_sum(accW);
  const float s2 = 2.0f / (float)R;
  float loss = 0.0f;
#pragma unroll
  for (int ch = 0; ch < C; ++ch) {
    const float d = accC[ch] - refv.gC[ch];
    up.gC[ch] = s2 * d;
    loss += d * d;
  }
  const float dd = accD - refv.gD;
  up.gD = s2 * ref.lambda_d * dd;
  loss += ref.lambda_d * dd * dd;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float dn = accN[a] - refv.gN[a];
    up.gN[a] = s2 * ref.lambda_n * dn;
    loss += ref.lambda_n * dn * dn;
  }
  if (ref.lambda_e != 0.0f) loss += ref.lambda_e * wave_sum(eik);
  up.gW = 0.0f;
  stage_gC<C>(up, sc);
  if (lane == 0) {
#pragma unroll
    for (int ch = 0; ch < C; ++ch) feat_out[(int64_t)C * r + ch] = accC[ch];
    depth[r] = accD;
    normal[3 * r] = accN[0];
    normal[3 * r + 1] = accN[1];
    normal[3 * r + 2] = accN[2];
    wsum[r] = accW;
    if (nsamples) nsamples[r] = n;
    if (ref.loss_ray) ref.loss_ray[r] = loss / (float)R;
  }
}

// The adjoint of the render (FUSED = false: upstream gradients are inputs),
// or the whole training step of the L2 rendering losses (FUSED = true: the
// forward outputs are written and the upstream gradients formed in
// registers from the reference values, then the same adjoint runs).
template <int C, bool FUSED, bool LIST>
__global__ __launch_bounds__(256) void k_render_bwd(
    GridView g, const float* __restrict__ vox, const float* __restrict__ rays, int64_t R, Params p,
    const int2* __restrict__ lq, const int32_t* __restrict__ lc,
    const float* __restrict__ g_feat, const float* __restrict__ g_depth,
    const float* __restrict__ g_normal, const float* __restrict__ g_wsum, L2Ref ref,
    float* __restrict__ feat_out, float* __restrict__ depth, float* __restrict__ normal,
    float* __restrict__ wsum, int32_t* __restrict__ nsamples, float* __restrict__ grad_vox,
    bool keep_v) {
  extern __shared__ int2 lds_q[];
  const int wpb = blockDim.x / kWave, lane = lane_id();
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int M = p.max_samples;
  // Per-sample state of multi-chunk rays: the last chunk's (the first one
  // pass 2 takes) in the scatter staging, which is free until that chunk's
  // scatter; the others (at most the whole chunks below max_samples - 1) in
  // their own entries.
  const int M_st = (M - 1) / kWave * kWave;
  int2* const q = lds_q + (int64_t)w * M;
  SampleState* st_base = reinterpret_cast<SampleState*>(lds_q + (int64_t)wpb * M);
  SampleState* st = st_base + (int64_t)w * M_st;
  Scat<C>* sc_base = reinterpret_cast<Scat<C>*>(st_base + (int64_t)wpb * M_st);
  Scat<C>* sc = sc_base + w;
  SampleState* st_last = reinterpret_cast<SampleState*>(sc->val);
  // Fused multi-chunk rays: grad f and features of every sample, kept from
  // pass 1 for pass 2 (structure of arrays [3 + C][max_samples]; t follows
  // from the lattice index again) when the launch has the room; otherwise
  // pass 2 interpolates again.
  float* vst = reinterpret_cast<float*>(sc_base + wpb) + (int64_t)w * (3 + C) * M;
  BatchRays rs((int64_t)blockIdx.x * wpb + w, (int64_t)gridDim.x * wpb, R);
  ListPrefetch pf;
  if (LIST) pf.load(lq, lc, M, rs.r, R);
  while (rs.next<!LIST>(rays, g, p)) {
    const int64_t r = rs.r;
    Upstream<C> pre, up;
    load_ray_inputs<C, FUSED>(r, g_feat, g_depth, g_normal, g_wsum, ref, pre);
    March m;
    const int n = ray_samples<LIST>(g, rs, p, lq, lc, pf, r, r + rs.stride, R, m, q);
    if constexpr (!FUSED) {
      if (n == 0) continue;  // wave-uniform: nothing to scatter
      up = pre;
      stage_gC<C>(up, sc);
    }
    if (n <= kWave) {
      // One chunk: every per-sample quantity stays in this lane's registers.
      const bool act = lane < n;
      float sd = 0.0f, f = 0.0f, grad[3] = {0.0f, 0.0f, 0.0f}, col[C > 0 ? C : 1];
#pragma unroll
      for (int ch = 0; ch < C; ++ch) col[ch] = 0.0f;
      Cell cell;
      cell.t = 0.0f;
      if (act) {
        locate(g, m, p, q[lane], cell);
        interpolate<C>(vox, cell, g.inv_h, f, grad, col);
        float e;
        sd = density(f, p, e) * p.step;
      }
      const float incl = wave_inclusive_sum(sd);
      const float excl = wave_shift_up(incl);
      float wt = 0.0f, tn = 0.0f;
      if (act) {
        wt = sample_weight(expf(-excl), sd);
        tn = expf(-incl);
      }
      float ce = 0.0f;  // Eikonal adjoint factor of this sample
      if constexpr (FUSED) {
        float accC[C > 0 ? C : 1], accN[3], eik = 0.0f;
        // the forward's first-chunk accumulation, fma onto zero
#pragma unroll
        for (int ch = 0; ch < C; ++ch) accC[ch] = fmaf(wt, col[ch], 0.0f);
        accN[0] = fmaf(wt, grad[0], 0.0f);
        accN[1] = fmaf(wt, grad[1], 0.0f);
        accN[2] = fmaf(wt, grad[2], 0.0f);
        if (ref.lambda_e != 0.0f && act) ce = eikonal_sample(grad, ref.lambda_e * (1.0f / (float)R), eik);
        write_outputs_and_l2_grad<C>(r, R, n, accC, fmaf(wt, cell.t, 0.0f), accN, wt, feat_out,
                                     depth, normal, wsum, nsamples, ref, pre, up, sc, eik);
        if (n == 0) continue;
      }
      float s = up.gD * cell.t + up.gW + up.gN[0] * grad[0] + up.gN[1] * grad[1] +
                up.gN[2] * grad[2];
#pragma unroll
      for (int ch = 0; ch < C; ++ch) s += up.gC[ch] * col[ch];
      const float later = wave_exclusive_suffix_sum(act ? wt * s : 0.0f);
      float df = 0.0f;
      if (act) {
        const float dsig = p.step * (tn * s - later);
        const float e = 0.5f * expf(-fabsf(f) * p.inv_beta);
        df = dsig * (-e * p.inv_beta * p.inv_beta);
      }
      const float gA[3] = {wt * up.gN[0] + ce * grad[0], wt * up.gN[1] + ce * grad[1],
                           wt * up.gN[2] + ce * grad[2]};
      scatter_chunk<C>(sc, act, cell, wt, df, gA, up.gC, g.inv_h, m, grad_vox);
      continue;
    }
    // Several chunks.  Pass 1: recompute the forward quantities of every
    // sample, in lattice order.
    float accC[C > 0 ? C : 1], accD = 0.0f, accN[3] = {0.0f, 0.0f, 0.0f}, accW = 0.0f;
#pragma unroll
    for (int ch = 0; ch < C; ++ch) accC[ch] = 0.0f;
    float tau = 0.0f, eik = 0.0f;
    const int last = (n - 1) / kWave * kWave;  // first chunk of pass 2
    for (int c0 = 0; c0 < n; c0 += kWave) {
      const int j = c0 + lane;
      const bool act = j < n;
      float sd = 0.0f, f = 0.0f, grad[3] = {0.0f, 0.0f, 0.0f}, col[C > 0 ? C : 1];
      Cell cell;
      cell.t = 0.0f;
      if (act) {
        locate(g, m, p, q[j], cell);
        interpolate<C>(vox, cell, g.inv_h, f, grad, col);
        float e;
        sd = density(f, p, e) * p.step;
      }
      const float incl = wave_inclusive_sum(sd);
      const float excl = wave_shift_up(incl);
      if (act) {
        SampleState s;
        s.w = sample_weight(expf(-(tau + excl)), sd);
        s.tn = expf(-(tau + incl));
        s.f = f;
        if constexpr (FUSED) {
          if (keep_v) {
            vst[j] = grad[0];
            vst[M + j] = grad[1];
            vst[2 * M + j] = grad[2];
#pragma unroll
            for (int ch = 0; ch < C; ++ch) vst[(3 + ch) * M + j] = col[ch];
          }
#pragma unroll
          for (int ch = 0; ch < C; ++ch) accC[ch] = fmaf(s.w, col[ch], accC[ch]);
          accD = fmaf(s.w, cell.t, accD);
          accN[0] = fmaf(s.w, grad[0], accN[0]);
          accN[1] = fmaf(s.w, grad[1], accN[1]);
          accN[2] = fmaf(s.w, grad[2], accN[2]);
          accW += s.w;
          if (ref.lambda_e != 0.0f) eikonal_sample(grad, 0.0f, eik);
          s.s = 0.0f;  // formed in pass 2, once the outputs are known
        } else {
          float dw = up.gD * cell.t + up.gW + up.gN[0] * grad[0] + up.gN[1] * grad[1] +
                     up.gN[2] * grad[2];
#pragma unroll
          for (int ch = 0; ch < C; ++ch) dw += up.gC[ch] * col[ch];
          s.s = dw;
        }
        if (j >= last) st_last[j - last] = s;
        else st[j] = s;
      }
      tau += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(incl), kWave - 1));
    }
    if constexpr (FUSED)
      write_outputs_and_l2_grad<C>(r, R, n, accC, accD, accN, accW, feat_out, depth, normal, wsum,
                                   nsamples, ref, pre, up, sc, eik);
    wave_sync();
    // Pass 2: chunks in reverse with lanes in reverse sample order (lane l
    // holds sample c0 + 63 - l), so sum_{j>k} w_j s_j is an exclusive prefix
    // sum over lanes.
    float carry = 0.0f;
    for (int c0 = last; c0 >= 0; c0 -= kWave) {
      const int j = c0 + (kWave - 1 - lane);
      const bool act = j < n;
      SampleState s = {0.0f, 0.0f, 0.0f, 0.0f};
      Cell cell;
      cell.t = 0.0f;
      float gA[3] = {0.0f, 0.0f, 0.0f};
      if (act) {
        s = j >= last ? st_last[j - last] : st[j];
        locate(g, m, p, q[j], cell);
#pragma unroll
        for (int a = 0; a < 3; ++a) gA[a] = s.w * up.gN[a];
        if constexpr (FUSED) {
          float f, grad[3], col[C > 0 ? C : 1];
          if (keep_v) {
            grad[0] = vst[j];
            grad[1] = vst[M + j];
            grad[2] = vst[2 * M + j];
#pragma unroll
            for (int ch = 0; ch < C; ++ch) col[ch] = vst[(3 + ch) * M + j];
          } else {
            interpolate<C>(vox, cell, g.inv_h, f, grad, col);
          }
          float dw = up.gD * cell.t + up.gW + up.gN[0] * grad[0] + up.gN[1] * grad[1] +
                     up.gN[2] * grad[2];
#pragma unroll
          for (int ch = 0; ch < C; ++ch) dw += up.gC[ch] * col[ch];
          s.s = dw;
          if (ref.lambda_e != 0.0f) {
            float unused = 0.0f;
            const float ce = eikonal_sample(grad, ref.lambda_e * (1.0f / (float)R), unused);
#pragma unroll
            for (int a = 0; a < 3; ++a) gA[a] += ce * grad[a];
          }
        }
      }
      const float ws = s.w * s.s;
      const float incl = wave_inclusive_sum(ws);
      const float later = wave_shift_up(incl);
      const float total = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(incl), kWave - 1));
      float df = 0.0f;
      if (act) {
        const float dsig = p.step * (s.tn * s.s - (carry + later));
        const float e = 0.5f * expf(-fabsf(s.f) * p.inv_beta);
        df = dsig * (-e * p.inv_beta * p.inv_beta);
      }
      scatter_chunk<C>(sc, act, cell, s.w, df, gA, up.gC, g.inv_h, m, grad_vox);
      carry += total;
    }
  }
}

// ---------------------------------------------------------------------------
// Footprint: per-ray (S, U, K) and the touched-voxel map.
__global__ __launch_bounds__(256) void k_footprint(GridView g, const float* __restrict__ rays,
                                                   int64_t R, Params p, int32_t* __restrict__ counts,
                                                   uint8_t* __restrict__ touched) {
  extern __shared__ int2 lds_q[];
  const int wpb = blockDim.x / kWave, lane = lane_id();
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  int2* q = lds_q + (int64_t)w * p.max_samples;
  RayStream rs(rays, (int64_t)blockIdx.x * wpb + w, (int64_t)gridDim.x * wpb, R);
  for (; rs.next(rays); rs.advance()) {
    const int64_t r = rs.r;
    March m;
    int n = 0;
    if (march_setup(g, rs.cur, p, m)) n = march_collect(g, m, p, q);
    int pi[3] = {0, 0, 0};  // base voxel of the previous chunk's last sample
    int vox_total = 0, blk_total = 0;
    for (int c0 = 0; c0 < n; c0 += kWave) {
      const int j = c0 + lane;
      const bool act = j < n;
      int i[3] = {0, 0, 0};
      if (act) {
        const float t = lattice_t(p, q[j].x);
#pragma unroll
        for (int a = 0; a < 3; ++a) i[a] = (int32_t)floorf(lattice_x(m.ov[a], m.dv[a], t));
        if (touched) {
          Cell cell;
          locate(g, m, p, q[j], cell);
#pragma unroll
          for (int a = 0; a < 8; ++a) touched[cell.off[a]] = 1;
        }
      }
      int prev[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int up = shfl(i[a], lane > 0 ? lane - 1 : 0);
        prev[a] = lane > 0 ? up : pi[a];
      }
      int nv = 0, nb = 0;
      if (act) {
        // voxels: the 2x2x2 corner cube minus its overlap with the previous
        // one (per-axis monotone positions: a voxel shared with any earlier
        // sample is shared with the previous one)
        int ov = 1, bsz = 1, bov = 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int d = abs(i[a] - prev[a]);
          ov *= d < 2 ? 2 - d : 0;
          const int lo = i[a] >> 3, hi = (i[a] + 1) >> 3;
          const int plo = prev[a] >> 3, phi = (prev[a] + 1) >> 3;
          bsz *= hi - lo + 1;
          const int o = min(hi, phi) - max(lo, plo) + 1;
          bov *= o > 0 ? o : 0;
        }
        const bool first = (j == 0);
        nv = 8 - (first ? 0 : ov);
        nb = bsz - (first ? 0 : bov);
      }
      vox_total += wave_sum_int(nv);
      blk_total += wave_sum_int(nb);
#pragma unroll
      for (int a = 0; a < 3; ++a) pi[a] = shfl(i[a], kWave - 1);
    }
    if (lane == 0) {
      counts[3 * r] = n;
      counts[3 * r + 1] = vox_total;
      counts[3 * r + 2] = blk_total;
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// Host side.
static bool supported_C(int C) {
  switch (C) {
    case 0: case 1: case 2: case 3: case 4: case 8: case 16: case 19: case 32:
      return true;
    default:
      return false;
  }
}

// Last lattice index k >= -1 with t_near + k*step <= t_far, evaluated with
// the same float32 operations as the kernels.
static int32_t last_lattice_index(float t_near, float step, float t_far) {
  double est = std::floor(((double)t_far - (double)t_near) / (double)step);
  int32_t k = (int32_t)std::fmin(std::fmax(est, -1.0), (double)kKMax);
  while (k + 1 <= kKMax && lattice_t(t_near, step, k + 1) <= t_far) ++k;
  while (k >= 0 && !(lattice_t(t_near, step, k) <= t_far)) --k;
  return k;
}

static int check_params(const sg_render_params* prm, Params& p) {
  if (!prm) return fail(SG_EINVAL, "params is NULL");
  if (!(prm->step > 0.0f) || !std::isfinite(prm->step)) return fail(SG_EINVAL, "step must be finite and > 0");
  if (!(prm->beta > 0.0f) || !std::isfinite(prm->beta)) return fail(SG_EINVAL, "beta must be finite and > 0");
  if (!std::isfinite(prm->t_near) || !std::isfinite(prm->t_far))
    return fail(SG_EINVAL, "t_near / t_far must be finite");
  if (prm->max_samples < 1 || prm->max_samples > SG_MAX_SAMPLES_LIMIT)
    return fail(SG_EINVAL, "max_samples must be in [1, 1024]");
  if (!((prm->t_far - prm->t_near) / prm->step < 16777216.0f))
    return fail(SG_EINVAL, "(t_far - t_near) / step must be below 2^24");
  p.step = prm->step;
  p.t_near = prm->t_near;
  p.t_far = prm->t_far;
  p.beta = prm->beta;
  p.inv_beta = 1.0f / prm->beta;
  p.max_samples = prm->max_samples;
  p.k_max = last_lattice_index(prm->t_near, prm->step, prm->t_far);
  p.inv_step = (float)(1.0 / (double)prm->step);
  return SG_OK;
}

struct Launch {
  unsigned blocks;
  unsigned threads;
  size_t lds;
};

// Waves loop over rays; the grid gives each wave about rays_per_wave rays.
// The backward kernels run one wave per workgroup: ray costs vary, and a
// workgroup's LDS is only released when all its waves are done, so single
// waves keep a CU's LDS in use (measured: the fused step 6% faster than
// with four waves per workgroup).  The forward and serving kernels measured
// best with four waves per workgroup (fewer if the per-wave LDS is large)
// and four rays per wave.
static Launch plan(int64_t R, size_t lds_per_wave, int wpb = 1, int rays_per_wave = 2) {
  while (wpb > 1 && lds_per_wave * wpb > 64 * 1024) wpb >>= 1;
  Launch l;
  l.threads = (unsigned)(wpb * kWave);
  int64_t blocks = (R + (int64_t)wpb * rays_per_wave - 1) / ((int64_t)wpb * rays_per_wave);
  const int64_t cap = 1 << 22;
  l.blocks = (unsigned)(blocks < 1 ? 1 : (blocks < cap ? blocks : cap));
  l.lds = lds_per_wave * wpb;
  return l;
}

// Rays per wave of the packed serving launches.
constexpr int kPackedRays = 16;

#define SG_DISPATCH_C(C, ...)                         \
  switch (C) {                                        \
    case 0: { constexpr int CC = 0; __VA_ARGS__; } break;   \
    case 1: { constexpr int CC = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int CC = 2; __VA_ARGS__; } break;   \
    case 3: { constexpr int CC = 3; __VA_ARGS__; } break;   \
    case 4: { constexpr int CC = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int CC = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int CC = 16; __VA_ARGS__; } break; \
    case 19: { constexpr int CC = 19; __VA_ARGS__; } break; \
    case 32: { constexpr int CC = 32; __VA_ARGS__; } break; \
    default: break;                                   \
  }

// LDS of one wave of k_render_bwd (without the pass-2 values): sample
// queue, per-sample state of all but the last chunk, scatter staging.
static size_t bwd_lds_per_wave(int C, int32_t M) {
  size_t scat = sizeof(ScatCore);
  SG_DISPATCH_C(C, scat = sizeof(Scat<CC>));
  return sizeof(int2) * (size_t)M + sizeof(SampleState) * (size_t)((M - 1) / kWave * kWave) +
         scat;
}

// Workspace of the sample lists: [R][max_samples] int2, then [R] int32.
static bool list_bytes(int64_t R, int32_t M, size_t& bytes) {
  const double b = (double)R * (double)M * 8.0 + (double)R * 4.0;
  if (R < 0 || M < 1 || b > 9.0e18) return false;
  bytes = (size_t)R * (size_t)M * 8u + (size_t)R * 4u;
  return true;
}

// Validate an optional sample-list buffer and view it.
static int list_view(const void* d_lists, size_t bytes, int64_t R, const Params& p, SampleList& L,
                     bool& use) {
  use = false;
  L = {nullptr, nullptr};
  if (!d_lists) {
    if (bytes != 0) return fail(SG_EINVAL, "list bytes given without a list buffer");
    return SG_OK;
  }
  size_t need;
  if (!list_bytes(R, p.max_samples, need)) return fail(SG_ERANGE, "list size overflows");
  if (bytes < need) return fail(SG_EINVAL, "list buffer smaller than sg_render_list_bytes");
  if (reinterpret_cast<uintptr_t>(d_lists) % 8 != 0)
    return fail(SG_EINVAL, "list buffer must be 8-byte aligned");
  char* base = static_cast<char*>(const_cast<void*>(d_lists));
  L.q = reinterpret_cast<int2*>(base);
  L.counts = reinterpret_cast<int32_t*>(base + (size_t)R * p.max_samples * 8u);
  use = true;
  return SG_OK;
}

}  // namespace sg

using namespace sg;

extern "C" {

size_t sg_render_list_bytes(int64_t n_rays, const sg_render_params* params) {
  Params p;
  if (n_rays < 0 || check_params(params, p)) return 0;
  size_t b;
  return list_bytes(n_rays, p.max_samples, b) ? b : 0;
}

int sg_render_march(const sg_grid* grid, const float* d_rays, int64_t n_rays,
                    const sg_render_params* params, void* d_lists, size_t lists_bytes,
                    sg_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  Params p;
  if ((rc = check_params(params, p))) return rc;
  if (n_rays < 0) return fail(SG_EINVAL, "n_rays must be >= 0");
  if (n_rays == 0) return SG_OK;
  if (!d_rays || !d_lists) return fail(SG_EINVAL, "a required pointer is NULL");
  SampleList L;
  bool list;
  if ((rc = list_view(d_lists, lists_bytes, n_rays, p, L, list))) return rc;
  const GridView g = view_of(grid);
  const Launch l = plan(n_rays, 0);
  hipLaunchKernelGGL(k_march, dim3(l.blocks), dim3(l.threads), 0, (hipStream_t)stream, g, d_rays,
                     n_rays, p, L);
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_render_forward(const sg_grid* grid, const float* d_vox, int32_t C, const float* d_rays,
                      int64_t n_rays, const sg_render_params* params, float* d_feat_out,
                      float* d_depth, float* d_normal, float* d_wsum, int32_t* d_nsamples,
                      const void* d_lists, size_t lists_bytes, sg_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  Params p;
  if ((rc = check_params(params, p))) return rc;
  if (!supported_C(C)) return fail(SG_EINVAL, "unsupported feature count C");
  if (n_rays < 0) return fail(SG_EINVAL, "n_rays must be >= 0");
  if (n_rays == 0) return SG_OK;
  if (!d_vox || !d_rays || !d_depth || !d_normal || !d_wsum || (C > 0 && !d_feat_out))
    return fail(SG_EINVAL, "a required pointer is NULL");
  const GridView g = view_of(grid);
  hipStream_t s = (hipStream_t)stream;
  SampleList L;
  bool list;
  if ((rc = list_view(d_lists, lists_bytes, n_rays, p, L, list))) return rc;
  const Launch l = plan(n_rays, sizeof(int2) * p.max_samples, 4, 4);
  if (list) {
    SG_DISPATCH_C(C, hipLaunchKernelGGL((k_render_fwd<CC, true>), dim3(l.blocks), dim3(l.threads),
                                        l.lds, s, g, d_vox, d_rays, n_rays, p, L.q, L.counts, d_feat_out,
                                        d_depth, d_normal, d_wsum, d_nsamples));
  } else {
    SG_DISPATCH_C(C, hipLaunchKernelGGL((k_render_fwd<CC, false>), dim3(l.blocks), dim3(l.threads),
                                        l.lds, s, g, d_vox, d_rays, n_rays, p, L.q, L.counts, d_feat_out,
                                        d_depth, d_normal, d_wsum, d_nsamples));
  }
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_render_backward(const sg_grid* grid, const float* d_vox, int32_t C, const float* d_rays,
                       int64_t n_rays, const sg_render_params* params, const float* d_g_feat,
                       const float* d_g_depth, const float* d_g_normal, const float* d_g_wsum,
                       float* d_grad_vox, const void* d_lists, size_t lists_bytes,
                       sg_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  Params p;
  if ((rc = check_params(params, p))) return rc;
  if (!supported_C(C)) return fail(SG_EINVAL, "unsupported feature count C");
  if (n_rays < 0) return fail(SG_EINVAL, "n_rays must be >= 0");
  if (n_rays == 0) return SG_OK;
  if (!d_vox || !d_rays || !d_g_depth || !d_g_normal || !d_grad_vox || (C > 0 && !d_g_feat))
    return fail(SG_EINVAL, "a required pointer is NULL");
  const GridView g = view_of(grid);
  hipStream_t s = (hipStream_t)stream;
  SampleList L;
  bool list;
  if ((rc = list_view(d_lists, lists_bytes, n_rays, p, L, list))) return rc;
  const Launch l = plan(n_rays, bwd_lds_per_wave(C, p.max_samples));
  const L2Ref none = {nullptr, nullptr, nullptr, 0.0f, 0.0f, 0.0f, nullptr};
  if (list) {
    SG_DISPATCH_C(C, hipLaunchKernelGGL((k_render_bwd<CC, false, true>), dim3(l.blocks),
                                        dim3(l.threads), l.lds, s, g, d_vox, d_rays, n_rays, p, L.q, L.counts,
                                        d_g_feat, d_g_depth, d_g_normal, d_g_wsum, none, nullptr,
                                        nullptr, nullptr, nullptr, nullptr, d_grad_vox, false));
  } else {
    SG_DISPATCH_C(C, hipLaunchKernelGGL((k_render_bwd<CC, false, false>), dim3(l.blocks),
                                        dim3(l.threads), l.lds, s, g, d_vox, d_rays, n_rays, p, L.q, L.counts,
                                        d_g_feat, d_g_depth, d_g_normal, d_g_wsum, none, nullptr,
                                        nullptr, nullptr, nullptr, nullptr, d_grad_vox, false));
  }
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_render_l2_step(const sg_grid* grid, const float* d_vox, int32_t C, const float* d_rays,
                      int64_t n_rays, const sg_render_params* params, const float* d_ref_feat,
                      const float* d_ref_depth, const float* d_ref_normal, float lambda_d,
                      float lambda_n, float lambda_e, float* d_feat_out, float* d_depth,
                      float* d_normal, float* d_wsum, int32_t* d_nsamples, float* d_loss_ray,
                      float* d_grad_vox, const void* d_lists, size_t lists_bytes,
                      sg_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  Params p;
  if ((rc = check_params(params, p))) return rc;
  if (!supported_C(C)) return fail(SG_EINVAL, "unsupported feature count C");
  if (n_rays < 0) return fail(SG_EINVAL, "n_rays must be >= 0");
  if (n_rays == 0) return SG_OK;
  if (!std::isfinite(lambda_d) || !std::isfinite(lambda_n) || !std::isfinite(lambda_e))
    return fail(SG_EINVAL, "lambda_d / lambda_n / lambda_e must be finite");
  if (!d_vox || !d_rays || !d_ref_depth || !d_ref_normal || !d_depth || !d_normal || !d_wsum ||
      !d_grad_vox || (C > 0 && (!d_ref_feat || !d_feat_out)))
    return fail(SG_EINVAL, "a required pointer is NULL");
  const GridView g = view_of(grid);
  hipStream_t s = (hipStream_t)stream;
  SampleList L;
  bool list;
  if ((rc = list_view(d_lists, lists_bytes, n_rays, p, L, list))) return rc;
  // Per-wave LDS: sample queue, per-sample state, scatter staging, and (when
  // the 12 waves a CU's registers allow, three per SIMD, still fit its
  // 160 KiB of LDS with them) the values pass 2 reuses.
  const size_t base = bwd_lds_per_wave(C, p.max_samples);
  const size_t vbytes = sizeof(float) * (size_t)(3 + C) * p.max_samples;
  const bool keep_v = (base + vbytes) * 12 <= 160 * 1024;
  const Launch l = plan(n_rays, base + (keep_v ? vbytes : 0));
  const L2Ref ref = {d_ref_feat, d_ref_depth, d_ref_normal, lambda_d, lambda_n, lambda_e,
                     d_loss_ray};
  if (list) {
    SG_DISPATCH_C(C, hipLaunchKernelGGL((k_render_bwd<CC, true, true>), dim3(l.blocks),
                                        dim3(l.threads), l.lds, s, g, d_vox, d_rays, n_rays, p, L.q, L.counts,
                                        nullptr, nullptr, nullptr, nullptr, ref, d_feat_out,
                                        d_depth, d_normal, d_wsum, d_nsamples, d_grad_vox, keep_v));
  } else {
    SG_DISPATCH_C(C, hipLaunchKernelGGL((k_render_bwd<CC, true, false>), dim3(l.blocks),
                                        dim3(l.threads), l.lds, s, g, d_vox, d_rays, n_rays, p, L.q, L.counts,
                                        nullptr, nullptr, nullptr, nullptr, ref, d_feat_out,
                                        d_depth, d_normal, d_wsum, d_nsamples, d_grad_vox, keep_v));
  }
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_packed_grid_desc(const sg_grid* grid, const float* d_vox, int32_t C,
                        const sg_render_params* params, sg_packed_grid* out) {
  int rc = check_grid(grid);
  if (rc) return rc;
  Params p;
  if ((rc = check_params(params, p))) return rc;
  if (!supported_C(C)) return fail(SG_EINVAL, "unsupported feature count C");
  if (!d_vox || !out) return fail(SG_EINVAL, "a required pointer is NULL");
  PackedGrid d;
  memset(&d, 0, sizeof(d));
  d.view = view_of(grid);
  d.vox = d_vox;
  d.params = p;
  d.C = C;
  d.owner = grid;
  d.generation = grid->generation;
  memset(out, 0, sizeof(*out));
  memcpy(out->opaque, &d, sizeof(d));
  return SG_OK;
}

int sg_packed_grid_check(const sg_grid* grid, const sg_packed_grid* desc) {
  if (!desc) return fail(SG_EINVAL, "desc is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  PackedGrid d;
  memcpy(&d, desc->opaque, sizeof(d));
  if (d.owner != grid) return fail(SG_ESTATE, "descriptor was made from another grid");
  if (d.generation != grid->generation)
    return fail(SG_ESTATE, "descriptor predates an sg_grid_extend of its grid (stale memory)");
  return SG_OK;
}

int sg_render_forward_packed(const sg_packed_grid* d_grids, int32_t n_grids,
                             const sg_render_slot* d_slots, const int32_t* d_n_slots,
                             int32_t max_slots, int32_t C, int32_t max_samples_cap,
                             int64_t launch_rays, sg_stream stream) {
  if (!d_grids || !d_slots || !d_n_slots) return fail(SG_EINVAL, "a required pointer is NULL");
  if (n_grids < 1 || max_slots < 1) return fail(SG_EINVAL, "n_grids and max_slots must be >= 1");
  if (!supported_C(C)) return fail(SG_EINVAL, "unsupported feature count C");
  if (max_samples_cap < 1 || max_samples_cap > SG_MAX_SAMPLES_LIMIT)
    return fail(SG_EINVAL, "max_samples_cap must be in [1, 1024]");
  if (launch_rays < 1) return fail(SG_EINVAL, "launch_rays must be >= 1");
  // 16 rays per wave: a batch's set-up (slot search, slot, descriptor: several
  // dependent memory round trips) is shared by more rays than the plain
  // forward's (one ray load) needs to be
  const Launch l = plan(launch_rays, sizeof(int2) * max_samples_cap, 4, kPackedRays);
  hipStream_t s = (hipStream_t)stream;
  if (reinterpret_cast<uintptr_t>(d_grids) % alignof(PackedGrid) != 0)
    return fail(SG_EINVAL, "d_grids must be 8-byte aligned");
  SG_DISPATCH_C(C, hipLaunchKernelGGL(k_render_packed<CC>, dim3(l.blocks), dim3(l.threads), l.lds,
                                      s, d_grids, n_grids, d_slots, d_n_slots, max_slots,
                                      max_samples_cap));
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_render_forward_slots(const sg_grid* grid, const float* d_vox, int32_t C,
                            const sg_render_params* params, const sg_render_slot* d_slots,
                            const int32_t* d_n_slots, int32_t max_slots, int64_t launch_rays,
                            sg_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  Params p;
  if ((rc = check_params(params, p))) return rc;
  if (!supported_C(C)) return fail(SG_EINVAL, "unsupported feature count C");
  if (!d_vox || !d_slots || !d_n_slots) return fail(SG_EINVAL, "a required pointer is NULL");
  if (max_slots < 1) return fail(SG_EINVAL, "max_slots must be >= 1");
  if (launch_rays < 1) return fail(SG_EINVAL, "launch_rays must be >= 1");
  const GridView g = view_of(grid);
  const Launch l = plan(launch_rays, sizeof(int2) * p.max_samples, 4, kPackedRays);
  SG_DISPATCH_C(C, hipLaunchKernelGGL(k_render_slots<CC>, dim3(l.blocks), dim3(l.threads), l.lds,
                                      (hipStream_t)stream, g, d_vox, p, d_slots, d_n_slots,
                                      max_slots));
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_query(const sg_grid* grid, const float* d_vox, int32_t C, const float* d_points,
             int64_t n_points, int32_t* d_valid, float* d_f, float* d_grad, float* d_feat,
             sg_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!supported_C(C)) return fail(SG_EINVAL, "unsupported feature count C");
  if (n_points < 0) return fail(SG_EINVAL, "n_points must be >= 0");
  if (n_points == 0) return SG_OK;
  if (!d_vox || !d_points) return fail(SG_EINVAL, "a required pointer is NULL");
  const GridView g = view_of(grid);
  const int64_t blocks = (n_points + 255) / 256;
  if (blocks > INT_MAX) return fail(SG_ERANGE, "too many points for one launch");
  SG_DISPATCH_C(C, hipLaunchKernelGGL(k_query<CC>, dim3((unsigned)blocks), dim3(256), 0,
                                      (hipStream_t)stream, g, d_vox, d_points, n_points, d_valid,
                                      d_f, d_grad, C > 0 ? d_feat : nullptr));
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_surface_points(const sg_grid* grid, const float* d_vox, int32_t C, const float* d_rays,
                      int64_t n_rays, const sg_render_params* params, float* d_points,
                      int32_t* d_hit, sg_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  Params p;
  if ((rc = check_params(params, p))) return rc;
  if (C < 0 || C > 64) return fail(SG_EINVAL, "C must be in [0, 64]");
  if (n_rays < 0) return fail(SG_EINVAL, "n_rays must be >= 0");
  if (n_rays == 0) return SG_OK;
  if (!d_vox || !d_rays || !d_points || !d_hit) return fail(SG_EINVAL, "a required pointer is NULL");
  const GridView g = view_of(grid);
  const Launch l = plan(n_rays, sizeof(int2) * p.max_samples, 4, 4);
  hipLaunchKernelGGL(k_surface, dim3(l.blocks), dim3(l.threads), l.lds, (hipStream_t)stream, g,
                     d_vox, 1 + C, d_rays, n_rays, p, d_points, d_hit);
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_query_backward(const sg_grid* grid, int32_t C, const float* d_points, int64_t n_points,
                      const float* d_g_f, const float* d_g_grad, const float* d_g_feat,
                      float* d_grad_vox, sg_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!supported_C(C)) return fail(SG_EINVAL, "unsupported feature count C");
  if (n_points < 0) return fail(SG_EINVAL, "n_points must be >= 0");
  if (n_points == 0) return SG_OK;
  if (!d_points || !d_grad_vox) return fail(SG_EINVAL, "a required pointer is NULL");
  const GridView g = view_of(grid);
  const int64_t blocks = (n_points + 255) / 256;
  if (blocks > INT_MAX) return fail(SG_ERANGE, "too many points for one launch");
  SG_DISPATCH_C(C, hipLaunchKernelGGL(k_query_backward<CC>, dim3((unsigned)blocks), dim3(256), 0,
                                      (hipStream_t)stream, g, d_points, n_points, d_g_f, d_g_grad,
                                      C > 0 ? d_g_feat : nullptr, d_grad_vox));
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_eikonal(const sg_grid* grid, const float* d_vox, int32_t C, const float* d_points,
               int64_t n_points, float weight, float* d_loss, float* d_grad_vox,
               sg_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!supported_C(C)) return fail(SG_EINVAL, "unsupported feature count C");
  if (!std::isfinite(weight)) return fail(SG_EINVAL, "weight must be finite");
  if (n_points < 0) return fail(SG_EINVAL, "n_points must be >= 0");
  if (n_points == 0) return SG_OK;
  if (!d_vox || !d_points) return fail(SG_EINVAL, "a required pointer is NULL");
  const GridView g = view_of(grid);
  const int64_t blocks = (n_points + 255) / 256;
  if (blocks > INT_MAX) return fail(SG_ERANGE, "too many points for one launch");
  hipLaunchKernelGGL(k_eikonal, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, g,
                     d_vox, 1 + C, d_points, n_points, weight, d_loss, d_grad_vox);
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_render_footprint(const sg_grid* grid, const float* d_rays, int64_t n_rays,
                        const sg_render_params* params, int32_t* d_counts, uint8_t* d_touched,
                        sg_stream stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  Params p;
  if ((rc = check_params(params, p))) return rc;
  if (n_rays < 0) return fail(SG_EINVAL, "n_rays must be >= 0");
  if (n_rays == 0) return SG_OK;
  if (!d_rays || !d_counts) return fail(SG_EINVAL, "a required pointer is NULL");
  const GridView g = view_of(grid);
  const Launch l = plan(n_rays, sizeof(int2) * p.max_samples);
  hipLaunchKernelGGL(k_footprint, dim3(l.blocks), dim3(l.threads), l.lds, (hipStream_t)stream, g,
                     d_rays, n_rays, p, d_counts, d_touched);
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

}  // extern "C"
