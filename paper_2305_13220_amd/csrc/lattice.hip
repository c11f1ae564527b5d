// Permutohedral-lattice Gaussian filtering on a collision-free hash of
// lattice points, and the mean-field update of the continuous CRF
// (Sec. 3.5.3): the message passing of the mean-field equation is a
// high-dimensional Gaussian filter, evaluated by splatting onto the
// vertices of each point's enclosing simplex, blurring along the d+1
// lattice directions and slicing back.
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace sg {

constexpr int kLatMaxD = 24;
constexpr int kLatMaxV = 32;

// Enclosing simplex of one scaled position (float32, no fused multiply-add,
// in this order, so the integer vertices match any other evaluation of the
// same steps): the position is lifted onto the plane sum x = 0 of R^{d+1},
// rounded to the nearest remainder-0 lattice point through the ranks of the
// residuals, and the barycentric weights follow from the sorted residuals.
// Vertex r has coordinates rem0[i] + r (rank[i] <= d - r) or
// rem0[i] + r - (d+1) otherwise; only the first d are stored.  MAXD bounds d
// at compile time: every loop runs to it with a guard, so the arrays stay in
// registers (a loop to the run-time d puts them in scratch memory).
template <int MAXD>
struct Simplex {
  int32_t rem0[MAXD + 1], rank[MAXD + 1];
  float w[MAXD + 2];
};

template <int MAXD>
__device__ inline void lattice_simplex(const float* __restrict__ pos, int d, Simplex<MAXD>& s) {
#pragma clang fp contract(off)
  float el[MAXD + 1];
  float sm = 0.0f;
#pragma unroll
  for (int i = MAXD; i >= 1; --i) {
    if (i <= d) {
      const float scale = (float)(d + 1) * sqrtf(2.0f / 3.0f) / sqrtf((float)(i * (i + 1)));
      const float cf = pos[i - 1] * scale;
      el[i] = sm - (float)i * cf;
      sm += cf;
    } else {
      el[i] = 0.0f;
    }
  }
  el[0] = sm;
  int sum = 0;
  const float inv = 1.0f / (float)(d + 1);
#pragma unroll
  for (int i = 0; i <= MAXD; ++i) {
    s.rem0[i] = 0;
    s.rank[i] = 0;
    if (i <= d) {
      const float v = el[i] * inv;
      const float up = ceilf(v) * (float)(d + 1), dn = floorf(v) * (float)(d + 1);
      s.rem0[i] = (int32_t)((up - el[i] < el[i] - dn) ? up : dn);
      sum += s.rem0[i] / (d + 1);
    }
  }
#pragma unroll
  for (int i = 0; i < MAXD; ++i)
#pragma unroll
    for (int j = i + 1; j <= MAXD; ++j) {
      if (j <= d) {
        const float di = el[i] - (float)s.rem0[i], dj = el[j] - (float)s.rem0[j];
        if (di < dj) ++s.rank[i];
        else ++s.rank[j];
      }
    }
#pragma unroll
  for (int i = 0; i <= MAXD; ++i) {
    if (i > d) continue;
    if (sum > 0) {
      if (s.rank[i] >= d + 1 - sum) {
        s.rank[i] -= d + 1 - sum;
        s.rem0[i] -= d + 1;
      } else {
        s.rank[i] += sum;
      }
    } else if (sum < 0) {
      if (s.rank[i] < -sum) {
        s.rank[i] += d + 1 + sum;
        s.rem0[i] += d + 1;
      } else {
        s.rank[i] += sum;
      }
    }
  }
  // w[d - rank_i] += t_i and w[d + 1 - rank_i] -= t_i, i in order: slot by
  // slot, the same updates in the same order, picked by compares rather than
  // an index into a register array
  float t[MAXD + 1];
#pragma unroll
  for (int i = 0; i <= MAXD; ++i) t[i] = i <= d ? (el[i] - (float)s.rem0[i]) * inv : 0.0f;
  float wd1 = 0.0f;  // w[d + 1]
#pragma unroll
  for (int q = 0; q <= MAXD + 1; ++q) {
    float wq = 0.0f;
#pragma unroll
    for (int i = 0; i <= MAXD; ++i) {
      if (i > d) continue;
      if (s.rank[i] == d - q) wq += t[i];
      if (s.rank[i] == d + 1 - q) wq -= t[i];
    }
    s.w[q] = wq;
    if (q == d + 1) wd1 = wq;
  }
  s.w[0] += 1.0f + wd1;
}

template <int MAXD>
__device__ inline int32_t vertex_coord(const Simplex<MAXD>& s, int d, int r, int i) {
  return s.rank[i] <= d - r ? s.rem0[i] + r : s.rem0[i] + r - (d + 1);
}

// 64-bit fingerprint of a key (never the empty marker): a mixed linear form
// sum_i k_i P_i (mod 2^64) with fixed pseudo-random odd multipliers P_i.  The
// form is additive, so the neighbours of a vertex along the lattice
// directions (key + the same offset vector, up to sign) are fingerprinted
// from the vertex's form with one multiply-add each.  Two keys share a
// fingerprint only if their forms collide; the build checks every vertex
// against its full key, and every neighbour found is checked too.
__host__ __device__ constexpr uint64_t lat_coef_of(int i) {
  uint64_t z = 0x632be59bd9b4e019ull * (uint64_t)(i + 1) + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return (z ^ (z >> 31)) | 1ull;
}
#define SG_LC(i) lat_coef_of(i)
__constant__ uint64_t kLatCoef[kLatMaxD] = {
    SG_LC(0),  SG_LC(1),  SG_LC(2),  SG_LC(3),  SG_LC(4),  SG_LC(5),  SG_LC(6),  SG_LC(7),
    SG_LC(8),  SG_LC(9),  SG_LC(10), SG_LC(11), SG_LC(12), SG_LC(13), SG_LC(14), SG_LC(15),
    SG_LC(16), SG_LC(17), SG_LC(18), SG_LC(19), SG_LC(20), SG_LC(21), SG_LC(22), SG_LC(23)};
#undef SG_LC
static_assert(kLatMaxD == 24, "one multiplier per key coordinate");

// (MAXD bounds d at compile time, so a key held in registers is indexed by
// constants: a loop to the run-time d would put it in scratch memory.)
template <int MAXD>
__device__ inline uint64_t key_lin(const int32_t* k, int d) {
  uint64_t h = 0;
#pragma unroll
  for (int i = 0; i < MAXD; ++i)
    if (i < d) h += (uint64_t)(int64_t)k[i] * kLatCoef[i];
  return h;
}
__device__ inline uint64_t lin_fp(uint64_t lin) {
  const uint64_t h = mix64(lin ^ 0x9e3779b97f4a7c15ull);
  return h == kEmptyKey ? h - 1 : h;
}
template <int MAXD>
__device__ inline uint64_t key_fp(const int32_t* k, int d) { return lin_fp(key_lin<MAXD>(k, d)); }

struct LatView {
  uint64_t* fp;    // [cap] fingerprints (kEmptyKey: free)
  int32_t* keys;   // [cap][ks]: the d coordinates, then zeros to ks
  uint64_t mask;   // cap - 1
  int d;
  int ks;          // row stride: d rounded up to a multiple of 4 (16-byte rows)
};

__host__ __device__ constexpr int lat_key_stride(int d) { return (d + 3) / 4 * 4; }

// A key row read with 16-byte loads (MAXD is a multiple of 4 and at least
// ks); k[c] = 0 for c >= d.
template <int MAXD>
__device__ inline void load_key(const LatView& L, int64_t s, int32_t k[MAXD]) {
  static_assert(MAXD % 4 == 0, "whole 16-byte pieces");
  const int4* row = reinterpret_cast<const int4*>(L.keys + s * L.ks);
#pragma unroll
  for (int q = 0; q < MAXD / 4; ++q) {
    const int4 v = 4 * q < L.d ? row[q] : make_int4(0, 0, 0, 0);
    k[4 * q] = v.x;
    k[4 * q + 1] = v.y;
    k[4 * q + 2] = v.z;
    k[4 * q + 3] = v.w;
  }
}

// Slot of a key of fingerprint f: insert (the CAS winner writes the full
// key) or find.
template <int MAXD>
__device__ inline int64_t lat_slot_fp(const LatView& L, const int32_t* k, uint64_t f,
                                      bool insert) {
  uint64_t s = mix64(f) & L.mask;
  for (;;) {
    const uint64_t cur = insert ? (uint64_t)atomicCAS((unsigned long long*)&L.fp[s],
                                                      (unsigned long long)kEmptyKey,
                                                      (unsigned long long)f)
                                : L.fp[s];
    if (cur == kEmptyKey) {
      if (!insert) return -1;
      // k[c] = 0 for c >= d, so the row's padding is written as zeros
      int4* row = reinterpret_cast<int4*>(L.keys + s * L.ks);
#pragma unroll
      for (int q = 0; q < MAXD / 4; ++q)
        if (4 * q < L.d) row[q] = make_int4(k[4 * q], k[4 * q + 1], k[4 * q + 2], k[4 * q + 3]);
      return (int64_t)s;
    }
    if (cur == f) return (int64_t)s;
    s = (s + 1) & L.mask;
  }
}

template <int MAXD>
__device__ inline int64_t lat_slot(const LatView& L, const int32_t* k, bool insert) {
  return lat_slot_fp<MAXD>(L, k, key_fp<MAXD>(k, L.d), insert);
}

// Per point: simplex, insertion of its d+1 vertices (mode 0), or the check
// that every vertex's slot holds its full key (mode 1: a fingerprint
// collision raises the error flag).
template <int MAXD>
__global__ __launch_bounds__(256) void k_lat_simplex(const float* __restrict__ pos, int64_t N, LatView L, int mode,
                              int32_t* __restrict__ vid, float* __restrict__ bw,
                              int* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int d = L.d;
  // Positions must be finite and moderate (|p| < 2^20), so that the lifted
  // coordinates and the vertex keys stay within int32 and the ranks form a
  // permutation; otherwise the build fails (error bit 2).
  for (int c = 0; c < d; ++c)
    if (!(fabsf(pos[i * d + c]) < 1048576.0f)) {
      atomicOr(err, 2);
      return;
    }
  Simplex<MAXD> s;
  lattice_simplex<MAXD>(pos + i * d, d, s);
  int32_t k[MAXD];
#pragma unroll
  for (int r = 0; r <= MAXD; ++r) {
    if (r > d) continue;
#pragma unroll
    for (int c = 0; c < MAXD; ++c) k[c] = c < d ? vertex_coord(s, d, r, c) : 0;
    if (mode == 0) {
      const int64_t slot = lat_slot<MAXD>(L, k, true);
      vid[i * (d + 1) + r] = (int32_t)slot;
      bw[i * (d + 1) + r] = s.w[r];
    } else {
      const int64_t slot = vid[i * (d + 1) + r];
      int32_t held[MAXD];
      load_key<MAXD>(L, slot, held);
      bool same = true;
#pragma unroll
      for (int c = 0; c < MAXD; ++c) same = same && (c >= d || held[c] == k[c]);
      if (!same) atomicOr(err, 1);
    }
  }
}

// List of the occupied slots (in no particular order) and their number.
// Each 1024-lane workgroup takes kLatCompactPer slots per lane (lane l's
// i-th is slot base + l + 1024 i, so every pass is coalesced), counts them
// per wave and pass into LDS, and takes its range of the list with one
// counter atomic: the atomics on the one counter are serialised, so with
// one per 1024 slots the 16M-slot table of a d = 22 build spent most of the
// compaction on them.
constexpr int kLatCompactT = 1024, kLatCompactPer = 16;
__global__ __launch_bounds__(kLatCompactT) void k_lat_compact(const uint64_t* __restrict__ fp,
                                                              int64_t cap,
                                                              unsigned long long* __restrict__ n,
                                                              int32_t* __restrict__ list) {
  constexpr int NW = kLatCompactT / kWave;
  __shared__ unsigned long long off[kLatCompactPer][NW];
  __shared__ unsigned long long bbase;
  const int w = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * kLatCompactT * kLatCompactPer + threadIdx.x;
  uint32_t used = 0;
#pragma unroll
  for (int i = 0; i < kLatCompactPer; ++i) {
    const int64_t s = base + (int64_t)i * kLatCompactT;
    const bool u = s < cap && fp[s] != kEmptyKey;
    used |= (uint32_t)u << i;
    const uint64_t b = __ballot(u);
    if (lane_id() == 0) off[i][w] = (unsigned long long)__popcll(b);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long acc = 0;
    for (int i = 0; i < kLatCompactPer; ++i)
      for (int k = 0; k < NW; ++k) {
        const unsigned long long c = off[i][k];
        off[i][k] = acc;
        acc += c;
      }
    bbase = acc ? atomicAdd(n, acc) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kLatCompactPer; ++i) {
    const bool u = (used >> i) & 1u;
    const uint64_t b = __ballot(u);
    if (u) list[bbase + off[i][w] + rank_below(b)] = (int32_t)(base + (int64_t)i * kLatCompactT);
  }
}

// Zero the value rows of the nv vertices (contiguous: rows are indexed by
// vertex number), 16-byte stores where the count allows.
__global__ void k_lat_zero(int64_t n, float* __restrict__ v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) v[t] = 0.0f;
}
__global__ void k_lat_zero4(int64_t n4, float4* __restrict__ v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n4) v[t] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Vertex numbers: vertex k of the occupied-slot list is number k; num is a
// slot-indexed scratch array.  The per-point vertex ids and the blur
// neighbours are then held as numbers, so the value rows are compact
// (rows 0..nv-1) rather than spread over the table's slots.
__global__ void k_lat_number(const int32_t* __restrict__ list, int64_t nv,
                             int32_t* __restrict__ num) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nv) num[list[k]] = (int32_t)k;
}
__global__ void k_lat_renumber(int32_t* __restrict__ vid, int64_t n,
                               const int32_t* __restrict__ num) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) vid[t] = num[vid[t]];
}

// Lanes laid out (point-vertex pair, channel): the channels of one vertex
// are consecutive, so an atomic instruction touches a few vertex rows
// rather than 64 (device float atomics are performed past the L2, one
// request per 64-byte piece an instruction touches).
__global__ void k_lat_splat(const int32_t* __restrict__ vid, const float* __restrict__ bw,
                            int64_t N, int d, const float* __restrict__ val, int vd,
                            float* __restrict__ lv) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * (d + 1) * vd) return;
  const int64_t pr = t / vd;
  const int c = (int)(t - pr * vd);
  const int64_t i = pr / (d + 1);
  unsafeAtomicAdd(lv + (int64_t)vid[pr] * vd + c, bw[pr] * val[i * vd + c]);
}

// Blur neighbours of every occupied vertex, found once at build: for list
// entry k and direction j, the vertex numbers of key -+ ((1,...,1) - (d+1) e_j)
// (first d coordinates), -1 where absent; filters then blur through this
// table.
template <int MAXD>
__global__ void k_lat_neighbors(LatView L, const int32_t* __restrict__ list, int64_t nv,
                                const int32_t* __restrict__ num, int32_t* __restrict__ nbr) {
  // one lane per vertex, every direction: the key is read once, and the
  // plus-side neighbour's fingerprint is the vertex's linear form plus the
  // direction's offset form
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int d = L.d;
  if (k >= nv) return;
  const int64_t s = list[k];
  int32_t key[MAXD];
  load_key<MAXD>(L, s, key);
  uint64_t lin = 0, sum = 0;
#pragma unroll
  for (int c = 0; c < MAXD; ++c) {
    if (c < d) {
      lin += (uint64_t)(int64_t)key[c] * kLatCoef[c];
      sum += kLatCoef[c];
    }
  }
  // The relation is symmetric: when B is A's neighbour on the plus side
  // of direction j, A is B's on the minus side.  So each vertex probes the
  // plus side only and writes both entries (the table starts at -1; each
  // entry has one writer, the vertex one step below along j).
  for (int j = 0; j <= d; ++j) {
    // offset of direction j: +1 on every coordinate, -d on coordinate j
    const uint64_t off = sum - (j < d ? (uint64_t)(d + 1) * kLatCoef[j] : 0ull);
    const int64_t n = lat_slot_fp<MAXD>(L, nullptr, lin_fp(lin + off), false);
    if (n >= 0) {
      int32_t cand[MAXD];
      load_key<MAXD>(L, n, cand);
      bool same = true;
#pragma unroll
      for (int c = 0; c < MAXD; ++c) same = same && (c >= d || cand[c] == key[c] + (c == j ? -d : 1));
      if (same) {  // otherwise a fingerprint alias of an absent key: no neighbour
        const int32_t b = num[n];
        nbr[2 * ((int64_t)j * nv + k) + 1] = b;
        nbr[2 * ((int64_t)j * nv + b)] = (int32_t)k;
      }
    }
  }
}

// Blur along direction j through the neighbour table, lanes laid out
// (vertex, channel): new = v/2 + (v(n-) + v(n+))/4.
__global__ void k_lat_blur_tab(const int32_t* __restrict__ nbr, int64_t nv,
                               const float* __restrict__ src, int vd, float* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nv * vd) return;
  const int64_t k = t / vd;
  const int c = (int)(t - k * vd);
  const int32_t a = nbr[2 * k], b = nbr[2 * k + 1];
  float v = 0.5f * src[t];
  if (a >= 0) v += 0.25f * src[(int64_t)a * vd + c];
  if (b >= 0) v += 0.25f * src[(int64_t)b * vd + c];
  dst[t] = v;
}

// The same with lanes laid out (vertex, four channels) where a row is a
// whole number of 16-byte pieces (vd a multiple of 4): a quarter of the
// memory instructions for the same per-channel arithmetic.
__global__ void k_lat_blur_tab4(const int32_t* __restrict__ nbr, int64_t nv,
                                const float* __restrict__ src, int vd, float* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int vq = vd / 4;
  if (t >= nv * vq) return;
  const int64_t k = t / vq;
  const int c = (int)(t - k * vq);
  const int2 ab = reinterpret_cast<const int2*>(nbr)[k];
  const float4* s4 = reinterpret_cast<const float4*>(src);
  const float4 o = s4[t];
  const float4 na = ab.x >= 0 ? s4[(int64_t)ab.x * vq + c] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const float4 nb = ab.y >= 0 ? s4[(int64_t)ab.y * vq + c] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  float v[4] = {0.5f * o.x, 0.5f * o.y, 0.5f * o.z, 0.5f * o.w};
  const float va[4] = {na.x, na.y, na.z, na.w}, vb[4] = {nb.x, nb.y, nb.z, nb.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (ab.x >= 0) v[e] += 0.25f * va[e];
    if (ab.y >= 0) v[e] += 0.25f * vb[e];
  }
  reinterpret_cast<float4*>(dst)[t] = make_float4(v[0], v[1], v[2], v[3]);
}

// Lanes laid out (point, channel): consecutive lanes read one vertex row.
__global__ void k_lat_slice(const int32_t* __restrict__ vid, const float* __restrict__ bw,
                            int64_t N, int d, const float* __restrict__ lv, int vd,
                            float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * vd) return;
  const int64_t i = t / vd;
  const int c = (int)(t - i * vd);
  float acc = 0.0f;
  for (int r = 0; r <= d; ++r) {
    const int64_t pr = i * (d + 1) + r;
    acc += bw[pr] * lv[(int64_t)vid[pr] * vd + c];
  }
  out[t] = acc;
}

// The same with lanes laid out (point, four channels) where a row is a
// whole number of 16-byte pieces; each channel sums the vertices in the
// same order.
__global__ void k_lat_slice4(const int32_t* __restrict__ vid, const float* __restrict__ bw,
                             int64_t N, int d, const float* __restrict__ lv, int vd,
                             float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int vq = vd / 4;
  if (t >= N * vq) return;
  const int64_t i = t / vq;
  const int c = (int)(t - i * vq);
  const float4* l4 = reinterpret_cast<const float4*>(lv);
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int r = 0; r <= d; ++r) {
    const int64_t pr = i * (d + 1) + r;
    const float w = bw[pr];
    const float4 x = l4[(int64_t)vid[pr] * vq + c];
    acc[0] += w * x.x;
    acc[1] += w * x.y;
    acc[2] += w * x.z;
    acc[3] += w * x.w;
  }
  reinterpret_cast<float4*>(out)[t] = make_float4(acc[0], acc[1], acc[2], acc[3]);
}

// Q = softmax(-unary + w_p * m) per point (m may be null: w_p ignored).
__global__ void k_softmax(const float* __restrict__ unary, const float* __restrict__ m, float w_p,
                          int64_t N, int Lb, float* __restrict__ Q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  float a[kLatMaxV];
  float mx = -INFINITY;
#pragma unroll
  for (int l = 0; l < kLatMaxV; ++l) {
    a[l] = l < Lb ? -unary[i * Lb + l] + (m ? w_p * m[i * Lb + l] : 0.0f) : -INFINITY;
    mx = fmaxf(mx, a[l]);
  }
  float s = 0.0f;
#pragma unroll
  for (int l = 0; l < kLatMaxV; ++l) {
    a[l] = l < Lb ? expf(a[l] - mx) : 0.0f;
    s += a[l];
  }
  const float inv = 1.0f / s;
#pragma unroll
  for (int l = 0; l < kLatMaxV; ++l)
    if (l < Lb) Q[i * Lb + l] = a[l] * inv;
}

// Mean-field update with a label compatibility matrix mu [Lb,Lb] (row l:
// mu(l, .)): Q(l) = softmax_l(-unary(l) - sum_k mu(l,k) m(k)).  The matrix
// indices are uniform across the wave, so mu is read through scalar loads;
// the loops are unrolled to the label limit so that the message row stays in
// registers.
__global__ void k_softmax_compat(const float* __restrict__ unary, const float* __restrict__ m,
                                 const float* __restrict__ mu, int64_t N, int Lb,
                                 float* __restrict__ Q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  float mm[kLatMaxV], a[kLatMaxV];
#pragma unroll
  for (int k = 0; k < kLatMaxV; ++k) mm[k] = k < Lb ? m[i * Lb + k] : 0.0f;
  float mx = -INFINITY;
#pragma unroll
  for (int l = 0; l < kLatMaxV; ++l) {
    float e = -INFINITY;
    if (l < Lb) {
      e = -unary[i * Lb + l];
#pragma unroll
      for (int k = 0; k < kLatMaxV; ++k)
        if (k < Lb) e -= mu[l * Lb + k] * mm[k];
    }
    a[l] = e;
    mx = fmaxf(mx, e);
  }
  float s = 0.0f;
#pragma unroll
  for (int l = 0; l < kLatMaxV; ++l) {
    a[l] = l < Lb ? expf(a[l] - mx) : 0.0f;
    s += a[l];
  }
  const float inv = 1.0f / s;
#pragma unroll
  for (int l = 0; l < kLatMaxV; ++l)
    if (l < Lb) Q[i * Lb + l] = a[l] * inv;
}

// Reverse step of the compatibility mean field, one lane per point, kMfT
// points per workgroup.  With Q = softmax(a), a = -unary - m mu^T:
//   ga = Q * (gQ - <Q, gQ>),  g_unary -= ga,
//   gm(k) = -sum_l ga(l) mu(l,k)               (HAS_M),
//   partial[block](l,k) = -sum_{points} ga(l) m(k)   (HAS_M),
// the last an outer-product sum over the workgroup's points staged in LDS
// (padded lanes contribute zeros), reduced later in a fixed order.
constexpr int kMfT = 128;
template <bool HAS_M>
__global__ __launch_bounds__(kMfT) void k_mf_bwd(const float* __restrict__ Q,
                                                 const float* __restrict__ gq,
                                                 const float* __restrict__ m,
                                                 const float* __restrict__ mu, int64_t N, int Lb,
                                                 float* __restrict__ g_unary,
                                                 float* __restrict__ gm,
                                                 float* __restrict__ partial) {
  __shared__ float s_ga[HAS_M ? kMfT * kLatMaxV : 1];
  __shared__ float s_m[HAS_M ? kMfT * kLatMaxV : 1];
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kMfT + tid;
  const bool ok = i < N;
  float q[kLatMaxV], ga[kLatMaxV];
  float dot = 0.0f;
#pragma unroll
  for (int l = 0; l < kLatMaxV; ++l) {
    const bool in = ok && l < Lb;
    q[l] = in ? Q[i * Lb + l] : 0.0f;
    ga[l] = in ? gq[i * Lb + l] : 0.0f;
    dot += q[l] * ga[l];
  }
#pragma unroll
  for (int l = 0; l < kLatMaxV; ++l) {
    ga[l] = q[l] * (ga[l] - dot);
    if (ok && l < Lb) g_unary[i * Lb + l] -= ga[l];
  }
  if constexpr (HAS_M) {
#pragma unroll
    for (int k = 0; k < kLatMaxV; ++k) {
      if (k < Lb) {
        float acc = 0.0f;
#pragma unroll
        for (int l = 0; l < kLatMaxV; ++l)
          if (l < Lb) acc -= ga[l] * mu[l * Lb + k];
        if (ok) gm[i * Lb + k] = acc;
        s_ga[tid * Lb + k] = ga[k];
        s_m[tid * Lb + k] = ok ? m[i * Lb + k] : 0.0f;
      }
    }
    __syncthreads();
    const int LL = Lb * Lb;
    for (int e = tid; e < LL; e += kMfT) {
      const int l = e / Lb, k = e - l * Lb;
      float acc = 0.0f;
      for (int p = 0; p < kMfT; ++p) acc += s_ga[p * Lb + l] * s_m[p * Lb + k];
      partial[(int64_t)blockIdx.x * LL + e] = -acc;
    }
  }
}

// g_compat[e] += sum over workgroups b of partial[b][e]: one workgroup per
// entry e, each lane summing a fixed stride of the partials, then a fixed
// LDS tree, so the result does not depend on timing.
constexpr int kMfRed = 256;
__global__ __launch_bounds__(kMfRed) void k_mf_reduce(const float* __restrict__ partial,
                                                      int64_t nblk, int LL,
                                                      float* __restrict__ g_compat) {
  __shared__ float red[kMfRed];
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  float acc = 0.0f;
  for (int64_t b = tid; b < nblk; b += kMfRed) acc += partial[b * LL + e];
  red[tid] = acc;
  __syncthreads();
  for (int w = kMfRed / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) g_compat[e] += red[0];
}

__global__ void k_fill_zero(float* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// Workspace of the mean-field backward: the marginals and the messages of
// every update, the running gradient of the marginals and of the messages,
// and the per-workgroup partial sums of the compatibility gradient.
struct MfWs {
  size_t qs, ms, gq, gm, part, total;
};
static MfWs mf_ws(int64_t n, int Lb, int T) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t nl = (size_t)n * Lb * sizeof(float);
  MfWs w;
  w.qs = 0;
  w.ms = al((size_t)(T + 1) * nl);
  w.gq = w.ms + al((size_t)T * nl);
  w.gm = w.gq + al(nl);
  w.part = w.gm + al(nl);
  w.total = w.part + al((size_t)((n + kMfT - 1) / kMfT) * Lb * Lb * sizeof(float));
  return w;
}

// Label loss of the CRF per node: x = softmax(logits), loss = weight *
// KL(x || Q), gradient weight * x_k (a_k - KL) with a = log x - log Q
// (Q a fixed target).  Row strides ld_s / ld_g (elements) let the logits
// be a column range of a feature array and the gradient be written into
// the matching columns of an upstream-gradient array.
__global__ void k_crf_label_loss(const float* __restrict__ logits, int64_t ld_s,
                                 const float* __restrict__ Q, int64_t N, int Lb, float weight,
                                 float* __restrict__ loss, float* __restrict__ g, int64_t ld_g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  float lx[kLatMaxV];
  float mx = -INFINITY;
#pragma unroll
  for (int l = 0; l < kLatMaxV; ++l) {
    lx[l] = l < Lb ? logits[i * ld_s + l] : -INFINITY;
    mx = fmaxf(mx, lx[l]);
  }
  float z = 0.0f;
#pragma unroll
  for (int l = 0; l < kLatMaxV; ++l) z += l < Lb ? expf(lx[l] - mx) : 0.0f;
  const float lz = logf(z);
  float kl = 0.0f;
#pragma unroll
  for (int l = 0; l < kLatMaxV; ++l) {
    if (l < Lb) {
      lx[l] = lx[l] - mx - lz;                       // log x_l
      const float a = lx[l] - logf(Q[i * Lb + l]);   // log x_l - log Q_l
      kl += expf(lx[l]) * a;
    }
  }
  if (loss) loss[i] = weight * kl;
  if (g) {
#pragma unroll
    for (int l = 0; l < kLatMaxV; ++l)
      if (l < Lb) g[i * ld_g + l] = weight * expf(lx[l]) * ((lx[l] - logf(Q[i * Lb + l])) - kl);
  }
}

// Colour / normal loss per node: Q = F(x) / F(1) from the filter of [x, 1]
// (a fixed target), loss = weight |x - Q|^2, gradient 2 weight (x - Q).
__global__ void k_crf_property_loss(const float* __restrict__ x, int64_t ld_x,
                                    const float* __restrict__ filt, int64_t N, int P, float weight,
                                    float* __restrict__ loss, float* __restrict__ g, int64_t ld_g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const float inv = 1.0f / filt[i * (P + 1) + P];
  float l = 0.0f;
  for (int k = 0; k < P; ++k) {
    const float d = x[i * ld_x + k] - filt[i * (P + 1) + k] * inv;
    l += d * d;
    if (g) g[i * ld_g + k] = 2.0f * weight * d;
  }
  if (loss) loss[i] = weight * l;
}

static unsigned grid_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace sg

struct sg_lattice {
  uint32_t magic;
  int device;  // the device current at build, which holds the arrays below
  int d, vmax;
  int64_t N, cap, n_vertices;
  uint64_t* fp;
  int32_t* keys;
  int32_t* list;  // [cap] occupied slots, n_vertices of them (vertex k at list[k])
  int32_t* vid;   // [N][d+1] vertex numbers of each point's simplex
  float* bw;
  float* v0;  // [n_vertices, vd] value rows by vertex number (allocated for cap rows)
  float* v1;
  float* m;  // [N, vmax] message buffer of the mean-field update
  int32_t* nbr;  // [d+1][n_vertices][2] blur neighbours' vertex numbers (-1: absent)
};

namespace sg {
constexpr uint32_t kLatMagic = 0x4c415454u;  // "LATT"
static int check_lat(const sg_lattice* L) {
  if (!L) return fail(SG_EINVAL, "lattice is NULL");
  if (L->magic != kLatMagic) return fail(SG_ESTATE, "lattice handle is not a live lattice");
  return SG_OK;
}
static void free_lat(sg_lattice* L) {
  (void)hipFree(L->fp);
  (void)hipFree(L->keys);
  (void)hipFree(L->list);
  (void)hipFree(L->vid);
  (void)hipFree(L->bw);
  (void)hipFree(L->v0);
  (void)hipFree(L->v1);
  (void)hipFree(L->m);
  (void)hipFree(L->nbr);
  delete L;
}
// reverse: blur directions in the order d..0, which makes the filter its
// own transpose (slice is the transpose of splat, each B_j is symmetric).
static int lat_filter(const sg_lattice* L, const float* d_val, int vd, float* d_out, hipStream_t s,
                      bool reverse = false) {
  const int T = 256;
  const int d = L->d;
  const LatView V = {L->fp, L->keys, (uint64_t)L->cap - 1, d, lat_key_stride(d)};
  const int64_t nv = L->n_vertices;
  if ((nv * vd) % 4 == 0)
    k_lat_zero4<<<grid_of(nv * vd / 4, T), T, 0, s>>>(nv * vd / 4, reinterpret_cast<float4*>(L->v0));
  else
    k_lat_zero<<<grid_of(nv * vd, T), T, 0, s>>>(nv * vd, L->v0);
  k_lat_splat<<<grid_of(L->N * (d + 1) * vd, T), T, 0, s>>>(L->vid, L->bw, L->N, d, d_val, vd,
                                                              L->v0);
  float* a = L->v0;
  float* b = L->v1;
  for (int jj = 0; jj <= d; ++jj) {
    const int j = reverse ? d - jj : jj;
    if (vd % 4 == 0)
      k_lat_blur_tab4<<<grid_of(nv * (vd / 4), T), T, 0, s>>>(L->nbr + (int64_t)j * nv * 2, nv, a,
                                                               vd, b);
    else
      k_lat_blur_tab<<<grid_of(nv * vd, T), T, 0, s>>>(L->nbr + (int64_t)j * nv * 2, nv, a, vd, b);
    float* t = a;
    a = b;
    b = t;
  }
  if (vd % 4 == 0 && reinterpret_cast<uintptr_t>(d_out) % 16 == 0)
    k_lat_slice4<<<grid_of(L->N * (vd / 4), T), T, 0, s>>>(L->vid, L->bw, L->N, d, a, vd, d_out);
  else
    k_lat_slice<<<grid_of(L->N * vd, T), T, 0, s>>>(L->vid, L->bw, L->N, d, a, vd, d_out);
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}
// Table capacity (a power of two, at least twice the n (d+1) vertex keys)
// and the byte sizes of the build's eight device arrays: fingerprints,
// keys, per-point vertex ids and weights, two value buffers, the slice
// output, the occupied-slot list.  The caller has checked
// n (d+1) < 2^30, so every size fits 64 bits.
static int64_t lat_sizes(int64_t n_points, int d, int max_values, size_t sz[8]) {
  int64_t cap = 1;
  while (cap < 2 * n_points * (d + 1)) cap <<= 1;
  sz[0] = sizeof(uint64_t) * cap;
  sz[1] = sizeof(int32_t) * cap * lat_key_stride(d);
  sz[2] = sizeof(int32_t) * n_points * (d + 1);
  sz[3] = sizeof(float) * n_points * (d + 1);
  sz[4] = sizeof(float) * cap * max_values;
  sz[5] = sizeof(float) * cap * max_values;
  sz[6] = sizeof(float) * n_points * max_values;
  sz[7] = sizeof(int32_t) * cap;
  return cap;
}

static bool lat_args_ok(int64_t n_points, int32_t d, int32_t max_values) {
  return d >= 1 && d <= kLatMaxD && max_values >= 1 && max_values <= kLatMaxV && n_points >= 1 &&
         n_points <= (int64_t)INT_MAX && n_points * (d + 1) <= (int64_t)INT_MAX / 2;
}


// The mean-field backward's checks shared by its two entry points (the
// caller-workspace one and the allocation-free one).
static bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char *pa = (const char*)a, *pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

static int mf_backward_check(const sg_lattice* L, const float* d_unary, int32_t n_labels,
                             const float* d_compat, int32_t iters, const float* d_gQ,
                             const float* d_g_unary, const float* d_g_compat) {
  int rc = check_lat(L);
  if (rc) return rc;
  if (n_labels < 1 || n_labels > L->vmax)
    return fail(SG_EINVAL, "n_labels must be in [1, max_values of the build]");
  if (iters < 0) return fail(SG_EINVAL, "iters must be >= 0");
  if (!d_unary || !d_compat || !d_gQ || !d_g_unary || !d_g_compat)
    return fail(SG_EINVAL, "a required pointer is NULL");
  const size_t nlb = (size_t)L->N * n_labels * sizeof(float);
  if (ranges_overlap(d_g_unary, nlb, d_gQ, nlb))
    return fail(SG_EINVAL, "d_g_unary must not overlap d_gQ");
  return SG_OK;
}

// Reverse mode through `iters` compatibility mean-field updates with the
// workspace at `base` (layout of mf_ws; every part is written before it is
// read, so nothing in it needs to start at zero).
static int mf_backward_run(const sg_lattice* L, const float* d_unary, int32_t n_labels,
                           const float* d_compat, int32_t iters, const float* d_gQ,
                           float* d_g_unary, float* d_g_compat, char* base, hipStream_t s) {
  const int64_t N = L->N;
  const MfWs w = mf_ws(N, n_labels, iters);
  float* Qs = (float*)(base + w.qs);
  float* ms = (float*)(base + w.ms);
  float* gq = (float*)(base + w.gq);
  float* gm = (float*)(base + w.gm);
  float* part = (float*)(base + w.part);
  const int64_t nl = N * n_labels;
  const int T = 256;
  int rc = SG_OK;
  // forward, keeping the marginals and the messages of every update
  k_softmax<<<grid_of(N, T), T, 0, s>>>(d_unary, nullptr, 0.0f, N, n_labels, Qs);
  for (int it = 1; it <= iters; ++it) {
    float* m = ms + (it - 1) * nl;
    if ((rc = lat_filter(L, Qs + (it - 1) * nl, n_labels, m, s))) return rc;
    k_softmax_compat<<<grid_of(N, T), T, 0, s>>>(d_unary, m, d_compat, N, n_labels, Qs + it * nl);
  }
  k_fill_zero<<<grid_of(nl, T), T, 0, s>>>(d_g_unary, nl);
  const int LL = n_labels * n_labels;
  k_fill_zero<<<grid_of(LL, T), T, 0, s>>>(d_g_compat, LL);
  const int64_t nblk = (N + kMfT - 1) / kMfT;
  const float* gin = d_gQ;
  for (int it = iters; it >= 1; --it) {
    k_mf_bwd<true><<<nblk, kMfT, 0, s>>>(Qs + it * nl, gin, ms + (it - 1) * nl, d_compat, N,
                                         n_labels, d_g_unary, gm, part);
    k_mf_reduce<<<LL, kMfRed, 0, s>>>(part, nblk, LL, d_g_compat);
    if ((rc = lat_filter(L, gm, n_labels, gq, s, true))) return rc;
    gin = gq;
  }
  k_mf_bwd<false><<<nblk, kMfT, 0, s>>>(Qs, gin, nullptr, d_compat, N, n_labels, d_g_unary,
                                        nullptr, nullptr);
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

// Fixed workspace of the allocation-free mean-field backward: one array in
// each device's copy of the code object, held until the process ends.  In
// host code `scratch` names a host-side stand-in, not device memory: kernels
// and copies take the address hipGetSymbolAddress returns for the current
// device, looked up once per device and kept in mf_scratch_ptr.
constexpr size_t kMfScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kMfScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex mf_scratch_mu;
static char* mf_scratch_ptr[kMaxDevices];

static int mf_scratch(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SG_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(mf_scratch_mu);
  if (!mf_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(SG_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    mf_scratch_ptr[dev] = (char*)p;
  }
  *out = mf_scratch_ptr[dev];
  return SG_OK;
}
}  // namespace sg

using namespace sg;

extern "C" {

size_t sg_lattice_bytes(int64_t n_points, int32_t d, int32_t max_values) {
  if (!lat_args_ok(n_points, d, max_values)) return 0;
  size_t sz[8];
  lat_sizes(n_points, d, max_values, sz);
  size_t total = 0;
  for (int k = 0; k < 8; ++k) total += sz[k];
  // blur neighbour table: 2 (d+1) slots per vertex, at most n (d+1) vertices
  return total + sizeof(int32_t) * 2 * (size_t)(d + 1) * (size_t)n_points * (size_t)(d + 1);
}

int sg_lattice_build(const float* d_pos, int64_t n_points, int32_t d, int32_t max_values,
                     sg_stream stream, sg_lattice** out) {
  if (!out) return fail(SG_EINVAL, "out is NULL");
  *out = nullptr;
  if (d < 1 || d > kLatMaxD) return fail(SG_EINVAL, "d must be in [1, 24]");
  if (max_values < 1 || max_values > kLatMaxV) return fail(SG_EINVAL, "max_values must be in [1, 32]");
  if (!lat_args_ok(n_points, d, max_values))
    return fail(SG_EINVAL, "n_points must be >= 1 and n_points * (d+1) < 2^30");
  if (!d_pos) return fail(SG_EINVAL, "d_pos is NULL");
  hipStream_t s = (hipStream_t)stream;
  int dev = -1;
  SG_HIP_CHECK(hipGetDevice(&dev));
  sg_lattice* L = new sg_lattice();
  memset(L, 0, sizeof(*L));
  L->device = dev;
  L->d = d;
  L->vmax = max_values;
  L->N = n_points;
  size_t sz[8];
  L->cap = lat_sizes(n_points, d, max_values, sz);
  void** ptrs[8] = {(void**)&L->fp, (void**)&L->keys, (void**)&L->vid, (void**)&L->bw,
                    (void**)&L->v0, (void**)&L->v1, (void**)&L->m, (void**)&L->list};
  for (int k = 0; k < 8; ++k)
    if (hipMalloc(ptrs[k], sz[k]) != hipSuccess) {
      (void)hipGetLastError();
      free_lat(L);
      return fail(SG_ENOMEM, "device allocation for the lattice failed");
    }
  int* d_err = nullptr;
  int64_t* d_n = nullptr;
  if (hipMalloc((void**)&d_err, sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&d_n, sizeof(int64_t)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(d_err);
    free_lat(L);
    return fail(SG_ENOMEM, "device allocation for the lattice failed");
  }
  const int T = 256;
  const LatView V = {L->fp, L->keys, (uint64_t)L->cap - 1, d, lat_key_stride(d)};
  int rc = SG_OK;
  int err = 0;
  int64_t nv = 0;
  if (hipMemsetAsync(L->fp, 0xff, sz[0], s) != hipSuccess ||
      hipMemsetAsync(d_err, 0, sizeof(int), s) != hipSuccess ||
      hipMemsetAsync(d_n, 0, sizeof(int64_t), s) != hipSuccess) {
    rc = fail(SG_EHIP, "hipMemsetAsync failed");
  } else {
    for (int mode = 0; mode < 2; ++mode) {
      if (d <= 8)
        k_lat_simplex<8><<<grid_of(n_points, T), T, 0, s>>>(d_pos, n_points, V, mode, L->vid, L->bw, d_err);
      else if (d <= 16)
        k_lat_simplex<16><<<grid_of(n_points, T), T, 0, s>>>(d_pos, n_points, V, mode, L->vid, L->bw, d_err);
      else
        k_lat_simplex<kLatMaxD><<<grid_of(n_points, T), T, 0, s>>>(d_pos, n_points, V, mode, L->vid, L->bw, d_err);
    }
    k_lat_compact<<<grid_of(L->cap, kLatCompactT * kLatCompactPer), kLatCompactT, 0, s>>>(
        L->fp, L->cap, (unsigned long long*)d_n, L->list);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&err, d_err, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&nv, d_n, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(e, "lattice build");
    else if (err & 2) rc = fail(SG_EINVAL, "a position is not finite or |p| >= 2^20");
    else if (err) rc = fail(SG_ERANGE, "lattice key fingerprint collision");
  }
  (void)hipFree(d_err);
  (void)hipFree(d_n);
  if (rc) {
    free_lat(L);
    return rc;
  }
  L->n_vertices = nv;
  {
    const size_t nb_bytes = sizeof(int32_t) * 2 * (size_t)(d + 1) * (size_t)(nv > 0 ? nv : 1);
    if (hipMalloc((void**)&L->nbr, nb_bytes) != hipSuccess) {
      (void)hipGetLastError();
      free_lat(L);
      return fail(SG_ENOMEM, "device allocation for the lattice failed");
    }
    if (nv > 0) {
      // slot -> vertex number in the second value buffer (cap >= nv int32 of
      // room; filters overwrite it later), then the point-vertex ids and the
      // neighbour table as numbers
      int32_t* num = reinterpret_cast<int32_t*>(L->v1);
      k_lat_number<<<grid_of(nv, T), T, 0, s>>>(L->list, nv, num);
      if (hipMemsetAsync(L->nbr, 0xff, nb_bytes, s) != hipSuccess) {  // every entry -1
        (void)hipGetLastError();
        free_lat(L);
        return fail(SG_EHIP, "hipMemsetAsync failed");
      }
      k_lat_renumber<<<grid_of(L->N * (d + 1), T), T, 0, s>>>(L->vid, L->N * (d + 1), num);
      if (d <= 8)
        k_lat_neighbors<8><<<grid_of(nv, T), T, 0, s>>>(V, L->list, nv, num, L->nbr);
      else if (d <= 16)
        k_lat_neighbors<16><<<grid_of(nv, T), T, 0, s>>>(V, L->list, nv, num, L->nbr);
      else
        k_lat_neighbors<kLatMaxD><<<grid_of(nv, T), T, 0, s>>>(V, L->list, nv, num, L->nbr);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        free_lat(L);
        return hip_fail(e, "lattice neighbours");
      }
    }
  }
  L->magic = kLatMagic;
  *out = L;
  return SG_OK;
}

int sg_lattice_num_vertices(const sg_lattice* L, int64_t* n) {
  int rc = check_lat(L);
  if (rc) return rc;
  if (!n) return fail(SG_EINVAL, "n is NULL");
  *n = L->n_vertices;
  return SG_OK;
}

int sg_lattice_filter(const sg_lattice* L, const float* d_val, int32_t n_values, float* d_out,
                      sg_stream stream) {
  int rc = check_lat(L);
  if (rc) return rc;
  if (n_values < 1 || n_values > L->vmax)
    return fail(SG_EINVAL, "n_values must be in [1, max_values of the build]");
  if (!d_val || !d_out) return fail(SG_EINVAL, "a required pointer is NULL");
  return lat_filter(L, d_val, n_values, d_out, (hipStream_t)stream);
}

int sg_crf_meanfield(const sg_lattice* L, const float* d_unary, int32_t n_labels, float w_p,
                     int32_t iters, float* d_Q, sg_stream stream) {
  int rc = check_lat(L);
  if (rc) return rc;
  if (n_labels < 1 || n_labels > L->vmax)
    return fail(SG_EINVAL, "n_labels must be in [1, max_values of the build]");
  if (iters < 0) return fail(SG_EINVAL, "iters must be >= 0");
  if (!std::isfinite(w_p)) return fail(SG_EINVAL, "w_p must be finite");
  if (!d_unary || !d_Q) return fail(SG_EINVAL, "a required pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  const int T = 256;
  k_softmax<<<grid_of(L->N, T), T, 0, s>>>(d_unary, nullptr, 0.0f, L->N, n_labels, d_Q);
  for (int it = 0; it < iters; ++it) {
    if ((rc = lat_filter(L, d_Q, n_labels, L->m, s))) return rc;
    k_softmax<<<grid_of(L->N, T), T, 0, s>>>(d_unary, L->m, w_p, L->N, n_labels, d_Q);
  }
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_crf_meanfield_compat(const sg_lattice* L, const float* d_unary, int32_t n_labels,
                            const float* d_compat, int32_t iters, float* d_Q, sg_stream stream) {
  int rc = check_lat(L);
  if (rc) return rc;
  if (n_labels < 1 || n_labels > L->vmax)
    return fail(SG_EINVAL, "n_labels must be in [1, max_values of the build]");
  if (iters < 0) return fail(SG_EINVAL, "iters must be >= 0");
  if (!d_unary || !d_Q || !d_compat) return fail(SG_EINVAL, "a required pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  const int T = 256;
  k_softmax<<<grid_of(L->N, T), T, 0, s>>>(d_unary, nullptr, 0.0f, L->N, n_labels, d_Q);
  for (int it = 0; it < iters; ++it) {
    if ((rc = lat_filter(L, d_Q, n_labels, L->m, s))) return rc;
    k_softmax_compat<<<grid_of(L->N, T), T, 0, s>>>(d_unary, L->m, d_compat, L->N, n_labels, d_Q);
  }
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

size_t sg_crf_meanfield_compat_backward_ws_bytes(int64_t n_points, int32_t n_labels,
                                                int32_t iters) {
  if (n_points < 1 || n_labels < 1 || n_labels > kLatMaxV || iters < 0) return 0;
  return mf_ws(n_points, n_labels, iters).total;
}

int sg_crf_meanfield_compat_backward(const sg_lattice* L, const float* d_unary, int32_t n_labels,
                                     const float* d_compat, int32_t iters, const float* d_gQ,
                                     float* d_g_unary, float* d_g_compat, void* d_ws,
                                     size_t ws_bytes, sg_stream stream) {
  int rc = mf_backward_check(L, d_unary, n_labels, d_compat, iters, d_gQ, d_g_unary, d_g_compat);
  if (rc) return rc;
  if (!d_ws) return fail(SG_EINVAL, "a required pointer is NULL");
  const MfWs w = mf_ws(L->N, n_labels, iters);
  if (ws_bytes < w.total) return fail(SG_EINVAL, "workspace smaller than the size query returns");
  if (ranges_overlap(d_ws, w.total, d_gQ, (size_t)L->N * n_labels * sizeof(float)))
    return fail(SG_EINVAL, "d_g_unary and d_ws must not overlap d_gQ");
  return mf_backward_run(L, d_unary, n_labels, d_compat, iters, d_gQ, d_g_unary, d_g_compat,
                         (char*)d_ws, (hipStream_t)stream);
}

size_t sg_crf_meanfield_compat_backward_noalloc_max_bytes(void) { return kMfScratchBytes; }

int sg_crf_meanfield_compat_backward_noalloc(const sg_lattice* L, const float* d_unary,
                                             int32_t n_labels, const float* d_compat,
                                             int32_t iters, const float* d_gQ, float* d_g_unary,
                                             float* d_g_compat, sg_stream stream) {
  int rc = mf_backward_check(L, d_unary, n_labels, d_compat, iters, d_gQ, d_g_unary, d_g_compat);
  if (rc) return rc;
  const MfWs w = mf_ws(L->N, n_labels, iters);
  if (w.total > kMfScratchBytes)
    return fail(SG_EINVAL, "n_points * n_labels * (2 iters + 3) floats plus the partial sums "
                           "exceed the library's fixed scratch of " +
                               std::to_string(kMfScratchBytes) + " bytes (" +
                               std::to_string(w.total) + " needed); use "
                               "sg_crf_meanfield_compat_backward with a caller workspace");
  int dev = -1;
  SG_HIP_CHECK(hipGetDevice(&dev));
  if (dev != L->device)
    return fail(SG_EINVAL, "the lattice's device must be the current device");
  char* base = nullptr;
  if ((rc = mf_scratch(dev, &base))) return rc;
  return mf_backward_run(L, d_unary, n_labels, d_compat, iters, d_gQ, d_g_unary, d_g_compat,
                         base, (hipStream_t)stream);
}

int sg_crf_label_loss(const float* d_logits, int64_t ld_logits, const float* d_Q, int64_t n,
                      int32_t n_labels, float weight, float* d_loss, float* d_g, int64_t ld_g,
                      sg_stream stream) {
  if (n < 0) return fail(SG_EINVAL, "n must be >= 0");
  if (n_labels < 1 || n_labels > kLatMaxV) return fail(SG_EINVAL, "n_labels must be in [1, 32]");
  if (ld_logits < n_labels || (d_g && ld_g < n_labels))
    return fail(SG_EINVAL, "row strides must be >= n_labels");
  if (!std::isfinite(weight)) return fail(SG_EINVAL, "weight must be finite");
  if (n == 0) return SG_OK;
  if (!d_logits || !d_Q) return fail(SG_EINVAL, "a required pointer is NULL");
  k_crf_label_loss<<<grid_of(n, 256), 256, 0, (hipStream_t)stream>>>(
      d_logits, ld_logits, d_Q, n, n_labels, weight, d_loss, d_g, ld_g);
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_crf_property_loss(const float* d_x, int64_t ld_x, const float* d_filtered, int64_t n,
                         int32_t n_props, float weight, float* d_loss, float* d_g, int64_t ld_g,
                         sg_stream stream) {
  if (n < 0) return fail(SG_EINVAL, "n must be >= 0");
  if (n_props < 1 || n_props >= kLatMaxV) return fail(SG_EINVAL, "n_props must be in [1, 31]");
  if (ld_x < n_props || (d_g && ld_g < n_props))
    return fail(SG_EINVAL, "row strides must be >= n_props");
  if (!std::isfinite(weight)) return fail(SG_EINVAL, "weight must be finite");
  if (n == 0) return SG_OK;
  if (!d_x || !d_filtered) return fail(SG_EINVAL, "a required pointer is NULL");
  k_crf_property_loss<<<grid_of(n, 256), 256, 0, (hipStream_t)stream>>>(
      d_x, ld_x, d_filtered, n, n_props, weight, d_loss, d_g, ld_g);
  SG_HIP_CHECK(hipGetLastError());
  return SG_OK;
}

int sg_lattice_destroy(sg_lattice* L) {
  if (!L) return SG_OK;
  if (L->magic != kLatMagic) return fail(SG_ESTATE, "lattice handle is not a live lattice");
  L->magic = 0;
  free_lat(L);
  return SG_OK;
}

}  // extern "C"
