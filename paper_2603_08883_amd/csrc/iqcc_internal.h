// Internal declarations of libiqcc (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace iqcc {

constexpr int kBlock = 256;              // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kMaxWords = 4;             // 256 qubits
constexpr int kGroupsPerHalf = 11;       // 3-qubit groups per 32-bit half word (10 full + 1 of 2)
constexpr int kGroupsPerWord = 2 * kGroupsPerHalf;
constexpr int kLutEntries = 64;          // 3 x-bits and 3 z-bits per group
constexpr int kMaxBucketBits = 28;

// ---------------------------------------------------------------------------
// GF(2)-linear 32-bit hash of a Pauli key.  Rotations, xors and xorshift
// rounds are all linear over GF(2), so hash(K ^ P) == hash(K) ^ hash(P); the
// rounds spread the strongly structured Jordan-Wigner keys evenly.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint64_t rotl64(uint64_t v, int r) {
  return r ? (v << r) | (v >> (64 - r)) : v;
}
__host__ __device__ __forceinline__ uint64_t xorshift64(uint64_t f) {
  f ^= f << 13;
  f ^= f >> 7;
  f ^= f << 17;
  return f;
}
template <int W>
__host__ __device__ __forceinline__ uint32_t bucket_hash(const uint64_t* x, const uint64_t* z) {
  uint64_t f = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) f ^= rotl64(x[w], (11 * w) & 63) ^ rotl64(z[w], (37 + 19 * w) & 63);
  f = xorshift64(xorshift64(xorshift64(f)));
  return (uint32_t)(f >> 32);
}
inline uint32_t bucket_hash_host(int W, const uint64_t* x, const uint64_t* z) {
  uint64_t f = 0;
  for (int w = 0; w < W; ++w) f ^= rotl64(x[w], (11 * w) & 63) ^ rotl64(z[w], (37 + 19 * w) & 63);
  f = xorshift64(xorshift64(xorshift64(f)));
  return (uint32_t)(f >> 32);
}

// Non-linear 32-bit mix for LDS hash tables.
template <int W>
__device__ __forceinline__ uint32_t table_hash(const uint64_t* x, const uint64_t* z) {
  uint64_t f = 0x9E3779B97F4A7C15ull;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    f = (f ^ x[w]) * 0xBF58476D1CE4E5B9ull;
    f = (f ^ z[w]) * 0x94D049BB133111EBull;
  }
  f ^= f >> 31;
  return (uint32_t)(f >> 32) ^ (uint32_t)f;
}

// ---------------------------------------------------------------------------
// Block-wide exclusive scan of a 64-bit value (fixed order: lanes, then waves).
// tmp: LDS scratch of kWaves uint64.  Contains two barriers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* tmp,
                                                         uint64_t& total) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  uint64_t s = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t y = __shfl_up(s, d, 64);
    if (lane >= d) s += y;
  }
  if (lane == 63) tmp[wid] = s;
  __syncthreads();
  uint64_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    uint64_t t = tmp[i];
    base += (i < wid) ? t : 0;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return base + s - v;
}

template <int NW>
__device__ __forceinline__ uint64_t block_exclusive_scan_n(uint64_t v, uint64_t* tmp,
                                                           uint64_t& total) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  uint64_t s = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t y = __shfl_up(s, d, 64);
    if (lane >= d) s += y;
  }
  if (lane == 63) tmp[wid] = s;
  __syncthreads();
  uint64_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    uint64_t t = tmp[i];
    base += (i < wid) ? t : 0;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return base + s - v;
}

template <int NW>
__device__ __forceinline__ double block_sum_n(double v, double* tmp) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_down(v, d, 64);
  if (lane == 0) tmp[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NW; ++i) s += tmp[i];
  }
  __syncthreads();
  return s;  // valid in thread 0
}

// Exact sums of doubles whose result does not depend on the order of the
// additions.  A value v with |v| < 2^31 is taken as the pair of integers
//   n1 = round(v * 2^20),  n0 = round((v - n1 * 2^-20) * 2^60),
// so v = n1 * 2^-20 + n0 * 2^-60 to within 2^-61; integer sums of the pairs
// are exact.  Adding 1.5 * 2^32 (resp. 1.5 * 2^-8) rounds to a multiple of
// 2^-20 (2^-60), and the difference of the bit patterns is that multiple as an
// integer (both sums stay in the binade of the constant).
struct FixedSum {
  long long hi = 0;    // units of 2^-20
  long long lo = 0;    // units of 2^-60
  double mag = 0.0;    // sum of |v| in any order: range check only
};

__device__ __forceinline__ void fixed_split(double v, long long& n1, long long& n0) {
  const double k1 = 0x1.8p32, k0 = 0x1.8p-8;
  const double a1 = v + k1;
  const double r = v - (a1 - k1);
  const double a0 = r + k0;
  n1 = __double_as_longlong(a1) - __double_as_longlong(k1);
  n0 = __double_as_longlong(a0) - __double_as_longlong(k0);
}

__device__ __forceinline__ void fixed_add(FixedSum& f, double v) {
  long long n1, n0;
  fixed_split(v, n1, n0);
  f.hi += n1;
  f.lo += n0;
  f.mag += fabs(v);
}

// Moves whole units of 2^-20 out of lo (|lo| < 2^40 afterwards).
__device__ __forceinline__ void fixed_normalize(FixedSum& f) {
  const long long carry = f.lo >> 40;
  f.hi += carry;
  f.lo -= carry * (1ll << 40);
}

// The value of a sum of at most 2^23 normalized parts whose values were
// finite and summed to magnitude below 2^31 (NaN otherwise).
__device__ __forceinline__ double fixed_value(long long hi, long long lo, double mag) {
  if (!(mag < 0x1p31)) return __builtin_nan("");
  return (double)hi * 0x1p-20 + (double)lo * 0x1p-60;
}

// Block sum of FixedSum parts (exact in hi and lo), valid in thread 0; the
// parts are normalized first.
template <int NW>
__device__ __forceinline__ FixedSum block_fixed_sum(FixedSum f, long long* tmp_hi, long long* tmp_lo,
                                                    double* tmp_mag) {
  fixed_normalize(f);
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    f.hi += __shfl_down(f.hi, d, 64);
    f.lo += __shfl_down(f.lo, d, 64);
    f.mag += __shfl_down(f.mag, d, 64);
  }
  if (lane == 0) {
    tmp_hi[wid] = f.hi;
    tmp_lo[wid] = f.lo;
    tmp_mag[wid] = f.mag;
  }
  __syncthreads();
  FixedSum t;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NW; ++i) {
      t.hi += tmp_hi[i];
      t.lo += tmp_lo[i];
      t.mag += tmp_mag[i];
    }
    fixed_normalize(t);
  }
  __syncthreads();
  return t;
}

// Block-wide sum of doubles in a fixed order (lane tree, then waves in order).
__device__ __forceinline__ double block_sum(double v, double* tmp) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_down(v, d, 64);
  if (lane == 0) tmp[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < kWaves; ++i) s += tmp[i];
  }
  __syncthreads();
  return s;  // valid in thread 0
}

// ---------------------------------------------------------------------------
// QMF expectation <K> = prod_j b_j(sigma_j) with a 3-qubit-group table.
// Qubits are grouped per 32-bit half word h (qubits 32h .. 32h+31) into 11
// groups of 3 (the last one of 2); group index gi = 11 h + g.
// lut[gi*64 + (xbits | zbits<<3)] = product of the group's single-qubit factors.
// Identity groups are skipped; four independent lookups per iteration keep
// several LDS reads in flight.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t div3_small(uint32_t b) { return (b * 11u) >> 5; }  // b < 32

// Bit 3g of the result is set when 3-qubit group g of a 32-bit half word has a
// non-identity qubit (nz = x | z of the half).
__device__ __forceinline__ uint32_t group_starts(uint32_t nz) {
  return (nz | (nz >> 1) | (nz >> 2)) & 0x49249249u;
}

// Table entry of the lowest remaining group in t (then cleared from t): group
// g * 64 + (x bits | z bits << 3).  Once t is empty it returns entry 0 of
// group 0, which is 1.0, so callers can run a fixed number of lookups without
// branching.
__device__ __forceinline__ uint32_t next_group_entry(uint32_t& t, uint32_t xh, uint32_t zh) {
  const uint32_t sh = (uint32_t)__builtin_ctz(t | 0x80000000u);   // 31 only when t == 0
  const uint32_t g = div3_small(sh);
  const uint32_t off = g * kLutEntries + (__builtin_amdgcn_ubfe(xh, sh, 3) |
                                          (__builtin_amdgcn_ubfe(zh, sh, 3) << 3));
  const uint32_t e = t ? off : 0u;
  t &= t - 1;
  return e;
}

template <int W>
__device__ __forceinline__ double expect_lut_sparse(const double* lut, const uint64_t* x,
                                             const uint64_t* z) {
  double p0 = 1.0, p1 = 1.0, p2 = 1.0, p3 = 1.0;
#pragma unroll
  for (int h = 0; h < 2 * W; ++h) {
    const uint32_t xh = (uint32_t)(x[h >> 1] >> (32 * (h & 1)));
    const uint32_t zh = (uint32_t)(z[h >> 1] >> (32 * (h & 1)));
    uint32_t t = group_starts(xh | zh);
    const double* lh = lut + h * kGroupsPerHalf * kLutEntries;
    while (t) {
      uint32_t e[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) e[k] = next_group_entry(t, xh, zh);
      p0 *= lh[e[0]];
      p1 *= lh[e[1]];
      p2 *= lh[e[2]];
      p3 *= lh[e[3]];
    }
  }
  return (p0 * p1) * (p2 * p3);
}

template <int W>
__device__ __forceinline__ double expect_lut(const double* lut, const uint64_t* x,
                                             const uint64_t* z) {
  if constexpr (W > 2) {
    return expect_lut_sparse<W>(lut, x, z);   // fewer registers for wide keys
  } else {
    // every group of every half word, identity groups included (table entry 0
    // is 1.0): no per-group branch or select; each iteration issues four
    // independent lookups per half word, so the product takes three LDS round
    // trips
    double p0 = 1.0, p1 = 1.0, p2 = 1.0, p3 = 1.0;
    uint32_t xh[2 * W], zh[2 * W];
#pragma unroll
    for (int h = 0; h < 2 * W; ++h) {
      xh[h] = (uint32_t)(x[h >> 1] >> (32 * (h & 1)));
      zh[h] = (uint32_t)(z[h >> 1] >> (32 * (h & 1)));
    }
#pragma unroll 1
    for (int g = 0; g < 12; g += 4) {
      const uint32_t s0 = 3 * g;
#pragma unroll
      for (int h = 0; h < 2 * W; ++h) {
        const double* lg = lut + (h * kGroupsPerHalf + g) * kLutEntries;
        p0 *= lg[__builtin_amdgcn_ubfe(xh[h], s0, 3) | (__builtin_amdgcn_ubfe(zh[h], s0, 3) << 3)];
        p1 *= lg[kLutEntries + (__builtin_amdgcn_ubfe(xh[h], s0 + 3, 3) | (__builtin_amdgcn_ubfe(zh[h], s0 + 3, 3) << 3))];
        p2 *= lg[2 * kLutEntries + (__builtin_amdgcn_ubfe(xh[h], s0 + 6, 3) | (__builtin_amdgcn_ubfe(zh[h], s0 + 6, 3) << 3))];
        if (g + 3 < kGroupsPerHalf)
          p3 *= lg[3 * kLutEntries + (__builtin_amdgcn_ubfe(xh[h], s0 + 9, 3) | (__builtin_amdgcn_ubfe(zh[h], s0 + 9, 3) << 3))];
      }
    }
    return (p0 * p1) * (p2 * p3);
  }
}

// <sigma> of one qubit of the QMF product state (Eq. 3) from sin/cos of its
// Bloch angles; op: 0 = I, 1 = X, 2 = Z, 3 = Y (bit0 = x, bit1 = z).
__device__ __forceinline__ double bloch_factor(int op, double st, double ct, double sp,
                                               double cp) {
  return op == 0 ? 1.0 : op == 1 ? st * cp : op == 2 ? ct : st * sp;
}

// Anticommutation of K with P: parity of |xK & zP| + |zK & xP|.
template <int W>
__device__ __forceinline__ bool anticommutes(const uint64_t* x, const uint64_t* z,
                                             const uint64_t* px, const uint64_t* pz) {
  uint64_t t = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) t ^= (x[w] & pz[w]) ^ (z[w] & px[w]);
  return __popcll(t) & 1;
}

// Phase exponent e of the product A*B = i^e Q (Hermitian-Y encoding):
// e = |xA&zA| + |xB&zB| + 2|zA&xB| - |xQ&zQ|  (mod 4).
template <int W>
__device__ __forceinline__ int product_phase(const uint64_t* xa, const uint64_t* za,
                                             const uint64_t* xb, const uint64_t* zb) {
  int s = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    s += __popcll(xa[w] & za[w]) + __popcll(xb[w] & zb[w]) + 2 * __popcll(za[w] & xb[w]) -
         __popcll((xa[w] ^ xb[w]) & (za[w] ^ zb[w]));
  }
  return s & 3;
}

// ---------------------------------------------------------------------------
// Device-side store descriptor (plain pointers).
// ---------------------------------------------------------------------------
struct StoreDev {
  uint64_t* x;       // [W][cap]
  uint64_t* z;       // [W][cap]
  double* c;         // [cap]
  int64_t cap;       // arena rows (= leading dimension)
  int64_t* off;      // [2^mcap] first row of each bucket
  int64_t* cnt;      // [2^mcap] live rows of each bucket
  int64_t* lim;      // [2^mcap] growth region of each bucket (see bucket_room)
  int* m;            // device scalar: bucket bits
  int64_t* total;    // device scalar: live terms
  int64_t* top;      // device scalar: arena rows reserved
  int* err;          // device scalar: 1 = arena overflow, 2 = bucket table overflow
  int64_t* stats;    // device [2]: anticommuting input terms, new terms of the last step
  int64_t* aux;      // device [8]: [0] change of `total` in an in-place step, [1] rows of
                     //   a bucket region, [2] first pool row, [3] work items of the last
                     //   in-place step that were relocated to the pool, [4] rows freed
                     //   by compression in the last in-place step
  int mcap;          // bucket table holds 2^mcap buckets
};

// Growth region of a bucket whose live rows are [off, off + cnt):
//   lim >= 0: the bucket grows upward; its region ends at row lim;
//   lim <  0: it grows downward; its region starts at row ~lim (= -lim - 1).
// Rows of the region outside the live rows belong to no other bucket.
__host__ __device__ __forceinline__ int64_t bucket_room(int64_t off, int64_t cnt, int64_t lim) {
  return lim >= 0 ? lim - off - cnt : off - ~lim;
}

struct Entangler {
  uint64_t px[kMaxWords];
  uint64_t pz[kMaxWords];
  uint32_t hp;       // bucket_hash(P)
  int piv_word;      // pivot bit of P (a set bit of x or z), used to pick one
  int piv_in_x;      //   member of each {K, K^P} pair for the join
  uint64_t piv_mask;
  // the 3-qubit groups P touches, for the split expectation product
  // <K> = A * B and <K^P> = A * B' (A over the other groups of K)
  uint32_t gbits[2 * kMaxWords];                        // per half word: bits of those groups
};

// ---------------------------------------------------------------------------
// Device helpers shared by the dressing kernels.
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ void load_key(const StoreDev& st, int64_t row, uint64_t* kx,
                                         uint64_t* kz, double& c) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    kx[w] = st.x[w * st.cap + row];
    kz[w] = st.z[w * st.cap + row];
  }
  c = st.c[row];
}

template <int W>
__device__ __forceinline__ void store_key(const StoreDev& st, int64_t row, const uint64_t* kx,
                                          const uint64_t* kz, double c) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    st.x[w * st.cap + row] = kx[w];
    st.z[w * st.cap + row] = kz[w];
  }
  st.c[row] = c;
}

template <int W>
__device__ __forceinline__ bool pivot_of(const Entangler& P, const uint64_t* kx,
                                         const uint64_t* kz) {
  uint64_t v = 0;
#pragma unroll
  for (int w = 0; w < W; ++w)
    if (w == P.piv_word) v = P.piv_in_x ? kx[w] : kz[w];
  return (v & P.piv_mask) != 0;
}

// residue classes use the high half of the representative hash; LDS table
// slots use the low bits
__device__ __forceinline__ uint32_t round_hash(uint32_t h) { return (h >> 16) | (h << 16); }

template <int W>
__device__ __forceinline__ uint32_t rep_hash(const Entangler& P, const uint64_t* kx,
                                             const uint64_t* kz) {
  uint64_t rx[W], rz[W];
  const bool piv = pivot_of<W>(P, kx, kz);
#pragma unroll
  for (int w = 0; w < W; ++w) {
    rx[w] = piv ? kx[w] ^ P.px[w] : kx[w];
    rz[w] = piv ? kz[w] ^ P.pz[w] : kz[w];
  }
  return table_hash<W>(rx, rz);
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ unsigned long long wave_bcast0(unsigned long long v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// <K> and <K^P> of the product state: A over the groups of K that P does not
// touch, B and B' over P's groups for K and K^P (two of P's groups per LDS
// round trip).
template <int W>
__device__ __forceinline__ void expect_split(const double* lut, const Entangler& P,
                                             const uint64_t* x, const uint64_t* z, double& ek,
                                             double& ekp) {
  double p0 = 1.0, p1 = 1.0, p2 = 1.0, p3 = 1.0, b = 1.0, b2 = 1.0, c1 = 1.0, c2 = 1.0;
  if constexpr (W > 2) {
    // A over the non-identity groups of K outside P's groups (fewer registers
    // for wide keys)
#pragma unroll
    for (int h = 0; h < 2 * W; ++h) {
      const uint32_t xh = (uint32_t)(x[h >> 1] >> (32 * (h & 1)));
      const uint32_t zh = (uint32_t)(z[h >> 1] >> (32 * (h & 1)));
      const double* lh = lut + h * kGroupsPerHalf * kLutEntries;
      uint32_t t = group_starts((xh | zh) & ~P.gbits[h]);
      while (t) {
        uint32_t e[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] = next_group_entry(t, xh, zh);
        p0 *= lh[e[0]];
        p1 *= lh[e[1]];
        p2 *= lh[e[2]];
        p3 *= lh[e[3]];
      }
    }
  } else {
    // A: every group of every half word with P's groups masked to the identity
    // (table entry 0 = 1.0); each iteration issues 4 independent lookups per
    // half word, so the whole product takes three LDS round trips
    uint32_t xa[2 * W], za[2 * W];
#pragma unroll
    for (int h = 0; h < 2 * W; ++h) {
      xa[h] = (uint32_t)(x[h >> 1] >> (32 * (h & 1))) & ~P.gbits[h];
      za[h] = (uint32_t)(z[h >> 1] >> (32 * (h & 1))) & ~P.gbits[h];
    }
#pragma unroll 1
    for (int g = 0; g < 12; g += 4) {
      const uint32_t s0 = 3 * g;
#pragma unroll
      for (int h = 0; h < 2 * W; ++h) {
        const double* lg = lut + (h * kGroupsPerHalf + g) * kLutEntries;
        p0 *= lg[__builtin_amdgcn_ubfe(xa[h], s0, 3) | (__builtin_amdgcn_ubfe(za[h], s0, 3) << 3)];
        p1 *= lg[kLutEntries + (__builtin_amdgcn_ubfe(xa[h], s0 + 3, 3) | (__builtin_amdgcn_ubfe(za[h], s0 + 3, 3) << 3))];
        p2 *= lg[2 * kLutEntries + (__builtin_amdgcn_ubfe(xa[h], s0 + 6, 3) | (__builtin_amdgcn_ubfe(za[h], s0 + 6, 3) << 3))];
        if (g + 3 < kGroupsPerHalf)
          p3 *= lg[3 * kLutEntries + (__builtin_amdgcn_ubfe(xa[h], s0 + 9, 3) | (__builtin_amdgcn_ubfe(za[h], s0 + 9, 3) << 3))];
      }
    }
  }
  // B and B' over P's groups, two per LDS round trip.  The groups come from
  // the uniform bit mask gbits (scalar registers): indexing an array of the
  // by-value kernel argument with a loop counter makes the compiler read it
  // from memory, and that wait would also wait for every store in flight.
#pragma unroll
  for (int h = 0; h < 2 * W; ++h) {
    const uint32_t xh = (uint32_t)(x[h >> 1] >> (32 * (h & 1)));
    const uint32_t zh = (uint32_t)(z[h >> 1] >> (32 * (h & 1)));
    const double* lh = lut + h * kGroupsPerHalf * kLutEntries;
    const uint32_t pxh = (uint32_t)(P.px[h >> 1] >> (32 * (h & 1)));
    const uint32_t pzh = (uint32_t)(P.pz[h >> 1] >> (32 * (h & 1)));
    uint32_t t = P.gbits[h] & 0x49249249u;   // the first bit of each of P's groups
    while (t) {
      {
        const uint32_t sh = (uint32_t)__builtin_ctz(t);
        t &= t - 1;
        const uint32_t g = div3_small(sh);
        const uint32_t code = __builtin_amdgcn_ubfe(xh, sh, 3) | (__builtin_amdgcn_ubfe(zh, sh, 3) << 3);
        const uint32_t pcode = __builtin_amdgcn_ubfe(pxh, sh, 3) | (__builtin_amdgcn_ubfe(pzh, sh, 3) << 3);
        b *= lh[g * kLutEntries + code];
        b2 *= lh[g * kLutEntries + (code ^ pcode)];
      }
      if (t) {
        const uint32_t sh = (uint32_t)__builtin_ctz(t);
        t &= t - 1;
        const uint32_t g = div3_small(sh);
        const uint32_t code = __builtin_amdgcn_ubfe(xh, sh, 3) | (__builtin_amdgcn_ubfe(zh, sh, 3) << 3);
        const uint32_t pcode = __builtin_amdgcn_ubfe(pxh, sh, 3) | (__builtin_amdgcn_ubfe(pzh, sh, 3) << 3);
        c1 *= lh[g * kLutEntries + code];
        c2 *= lh[g * kLutEntries + (code ^ pcode)];
      }
    }
  }
  const double a = (p0 * p1) * (p2 * p3);
  ek = a * (b * c1);
  ekp = a * (b2 * c2);
}

__device__ __forceinline__ void pair_buckets(int64_t pi, uint32_t f, int thi, uint32_t& b0,
                                             uint32_t& b1) {
  if (f) {
    const uint32_t lo = (uint32_t)pi & ((1u << thi) - 1);
    b0 = (((uint32_t)pi >> thi) << (thi + 1)) | lo;
    b1 = b0 ^ f;
  } else {
    b0 = b1 = (uint32_t)pi;
  }
}

// ---------------------------------------------------------------------------
// Host launchers (defined in the kernel files).
// ---------------------------------------------------------------------------
void launch_build_lut(int W, int nq, const double* theta, const double* phi, double* lut,
                      hipStream_t s);
void launch_zero_counters(StoreDev out, hipStream_t s);
// Load of flat rows into packed buckets, each bucket's rows in ascending key
// order (the same rows whatever the input order).  scratch: B + B/1024 + 16 + n.
int launch_store_load(int W, StoreDev st, const uint64_t* x, const uint64_t* z, const double* c,
                      int64_t n, int64_t ld, int m, int64_t* scratch, hipStream_t s);
void launch_store_export(int W, StoreDev st, int m, uint64_t* x, uint64_t* z, double* c, int64_t ld,
                         int64_t* dest_off, int64_t* scratch, hipStream_t s);
void launch_sum_squares(const StoreDev& st, int grid, double* partial, hipStream_t s);
void launch_lookup(int W, const StoreDev& st, const uint64_t* qx, const uint64_t* qz, int64_t n,
                   int64_t ld, int8_t* found, double* val, hipStream_t s);
void launch_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* scratch, hipStream_t s);

struct DressConfig {
  double C, S, eps;
  int64_t split_thr;
  int anti_cap;
  int grid;
  const double* lut;   // null: no fused energy
  int delta;           // 1: e_partial accumulates only the change of the energy
  double* e_partial;   // [grid]
  int32_t* tape_self;     // null, or per input arena row: output row of K (-1 dropped)
  int32_t* tape_partner;  //   and -1 for a commuting row; for an anticommuting row
                          //   2 * (output row of K^P + 1) + [s_K = +1], where the
                          //   output row is -1 when K^P is absent or dropped
  int unit_pairs;         // batched dressing: consecutive bucket pairs per work unit
};
void launch_dress(int W, const StoreDev& in, const StoreDev& out, const Entangler& P,
                  const DressConfig& cfg, hipStream_t s);

// In-place dressing of a store laid out in bucket regions (kernels_inplace.hip).
struct InplaceConfig {
  double C, S, eps;
  int cap;              // stash entries per wave (inplace_cap)
  int item_terms;       // input terms per work item while buckets are small
  const double* theta;  // null: no energy; else the QMF angles (the group
  const double* phi;    //   table is built in each workgroup's LDS)
  int nq;
  int delta;            // 1: e_partial accumulates only the change of the energy
  double* e_partial;    // [grid * inplace_waves_per_block()]
  int64_t* counts;      // [grid * inplace_waves_per_block()][5]: anticommuting
                        //   inputs, new keys, change of the term count,
                        //   relocated items, freed rows, per wavefront
};
size_t inplace_lds_bytes(int W, int cap, bool energy);
int inplace_cap(int W, bool energy, size_t lds_budget);
int inplace_waves_per_block();
// The step and its finishing kernel (counters of the store, and the energy
// into energy_out, plus *energy_in when given, if energy_out is not null).
void launch_dress_inplace(int W, const StoreDev& st, const Entangler& P, const InplaceConfig& cfg, int grid,
                          const double* energy_in, double* energy_out, hipStream_t s);
// Bucket regions: bucket b gets max(R, 2 cnt_b rounded up to 16) rows; the
// pool starts after the last region.  Load of flat rows (as launch_store_load;
// scratch 3 B + B/1024 + 16 + n) and copy of a store (deterministic: each
// destination bucket takes its rows in source order).  Both set err = 1 when
// the regions do not fit the arena.
int launch_store_load_regions(int W, StoreDev st, const uint64_t* x, const uint64_t* z, const double* c,
                              int64_t n, int64_t ld, int m, int64_t R, int64_t* scratch, hipStream_t s);
// same_m: the source has the same bucket count m (its current m is known on
// the host), so every bucket keeps its terms.
void launch_store_copy_regions(int W, const StoreDev& src, StoreDev dst, int m, int64_t R, int64_t* scratch,
                               hipStream_t s, bool same_m);

// One Hamiltonian of a batched dressing launch.
struct BatchItem {
  StoreDev in, out;
  Entangler P;
  double C, S;
};
// Device-side sizing of one Hamiltonian's step (written by the plan kernel).
struct BatchPlan {
  int64_t item_start;   // first work unit (up to unit_pairs bucket pairs) of this Hamiltonian
  int64_t npairs;
  uint32_t f;
  int m, split, thi;
};
void set_dress_batch_attributes(int W, int anti_cap);
void launch_dress_batch(int W, int n_ham, const BatchItem* items, BatchPlan* plan,
                        const DressConfig& cfg, int64_t* queue, hipStream_t s);
size_t dress_lds_bytes(int W, int anti_cap, bool energy, bool tape);
void launch_count_anti(int W, const StoreDev& st, const Entangler& P, unsigned long long* out,
                       int grid, hipStream_t s);
void launch_pauli_products(int W, const uint64_t* x1, const uint64_t* z1, const uint64_t* x2,
                           const uint64_t* z2, int64_t n, int64_t ld, uint64_t* x3, uint64_t* z3,
                           int8_t* e, hipStream_t s);
void launch_dress_raw(int W, const uint64_t* x, const uint64_t* z, const double* c, int64_t n,
                      int64_t ld, const Entangler& P, double C, double S, uint64_t* ox,
                      uint64_t* oz, double* oc, int8_t* flag, int64_t ld_out, hipStream_t s);
// *out = (base ? *base : 0) + (scale ? *scale : 1) * sum(partial[0..n)); out may alias base.
void launch_finalize_sum(const double* partial, int n, const double* scale, double* out,
                         hipStream_t s, const double* base = nullptr);
// *out = exact sum of n FixedSum parts stored as three 8-byte words each
// (hi, lo, mag), NaN when the values were out of range.
void launch_finalize_fixed(const double* parts, int n, double* out, hipStream_t s);

// Device state of the term-limit selection (kernels_select.hip).
struct SelState {
  uint64_t prefix;               // digits fixed so far
  int64_t need;                  // terms still to take among those matching the prefix
  int64_t passed;                // terms in bins passed over so far
  uint64_t T;                    // |c| bits of the M-th largest term
  int64_t ties;                  // terms with |c| bits == T
  int64_t at;                    // terms in the digit picked last
  int key_mode;                  // 1: keep only ties with canonical key <= kthr
  int pad;
  uint64_t kthr[2 * kMaxWords];  // canonical key threshold among the ties
};
// First |c| digit over every term (sets ss->at, the terms that share it);
// then the remaining digits, copying the |c| bits of those terms to cand
// (capacity >= ss->at) on the second pass and reading only them afterwards.
void launch_abs_select_first(int W, const StoreDev& st, SelState* ss, unsigned* hist, int grid,
                             hipStream_t s);
void launch_abs_select_rest(int W, const StoreDev& st, SelState* ss, unsigned* hist, int grid,
                            uint64_t* cand, int64_t cand_cap, unsigned long long* cand_count,
                            hipStream_t s);
void launch_collect_ties(int W, const StoreDev& st, const SelState* ss, uint64_t* keys, int64_t cap,
                         unsigned long long* count, int grid, hipStream_t s);
void launch_key_select(int W, const uint64_t* keys, int64_t n, SelState* ss, unsigned* hist,
                       hipStream_t s);
// keep_all: 1 every term, 0 the selection in ss, -1 none
void launch_select_compact(int W, const StoreDev& in, const StoreDev& out, const SelState* ss,
                           int keep_all, int grid, hipStream_t s);

// A Pauli key passed by value to a kernel.
struct PauliKey {
  uint64_t x[kMaxWords], z[kMaxWords];
};
// Sortless dressing of a flat, canonically sorted Hamiltonian (kernels_sortless.hip).
// nbits = popcount(P.x) + popcount(P.z); synchronises; hipErrorInvalidValue when the
// result exceeds cap (*n_out is set).
hipError_t sortless_dress_run(int W, const uint64_t* x, const uint64_t* z, const double* c, int64_t n,
                              int64_t ld, const PauliKey& P, int nbits, double C, double S, double eps,
                              uint64_t* ox, uint64_t* oz, double* oc, int64_t cap, int64_t ld_out,
                              int64_t* n_out, hipStream_t s);
void launch_flip_rows(int W, const StoreDev& st, int w_max, uint64_t* ox, uint64_t* oz, double* oc,
                      int64_t ld, unsigned long long* count, int grid, hipStream_t s);
void launch_energy_anti(int W, const StoreDev& st, const PauliKey& P, int grid, const double* lut,
                        double* partial, hipStream_t s);
// Stand-alone energy: builds the table (4-qubit groups for keys of up to two
// words, else 3-qubit groups) into `lut` (energy_lut_doubles(W) doubles) and
// writes grid partial sums.
int energy_lut_doubles(int W);
void launch_energy_table(int W, int nq, const StoreDev& st, int grid, const double* theta,
                         const double* phi, double* lut, double* partial, hipStream_t s);
void launch_energy(int W, const StoreDev& st, int grid, const double* lut, double* e_partial,
                   hipStream_t s);
int energy_bwd_blocks_per_cu(int W);
void launch_energy_backward(int W, int nq, const StoreDev& st, int grid, const double* theta,
                            const double* phi, const double* lut, const double* dE,
                            double* lam /*null or [arena rows]*/, double* acc /*[grid][3*nq]*/,
                            hipStream_t s);
void launch_backward_finalize(int nq, int grid, const double* acc, const double* theta,
                              const double* phi, const double* dE, double* dtheta, double* dphi,
                              hipStream_t s);

int dis_one_blocks_per_cu(int W);
void launch_dis(int W, const StoreDev& st, const double* lut, const uint64_t* cx,
                const uint64_t* cz, int64_t n_cand, int64_t ld_cand, int mode, int tile,
                int grid, double* partial /*[grid_terms][n_cand]*/, int grid_terms,
                double* g, hipStream_t s, const double* theta, const double* phi, int nq,
                double* tables /*dis_tables_doubles(W), batched mode*/);
int64_t dis_tables_doubles(int W);
int64_t dis_tile();   // candidates per workgroup of the batched kernel

void launch_dress_backward(int W, const StoreDev& in, double C, double S,
                           const int32_t* tape_self, const int32_t* tape_partner,
                           const double* lam_out, double* lam_in, double* partial, int grid,
                           hipStream_t s);
void launch_expectations(int W, const StoreDev& st, const double* lut, const double* scale,
                         double* out, int grid, hipStream_t s);
int64_t merge_scratch_len(int W, int64_t n, int m);
void launch_merge_buckets(int W, StoreDev st, const uint64_t* x, const uint64_t* z,
                          const double* c, int64_t n, int64_t ld, int m, double eps,
                          int64_t* scratch, int64_t scratch_len, hipStream_t s);

}  // namespace iqcc
