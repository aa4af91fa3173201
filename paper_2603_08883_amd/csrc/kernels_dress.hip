// Fused dressing step on gfx950:
//   classify (anticommutation with P), split (cos/sin rotation, product phase),
//   route (new key K^P goes to bucket b ^ f(P)), merge D = H + I inside the
//   bucket pair, compression |c| < eps, optional QMF energy of the output.
//
// Closed-form dressing: Sec. II, Eq. 5.  Merge D = H + I: App. D.
// Pairwise routing between partitions that differ in the flipped bits: App. B/C.
// Compression of small terms: App. A, iterative procedure.
//
// One 512-thread workgroup handles one bucket pair {b, b ^ f} at a time
// (persistent grid, static round-robin over pairs, one arena reservation per
// workgroup).  Every key of the output receives at most two contributions,
// from K and from K ^ P, so the pair's anticommuting terms are joined in an
// LDS hash table on one member of each {K, K^P} pair (the one whose pivot bit
// is 0) and each coefficient is a single IEEE addition.  Commuting terms
// stream straight through.  Bucket b's outputs fill its region from the front
// (child 0) and, when the step doubles the bucket count, from the back
// (child 1).  The energy of every output is formed while the input term is in
// registers: <K> = A * B and <K^P> = A * B', where B, B' run over the few
// 3-qubit groups P touches and A over the rest of K.
#include "iqcc_internal.h"

#pragma clang fp contract(off)

namespace iqcc {

constexpr int kDB = 512;                  // threads per dressing workgroup
constexpr int kDW = kDB / 64;             // waves per dressing workgroup
constexpr int kFieldBits = 12;            // packed per-category counters (<= 1024 per round)
constexpr uint64_t kFieldMask = (1u << kFieldBits) - 1;

__host__ __device__ inline int next_pow2_int(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

size_t dress_lds_bytes(int W, int cap, bool energy, bool tape) {
  size_t o = energy ? (size_t)W * kGroupsPerWord * kLutEntries * 8 : 0;
  o += (size_t)W * cap * 8 * 2;                  // keys
  o += (size_t)cap * 8;                          // coefficients
  if (energy) o += (size_t)cap * 8 * 2;          // <K>, <K^P>
  o += (size_t)next_pow2_int(2 * cap) * 4;       // hash table
  o += (size_t)cap * 2;                          // partner
  o += ((size_t)cap + 7) & ~(size_t)7;           // side
  o += 8 * 8 + 8 * 8 + 8 * 8 + 256 * 4;          // scan, reduce, misc, round stack
  if (tape) o += (size_t)cap * 8 * 2;            // tape: input row, own output row
  return o;
}

template <int W>
struct Smem {
  double* lut;
  uint64_t* ax;
  uint64_t* az;
  double* ac;
  double* ek;     // <K> of each anticommuting entry
  double* ekp;    // <K^P>
  int* tab;
  int16_t* partner;
  uint8_t* side;
  uint64_t* scan;
  double* red;
  int64_t* misc;
  int* stack;
  int64_t* arow;   // tape: input row of each anticommuting entry
  int64_t* orow;   // tape: output row of its own key (-1 if dropped)
  int cap, ts;
};

template <int W, bool ENERGY>
__device__ __forceinline__ Smem<W> carve(unsigned char* smem, int cap, bool tape) {
  Smem<W> s;
  size_t o = 0;
  s.lut = (double*)(smem + o);
  o += ENERGY ? (size_t)W * kGroupsPerWord * kLutEntries * 8 : 0;
  s.ax = (uint64_t*)(smem + o); o += (size_t)W * cap * 8;
  s.az = (uint64_t*)(smem + o); o += (size_t)W * cap * 8;
  s.ac = (double*)(smem + o); o += (size_t)cap * 8;
  s.ek = (double*)(smem + o); o += ENERGY ? (size_t)cap * 8 : 0;
  s.ekp = (double*)(smem + o); o += ENERGY ? (size_t)cap * 8 : 0;
  s.ts = next_pow2_int(2 * cap);
  s.tab = (int*)(smem + o); o += (size_t)s.ts * 4;
  s.partner = (int16_t*)(smem + o); o += (size_t)cap * 2;
  s.side = (uint8_t*)(smem + o); o += ((size_t)cap + 7) & ~(size_t)7;
  s.scan = (uint64_t*)(smem + o); o += 64;
  s.red = (double*)(smem + o); o += 64;
  s.misc = (int64_t*)(smem + o); o += 64;
  s.stack = (int*)(smem + o); o += 256 * 4;
  // tape rows (only carved, and only touched, when the step records a tape)
  s.arow = (int64_t*)(smem + o); o += tape ? (size_t)cap * 8 : 0;
  s.orow = (int64_t*)(smem + o);
  s.cap = cap;
  return s;
}

struct PairState {
  int64_t n0, n1, off0, off1, ntot;
  int64_t reg0, reg1, bound0, bound1;
  int64_t c00, c01, c10, c11;   // outputs written per (side, child); category = 2*side + child
  uint32_t b0, b1;
  bool self;
  __device__ __forceinline__ int64_t cnt(int cat) const {
    return cat == 0 ? c00 : cat == 1 ? c01 : cat == 2 ? c10 : c11;
  }
  __device__ __forceinline__ void add_packed(uint64_t total) {
    c00 += (int64_t)(total & kFieldMask);
    c01 += (int64_t)((total >> kFieldBits) & kFieldMask);
    c10 += (int64_t)((total >> (2 * kFieldBits)) & kFieldMask);
    c11 += (int64_t)((total >> (3 * kFieldBits)) & kFieldMask);
  }
  __device__ __forceinline__ int64_t row(int cat, int64_t k) const {
    const int64_t reg = (cat >> 1) ? reg1 : reg0;
    const int64_t bound = (cat >> 1) ? bound1 : bound0;
    return (cat & 1) == 0 ? reg + k : reg + bound - 1 - k;
  }
};

template <int W>
__device__ __forceinline__ void load_key(const StoreDev& st, int64_t row, uint64_t* kx,
                                         uint64_t* kz, double& c) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    kx[w] = __builtin_nontemporal_load(&st.x[w * st.cap + row]);
    kz[w] = __builtin_nontemporal_load(&st.z[w * st.cap + row]);
  }
  c = __builtin_nontemporal_load(&st.c[row]);
}

template <int W>
__device__ __forceinline__ void store_key(const StoreDev& st, int64_t row, const uint64_t* kx,
                                          const uint64_t* kz, double c) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    __builtin_nontemporal_store(kx[w], &st.x[w * st.cap + row]);
    __builtin_nontemporal_store(kz[w], &st.z[w * st.cap + row]);
  }
  __builtin_nontemporal_store(c, &st.c[row]);
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

// <K> and <K^P> of the product state: A over the non-identity groups of K
// that P does not touch (four independent lookups per iteration), B and B'
// over P's groups for K and K^P.
template <int W>
__device__ __forceinline__ void expect_split(const double* lut, const Entangler& P,
                                             const uint64_t* x, const uint64_t* z, double& ek,
                                             double& ekp) {
  double p0 = 1.0, p1 = 1.0, p2 = 1.0, p3 = 1.0, b = 1.0, b2 = 1.0;
#pragma unroll
  for (int h = 0; h < 2 * W; ++h) {
    const uint32_t xh = (uint32_t)(x[h >> 1] >> (32 * (h & 1)));
    const uint32_t zh = (uint32_t)(z[h >> 1] >> (32 * (h & 1)));
    const double* lh = lut + h * kGroupsPerHalf * kLutEntries;
    uint32_t nz = (xh | zh) & ~P.gbits[h];
    while (nz) {
      uint32_t e[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        uint32_t off = 0;   // entry 0 of group 0 is 1.0: the identity once nz is empty
        if (nz) {
          const uint32_t g = div3_small((uint32_t)__builtin_ctz(nz));
          const uint32_t sh = 3 * g;
          off = g * kLutEntries + (__builtin_amdgcn_ubfe(xh, sh, 3) | (__builtin_amdgcn_ubfe(zh, sh, 3) << 3));
          nz &= ~(7u << sh);
        }
        e[k] = off;
      }
      p0 *= lh[e[0]];
      p1 *= lh[e[1]];
      p2 *= lh[e[2]];
      p3 *= lh[e[3]];
    }
    const uint32_t pxh = (uint32_t)(P.px[h >> 1] >> (32 * (h & 1)));
    const uint32_t pzh = (uint32_t)(P.pz[h >> 1] >> (32 * (h & 1)));
    for (int t = P.gstart[h]; t < P.gstart[h + 1]; ++t) {
      const uint32_t sh = 3 * (uint32_t)P.glist[t];
      const uint32_t ix = __builtin_amdgcn_ubfe(xh, sh, 3), iz = __builtin_amdgcn_ubfe(zh, sh, 3);
      const uint32_t base = (uint32_t)P.glist[t] * kLutEntries;
      b *= lh[base + (ix | (iz << 3))];
      b2 *= lh[base + ((ix ^ __builtin_amdgcn_ubfe(pxh, sh, 3)) | ((iz ^ __builtin_amdgcn_ubfe(pzh, sh, 3)) << 3))];
    }
  }
  const double a = (p0 * p1) * (p2 * p3);
  ek = a * b;
  ekp = a * b2;
}

// One pass over the pair's input terms (one term per thread per round).
// Commuting terms are written to the output when `full`; anticommuting terms
// whose representative hash falls in residue class `rem` mod `mod` are
// appended to the LDS list (up to cap).  Returns the number of such
// anticommuting terms (block-uniform).
template <int W, bool ENERGY>
__device__ int64_t scan_pair(const StoreDev& in, const StoreDev& out, const Entangler& P,
                             const Smem<W>& sm, PairState& ps, int split, int m, bool full,
                             uint32_t mod, uint32_t rem, double eps, int64_t* tape_self,
                             int64_t* tape_partner, double& eacc) {
  const int tid = threadIdx.x;
  int64_t n_anti = 0;
  for (int64_t i0 = 0; i0 < ps.ntot; i0 += kDB) {
    const int64_t idx = i0 + tid;
    const bool valid = idx < ps.ntot;
    const int kside = idx >= ps.n0;
    const int64_t krow = kside ? ps.off1 + (idx - ps.n0) : ps.off0 + idx;
    uint64_t kx[W], kz[W];
    double kc = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) kx[w] = kz[w] = 0;
    if (valid) load_key<W>(in, krow, kx, kz, kc);
    int cat = -1;
    if (valid) {
      if (anticommutes<W>(kx, kz, P.px, P.pz)) {
        if (mod == 1 || (round_hash(rep_hash<W>(P, kx, kz)) & (mod - 1)) == rem) cat = 4;
      } else if (full) {
        if (!(fabs(kc) < eps)) {
          // commuting terms keep their coefficient; compression applies to them too
          const int child = split ? (int)((bucket_hash<W>(kx, kz) >> m) & 1u) : 0;
          cat = kside * 2 + child;
        } else if (tape_self) {
          tape_self[krow] = -1;
          tape_partner[krow] = -2;
        }
      }
    }
    double ek = 0.0, ekp = 0.0;
    if (ENERGY && cat >= 0) expect_split<W>(sm.lut, P, kx, kz, ek, ekp);
    uint64_t total;
    const uint64_t ex = block_exclusive_scan_n<kDW>(cat >= 0 ? 1ull << (kFieldBits * cat) : 0ull,
                                                    sm.scan, total);
    if (cat >= 0) {
      const int64_t k = (int64_t)((ex >> (kFieldBits * cat)) & kFieldMask);
      if (cat == 4) {
        const int64_t slot = n_anti + k;
        if (slot < sm.cap) {
#pragma unroll
          for (int w = 0; w < W; ++w) {
            sm.ax[w * sm.cap + slot] = kx[w];
            sm.az[w * sm.cap + slot] = kz[w];
          }
          sm.ac[slot] = kc;
          sm.side[slot] = (uint8_t)kside;
          if (ENERGY) {
            sm.ek[slot] = ek;
            sm.ekp[slot] = ekp;
          }
          if (tape_self) sm.arow[slot] = krow;
        }
      } else {
        const int64_t orow = ps.row(cat, ps.cnt(cat) + k);
        store_key<W>(out, orow, kx, kz, kc);
        if (ENERGY) eacc += kc * ek;
        if (tape_self) {
          tape_self[krow] = orow;
          tape_partner[krow] = -2;
        }
      }
    }
    ps.add_packed(total);
    n_anti += (int64_t)((total >> (kFieldBits * 4)) & kFieldMask);
  }
  return n_anti;
}

// Join the n (<= cap) anticommuting terms held in LDS and emit the rotated
// and new terms.
template <int W, bool ENERGY>
__device__ void emit_anti(const StoreDev& out, const Entangler& P, const Smem<W>& sm,
                          PairState& ps, int n, int split, int m, double C, double S,
                          double eps, int64_t* tape_self, int64_t* tape_partner,
                          double& eacc) {
  const int tid = threadIdx.x;
  const uint32_t tmask = (uint32_t)sm.ts - 1;
  for (int i = tid; i < sm.ts; i += kDB) sm.tab[i] = -1;
  for (int i = tid; i < n; i += kDB) sm.partner[i] = -1;
  __syncthreads();
  // insert the members whose pivot bit is 0
  for (int i = tid; i < n; i += kDB) {
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      kx[w] = sm.ax[w * sm.cap + i];
      kz[w] = sm.az[w * sm.cap + i];
    }
    if (pivot_of<W>(P, kx, kz)) continue;
    uint32_t h = table_hash<W>(kx, kz) & tmask;
    while (atomicCAS(&sm.tab[h], -1, i) != -1) h = (h + 1) & tmask;
  }
  __syncthreads();
  // the members whose pivot bit is 1 look up K ^ P
  for (int i = tid; i < n; i += kDB) {
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      kx[w] = sm.ax[w * sm.cap + i] ^ P.px[w];
      kz[w] = sm.az[w * sm.cap + i] ^ P.pz[w];
    }
    if (pivot_of<W>(P, kx, kz)) continue;  // pivot of K was 0: K is in the table itself
    uint32_t h = table_hash<W>(kx, kz) & tmask;
    for (;;) {
      const int j = sm.tab[h];
      if (j < 0) break;
      bool eq = true;
#pragma unroll
      for (int w = 0; w < W; ++w)
        eq = eq && (sm.ax[w * sm.cap + j] == kx[w]) && (sm.az[w * sm.cap + j] == kz[w]);
      if (eq) {
        sm.partner[i] = (int16_t)j;
        sm.partner[j] = (int16_t)i;
        break;
      }
      h = (h + 1) & tmask;
    }
  }
  __syncthreads();
  const int child_p = split ? (int)((P.hp >> m) & 1u) : 0;
  for (int i0 = 0; i0 < n; i0 += kDB) {
    const int i = i0 + tid;
    const bool valid = i < n;
    uint64_t kx[W], kz[W];
    double v_own = 0.0, v_new = 0.0;
    int cat_own = -1, cat_new = -1;
    if (valid) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        kx[w] = sm.ax[w * sm.cap + i];
        kz[w] = sm.az[w * sm.cap + i];
      }
      const double a = sm.ac[i];
      const int side = sm.side[i];
      const int j = sm.partner[i];
      const int child = split ? (int)((bucket_hash<W>(kx, kz) >> m) & 1u) : 0;
      const double rot = __dmul_rn(C, a);
      if (j >= 0) {
        // partner K ^ P present: its new term lands on K
        uint64_t jx[W], jz[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
          jx[w] = sm.ax[w * sm.cap + j];
          jz[w] = sm.az[w * sm.cap + j];
        }
        const int ej = product_phase<W>(P.px, P.pz, jx, jz);
        const double sj = __dmul_rn(S, sm.ac[j]);
        v_own = __dadd_rn(rot, ej == 3 ? sj : -sj);
      } else {
        v_own = rot;
        const int e = product_phase<W>(P.px, P.pz, kx, kz);
        const double si = __dmul_rn(S, a);
        v_new = e == 3 ? si : -si;
        if (!(fabs(v_new) < eps)) {
          const int oside = ps.self ? 0 : side ^ 1;
          cat_new = oside * 2 + (child ^ child_p);
        }
      }
      if (!(fabs(v_own) < eps)) cat_own = side * 2 + child;
    }
    uint64_t packed = 0;
    if (cat_own >= 0) packed += 1ull << (kFieldBits * cat_own);
    if (cat_new >= 0) packed += 1ull << (kFieldBits * cat_new);
    uint64_t total;
    uint64_t ex = block_exclusive_scan_n<kDW>(packed, sm.scan, total);
    int64_t own_row = -1, new_row = -1;
    if (cat_own >= 0) {
      const int64_t k = (int64_t)((ex >> (kFieldBits * cat_own)) & kFieldMask);
      ex += 1ull << (kFieldBits * cat_own);
      own_row = ps.row(cat_own, ps.cnt(cat_own) + k);
      store_key<W>(out, own_row, kx, kz, v_own);
      if (ENERGY) eacc += v_own * sm.ek[i];
    }
    if (cat_new >= 0) {
      atomicAdd((unsigned long long*)&sm.misc[3], 1ull);
      const int64_t k = (int64_t)((ex >> (kFieldBits * cat_new)) & kFieldMask);
      new_row = ps.row(cat_new, ps.cnt(cat_new) + k);
      uint64_t qx[W], qz[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        qx[w] = kx[w] ^ P.px[w];
        qz[w] = kz[w] ^ P.pz[w];
      }
      store_key<W>(out, new_row, qx, qz, v_new);
      if (ENERGY) eacc += v_new * sm.ekp[i];
    }
    if (tape_self && valid) {
      sm.orow[i] = own_row;
      tape_self[sm.arow[i]] = own_row;
      if (sm.partner[i] < 0) tape_partner[sm.arow[i]] = new_row;
    }
    ps.add_packed(total);
  }
  __syncthreads();
  if (tape_self) {
    // the partner K^P of a paired entry is the other member's own output row
    for (int i = tid; i < n; i += kDB) {
      const int j = sm.partner[i];
      if (j >= 0) tape_partner[sm.arow[i]] = sm.orow[j];
    }
    __syncthreads();
  }
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

// Rows a pair reserves in the output arena: the worst case 2 (n_b + n_b').
__device__ __forceinline__ int64_t pair_need(const StoreDev& in, int64_t pi, uint32_t f, int thi) {
  uint32_t b0, b1;
  pair_buckets(pi, f, thi, b0, b1);
  const int64_t n0 = in.cnt[b0];
  return f ? 2 * (n0 + in.cnt[b1]) : 2 * n0;
}

// Rows for every pair this workgroup owns (pi = first, first + stride, ...),
// reserved with one atomic; returns the base (block-uniform) or -1 when the
// arena is too small.
__device__ int64_t reserve_rows(const StoreDev& in, const StoreDev& out, int64_t first,
                                int64_t stride, int64_t npairs, uint32_t f, int thi,
                                uint64_t* scan_tmp, int64_t* misc) {
  int64_t mine = 0;
  const int64_t count = first < npairs ? (npairs - first + stride - 1) / stride : 0;
  for (int64_t k = threadIdx.x; k < count; k += kDB) mine += pair_need(in, first + k * stride, f, thi);
  uint64_t total;
  block_exclusive_scan_n<kDW>((uint64_t)mine, scan_tmp, total);
  if (threadIdx.x == 0) {
    int64_t base = total ? (int64_t)atomicAdd((unsigned long long*)out.top, (unsigned long long)total) : 0;
    if (base + (int64_t)total > out.cap) {
      atomicOr(out.err, 1);
      base = -1;
    }
    misc[5] = base;
  }
  __syncthreads();
  const int64_t base = misc[5];
  __syncthreads();
  return base;
}

// Per-workgroup totals of one step, flushed to the output store's device
// counters once at the end (same-address global atomics serialise in L2).
struct StepCounts {
  int64_t produced = 0, anti = 0, fresh = 0;
};

// Everything one workgroup does for bucket pair `pi` of one dressing step;
// `base` is the first arena row reserved for it (-1: no room, write nothing).
template <int W, bool ENERGY>
__device__ void process_pair(const StoreDev& in, const StoreDev& out, const Entangler& P,
                             const DressConfig& cfg, const Smem<W>& sm, int64_t pi, int m,
                             int split, uint32_t f, int thi, int64_t base, double& eacc,
                             StepCounts& counts) {
  const int tid = threadIdx.x;
  PairState ps;
  pair_buckets(pi, f, thi, ps.b0, ps.b1);
  ps.self = (f == 0);
  ps.n0 = in.cnt[ps.b0];
  ps.off0 = in.off[ps.b0];
  ps.n1 = ps.self ? 0 : in.cnt[ps.b1];
  ps.off1 = ps.self ? 0 : in.off[ps.b1];
  ps.ntot = ps.n0 + ps.n1;
  ps.bound0 = ps.self ? 2 * ps.n0 : ps.n0 + ps.n1;
  ps.bound1 = ps.self ? 0 : ps.n0 + ps.n1;
  const bool bad = base < 0;
  if (tid == 0) {
    sm.misc[2] = 0;   // round stack depth
    sm.misc[3] = 0;   // new terms of this pair
  }
  __syncthreads();
  ps.reg0 = base;
  ps.reg1 = base + ps.bound0;
  ps.c00 = ps.c01 = ps.c10 = ps.c11 = 0;
  int64_t pair_anti = 0;
  if (!bad) {
    // The first pass writes the commuting terms and collects all
    // anticommuting ones.  If they do not fit in LDS they are processed in
    // residue classes of a hash of the pair representative (both members of
    // a {K, K^P} pair fall in the same class); oversized classes split.  One
    // call site each for the scan and the join keeps the code small.
    int* stk = sm.stack;   // pairs (mod, rem), written by thread 0
    bool full = true;
    uint32_t mod = 1, rem = 0;
    for (;;) {
      const int64_t na = scan_pair<W, ENERGY>(in, out, P, sm, ps, split, m, full, mod, rem, cfg.eps,
                                              cfg.tape_self, cfg.tape_partner, eacc);
      __syncthreads();
      if (full) pair_anti = na;
      if (na <= sm.cap) {
        emit_anti<W, ENERGY>(out, P, sm, ps, (int)na, split, m, cfg.C, cfg.S, cfg.eps,
                             cfg.tape_self, cfg.tape_partner, eacc);
      } else if (tid == 0) {
        int t = (int)sm.misc[2];
        if (full) {
          int r0 = 1;
          while (r0 * (int64_t)sm.cap < 2 * na && r0 < 32) r0 <<= 1;
          for (int r = r0 - 1; r >= 0; --r) {
            stk[2 * t] = r0;
            stk[2 * t + 1] = r;
            ++t;
          }
        } else if (t + 2 <= 120 && mod < (1u << 30)) {
          stk[2 * t] = (int)(2 * mod); stk[2 * t + 1] = (int)(rem + mod);
          stk[2 * t + 2] = (int)(2 * mod); stk[2 * t + 3] = (int)rem;
          t += 2;
        } else {
          atomicOr(out.err, 4);
        }
        sm.misc[2] = t;
      }
      __syncthreads();
      const int sp = (int)sm.misc[2];
      if (sp == 0) break;
      mod = (uint32_t)stk[2 * (sp - 1)];
      rem = (uint32_t)stk[2 * (sp - 1) + 1];
      full = false;
      __syncthreads();
      if (tid == 0) sm.misc[2] = sp - 1;
    }
  }
  // bucket table of the output
  if (tid == 0) {
    int64_t produced = 0;
    const int nside = ps.self ? 1 : 2;
    for (int s = 0; s < nside; ++s) {
      const uint32_t b = s ? ps.b1 : ps.b0;
      for (int ch = 0; ch < 1 + split; ++ch) {
        const uint32_t ob = b + ((uint32_t)ch << m);
        const int64_t k = bad ? 0 : ps.cnt(2 * s + ch);
        out.cnt[ob] = k;
        out.off[ob] = ps.row(2 * s + ch, k - 1) - (ch ? 0 : k - 1);
        produced += k;
      }
    }
    counts.produced += produced;
    counts.anti += pair_anti;
    counts.fresh += sm.misc[3];
  }
  __syncthreads();
}

__device__ __forceinline__ void flush_counts(const StoreDev& out, const StepCounts& counts) {
  if (threadIdx.x == 0) {
    if (counts.produced) atomicAdd((unsigned long long*)out.total, (unsigned long long)counts.produced);
    if (counts.anti) atomicAdd((unsigned long long*)&out.stats[0], (unsigned long long)counts.anti);
    if (counts.fresh) atomicAdd((unsigned long long*)&out.stats[1], (unsigned long long)counts.fresh);
  }
}

template <int W, bool ENERGY>
__global__ __launch_bounds__(kDB) __attribute__((amdgpu_waves_per_eu(4))) void k_dress(StoreDev in, StoreDev out, Entangler P,
                                               DressConfig cfg) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Smem<W> sm = carve<W, ENERGY>(smem, cfg.anti_cap, cfg.tape_self != nullptr);
  const int tid = threadIdx.x;
  if (*in.err) {
    // the input is the invalid output of an earlier step: propagate, read nothing
    if (blockIdx.x == 0 && tid == 0) atomicOr(out.err, *in.err);
    return;
  }
  const int m = *in.m;
  const int64_t n_in = *in.total;
  const int split = (m < out.mcap) && (n_in > (cfg.split_thr << m)) ? 1 : 0;
  if (m + split > out.mcap) {
    if (blockIdx.x == 0 && tid == 0) atomicOr(out.err, 2);
    return;
  }
  const uint32_t mask = (uint32_t)((1ull << m) - 1);
  const uint32_t f = P.hp & mask;
  const int64_t npairs = f ? (1ll << (m - 1)) : (1ll << m);
  const int thi = f ? 31 - __clz(f) : 0;
  if (blockIdx.x == 0 && tid == 0) *out.m = m + split;
  if (ENERGY) {
    for (int i = tid; i < W * kGroupsPerWord * kLutEntries; i += kDB) sm.lut[i] = cfg.lut[i];
    __syncthreads();
  }
  double eacc = 0.0;
  StepCounts counts;
  int64_t base = reserve_rows(in, out, blockIdx.x, gridDim.x, npairs, f, thi, sm.scan, sm.misc);
  for (int64_t pi = blockIdx.x; pi < npairs; pi += gridDim.x) {
    process_pair<W, ENERGY>(in, out, P, cfg, sm, pi, m, split, f, thi, base, eacc, counts);
    if (base >= 0) base += pair_need(in, pi, f, thi);
  }
  flush_counts(out, counts);
  if (ENERGY) {
    const double s = block_sum_n<kDW>(eacc, sm.red);
    if (tid == 0) cfg.e_partial[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// Batched dressing of many independent Hamiltonians (one entangler each) in
// one persistent launch.  A plan kernel sizes every Hamiltonian's step on the
// device (no host synchronisation, so the pair of launches can be captured in
// a HIP graph); workgroups then take (Hamiltonian, bucket pair) items from an
// atomic queue, so uneven sizes balance across the chip.
// ---------------------------------------------------------------------------
__global__ void k_batch_plan(int n_ham, const BatchItem* items, BatchPlan* plan,
                             int64_t split_thr, int64_t* queue) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t start = 0;
  for (int i = 0; i < n_ham; ++i) {
    const BatchItem& it = items[i];
    BatchPlan p{};
    p.item_start = start;
    *it.out.total = 0;
    *it.out.top = 0;
    *it.out.err = 0;
    it.out.stats[0] = 0;
    it.out.stats[1] = 0;
    const int ierr = *it.in.err;
    const int m = *it.in.m;
    const int64_t n_in = *it.in.total;
    const int split = (m < it.out.mcap) && (n_in > (split_thr << m)) ? 1 : 0;
    if (ierr || m + split > it.out.mcap) {
      *it.out.err = ierr ? ierr : 2;
      p.npairs = 0;
    } else {
      const uint32_t f = it.P.hp & (uint32_t)((1ull << m) - 1);
      p.m = m;
      p.split = split;
      p.f = f;
      p.thi = f ? 31 - __clz(f) : 0;
      p.npairs = f ? (1ll << (m - 1)) : (1ll << m);
      *it.out.m = m + split;
    }
    start += p.npairs;
    plan[i] = p;
  }
  plan[n_ham].item_start = start;
  *queue = 0;
}

template <int W>
__global__ __launch_bounds__(kDB) __attribute__((amdgpu_waves_per_eu(4))) void k_dress_batch(int n_ham, const BatchItem* items,
                                                     const BatchPlan* plan, DressConfig cfg,
                                                     int64_t* queue) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Smem<W> sm = carve<W, false>(smem, cfg.anti_cap, false);
  const int64_t total = plan[n_ham].item_start;
  double eacc = 0.0;
  constexpr int64_t kGrab = 4;   // items taken per queue atomic
  int64_t item = 0, left = 0;
  for (;;) {
    if (left == 0) {
      if (threadIdx.x == 0) sm.misc[4] = (int64_t)atomicAdd((unsigned long long*)queue, (unsigned long long)kGrab);
      __syncthreads();
      item = sm.misc[4];
      __syncthreads();
      left = kGrab;
    }
    if (item >= total) break;
    int lo = 0, hi = n_ham - 1;   // last i with item_start <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (plan[mid].item_start <= item) lo = mid; else hi = mid - 1;
    }
    const BatchItem& it = items[lo];
    const BatchPlan p = plan[lo];
    DressConfig c = cfg;
    c.C = it.C;
    c.S = it.S;
    // items come from a dynamic queue: reserve per pair
    const int64_t pi = item - p.item_start;
    const int64_t need = pair_need(it.in, pi, p.f, p.thi);
    if (threadIdx.x == 0) {
      int64_t b = need ? (int64_t)atomicAdd((unsigned long long*)it.out.top, (unsigned long long)need) : 0;
      if (b + need > it.out.cap) {
        atomicOr(it.out.err, 1);
        b = -1;
      }
      sm.misc[5] = b;
    }
    __syncthreads();
    const int64_t base = sm.misc[5];
    __syncthreads();
    StepCounts counts;
    process_pair<W, false>(it.in, it.out, it.P, c, sm, pi, p.m, p.split, p.f, p.thi, base, eacc, counts);
    flush_counts(it.out, counts);
    ++item;
    --left;
  }
}

void set_dress_batch_attributes(int W, int anti_cap) {
  const int lds = (int)dress_lds_bytes(W, anti_cap, false, false);
  switch (W) {
    case 1: hipFuncSetAttribute((const void*)k_dress_batch<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds); break;
    case 2: hipFuncSetAttribute((const void*)k_dress_batch<2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds); break;
    case 3: hipFuncSetAttribute((const void*)k_dress_batch<3>, hipFuncAttributeMaxDynamicSharedMemorySize, lds); break;
    default: hipFuncSetAttribute((const void*)k_dress_batch<4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds); break;
  }
}

// Launches only (no attribute calls), so the pair can be captured in a graph.
void launch_dress_batch(int W, int n_ham, const BatchItem* items, BatchPlan* plan,
                        const DressConfig& cfg, int64_t* queue, hipStream_t s) {
  const size_t lds = dress_lds_bytes(W, cfg.anti_cap, false, false);
  hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(64), 0, s, n_ham, items, plan, cfg.split_thr, queue);
  const BatchPlan* cp = plan;
  switch (W) {
    case 1: hipLaunchKernelGGL(k_dress_batch<1>, dim3(cfg.grid), dim3(kDB), lds, s, n_ham, items, cp, cfg, queue); break;
    case 2: hipLaunchKernelGGL(k_dress_batch<2>, dim3(cfg.grid), dim3(kDB), lds, s, n_ham, items, cp, cfg, queue); break;
    case 3: hipLaunchKernelGGL(k_dress_batch<3>, dim3(cfg.grid), dim3(kDB), lds, s, n_ham, items, cp, cfg, queue); break;
    default: hipLaunchKernelGGL(k_dress_batch<4>, dim3(cfg.grid), dim3(kDB), lds, s, n_ham, items, cp, cfg, queue); break;
  }
}

template <int W, bool E>
static void launch_dress_t(const StoreDev& in, const StoreDev& out, const Entangler& P,
                           const DressConfig& cfg, hipStream_t s) {
  const size_t lds = dress_lds_bytes(W, cfg.anti_cap, E, cfg.tape_self != nullptr);
  hipFuncSetAttribute((const void*)k_dress<W, E>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds);
  hipLaunchKernelGGL((k_dress<W, E>), dim3(cfg.grid), dim3(kDB), lds, s, in, out, P, cfg);
}

void launch_dress(int W, const StoreDev& in, const StoreDev& out, const Entangler& P,
                  const DressConfig& cfg, hipStream_t s) {
  const bool e = cfg.lut != nullptr;
  switch (W) {
    case 1: e ? launch_dress_t<1, true>(in, out, P, cfg, s) : launch_dress_t<1, false>(in, out, P, cfg, s); break;
    case 2: e ? launch_dress_t<2, true>(in, out, P, cfg, s) : launch_dress_t<2, false>(in, out, P, cfg, s); break;
    case 3: e ? launch_dress_t<3, true>(in, out, P, cfg, s) : launch_dress_t<3, false>(in, out, P, cfg, s); break;
    default: e ? launch_dress_t<4, true>(in, out, P, cfg, s) : launch_dress_t<4, false>(in, out, P, cfg, s); break;
  }
}

// ---------------------------------------------------------------------------
// Raw dressing of flat rows (no merge): row 2i = rotated/copied term, row
// 2i+1 = new term for anticommuting rows.
// ---------------------------------------------------------------------------
template <int W>
__global__ void k_dress_raw(const uint64_t* __restrict__ x, const uint64_t* __restrict__ z,
                            const double* __restrict__ c, int64_t n, int64_t ld, Entangler P,
                            double C, double S, uint64_t* ox, uint64_t* oz, double* oc,
                            int8_t* flag, int64_t ldo) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      kx[w] = x[w * ld + i];
      kz[w] = z[w * ld + i];
    }
    const double a = c[i];
    const bool anti = anticommutes<W>(kx, kz, P.px, P.pz);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      ox[w * ldo + 2 * i] = kx[w];
      oz[w * ldo + 2 * i] = kz[w];
      ox[w * ldo + 2 * i + 1] = kx[w] ^ P.px[w];
      oz[w * ldo + 2 * i + 1] = kz[w] ^ P.pz[w];
    }
    if (anti) {
      const int e = product_phase<W>(P.px, P.pz, kx, kz);
      const double si = __dmul_rn(S, a);
      oc[2 * i] = __dmul_rn(C, a);
      oc[2 * i + 1] = e == 3 ? si : -si;
    } else {
      oc[2 * i] = a;
      oc[2 * i + 1] = __builtin_nan("");
    }
    flag[i] = anti ? 1 : 0;
  }
}

void launch_dress_raw(int W, const uint64_t* x, const uint64_t* z, const double* c, int64_t n,
                      int64_t ld, const Entangler& P, double C, double S, uint64_t* ox,
                      uint64_t* oz, double* oc, int8_t* flag, int64_t ld_out, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  switch (W) {
    case 1: hipLaunchKernelGGL(k_dress_raw<1>, dim3(blocks), dim3(kBlock), 0, s, x, z, c, n, ld, P, C, S, ox, oz, oc, flag, ld_out); break;
    case 2: hipLaunchKernelGGL(k_dress_raw<2>, dim3(blocks), dim3(kBlock), 0, s, x, z, c, n, ld, P, C, S, ox, oz, oc, flag, ld_out); break;
    case 3: hipLaunchKernelGGL(k_dress_raw<3>, dim3(blocks), dim3(kBlock), 0, s, x, z, c, n, ld, P, C, S, ox, oz, oc, flag, ld_out); break;
    default: hipLaunchKernelGGL(k_dress_raw<4>, dim3(blocks), dim3(kBlock), 0, s, x, z, c, n, ld, P, C, S, ox, oz, oc, flag, ld_out); break;
  }
}

}  // namespace iqcc
