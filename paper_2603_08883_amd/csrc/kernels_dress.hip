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
// (child 1).
//
// Output positions come from per-wave reservations: each wave ranks its lanes
// per output category with ballots and takes a block of rows with one LDS
// atomic per counter word, so the streaming passes have no workgroup barrier
// (rows within a category are in wave-arrival order; the set of terms is
// unique).  The energy of an anticommuting term is formed once, after
// compaction into LDS: <K> = A * B and <K^P> = A * B', where B, B' run over
// the few 3-qubit groups P touches and A over the rest of K.
#include "iqcc_internal.h"

#pragma clang fp contract(off)

namespace iqcc {

constexpr int kDB = 512;                  // threads per dressing workgroup
constexpr int kDW = kDB / 64;             // waves per dressing workgroup

__host__ __device__ inline int next_pow2_int(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

size_t dress_lds_bytes(int W, int cap, bool energy, bool tape) {
  size_t o = energy ? (size_t)W * kGroupsPerWord * kLutEntries * 8 : 0;
  o += (size_t)W * cap * 8 * 2;                  // keys
  o += (size_t)cap * 8;                          // coefficients
  o += (size_t)next_pow2_int(2 * cap) * 4;       // hash table
  o += (size_t)cap * 2;                          // partner
  o += ((size_t)cap + 7) & ~(size_t)7;           // side
  o += 8 * 8 + 8 * 8 + 8 * 8 + 256 * 4 + 4 * 8;  // scan, reduce, misc, round stack, counters
  if (tape) o += (size_t)cap * 8 * 2;            // tape: input row, own output row
  return o;
}

template <int W>
struct Smem {
  double* lut;
  uint64_t* ax;
  uint64_t* az;
  double* ac;
  int* tab;
  int16_t* partner;
  uint8_t* side;
  uint64_t* scan;
  double* red;
  int64_t* misc;
  int* stack;
  unsigned long long* ctr;   // per-pair output counters: [c00|c01<<32, c10|c11<<32, anti]
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
  s.ts = next_pow2_int(2 * cap);
  s.tab = (int*)(smem + o); o += (size_t)s.ts * 4;
  s.partner = (int16_t*)(smem + o); o += (size_t)cap * 2;
  s.side = (uint8_t*)(smem + o); o += ((size_t)cap + 7) & ~(size_t)7;
  s.scan = (uint64_t*)(smem + o); o += 64;
  s.red = (double*)(smem + o); o += 64;
  s.misc = (int64_t*)(smem + o); o += 64;
  s.stack = (int*)(smem + o); o += 256 * 4;
  s.ctr = (unsigned long long*)(smem + o); o += 4 * 8;
  // tape rows (only carved, and only touched, when the step records a tape)
  s.arow = (int64_t*)(smem + o); o += tape ? (size_t)cap * 8 : 0;
  s.orow = (int64_t*)(smem + o);
  s.cap = cap;
  return s;
}

// Output category of a term: 2 * side + child (side: which bucket of the
// pair, child: which half after a split).  Category 4: anticommuting, to LDS.
struct PairState {
  int64_t n0, n1, off0, off1, ntot;
  int64_t reg0, reg1, bound0, bound1;
  uint32_t b0, b1;
  bool self;
  __device__ __forceinline__ int64_t row(int cat, int64_t k) const {
    const int64_t reg = (cat >> 1) ? reg1 : reg0;
    const int64_t bound = (cat >> 1) ? bound1 : bound0;
    return (cat & 1) == 0 ? reg + k : reg + bound - 1 - k;
  }
};

// Row positions for up to two entries per lane (categories a and b in
// [0, 2 * NWORD), -1 for none) from the LDS counters ctr[0..NWORD), which hold
// two 32-bit fields each (category 2k in the low field of word k, 2k + 1 in
// the high field).  Within a wave, all a-entries of a category precede its
// b-entries, each in lane order; the wave's block comes from one LDS atomic
// per counter word it touches.  Must be called by the whole wave (every lane
// active, wave-uniform control flow).  Returns the number of b-entries of the
// wave (wave-uniform).
template <int NWORD, bool TWO>
__device__ __forceinline__ uint32_t wave_positions(unsigned long long* ctr, int a, int b,
                                                   uint32_t& pa, uint32_t& pb) {
  uint32_t nb = 0;
#pragma unroll
  for (int k = 0; k < NWORD; ++k) {
    const uint64_t ma0 = __ballot(a == 2 * k);
    const uint64_t ma1 = __ballot(a == 2 * k + 1);
    const uint64_t mb0 = TWO ? __ballot(b == 2 * k) : 0ull;
    const uint64_t mb1 = TWO ? __ballot(b == 2 * k + 1) : 0ull;
    if ((ma0 | ma1 | mb0 | mb1) == 0) continue;
    const uint32_t na0 = (uint32_t)__popcll(ma0), na1 = (uint32_t)__popcll(ma1);
    const uint32_t nb0 = (uint32_t)__popcll(mb0), nb1 = (uint32_t)__popcll(mb1);
    nb += nb0 + nb1;
    const unsigned long long inc = (unsigned long long)(na0 + nb0) |
                                   ((unsigned long long)(na1 + nb1) << 32);
    unsigned long long old = 0;
    if ((threadIdx.x & 63) == 0) old = atomicAdd(&ctr[k], inc);
    old = wave_bcast0(old);
    const uint32_t lo = (uint32_t)old, hi = (uint32_t)(old >> 32);
    if (a == 2 * k) pa = lo + lanes_below(ma0);
    if (a == 2 * k + 1) pa = hi + lanes_below(ma1);
    if (TWO) {
      if (b == 2 * k) pb = lo + na0 + lanes_below(mb0);
      if (b == 2 * k + 1) pb = hi + na1 + lanes_below(mb1);
    }
  }
  return nb;
}

// One pass over the pair's input terms, each wave on its own 64-term slices
// (no workgroup barrier).  Commuting terms are written to the output when
// `full`; anticommuting terms whose representative hash falls in residue
// class `rem` mod `mod` are appended to the LDS list (up to cap; the count is
// in ctr[2] afterwards).
template <int W, bool ENERGY>
__device__ void scan_pair(const StoreDev& in, const StoreDev& out, const Entangler& P,
                          const Smem<W>& sm, const PairState& ps, int split, int m, bool full,
                          uint32_t mod, uint32_t rem, double eps, int delta,
                          int32_t* tape_self, int32_t* tape_partner, double& eacc) {
  const int lane = threadIdx.x & 63;
  for (int64_t i0 = (threadIdx.x & ~63); i0 < ps.ntot; i0 += kDB) {
    const int64_t idx = i0 + lane;
    const bool valid = idx < ps.ntot;
    const int kside = idx >= ps.n0;
    const int64_t krow = kside ? ps.off1 + (idx - ps.n0) : ps.off0 + idx;
    uint64_t kx[W], kz[W];
    double kc = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) kx[w] = kz[w] = 0;
    if (valid) load_key<W>(in, krow, kx, kz, kc);
    int cat = -1;
    bool dropped = false;   // a commuting term removed by compression
    if (valid) {
      if (anticommutes<W>(kx, kz, P.px, P.pz)) {
        if (mod == 1 || (round_hash(rep_hash<W>(P, kx, kz)) & (mod - 1)) == rem) cat = 4;
      } else if (full) {
        if (!(fabs(kc) < eps)) {
          // commuting terms keep their coefficient; compression applies to them too
          const int child = split ? (int)((bucket_hash<W>(kx, kz) >> m) & 1u) : 0;
          cat = kside * 2 + child;
        } else {
          dropped = true;
          if (tape_self) {
            tape_self[krow] = -1;
            tape_partner[krow] = -1;   // commuting
          }
        }
      }
    }
    // Energy of commuting terms: every kept one, or (delta) only those that
    // compression removes.  Anticommuting terms are evaluated after the join.
    if (ENERGY && (delta ? dropped : (cat >= 0 && cat < 4))) {
      const double ek = expect_lut<W>(sm.lut, kx, kz);
      eacc += dropped ? -(kc * ek) : kc * ek;
    }
    uint32_t pos = 0, unused = 0;
    wave_positions<3, false>(sm.ctr, cat, -1, pos, unused);
    if (cat == 4) {
      if ((int)pos < sm.cap) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          sm.ax[w * sm.cap + pos] = kx[w];
          sm.az[w * sm.cap + pos] = kz[w];
        }
        sm.ac[pos] = kc;
        sm.side[pos] = (uint8_t)kside;
        if (tape_self) sm.arow[pos] = krow;
      }
    } else if (cat >= 0) {
      const int64_t orow = ps.row(cat, pos);
      store_key<W>(out, orow, kx, kz, kc);
      if (tape_self) {
        tape_self[krow] = (int32_t)orow;
        tape_partner[krow] = -1;   // commuting
      }
    }
  }
}

// Join the n (<= cap) anticommuting terms held in LDS and emit the rotated
// and new terms.
template <int W, bool ENERGY>
__device__ void emit_anti(const StoreDev& out, const Entangler& P, const Smem<W>& sm,
                          const PairState& ps, int n, int split, int m, double C, double S,
                          double eps, int delta, int32_t* tape_self, int32_t* tape_partner,
                          double& eacc, int64_t& fresh) {
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
  const int lane = threadIdx.x & 63;
  for (int i0 = (threadIdx.x & ~63); i0 < n; i0 += kDB) {   // wave-uniform
    const int i = i0 + lane;
    const bool valid = i < n;
    uint64_t kx[W], kz[W];
    double v_own = 0.0, v_new = 0.0, a = 0.0;
    int cat_own = -1, cat_new = -1;
    int sa = 0;   // 1 when s_K = +1 (P K = i^3 (K^P)), for the tape
    if (valid) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        kx[w] = sm.ax[w * sm.cap + i];
        kz[w] = sm.az[w * sm.cap + i];
      }
      a = sm.ac[i];
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
        sa = ej == 3 ? 0 : 1;   // the two members of a pair have opposite signs
        const double sj = __dmul_rn(S, sm.ac[j]);
        v_own = __dadd_rn(rot, ej == 3 ? sj : -sj);
      } else {
        v_own = rot;
        const int e = product_phase<W>(P.px, P.pz, kx, kz);
        sa = e == 3 ? 1 : 0;
        const double si = __dmul_rn(S, a);
        v_new = e == 3 ? si : -si;
        if (!(fabs(v_new) < eps)) {
          const int oside = ps.self ? 0 : side ^ 1;
          cat_new = oside * 2 + (child ^ child_p);
        }
      }
      if (!(fabs(v_own) < eps)) cat_own = side * 2 + child;
      if (ENERGY) {
        // <K> and <K^P>; (delta) A's contribution before the step is removed
        double ek, ekp;
        expect_split<W>(sm.lut, P, kx, kz, ek, ekp);
        if (cat_own >= 0) eacc += v_own * ek;
        if (cat_new >= 0) eacc += v_new * ekp;
        if (delta) eacc -= a * ek;
      }
    }
    uint32_t own_pos = 0, new_pos = 0;
    fresh += wave_positions<2, true>(sm.ctr, cat_own, cat_new, own_pos, new_pos);
    int64_t own_row = -1, new_row = -1;
    if (cat_own >= 0) {
      own_row = ps.row(cat_own, own_pos);
      store_key<W>(out, own_row, kx, kz, v_own);
    }
    if (cat_new >= 0) {
      new_row = ps.row(cat_new, new_pos);
      uint64_t qx[W], qz[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        qx[w] = kx[w] ^ P.px[w];
        qz[w] = kz[w] ^ P.pz[w];
      }
      store_key<W>(out, new_row, qx, qz, v_new);
    }
    if (tape_self && valid) {
      // tape_partner of an anticommuting row: 2 * (output row of K^P + 1) + [s_K = +1]
      sm.orow[i] = own_row;
      tape_self[sm.arow[i]] = (int32_t)own_row;
      if (sm.partner[i] < 0) tape_partner[sm.arow[i]] = (int32_t)(2 * (new_row + 1) + sa);
      else sm.side[i] = (uint8_t)(sm.side[i] | (sa << 1));   // only this lane reads side[i]
    }
  }
  __syncthreads();
  if (tape_self) {
    // the partner K^P of a paired entry is the other member's own output row
    for (int i = tid; i < n; i += kDB) {
      const int j = sm.partner[i];
      if (j >= 0) tape_partner[sm.arow[i]] = (int32_t)(2 * (sm.orow[j] + 1) + ((sm.side[i] >> 1) & 1));
    }
    __syncthreads();
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
  int64_t produced = 0, anti = 0;   // thread 0 of the workgroup
  int64_t fresh = 0;                // per wave (lane 0 flushes)
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
    sm.ctr[0] = sm.ctr[1] = sm.ctr[2] = 0;
  }
  __syncthreads();
  ps.reg0 = base;
  ps.reg1 = base + ps.bound0;
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
      scan_pair<W, ENERGY>(in, out, P, sm, ps, split, m, full, mod, rem, cfg.eps, cfg.delta,
                           cfg.tape_self, cfg.tape_partner, eacc);
      __syncthreads();
      const int64_t na = (int64_t)(uint32_t)sm.ctr[2];
      if (full) pair_anti = na;
      if (na <= sm.cap) {
        emit_anti<W, ENERGY>(out, P, sm, ps, (int)na, split, m, cfg.C, cfg.S, cfg.eps, cfg.delta,
                             cfg.tape_self, cfg.tape_partner, eacc, counts.fresh);
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
      if (tid == 0) {
        sm.misc[2] = sp - 1;
        sm.ctr[2] = 0;   // the next round counts its own class
      }
      __syncthreads();
    }
  }
  // bucket table of the output
  if (tid == 0) {
    int64_t produced = 0;
    const int nside = ps.self ? 1 : 2;
    for (int s = 0; s < nside; ++s) {
      const uint32_t b = s ? ps.b1 : ps.b0;
      const unsigned long long word = sm.ctr[s];
      const int64_t reg = bad ? 0 : (s ? ps.reg1 : ps.reg0);
      const int64_t bound = bad ? 0 : (s ? ps.bound1 : ps.bound0);
      const int64_t k0 = bad ? 0 : (int64_t)(uint32_t)word;
      const int64_t k1 = (bad || !split) ? 0 : (int64_t)(uint32_t)(word >> 32);
      // child 0 fills the side's region from the front and grows upward;
      // child 1 fills it from the back and grows downward; the gap between
      // them is shared half and half
      out.cnt[b] = k0;
      out.off[b] = reg;
      if (split) {
        const int64_t mid = reg + k0 + (bound - k0 - k1) / 2;
        const uint32_t ob = b + (1u << m);
        out.lim[b] = mid;
        out.cnt[ob] = k1;
        out.off[ob] = reg + bound - k1;
        out.lim[ob] = ~mid;
      } else {
        out.lim[b] = reg + bound;
      }
      produced += k0 + k1;
    }
    counts.produced += produced;
    counts.anti += pair_anti;
  }
  __syncthreads();
}

__device__ __forceinline__ void flush_counts(const StoreDev& out, const StepCounts& counts) {
  if (threadIdx.x == 0) {
    if (counts.produced) atomicAdd((unsigned long long*)out.total, (unsigned long long)counts.produced);
    if (counts.anti) atomicAdd((unsigned long long*)&out.stats[0], (unsigned long long)counts.anti);
  }
  if ((threadIdx.x & 63) == 0 && counts.fresh)
    atomicAdd((unsigned long long*)&out.stats[1], (unsigned long long)counts.fresh);
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
// device, one thread per Hamiltonian and a scan (no host synchronisation, so
// the pair of launches can be captured in a HIP graph); workgroups then take
// work units -- up to unit_pairs consecutive bucket pairs of one Hamiltonian --
// from an atomic queue, so uneven sizes balance across the chip while the
// queue, the Hamiltonian lookup, the row reservation and the counter flush
// are paid once per unit.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_batch_plan(int n_ham, const BatchItem* items,
                                                       BatchPlan* plan, int64_t split_thr,
                                                       int unit_pairs, int64_t* queue) {
  __shared__ uint64_t scan_tmp[kWaves];
  int64_t start = 0;
  for (int base = 0; base < n_ham; base += kBlock) {
    const int i = base + threadIdx.x;
    BatchPlan p{};
    int64_t units = 0;
    if (i < n_ham) {
      const BatchItem& it = items[i];
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
      units = (p.npairs + unit_pairs - 1) / unit_pairs;
    }
    uint64_t total;
    const uint64_t ex = block_exclusive_scan((uint64_t)units, scan_tmp, total);
    if (i < n_ham) {
      p.item_start = start + (int64_t)ex;
      plan[i] = p;
    }
    start += (int64_t)total;
  }
  if (threadIdx.x == 0) {
    plan[n_ham].item_start = start;
    *queue = 0;
  }
}

template <int W>
__global__ __launch_bounds__(kDB) __attribute__((amdgpu_waves_per_eu(4))) void k_dress_batch(int n_ham, const BatchItem* items,
                                                     const BatchPlan* plan, DressConfig cfg,
                                                     int64_t* queue) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Smem<W> sm = carve<W, false>(smem, cfg.anti_cap, false);
  __shared__ __align__(16) BatchItem s_item;
  static_assert(sizeof(BatchItem) % 8 == 0, "BatchItem is copied as 64-bit words");
  const int64_t total = plan[n_ham].item_start;
  double eacc = 0.0;
  for (;;) {
    if (threadIdx.x == 0) {
      const int64_t unit = (int64_t)atomicAdd((unsigned long long*)queue, 1ull);
      int lo = 0, hi = n_ham - 1;   // last Hamiltonian whose first unit is <= unit
      if (unit < total) {
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (plan[mid].item_start <= unit) lo = mid; else hi = mid - 1;
        }
      }
      sm.misc[4] = unit;
      sm.misc[6] = lo;
    }
    __syncthreads();
    const int64_t unit = sm.misc[4];
    const int h = (int)sm.misc[6];
    if (unit >= total) break;
    // the unit's Hamiltonian descriptors, copied once into LDS (read there
    // by every pair of the unit instead of from global memory)
    constexpr int kItemWords = (int)(sizeof(BatchItem) / 8);
    for (int k = threadIdx.x; k < kItemWords; k += kDB)
      reinterpret_cast<uint64_t*>(&s_item)[k] = reinterpret_cast<const uint64_t*>(items + h)[k];
    __syncthreads();
    const StoreDev& in = s_item.in;
    const StoreDev& out = s_item.out;
    const Entangler& P = s_item.P;
    const BatchPlan p = plan[h];
    DressConfig c = cfg;
    c.C = s_item.C;
    c.S = s_item.S;
    const int64_t p0 = (unit - p.item_start) * cfg.unit_pairs;
    const int64_t p1 = p0 + cfg.unit_pairs < p.npairs ? p0 + cfg.unit_pairs : p.npairs;
    int64_t base = reserve_rows(in, out, p0, 1, p1, p.f, p.thi, sm.scan, sm.misc);
    StepCounts counts;
    for (int64_t pi = p0; pi < p1; ++pi) {
      process_pair<W, false>(in, out, P, c, sm, pi, p.m, p.split, p.f, p.thi, base, eacc, counts);
      if (base >= 0) base += pair_need(in, pi, p.f, p.thi);
    }
    flush_counts(out, counts);
    __syncthreads();   // every thread is done with s_item before the next copy
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
  hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(kBlock), 0, s, n_ham, items, plan, cfg.split_thr,
                     cfg.unit_pairs, queue);
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

// ---------------------------------------------------------------------------
// Sizing count: terms of the store that anticommute with P (one integer
// atomic per workgroup, so the count is exact and order-independent).
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kBlock) void k_count_anti(StoreDev st, Entangler P,
                                                       unsigned long long* out) {
  __shared__ uint64_t tmp[kWaves];
  const int64_t B = 1ll << *st.m;
  uint64_t mine = 0;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = st.cnt[b], off = st.off[b];
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
      uint64_t kx[W], kz[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        kx[w] = st.x[w * st.cap + off + i];
        kz[w] = st.z[w * st.cap + off + i];
      }
      mine += anticommutes<W>(kx, kz, P.px, P.pz) ? 1u : 0u;
    }
  }
  uint64_t total;
  block_exclusive_scan(mine, tmp, total);
  if (threadIdx.x == 0 && total) atomicAdd(out, (unsigned long long)total);
}

void launch_count_anti(int W, const StoreDev& st, const Entangler& P, unsigned long long* out,
                       int grid, hipStream_t s) {
  switch (W) {
    case 1: hipLaunchKernelGGL(k_count_anti<1>, dim3(grid), dim3(kBlock), 0, s, st, P, out); break;
    case 2: hipLaunchKernelGGL(k_count_anti<2>, dim3(grid), dim3(kBlock), 0, s, st, P, out); break;
    case 3: hipLaunchKernelGGL(k_count_anti<3>, dim3(grid), dim3(kBlock), 0, s, st, P, out); break;
    default: hipLaunchKernelGGL(k_count_anti<4>, dim3(grid), dim3(kBlock), 0, s, st, P, out); break;
  }
}

// ---------------------------------------------------------------------------
// P1 P2 = i^e P3 for n pairs of words (the phase rule of product_phase).
// ---------------------------------------------------------------------------
template <int W>
__global__ void k_pauli_products(const uint64_t* x1, const uint64_t* z1, const uint64_t* x2,
                                 const uint64_t* z2, int64_t n, int64_t ld, uint64_t* x3,
                                 uint64_t* z3, int8_t* e) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t ax[W], az[W], bx[W], bz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      ax[w] = x1[w * ld + i]; az[w] = z1[w * ld + i];
      bx[w] = x2[w * ld + i]; bz[w] = z2[w * ld + i];
    }
    e[i] = (int8_t)product_phase<W>(ax, az, bx, bz);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      x3[w * ld + i] = ax[w] ^ bx[w];
      z3[w * ld + i] = az[w] ^ bz[w];
    }
  }
}

void launch_pauli_products(int W, const uint64_t* x1, const uint64_t* z1, const uint64_t* x2,
                           const uint64_t* z2, int64_t n, int64_t ld, uint64_t* x3, uint64_t* z3,
                           int8_t* e, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  switch (W) {
    case 1: hipLaunchKernelGGL(k_pauli_products<1>, dim3(blocks), dim3(kBlock), 0, s, x1, z1, x2, z2, n, ld, x3, z3, e); break;
    case 2: hipLaunchKernelGGL(k_pauli_products<2>, dim3(blocks), dim3(kBlock), 0, s, x1, z1, x2, z2, n, ld, x3, z3, e); break;
    case 3: hipLaunchKernelGGL(k_pauli_products<3>, dim3(blocks), dim3(kBlock), 0, s, x1, z1, x2, z2, n, ld, x3, z3, e); break;
    default: hipLaunchKernelGGL(k_pauli_products<4>, dim3(blocks), dim3(kBlock), 0, s, x1, z1, x2, z2, n, ld, x3, z3, e); break;
  }
}

}  // namespace iqcc
