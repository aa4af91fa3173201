// In-place dressing step on gfx950 for stores laid out in bucket regions.
//
// The step computes what the out-of-place kernel computes (closed-form
// dressing: Sec. II, Eq. 5; merge D = H + I: App. D; compression |c| < eps:
// App. A, iterative procedure), but rewrites only what changes.  Every bucket
// owns a region of rows with free rows after its live ones:
//   - a term that commutes with P keeps its row, key and coefficient, so it is
//     read (to classify it) and never written;
//   - an anticommuting term K gets RN(cos tau c_K) + RN(s sin tau c_{K^P}) in
//     its own row (8 bytes written);
//   - a new key K^P (no partner in the input) goes to its bucket b ^ f: first
//     into rows freed by compression, then after the live rows;
//   - when compression frees more rows of a bucket than new keys arrive, the
//     last live rows of the bucket move down into the remaining free rows, so
//     the live rows stay contiguous.
// A work item whose buckets would outgrow their regions (or whose
// anticommuting terms do not fit the wave's LDS stash) is written to fresh
// regions from the store's pool instead.
//
// Work split: one wavefront per work item, with no workgroup barrier after
// the table load.  A work item is a bucket pair {b, b ^ f} (the single-device
// form of the pairwise exchange between partitions, App. B/C), or up to 32
// consecutive pairs while buckets are small.  Wave g of the grid takes items
// g, g + waves, g + 2 waves, ..., and loads the bucket table of its next item
// while it works on the current one.  Every row position, every sum and the
// energy partials are the same on every run.  Inside an item the
// anticommuting terms are staged in the wave's LDS segment, joined on one
// member of each {K, K^P} pair in an LDS hash table, and every output
// position comes from ballots in stash order.  Lane s of the wave holds the
// bucket table entry of the item's slot s.
#include "iqcc_internal.h"

#pragma clang fp contract(off)

namespace iqcc {

#ifndef IQCC_INPLACE_WAVES
#define IQCC_INPLACE_WAVES 12
#endif
constexpr int kIPW = IQCC_INPLACE_WAVES;   // waves per workgroup (one workgroup per CU)
constexpr int kIPB = 64 * kIPW;
constexpr int kIPSlots = 64;      // buckets per work item (one per lane)
#ifndef IQCC_INPLACE_UNROLL
#define IQCC_INPLACE_UNROLL 2
#endif
constexpr int kIPU = IQCC_INPLACE_UNROLL;   // 64-term slices of the scan in flight per wave

enum : uint8_t { kFComm = 1, kFHole = 2, kFNew = 4 };

// Per-wave LDS segment: the stash of up to `cap` entries, its join table and
// per-slot counters of the item.
constexpr int kIPSlotArrays = 4;

// Join table entries: 11/8 of the stash.  At most one member of each {K, K^P}
// pair is inserted, so the table is seldom more than ~40 % full and always has
// an empty entry (probes end); it has at least `cap` entries because it later
// lists the freed rows.  (With the energy table at W = 2 this size keeps the
// stash at 200 entries; a fuller table lengthens the slowest probe of the wave.)
__host__ __device__ inline int ip_tsize(int cap) { return (11 * cap / 8 + 7) & ~7; }

__host__ __device__ inline size_t seg_bytes(int W, int cap) {
  size_t o = (size_t)W * cap * 16 + (size_t)cap * 8       // keys, coefficient
           + (size_t)ip_tsize(cap) * 4 + (size_t)cap * 4   // join table (later the freed rows), row
           + (size_t)kIPSlotArrays * (kIPSlots + 1) * 4    // per-slot counters
           + (size_t)cap * 2 + (size_t)cap * 2;            // partner, slot + flag
  return (o + 15) & ~(size_t)15;
}

size_t inplace_lds_bytes(int W, int cap, bool energy) {
  return (energy ? (size_t)W * kGroupsPerWord * kLutEntries * 8 : 0) + kIPW * seg_bytes(W, cap);
}

int inplace_cap(int W, bool energy, size_t budget) {
  int cap = 512;
  while (cap > 8 && inplace_lds_bytes(W, cap, energy) > budget) cap -= 8;
  return cap;
}

template <int W>
struct Seg {
  uint64_t* ax;      // [W][cap]
  uint64_t* az;
  double* ac;        // [cap]
  int32_t* tab;      // [tsize] join table; afterwards the freed rows of every slot
  int32_t* arel;     // [cap] row of the entry relative to its bucket's first row
  int32_t* s_nnew;   // [kIPSlots + 1] new keys arriving in the slot
  int32_t* s_nhole;  // rows of the slot freed by compression
  int32_t* s_hfirst; // first freed row of the slot in the list
  int32_t* s_ctr;    // rows placed so far
  int16_t* partner;  // [cap]
  uint8_t* aslot;    // [cap]
  uint8_t* aflag;    // [cap]
  int cap, tsize;
};

template <int W>
__device__ __forceinline__ Seg<W> carve_seg(unsigned char* p, int cap) {
  Seg<W> g;
  size_t o = 0;
  g.ax = (uint64_t*)(p + o); o += (size_t)W * cap * 8;
  g.az = (uint64_t*)(p + o); o += (size_t)W * cap * 8;
  g.ac = (double*)(p + o); o += (size_t)cap * 8;
  g.tsize = ip_tsize(cap);
  g.tab = (int32_t*)(p + o); o += (size_t)g.tsize * 4;
  g.arel = (int32_t*)(p + o); o += (size_t)cap * 4;
  int32_t* sa = (int32_t*)(p + o); o += (size_t)kIPSlotArrays * (kIPSlots + 1) * 4;
  g.s_nnew = sa;
  g.s_nhole = sa + 1 * (kIPSlots + 1);
  g.s_hfirst = sa + 2 * (kIPSlots + 1);
  g.s_ctr = sa + 3 * (kIPSlots + 1);
  g.partner = (int16_t*)(p + o); o += (size_t)cap * 2;
  g.aslot = (uint8_t*)(p + o); o += (size_t)cap;
  g.aflag = (uint8_t*)(p + o);
  g.cap = cap;
  return g;
}

// LDS written by some lanes of this wave is read by others next.  The LDS
// unit executes one wave's operations in issue order, so only the compiler
// must not move LDS accesses across this point: a wavefront-scope fence (no
// wait instruction; a workgroup-scope fence would also wait for every
// outstanding global store of the wave).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t table_slot(uint32_t h, int tsize) {
  return (uint32_t)(((uint64_t)h * (uint32_t)tsize) >> 32);
}

__device__ __forceinline__ bool sorted_contains(const int32_t* h, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (h[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo < n && h[lo] == v;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(v, d, 64);
    if (lane >= d) v += y;
  }
  return v;
}

// Sum over the wave, returned as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return __builtin_amdgcn_readfirstlane(v);
}

struct Geo {
  uint32_t f;
  int thi, selfp, ppi;
  int64_t npairs, nitems;
};

// Bucket table entry of slot `lane` of a work item (lanes >= nslots: empty).
struct SlotDesc {
  int off = 0, cnt = 0, lim = 0;   // rows of an in-place store are below 2^31
  uint32_t b = 0;
  int nslots = 0;
};

// The item's buckets: slot s of pair k is bucket b0 (s = 2k) or b0 ^ f (s = 2k + 1),
// or b0 alone when f = 0.
__device__ __forceinline__ SlotDesc load_desc(const StoreDev& st, const Geo& G, int64_t it) {
  const int lane = threadIdx.x & 63;
  SlotDesc d;
  const int64_t q0 = it * G.ppi;
  const int64_t left = G.npairs - q0;
  const int np = (int)(left < G.ppi ? left : G.ppi);
  d.nslots = G.selfp ? np : 2 * np;
  if (lane < d.nslots) {
    const int64_t q = q0 + (G.selfp ? lane : (lane >> 1));
    uint32_t b0, b1;
    pair_buckets(q, G.f, G.thi, b0, b1);
    d.b = (!G.selfp && (lane & 1)) ? b1 : b0;
    d.off = (int)st.off[d.b];
    d.cnt = (int)st.cnt[d.b];
    d.lim = (int)st.lim[d.b];
  }
  return d;
}

// Per-lane (slot = lane) state of the item being processed.
struct Item {
  int off, cnt, room;   // first row, live rows, rows of the region (input layout)
  int noff;             // first row of the fresh region (relocated items)
  uint32_t b;
  int pre;              // flat index of the slot's first term
  int pre1;             // flat index of slot 1 (wave-uniform)
  int nslots, n;
};

// Slot of flat index i: the largest s < nslots with pre_s <= i, where lane s
// holds pre_s (non-decreasing, pre_0 = 0).  Called by the whole wave.
__device__ __forceinline__ int slot_of(const Item& I, int i) {
  if (I.nslots <= 2) return (I.nslots == 2 && i >= I.pre1) ? 1 : 0;
  int s = 0;
#pragma unroll
  for (int step = kIPSlots / 2; step; step >>= 1) {
    const int c = s + step;
    const int pc = __shfl(I.pre, c < kIPSlots ? c : kIPSlots - 1, 64);
    if (c < I.nslots && pc <= i) s = c;
  }
  return s;
}

// The item's per-lane state from its bucket table entries.
__device__ __forceinline__ Item make_item(const SlotDesc& d) {
  Item I;
  I.nslots = d.nslots;
  I.off = d.off;
  I.cnt = d.cnt;
  I.room = d.lim - d.off;
  I.b = d.b;
  I.noff = 0;
  const int incl = wave_incl_scan(I.cnt);
  I.pre = incl - I.cnt;
  I.n = __shfl(incl, 63, 64);
  I.pre1 = __shfl(I.pre, 1, 64);
  return I;
}

// U slices of 64 input terms of an item, loaded ahead of their use.
template <int W, int U>
struct Slices {
  uint64_t kx[U][W], kz[U][W];
  double kc[U];
  int slot[U], rel[U];
};

// Issue the loads of flat indices [base, base + 64 U) of item I.
template <int W, int U>
__device__ __forceinline__ void issue_slices(const StoreDev& st, const Item& I, int base, Slices<W, U>& S) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = base + 64 * u + lane;
    const bool valid = i < I.n;
    const int sl = slot_of(I, i);
    const int pre = __shfl(I.pre, sl, 64);
    const int off = __shfl(I.off, sl, 64);
    S.slot[u] = sl;
    S.rel[u] = i - pre;
    S.kc[u] = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) S.kx[u][w] = S.kz[u][w] = 0;
    if (valid) load_key<W>(st, (int64_t)off + S.rel[u], S.kx[u], S.kz[u], S.kc[u]);
  }
}

// Per-wavefront tallies of a step, kept in scalar registers: each is bounded
// by the store's rows (below 2^31) or by the number of work items.
struct WaveCounts {
  int anti = 0, fresh = 0, delta = 0, reloc = 0, freed = 0;
};

// Rows for the entries with `has` set, placed in their slot `d` in stash
// order.  MODE 0 (in place): first the slot's freed rows, in ascending order,
// then the rows after its live ones; MODE 1: the slot's fresh region.
// Lanes with the same d are consecutive (the stash and the scan are in
// slot-major order, and a new key goes to slot s ^ 1 or s), so a lane's rank
// is the slot's count so far plus the `has` lanes between the start of its
// run of equal d and itself; the last lane of each run advances the count.
// Lanes past the end of the data pass d = -1.
template <int W, int MODE>
__device__ __forceinline__ void put_rows(const StoreDev& st, const Seg<W>& g, const Item& I, bool has, int d,
                                         const uint64_t* kx, const uint64_t* kz, double c) {
  const int lane = threadIdx.x & 63;
  const uint64_t hm = __ballot(has);
  if (hm == 0) return;
  const int dprev = __shfl_up(d, 1, 64);
  const uint64_t heads = __ballot(lane == 0 || d != dprev);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);   // lanes <= this one
  const int start = 63 - __clzll(heads & upto);
  const uint64_t run_below = ((1ull << lane) - 1) & ~((1ull << start) - 1);
  const int before = __popcll(hm & run_below);
  const bool tail = lane == 63 || ((heads >> (lane + 1)) & 1);
  const int dd = d < 0 ? 0 : d;
  const int base = d >= 0 ? g.s_ctr[dd] : 0;
  const int o = __shfl(MODE == 0 ? I.off : I.noff, dd, 64);
  const int ct = __shfl(I.cnt, dd, 64);
  if (has) {
    const int rank = base + before;
    int64_t row;
    if (MODE == 0) {
      const int nh = g.s_nhole[dd];
      row = rank < nh ? (int64_t)o + g.tab[g.s_hfirst[dd] + rank] : (int64_t)o + ct + (rank - nh);
    } else {
      row = (int64_t)o + rank;
    }
    store_key<W>(st, row, kx, kz, c);
  }
  wave_sync();
  if (tail && d >= 0) g.s_ctr[dd] = base + before + (has ? 1 : 0);
  wave_sync();
}

// Classify U loaded slices (flat indices base + 64 u + lane):
//   mode 0: stash the anticommuting terms and the commuting terms that
//           compression drops (flag kFComm); energy of the commuting terms;
//   mode 1: put the kept commuting terms into the fresh regions, stash the
//           anticommuting terms of residue class `rem` mod `mod`;
//   mode 2: stash the anticommuting terms of class `rem` only.
// nst counts the stash candidates (entries beyond cap are not written); nanti
// the anticommuting terms.
template <int W, bool ENERGY, int U>
__device__ __forceinline__ void classify_slices(const StoreDev& st, const Entangler& P, double eps, int delta,
                                                const double* lut, const Seg<W>& g, const Item& I, int base,
                                                const Slices<W, U>& S, int mode, uint32_t mod, uint32_t rem,
                                                double& eacc, int& nst, int& nanti) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const bool valid = base + 64 * u + lane < I.n;
    const bool anti = valid && anticommutes<W>(S.kx[u], S.kz[u], P.px, P.pz);
    nanti += (int)__popcll(__ballot(anti));
    const bool comm_drop = valid && !anti && fabs(S.kc[u]) < eps;
    const bool comm_keep = valid && !anti && !comm_drop;
    bool stash = anti;
    if (anti && mode != 0 && mod > 1)
      stash = (round_hash(rep_hash<W>(P, S.kx[u], S.kz[u])) & (mod - 1)) == rem;
    uint8_t flag = 0;
    if (mode == 0 && comm_drop) {
      stash = true;
      flag = kFComm;
    }
    if (ENERGY && mode == 0) {
      // commuting terms: every kept one, or (delta) only those compression drops
      if (delta ? comm_drop : comm_keep) {
        const double ek = expect_lut<W>(lut, S.kx[u], S.kz[u]);
        eacc += comm_drop ? -(S.kc[u] * ek) : S.kc[u] * ek;
      }
    }
    if (mode == 1) put_rows<W, 1>(st, g, I, comm_keep, valid ? S.slot[u] : -1, S.kx[u], S.kz[u], S.kc[u]);
    const uint64_t bm = __ballot(stash);
    const int pos = nst + (int)lanes_below(bm);
    if (stash && pos < g.cap) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        g.ax[w * g.cap + pos] = S.kx[u][w];
        g.az[w * g.cap + pos] = S.kz[u][w];
      }
      g.ac[pos] = S.kc[u];
      g.arel[pos] = S.rel[u];
      g.aslot[pos] = (uint8_t)S.slot[u];
      g.aflag[pos] = flag;
    }
    nst += (int)__popcll(bm);
  }
}

// One pass over the item's input terms from flat index `from` on, U slices
// per iteration (their loads in flight before any is classified).
template <int W, bool ENERGY, int U>
__device__ void item_scan(const StoreDev& st, const Entangler& P, double eps, int delta, const double* lut,
                          const Seg<W>& g, const Item& I, int from, int mode, uint32_t mod, uint32_t rem,
                          double& eacc, int& nst, int& nanti) {
  for (int base = from; base < I.n; base += 64 * U) {
    Slices<W, U> S;
    issue_slices<W, U>(st, I, base, S);
    classify_slices<W, ENERGY, U>(st, P, eps, delta, lut, g, I, base, S, mode, mod, rem, eacc, nst, nanti);
  }
}

template <int W>
__device__ __forceinline__ void entry_key(const Seg<W>& g, int i, uint64_t* kx, uint64_t* kz) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    kx[w] = g.ax[w * g.cap + i];
    kz[w] = g.az[w * g.cap + i];
  }
}

// Pair each stashed anticommuting K with K^P: the members whose pivot bit is
// 0 go into the table, the others look up K^P.  A table entry holds the
// stash index in its low 16 bits and the low 16 bits of the key's hash above
// them (the slot comes from the high bits), so a probe that meets another key
// is mostly rejected without reading its words (-1 marks an empty entry; the
// stash holds at most 512 entries).
template <int W>
__device__ void item_join(const Entangler& P, const Seg<W>& g, int n) {
  const int lane = threadIdx.x & 63;
  for (int i = lane; i < g.tsize; i += 64) g.tab[i] = -1;
  for (int i = lane; i < n; i += 64) g.partner[i] = -1;
  wave_sync();
  for (int i = lane; i < n; i += 64) {
    if (g.aflag[i] & kFComm) continue;
    uint64_t kx[W], kz[W];
    entry_key<W>(g, i, kx, kz);
    if (pivot_of<W>(P, kx, kz)) continue;
    const uint32_t hk = table_hash<W>(kx, kz);
    const int32_t e = (int32_t)((hk << 16) | (uint32_t)i);
    uint32_t h = table_slot(hk, g.tsize);
    while (atomicCAS(&g.tab[h], -1, e) != -1) h = (h + 1 == (uint32_t)g.tsize) ? 0 : h + 1;
  }
  wave_sync();
  for (int i = lane; i < n; i += 64) {
    if (g.aflag[i] & kFComm) continue;
    uint64_t kx[W], kz[W];
    entry_key<W>(g, i, kx, kz);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      kx[w] ^= P.px[w];
      kz[w] ^= P.pz[w];
    }
    if (pivot_of<W>(P, kx, kz)) continue;   // the pivot bit of K is 0: K is in the table
    const uint32_t hk = table_hash<W>(kx, kz);
    const uint32_t fp = hk << 16;
    uint32_t h = table_slot(hk, g.tsize);
    for (;;) {
      const int32_t e = g.tab[h];
      if (e == -1) break;
      if (((uint32_t)e & 0xFFFF0000u) == fp) {
        const int j = e & 0xFFFF;
        bool eq = true;
#pragma unroll
        for (int w = 0; w < W; ++w) eq = eq && g.ax[w * g.cap + j] == kx[w] && g.az[w * g.cap + j] == kz[w];
        if (eq) {
          g.partner[i] = (int16_t)j;
          g.partner[j] = (int16_t)i;
          break;
        }
      }
      h = (h + 1 == (uint32_t)g.tsize) ? 0 : h + 1;
    }
  }
  wave_sync();
}

// Output values of stash entry i (an anticommuting term K with coefficient a):
// own = RN(cos tau a) + RN(s_{K^P} sin tau a_{K^P}) when K^P is present, else
// RN(cos tau a) together with the new term K^P of value s_K RN(sin tau a),
// where s_A = +1 when P A = i^3 (A^P) and -1 when P A = i^1 (A^P).
template <int W>
__device__ __forceinline__ void entry_values(const Entangler& P, double C, double S, const Seg<W>& g, int i,
                                             const uint64_t* kx, const uint64_t* kz, double& a,
                                             double& v_own, double& v_new, bool& paired) {
  a = g.ac[i];
  const int j = g.partner[i];
  const double rot = __dmul_rn(C, a);
  paired = j >= 0;
  if (paired) {
    uint64_t jx[W], jz[W];
    entry_key<W>(g, j, jx, jz);
    const int ej = product_phase<W>(P.px, P.pz, jx, jz);
    const double sj = __dmul_rn(S, g.ac[j]);
    v_own = __dadd_rn(rot, ej == 3 ? sj : -sj);
    v_new = 0.0;
  } else {
    v_own = rot;
    const int e = product_phase<W>(P.px, P.pz, kx, kz);
    const double si = __dmul_rn(S, a);
    v_new = e == 3 ? si : -si;
  }
}

// In-place path, first emission pass: which entries free their row and which
// add a new key, and how many per slot.
template <int W>
__device__ void count_outputs(const Entangler& P, double C, double S, double eps, const Seg<W>& g, int n,
                              int selfp) {
  const int lane = threadIdx.x & 63;
  for (int i = lane; i < n; i += 64) {
    uint8_t fl = g.aflag[i];
    const int s = g.aslot[i];
    if (fl & kFComm) {
      fl |= kFHole;
    } else {
      uint64_t kx[W], kz[W];
      entry_key<W>(g, i, kx, kz);
      double a, vo, vn;
      bool paired;
      entry_values<W>(P, C, S, g, i, kx, kz, a, vo, vn, paired);
      if (fabs(vo) < eps) fl |= kFHole;
      if (!paired && !(fabs(vn) < eps)) {
        fl |= kFNew;
        atomicAdd(&g.s_nnew[selfp ? s : s ^ 1], 1);
      }
    }
    if (fl & kFHole) atomicAdd(&g.s_nhole[s], 1);
    g.aflag[i] = fl;
  }
  wave_sync();
}

// The freed rows of every slot, ascending within the slot (the stash is in
// flat order: slot-major, rows ascending), into g.tab; returns their number.
template <int W>
__device__ int list_holes(const Seg<W>& g, const Item& I, int n) {
  const int lane = threadIdx.x & 63;
  const int h = lane < I.nslots ? g.s_nhole[lane] : 0;
  const int incl = wave_incl_scan(h);
  const int total = __shfl(incl, 63, 64);
  if (total == 0) return 0;
  if (lane < I.nslots) g.s_hfirst[lane] = incl - h;
  int k = 0;
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int i = i0 + lane;
    const bool ho = i < n && (g.aflag[i] & kFHole);
    const uint64_t bm = __ballot(ho);
    if (ho) g.tab[k + (int)lanes_below(bm)] = g.arel[i];
    k += (int)__popcll(bm);
  }
  wave_sync();
  return total;
}

// In-place path, second emission pass: rotated coefficients into their own
// rows, new keys into the partner slot (freed rows first), energy.
template <int W, bool ENERGY>
__device__ void emit_inplace(const StoreDev& st, const Entangler& P, double C, double S, int delta,
                             const double* lut, const Seg<W>& g, const Item& I, int n, int selfp,
                             double& eacc) {
  const int lane = threadIdx.x & 63;
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int i = i0 + lane;
    const bool valid = i < n;
    const uint8_t fl = valid ? g.aflag[i] : (uint8_t)0;
    const bool live = valid && !(fl & kFComm);
    const int s = valid ? g.aslot[i] : 0;
    const int off = __shfl(I.off, s, 64);
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) kx[w] = kz[w] = 0;
    double a = 0.0, vo = 0.0, vn = 0.0;
    if (live) {
      entry_key<W>(g, i, kx, kz);
      bool paired;
      entry_values<W>(P, C, S, g, i, kx, kz, a, vo, vn, paired);
      if (!(fl & kFHole)) st.c[(int64_t)off + g.arel[i]] = vo;
      if (ENERGY) {
        double ek, ekp;
        expect_split<W>(lut, P, kx, kz, ek, ekp);
        if (!(fl & kFHole)) eacc += vo * ek;
        if (fl & kFNew) eacc += vn * ekp;
        if (delta) eacc -= a * ek;
      }
    }
    uint64_t qx[W], qz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      qx[w] = kx[w] ^ P.px[w];
      qz[w] = kz[w] ^ P.pz[w];
    }
    put_rows<W, 0>(st, g, I, live && (fl & kFNew), valid ? (selfp ? s : s ^ 1) : -1, qx, qz, vn);
  }
  wave_sync();
}

// Slots that lost more rows than new keys arrived: the live rows at or above
// the slot's new count move, in order, into the freed rows below it that no
// new key took.  A moved row is either an anticommuting term of the stash
// (its new coefficient is recomputed from the stash) or a commuting term that
// this step has not written (read from the store).  The windows [fin, cnt) of
// all such slots are walked together, 64 rows per pass (one lane per row,
// slot-major, so the lanes of one slot are consecutive); a row's destination
// is the slot's freed row number nn + (live rows of its window below it).
// Reads are at rows >= fin and writes below fin, so no row is read after it
// is overwritten.
template <int W>
__device__ void refill(const StoreDev& st, const Entangler& P, double C, double S, const Seg<W>& g,
                       const Item& I, int n) {
  const int lane = threadIdx.x & 63;
  // lane s: the length of slot s's window and the slot's stash range
  // (the stash is slot-major: aslot is non-decreasing)
  int len = 0, e0 = 0, e1 = 0;
  if (lane < I.nslots) {
    const int nh = g.s_nhole[lane], nn = g.s_nnew[lane];
    len = nh > nn ? nh - nn : 0;
    if (len) {
      int lo = 0, hi = n;
      while (lo < hi) { const int m = (lo + hi) >> 1; if (g.aslot[m] < lane) lo = m + 1; else hi = m; }
      e0 = lo;
      hi = n;
      while (lo < hi) { const int m = (lo + hi) >> 1; if (g.aslot[m] <= lane) lo = m + 1; else hi = m; }
      e1 = lo;
    }
    g.s_ctr[lane] = 0;
  }
  const int incl = wave_incl_scan(len);
  const int pre = incl - len;
  const int total = __shfl(incl, 63, 64);
  wave_sync();
  for (int f0 = 0; f0 < total; f0 += 64) {
    const int f = f0 + lane;
    const bool act = f < total;
    // the slot of f: the largest s < nslots with pre_s <= f
    int s = 0;
#pragma unroll
    for (int step = kIPSlots / 2; step; step >>= 1) {
      const int cand = s + step;
      const int pc = __shfl(pre, cand < kIPSlots ? cand : kIPSlots - 1, 64);
      if (cand < I.nslots && pc <= f) s = cand;
    }
    const int ps = __shfl(pre, s, 64);
    const int cnt = __shfl(I.cnt, s, 64);
    const int off = __shfl(I.off, s, 64);
    const int se0 = __shfl(e0, s, 64), se1 = __shfl(e1, s, 64);
    const int nh = g.s_nhole[s], nn = g.s_nnew[s];
    const int32_t* H = g.tab + g.s_hfirst[s];
    const int r = cnt - (nh - nn) + (f - ps);
    const bool lv = act && !sorted_contains(H, nh, r);
    // rank among the live rows of the slot: its count so far plus the live
    // lanes between the start of its run of equal slots and this lane
    const int d = act ? s : -1;
    const uint64_t hm = __ballot(lv);
    const int dprev = __shfl_up(d, 1, 64);
    const uint64_t heads = __ballot(lane == 0 || d != dprev);
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    const int start = 63 - __clzll(heads & upto);
    const uint64_t run_below = ((1ull << lane) - 1) & ~((1ull << start) - 1);
    const int before = __popcll(hm & run_below);
    const bool tail = lane == 63 || ((heads >> (lane + 1)) & 1);
    const int base = act ? g.s_ctr[s] : 0;
    if (lv) {
      const int dst = H[nn + base + before];
      int a0 = se0, a1 = se1;   // stash entry with row r (rows ascend within the slot)
      while (a0 < a1) { const int m = (a0 + a1) >> 1; if (g.arel[m] < r) a0 = m + 1; else a1 = m; }
      uint64_t kx[W], kz[W];
      double c;
      if (a0 < se1 && g.arel[a0] == r) {
        entry_key<W>(g, a0, kx, kz);
        double a, vn;
        bool paired;
        entry_values<W>(P, C, S, g, a0, kx, kz, a, c, vn, paired);
      } else {
        load_key<W>(st, (int64_t)off + r, kx, kz, c);
      }
      store_key<W>(st, (int64_t)off + dst, kx, kz, c);
    }
    wave_sync();
    if (tail && act) g.s_ctr[s] = base + before + (lv ? 1 : 0);
    wave_sync();
  }
}

template <int W, bool ENERGY>
__device__ bool relocate_item(const StoreDev& st, const Entangler& P, const InplaceConfig& cfg,
                              const double* lut, const Seg<W>& g, Item& I, int selfp, int nanti,
                              double& eacc, WaveCounts& wc) {
  const int lane = threadIdx.x & 63;
  // fresh regions from the pool: own rows + the partner's (worst case output)
  const int cp = __shfl(I.cnt, selfp ? lane : (lane ^ 1), 64);
  const int need = lane < I.nslots ? ((I.cnt + cp + 15) & ~15) : 0;
  const int incl = wave_incl_scan(need);
  const int total = __shfl(incl, 63, 64);
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd((unsigned long long*)st.top, (unsigned long long)total);
  base = wave_bcast0(base);
  if ((int64_t)base + total > st.cap) {
    if (lane == 0) atomicOr(st.err, 1);
    return false;
  }
  I.noff = (int)(base + (incl - need));
  // residue classes of a hash of the pair representative (both members of a
  // {K, K^P} pair share the class), about cap/4 terms each; if a class still
  // overflows the stash, the item is redone with twice as many classes (the
  // fresh regions are rewritten from their start)
  uint32_t R = 1;
  while ((int64_t)R * (g.cap / 4) < nanti && R < (1u << 20)) R <<= 1;
  for (;;) {
    double e_try = 0.0;
    int fresh_try = 0;
    if (lane < I.nslots) g.s_ctr[lane] = 0;
    wave_sync();
    bool ok = true;
    for (uint32_t r = 0; r < R; ++r) {
      // one slice at a time: the next item's slices may be in flight
      int nst = 0, na = 0;
      item_scan<W, ENERGY, 1>(st, P, cfg.eps, cfg.delta, lut, g, I, 0, r == 0 ? 1 : 2, R, r, e_try, nst, na);
      wave_sync();
      if (nst > g.cap) {
        ok = false;
        break;
      }
      item_join<W>(P, g, nst);
      // every kept output into the fresh region of its slot
      for (int i0 = 0; i0 < nst; i0 += 64) {
        const int i = i0 + lane;
        const bool valid = i < nst;
        const int s = valid ? g.aslot[i] : 0;
        uint64_t kx[W], kz[W];
#pragma unroll
        for (int w = 0; w < W; ++w) kx[w] = kz[w] = 0;
        double a = 0.0, vo = 0.0, vn = 0.0;
        bool paired = true;
        if (valid) {
          entry_key<W>(g, i, kx, kz);
          entry_values<W>(P, cfg.C, cfg.S, g, i, kx, kz, a, vo, vn, paired);
        }
        const bool keep_own = valid && !(fabs(vo) < cfg.eps);
        const bool keep_new = valid && !paired && !(fabs(vn) < cfg.eps);
        if (ENERGY && valid) {
          double ek, ekp;
          expect_split<W>(lut, P, kx, kz, ek, ekp);
          if (keep_own) e_try += vo * ek;
          if (keep_new) e_try += vn * ekp;
          if (cfg.delta) e_try -= a * ek;
        }
        fresh_try += __popcll(__ballot(keep_new));
        put_rows<W, 1>(st, g, I, keep_own, valid ? s : -1, kx, kz, vo);
        uint64_t qx[W], qz[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
          qx[w] = kx[w] ^ P.px[w];
          qz[w] = kz[w] ^ P.pz[w];
        }
        put_rows<W, 1>(st, g, I, keep_new, valid ? (selfp ? s : s ^ 1) : -1, qx, qz, vn);
      }
      wave_sync();
    }
    if (ok) {
      eacc += e_try;
      wc.fresh += fresh_try;
      break;
    }
    if (R >= (1u << 20)) {
      if (lane == 0) atomicOr(st.err, 4);
      return false;
    }
    R <<= 1;
  }
  int dl = 0;
  if (lane < I.nslots) {
    const int cnt_new = g.s_ctr[lane];
    st.off[I.b] = I.noff;
    st.lim[I.b] = (int64_t)I.noff + need;
    st.cnt[I.b] = cnt_new;
    dl = cnt_new - I.cnt;
  }
  wc.delta += wave_sum(dl);
  wc.reloc += 1;
  return true;
}

// One work item.  S holds the loads of its first kIPU slices, issued while
// the previous item was processed; once this item's input is stashed, the
// loads of the next item's first slices (item In, from descriptor dn) are
// issued into S, so they are in flight while this item is joined and emitted.
template <int W, bool ENERGY>
__device__ void process_item(const StoreDev& st, const Entangler& P, const InplaceConfig& cfg, const Geo& G,
                             const double* lut, const Seg<W>& g, Item& I, Slices<W, kIPU>& S, bool have_next,
                             const SlotDesc& dn, Item& In, double& eacc, WaveCounts& wc) {
  const int lane = threadIdx.x & 63;
  if (I.n == 0) {
    if (have_next) {
      In = make_item(dn);
      issue_slices<W, kIPU>(st, In, 0, S);
    }
    return;
  }
  if (lane < I.nslots) {
    g.s_nnew[lane] = 0;
    g.s_nhole[lane] = 0;
    g.s_ctr[lane] = 0;
  }
  wave_sync();
  int nst = 0, nanti = 0;
  classify_slices<W, ENERGY, kIPU>(st, P, cfg.eps, cfg.delta, lut, g, I, 0, S, 0, 1, 0, eacc, nst, nanti);
  item_scan<W, ENERGY, kIPU>(st, P, cfg.eps, cfg.delta, lut, g, I, 64 * kIPU, 0, 1, 0, eacc, nst, nanti);
  wave_sync();
  if (have_next) {
    In = make_item(dn);
    issue_slices<W, kIPU>(st, In, 0, S);
  }
  wc.anti += nanti;
  if (nst > g.cap) {
    relocate_item<W, ENERGY>(st, P, cfg, lut, g, I, G.selfp, nanti, eacc, wc);
    return;
  }
  item_join<W>(P, g, nst);
  count_outputs<W>(P, cfg.C, cfg.S, cfg.eps, g, nst, G.selfp);
  int nn = 0, nh = 0;
  bool fits = true;
  if (lane < I.nslots) {
    nn = g.s_nnew[lane];
    nh = g.s_nhole[lane];
    fits = I.cnt + (nn > nh ? nn - nh : 0) <= I.room;
  }
  if (__ballot(!fits)) {
    relocate_item<W, ENERGY>(st, P, cfg, lut, g, I, G.selfp, nanti, eacc, wc);
    return;
  }
  const int freed = list_holes<W>(g, I, nst);
  emit_inplace<W, ENERGY>(st, P, cfg.C, cfg.S, cfg.delta, lut, g, I, nst, G.selfp, eacc);
  if (__ballot(nh > nn)) refill<W>(st, P, cfg.C, cfg.S, g, I, nst);
  if (lane < I.nslots) st.cnt[I.b] = I.cnt + nn - nh;
  wc.delta += wave_sum(nn - nh);
  wc.fresh += wave_sum(nn);
  wc.freed += __builtin_amdgcn_readfirstlane(freed);
}

template <int W, bool ENERGY>
__global__ __launch_bounds__(kIPB) void k_dress_inplace(StoreDev st, Entangler P, InplaceConfig cfg) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: segment pointers stay scalar
  const int lane = threadIdx.x & 63;
  const size_t lut_bytes = ENERGY ? (size_t)W * kGroupsPerWord * kLutEntries * 8 : 0;
  double* lut = (double*)smem;
  if (ENERGY) {
    // the 3-qubit group table of the QMF state, built in LDS from the angles;
    // the per-qubit factors sit in the (not yet used) wave segments
    double* fq = (double*)(smem + lut_bytes);
    for (int q = threadIdx.x; q < 64 * W; q += kIPB) {
      double st_ = 0.0, ct = 1.0, sp = 0.0, cp = 1.0;
      if (q < cfg.nq) {
        sincos(cfg.theta[q], &st_, &ct);
        sincos(cfg.phi[q], &sp, &cp);
      }
#pragma unroll
      for (int op = 0; op < 4; ++op) fq[4 * q + op] = bloch_factor(op, st_, ct, sp, cp);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < W * kGroupsPerWord * kLutEntries; i += kIPB) {
      const int code = i % kLutEntries, gi = i / kLutEntries;
      const int h = gi / kGroupsPerHalf, gg = gi % kGroupsPerHalf;
      double p = 1.0;
      for (int r = 0; r < 3; ++r) {
        const int bit = 3 * gg + r, q = 32 * h + bit;
        if (bit >= 32 || q >= cfg.nq) continue;
        const int op = ((code >> r) & 1) | (((code >> (3 + r)) & 1) << 1);
        if (op != 0) p *= fq[4 * q + op];
      }
      lut[i] = p;
    }
  }
  __syncthreads();
  const Seg<W> g = carve_seg<W>(smem + lut_bytes + (size_t)wave * seg_bytes(W, cfg.cap), cfg.cap);
  const int64_t gw = (int64_t)blockIdx.x * kIPW + wave;
  double eacc = 0.0;
  WaveCounts wc;
  if (*st.err == 0) {
    const int m = *st.m;
    const int64_t n_in = *st.total;
    Geo G;
    const uint32_t mask = (uint32_t)((1ull << m) - 1);
    G.f = P.hp & mask;
    G.selfp = G.f == 0;
    G.thi = G.f ? 31 - __clz(G.f) : 0;
    G.npairs = G.f ? (1ll << (m - 1)) : (1ll << m);
    const int64_t mean = (n_in >> m) > 0 ? (n_in >> m) : 1;
    const int64_t pair_terms = G.selfp ? mean : 2 * mean;
    const int maxp = G.selfp ? kIPSlots : kIPSlots / 2;
    int ppi = 1;
    while (ppi * 2 <= maxp && (int64_t)ppi * 2 * pair_terms <= cfg.item_terms) ppi *= 2;
    G.ppi = ppi;
    G.nitems = (G.npairs + ppi - 1) / ppi;
    const int64_t nw = (int64_t)gridDim.x * kIPW;
    // bucket tables two items ahead, term slices one item ahead
    SlotDesc d_next;
    if (gw + nw < G.nitems) d_next = load_desc(st, G, gw + nw);
    Item I;
    Slices<W, kIPU> S;
    if (gw < G.nitems) {
      I = make_item(load_desc(st, G, gw));
      issue_slices<W, kIPU>(st, I, 0, S);
    }
    for (int64_t it = gw; it < G.nitems; it += nw) {
      const bool have_next = it + nw < G.nitems;
      const SlotDesc dn = d_next;
      if (it + 2 * nw < G.nitems) d_next = load_desc(st, G, it + 2 * nw);
      Item In;
      process_item<W, ENERGY>(st, P, cfg, G, lut, g, I, S, have_next, dn, In, eacc, wc);
      I = In;
    }
  }
  // per-wavefront counts (summed by k_inplace_end, no atomics)
  if (lane == 0) {
    int64_t* c = cfg.counts + 5 * gw;
    c[0] = wc.anti;
    c[1] = wc.fresh;
    c[2] = wc.delta;
    c[3] = wc.reloc;
    c[4] = wc.freed;
  }
  if (ENERGY) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) eacc += __shfl_down(eacc, d, 64);
    if (lane == 0) cfg.e_partial[gw] = eacc;
  }
}

// Finishes a step in one workgroup: sums the per-wavefront counts into the
// store's counters (integer sums) and the energy partials in a fixed order
// (each thread a strided share, then the lane tree and the waves in order).
__global__ __launch_bounds__(kBlock) void k_inplace_end(StoreDev st, const int64_t* counts,
                                                        const double* e_partial, int nparts,
                                                        const double* energy_in, double* energy_out) {
  __shared__ double red[kWaves];
  __shared__ unsigned long long s_cnt[5];
  if (threadIdx.x < 5) s_cnt[threadIdx.x] = 0ull;
  __syncthreads();
  unsigned long long mine[5] = {0ull, 0ull, 0ull, 0ull, 0ull};
  double e = 0.0;
  // four strided partials per round, their loads issued together; the
  // energy adds stay in increasing partial order
  constexpr int kU = 4;
  for (int i0 = threadIdx.x; i0 < nparts; i0 += kU * kBlock) {
    int64_t cv[kU][5];
    double ev[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * kBlock;
      const bool ok = i < nparts;
#pragma unroll
      for (int k = 0; k < 5; ++k) cv[u][k] = ok ? counts[5 * i + k] : 0;
      ev[u] = (ok && energy_out) ? e_partial[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
#pragma unroll
      for (int k = 0; k < 5; ++k) mine[k] += (unsigned long long)cv[u][k];
      if (i0 + u * kBlock < nparts && energy_out) e += ev[u];
    }
  }
#pragma unroll
  for (int k = 0; k < 5; ++k)
    if (mine[k]) atomicAdd(&s_cnt[k], mine[k]);
  const double es = block_sum(e, red);   // also orders the LDS adds above
  if (threadIdx.x == 0) {
    st.stats[0] = (int64_t)s_cnt[0];
    st.stats[1] = (int64_t)s_cnt[1];
    st.aux[0] = (int64_t)s_cnt[2];
    st.aux[3] = (int64_t)s_cnt[3];
    st.aux[4] = (int64_t)s_cnt[4];
    *st.total += (int64_t)s_cnt[2];
    if (energy_out) *energy_out = energy_in ? *energy_in + es : es;
  }
}

template <int W, bool E>
static void launch_inplace_t(const StoreDev& st, const Entangler& P, const InplaceConfig& cfg, int grid,
                             hipStream_t s) {
  const size_t lds = inplace_lds_bytes(W, cfg.cap, E);
  (void)hipFuncSetAttribute((const void*)k_dress_inplace<W, E>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL((k_dress_inplace<W, E>), dim3(grid), dim3(kIPB), lds, s, st, P, cfg);
}

void launch_dress_inplace(int W, const StoreDev& st, const Entangler& P, const InplaceConfig& cfg, int grid,
                          const double* energy_in, double* energy_out, hipStream_t s) {
  const bool e = cfg.theta != nullptr;
  switch (W) {
    case 1: e ? launch_inplace_t<1, true>(st, P, cfg, grid, s) : launch_inplace_t<1, false>(st, P, cfg, grid, s); break;
    case 2: e ? launch_inplace_t<2, true>(st, P, cfg, grid, s) : launch_inplace_t<2, false>(st, P, cfg, grid, s); break;
    case 3: e ? launch_inplace_t<3, true>(st, P, cfg, grid, s) : launch_inplace_t<3, false>(st, P, cfg, grid, s); break;
    default: e ? launch_inplace_t<4, true>(st, P, cfg, grid, s) : launch_inplace_t<4, false>(st, P, cfg, grid, s); break;
  }
  hipLaunchKernelGGL(k_inplace_end, dim3(1), dim3(kBlock), 0, s, st, cfg.counts, cfg.e_partial,
                     grid * kIPW, energy_in, energy_out);
}

int inplace_waves_per_block() { return kIPW; }

}  // namespace iqcc
