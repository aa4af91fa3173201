// Term-store kernels: load (bucket partition), export (compaction), scans.
//
// Bucket partition = the single-device form of the bit-wise partitioning of
// App. B: a term's bucket is the low m bits of a GF(2)-linear hash of its key.
#include "iqcc_internal.h"

namespace iqcc {

__global__ void k_zero_counters(StoreDev st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *st.total = 0;
    *st.top = 0;
    *st.err = 0;
    st.stats[0] = 0;
    st.stats[1] = 0;
  }
}

void launch_zero_counters(StoreDev out, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, out);
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static void fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, n, v);
}

// ---------------------------------------------------------------------------
// Exclusive scan of int64 (three passes: block sums, scan of sums, apply).
// scratch: ceil(n/1024) + 1 int64.
// ---------------------------------------------------------------------------
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__global__ void k_scan_blocksum(const int64_t* in, int64_t n, int64_t* sums) {
  __shared__ uint64_t tmp[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + (int64_t)threadIdx.x * kScanItems + r;
    if (i < n) s += in[i];
  }
  uint64_t total;
  block_exclusive_scan((uint64_t)s, tmp, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = (int64_t)total;
}

__global__ void k_scan_sums(int64_t* sums, int64_t nb) {
  __shared__ uint64_t tmp[kWaves];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
    int64_t i = b0 + threadIdx.x;
    int64_t v = i < nb ? sums[i] : 0;
    uint64_t total;
    uint64_t ex = block_exclusive_scan((uint64_t)v, tmp, total);
    int64_t c0 = carry;
    if (i < nb) sums[i] = c0 + (int64_t)ex;
    __syncthreads();
    if (threadIdx.x == 0) carry = c0 + (int64_t)total;
    __syncthreads();
  }
}

__global__ void k_scan_apply(const int64_t* in, int64_t* out, int64_t n, const int64_t* sums) {
  __shared__ uint64_t tmp[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t v[kScanItems];
  int64_t s = 0;
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + (int64_t)threadIdx.x * kScanItems + r;
    v[r] = i < n ? in[i] : 0;
    s += v[r];
  }
  uint64_t total;
  int64_t ex = (int64_t)block_exclusive_scan((uint64_t)s, tmp, total) + sums[blockIdx.x];
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + (int64_t)threadIdx.x * kScanItems + r;
    if (i < n) out[i] = ex;
    ex += v[r];
  }
}

void launch_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* scratch,
                     hipStream_t s) {
  if (n <= 0) return;
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_blocksum, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, scratch);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, scratch, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n, scratch);
}

// ---------------------------------------------------------------------------
// Load: flat rows -> bucketed store.
// ---------------------------------------------------------------------------
template <int W>
__global__ void k_load_hist(const uint64_t* __restrict__ x, const uint64_t* __restrict__ z,
                            int64_t n, int64_t ld, uint32_t mask, int64_t* cnt) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      kx[w] = x[w * ld + i];
      kz[w] = z[w * ld + i];
    }
    uint32_t b = bucket_hash<W>(kx, kz) & mask;
    atomicAdd((unsigned long long*)&cnt[b], 1ull);
  }
}

// Load, second pass: the input index of every term into its bucket's slot
// list (lists packed at poff); the order inside a list follows the atomics
// and is undone by the third pass.  err (optional): skip when it is set.
template <int W>
__global__ void k_load_slots(const uint64_t* __restrict__ x, const uint64_t* __restrict__ z, int64_t n,
                             int64_t ld, uint32_t mask, const int64_t* poff, int64_t* fill, int64_t* slots,
                             const int* err) {
  if (err && *err) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      kx[w] = x[w * ld + i];
      kz[w] = z[w * ld + i];
    }
    const uint32_t b = bucket_hash<W>(kx, kz) & mask;
    slots[poff[b] + (int64_t)atomicAdd((unsigned long long*)&fill[b], 1ull)] = i;
  }
}

__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int t) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, t);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), t);
  return ((uint64_t)hi << 32) | lo;
}

// -1, 0 or +1 as a is below, equal to or above b; `ord` carries the verdict of
// the more significant words.
__device__ __forceinline__ int cmp_next(int ord, uint64_t a, uint64_t b) {
  return ord ? ord : (a < b ? -1 : (a > b ? 1 : 0));
}

// Load, third pass: one wavefront per bucket writes the bucket's terms in
// ascending key order (x words, then z words, most significant first; ties,
// which a valid input does not have, by input index), so a loaded store's
// rows depend only on the terms, not on the order of the second pass's
// atomics or of the input.  A term's row is off_b plus the number of the
// bucket's terms that precede it; candidates are broadcast from lane
// registers 64 at a time, O(cnt^2 / 64) steps per bucket.  Terms are read
// from the input and written to the store, so no row is overwritten early.
template <int W>
__global__ void k_load_place(const uint64_t* __restrict__ x, const uint64_t* __restrict__ z,
                             const double* __restrict__ c, int64_t ld, int64_t B, const int64_t* poff,
                             const int64_t* slots, StoreDev st, int guarded) {
  if (guarded && *st.err) return;   // the regions do not fit the arena: write nothing
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int nw = (int)(gridDim.x * (blockDim.x >> 6));
  for (int64_t b = wid; b < B; b += nw) {
    const int64_t cnt = st.cnt[b], base = poff[b], out = st.off[b];
    for (int64_t j0 = 0; j0 < cnt; j0 += 64) {
      const bool has = j0 + lane < cnt;
      int64_t ij = 0;
      uint64_t jx[W], jz[W];
#pragma unroll
      for (int w = 0; w < W; ++w) jx[w] = jz[w] = 0;
      if (has) {
        ij = slots[base + j0 + lane];
#pragma unroll
        for (int w = 0; w < W; ++w) {
          jx[w] = x[w * ld + ij];
          jz[w] = z[w * ld + ij];
        }
      }
      int64_t rank = 0;
      for (int64_t k0 = 0; k0 < cnt; k0 += 64) {
        int64_t ik = 0;
        uint64_t kx[W], kz[W];
#pragma unroll
        for (int w = 0; w < W; ++w) kx[w] = kz[w] = 0;
        if (k0 + lane < cnt) {
          ik = slots[base + k0 + lane];
#pragma unroll
          for (int w = 0; w < W; ++w) {
            kx[w] = x[w * ld + ik];
            kz[w] = z[w * ld + ik];
          }
        }
        const int kn = (int)(cnt - k0 < 64 ? cnt - k0 : 64);
        for (int t = 0; t < kn; ++t) {
          int ord = 0;
#pragma unroll
          for (int w = W - 1; w >= 0; --w) ord = cmp_next(ord, lane_u64(kx[w], t), jx[w]);
#pragma unroll
          for (int w = W - 1; w >= 0; --w) ord = cmp_next(ord, lane_u64(kz[w], t), jz[w]);
          ord = cmp_next(ord, lane_u64((uint64_t)ik, t), (uint64_t)ij);
          rank += ord < 0;
        }
      }
      if (has) {
        const int64_t row = out + rank;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          st.x[w * st.cap + row] = jx[w];
          st.z[w * st.cap + row] = jz[w];
        }
        st.c[row] = c[ij];
      }
    }
  }
}

// The second and third passes of a load (the bucket counts, their packed
// offsets poff and the rows' offsets st.off are in place).
static void load_place_rows(int W, StoreDev st, const uint64_t* x, const uint64_t* z, const double* c,
                            int64_t n, int64_t ld, uint32_t mask, int64_t B, const int64_t* poff,
                            int64_t* fill, int64_t* slots, bool guarded, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  const int* err = guarded ? st.err : nullptr;
  int64_t pb = (B + kWaves - 1) / kWaves;
  if (pb > 8192) pb = 8192;
  const int g = guarded ? 1 : 0;
  switch (W) {
    case 1:
      hipLaunchKernelGGL(k_load_slots<1>, dim3(blocks), dim3(kBlock), 0, s, x, z, n, ld, mask, poff, fill, slots, err);
      hipLaunchKernelGGL(k_load_place<1>, dim3(pb), dim3(kBlock), 0, s, x, z, c, ld, B, poff, slots, st, g);
      break;
    case 2:
      hipLaunchKernelGGL(k_load_slots<2>, dim3(blocks), dim3(kBlock), 0, s, x, z, n, ld, mask, poff, fill, slots, err);
      hipLaunchKernelGGL(k_load_place<2>, dim3(pb), dim3(kBlock), 0, s, x, z, c, ld, B, poff, slots, st, g);
      break;
    case 3:
      hipLaunchKernelGGL(k_load_slots<3>, dim3(blocks), dim3(kBlock), 0, s, x, z, n, ld, mask, poff, fill, slots, err);
      hipLaunchKernelGGL(k_load_place<3>, dim3(pb), dim3(kBlock), 0, s, x, z, c, ld, B, poff, slots, st, g);
      break;
    default:
      hipLaunchKernelGGL(k_load_slots<4>, dim3(blocks), dim3(kBlock), 0, s, x, z, n, ld, mask, poff, fill, slots, err);
      hipLaunchKernelGGL(k_load_place<4>, dim3(pb), dim3(kBlock), 0, s, x, z, c, ld, B, poff, slots, st, g);
      break;
  }
}

// Loaded buckets are packed: each bucket's region is exactly its rows.
__global__ void k_set_packed_lim(StoreDev st, int64_t B) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < B;
       b += (int64_t)gridDim.x * blockDim.x)
    st.lim[b] = st.off[b] + st.cnt[b];
}

__global__ void k_load_finish(StoreDev st, int m, int64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *st.m = m;
    *st.total = n;
    *st.top = n;
    *st.err = 0;
    st.stats[0] = 0;
    st.stats[1] = 0;
  }
}

// scratch: B + ceil(B/1024) + 16 + n int64 (fill, scan, slot lists).
int launch_store_load(int W, StoreDev st, const uint64_t* x, const uint64_t* z, const double* c,
                      int64_t n, int64_t ld, int m, int64_t* scratch, hipStream_t s) {
  const int64_t B = 1ll << m;
  const uint32_t mask = (uint32_t)(B - 1);
  int64_t* fill = scratch;                       // B
  int64_t* scan_tmp = scratch + B;               // ceil(B/1024)+1
  int64_t* slots = scratch + B + B / 1024 + 16;  // n
  fill_i64(st.cnt, B, 0, s);
  fill_i64(fill, B, 0, s);
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  if (n > 0) {
    switch (W) {
      case 1: hipLaunchKernelGGL(k_load_hist<1>, dim3(blocks), dim3(kBlock), 0, s, x, z, n, ld, mask, st.cnt); break;
      case 2: hipLaunchKernelGGL(k_load_hist<2>, dim3(blocks), dim3(kBlock), 0, s, x, z, n, ld, mask, st.cnt); break;
      case 3: hipLaunchKernelGGL(k_load_hist<3>, dim3(blocks), dim3(kBlock), 0, s, x, z, n, ld, mask, st.cnt); break;
      default: hipLaunchKernelGGL(k_load_hist<4>, dim3(blocks), dim3(kBlock), 0, s, x, z, n, ld, mask, st.cnt); break;
    }
  }
  launch_scan_i64(st.cnt, st.off, B, scan_tmp, s);
  // packed rows: the slot lists and the rows share their offsets
  load_place_rows(W, st, x, z, c, n, ld, mask, B, st.off, fill, slots, false, s);
  {
    int64_t lb = (B + kBlock - 1) / kBlock;
    if (lb > 4096) lb = 4096;
    hipLaunchKernelGGL(k_set_packed_lim, dim3((unsigned)lb), dim3(kBlock), 0, s, st, B);
  }
  hipLaunchKernelGGL(k_load_finish, dim3(1), dim3(64), 0, s, st, m, n);
  return 0;
}

// ---------------------------------------------------------------------------
// Bucket regions (stores dressed in place): bucket b owns rows
// [off_b, off_b + reg_b) with reg_b = max(R, 2 cnt_b rounded up to 16), so it
// can grow after its live rows; the pool for buckets that outgrow their
// region starts after the last region.
// ---------------------------------------------------------------------------
__global__ void k_region_sizes(const int64_t* cnt, int64_t B, int64_t R, int64_t* reg) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < B;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = (2 * cnt[b] + 15) & ~(int64_t)15;
    reg[b] = r > R ? r : R;
  }
}

__global__ void k_region_lim(StoreDev st, const int64_t* reg, int64_t B) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < B;
       b += (int64_t)gridDim.x * blockDim.x)
    st.lim[b] = st.off[b] + reg[b];
}

// n >= 0: the live terms; n < 0: take them (and an error flag) from src.
__global__ void k_regions_finish(StoreDev st, const int64_t* reg, int64_t B, int m, int64_t R, int64_t n,
                                 StoreDev src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int64_t end = st.off[B - 1] + reg[B - 1];
    const int serr = n < 0 ? *src.err : 0;
    *st.m = m;
    *st.total = n < 0 ? *src.total : n;
    *st.top = end;
    *st.err = serr ? serr : (end > st.cap ? 1 : 0);
    st.stats[0] = 0;
    st.stats[1] = 0;
    st.aux[0] = 0;
    st.aux[1] = R;
    st.aux[2] = end;
    st.aux[3] = 0;
    st.aux[4] = 0;
  }
}

static void regions_from_counts(StoreDev st, int64_t B, int m, int64_t R, int64_t n, const StoreDev& src,
                                int64_t* reg, int64_t* scan_tmp, hipStream_t s) {
  int64_t lb = (B + kBlock - 1) / kBlock;
  if (lb > 4096) lb = 4096;
  hipLaunchKernelGGL(k_region_sizes, dim3((unsigned)lb), dim3(kBlock), 0, s, st.cnt, B, R, reg);
  launch_scan_i64(reg, st.off, B, scan_tmp, s);
  hipLaunchKernelGGL(k_region_lim, dim3((unsigned)lb), dim3(kBlock), 0, s, st, reg, B);
  hipLaunchKernelGGL(k_regions_finish, dim3(1), dim3(64), 0, s, st, reg, B, m, R, n, src);
}

// scratch: 3 B + ceil(B/1024) + 16 + n int64 (fill, region sizes, scan,
// packed slot offsets, slot lists).
int launch_store_load_regions(int W, StoreDev st, const uint64_t* x, const uint64_t* z, const double* c,
                              int64_t n, int64_t ld, int m, int64_t R, int64_t* scratch, hipStream_t s) {
  const int64_t B = 1ll << m;
  const uint32_t mask = (uint32_t)(B - 1);
  int64_t* fill = scratch;                           // B
  int64_t* reg = scratch + B;                        // B
  int64_t* scan_tmp = scratch + 2 * B;               // ceil(B/1024)+1
  int64_t* poff = scratch + 2 * B + B / 1024 + 16;   // B
  int64_t* slots = poff + B;                         // n
  fill_i64(st.cnt, B, 0, s);
  fill_i64(fill, B, 0, s);
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  if (n > 0) {
    switch (W) {
      case 1: hipLaunchKernelGGL(k_load_hist<1>, dim3(blocks), dim3(kBlock), 0, s, x, z, n, ld, mask, st.cnt); break;
      case 2: hipLaunchKernelGGL(k_load_hist<2>, dim3(blocks), dim3(kBlock), 0, s, x, z, n, ld, mask, st.cnt); break;
      case 3: hipLaunchKernelGGL(k_load_hist<3>, dim3(blocks), dim3(kBlock), 0, s, x, z, n, ld, mask, st.cnt); break;
      default: hipLaunchKernelGGL(k_load_hist<4>, dim3(blocks), dim3(kBlock), 0, s, x, z, n, ld, mask, st.cnt); break;
    }
  }
  regions_from_counts(st, B, m, R, n, st, reg, scan_tmp, s);
  launch_scan_i64(st.cnt, poff, B, scan_tmp, s);
  load_place_rows(W, st, x, z, c, n, ld, mask, B, poff, fill, slots, true, s);
  return 0;
}

// One wave per destination bucket d (m bits): its terms are those of source
// bucket d mod 2^ms whose hash has low bits d (m >= ms), or every term of the
// source buckets d + k 2^m in order (m < ms).  COUNT: live rows only; else the
// rows, in source order (ballot ranks).
template <int W, bool COUNT>
__global__ void k_copy_regions(StoreDev src, StoreDev dst, int m) {
  if (*src.err || (!COUNT && *dst.err)) return;   // an invalid source is not read
  const int lane = threadIdx.x & 63;
  const int ms = *src.m;
  const int64_t B = 1ll << m;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const uint32_t mask = (uint32_t)(B - 1);
  const int64_t nsrc = m >= ms ? 1 : (1ll << (ms - m));
  for (int64_t d = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); d < B; d += waves) {
    int64_t k = 0;
    const int64_t base = COUNT ? 0 : dst.off[d];
    for (int64_t t = 0; t < nsrc; ++t) {
      const int64_t sb = m >= ms ? (d & ((1ll << ms) - 1)) : d + (t << m);
      const int64_t n = src.cnt[sb], off = src.off[sb];
      for (int64_t i0 = 0; i0 < n; i0 += 64) {
        const int64_t i = i0 + lane;
        uint64_t kx[W], kz[W];
        double c = 0.0;
        bool sel = false;
        if (i < n) {
          load_key<W>(src, off + i, kx, kz, c);
          sel = m < ms || (bucket_hash<W>(kx, kz) & mask) == (uint32_t)d;
        }
        const uint64_t bm = __ballot(sel);
        if (!COUNT && sel) store_key<W>(dst, base + k + (int64_t)lanes_below(bm), kx, kz, c);
        k += __popcll(bm);
      }
    }
    if (COUNT && lane == 0) dst.cnt[d] = k;
  }
}

// Same bucket count on both sides: bucket b keeps its terms.  Counts first,
// then the rows: one wave per 64 consecutive buckets, lanes over the flat
// index of their rows (coalesced for large buckets, dense for small ones).
__global__ void k_copy_counts_same(StoreDev src, StoreDev dst, int64_t B) {
  if (*src.err) return;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < B;
       b += (int64_t)gridDim.x * blockDim.x)
    dst.cnt[b] = src.cnt[b];
}

template <int W>
__global__ void k_copy_rows_same(StoreDev src, StoreDev dst, int64_t B) {
  if (*src.err || *dst.err) return;
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t g = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); g * 64 < B; g += waves) {
    const int64_t b = g * 64 + lane;
    const int64_t cnt = b < B ? src.cnt[b] : 0;
    const int64_t soff = b < B ? src.off[b] : 0;
    const int64_t doff = b < B ? dst.off[b] : 0;
    int64_t incl = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    const int64_t pre = incl - cnt;
    const int64_t n = __shfl(incl, 63, 64);
    for (int64_t i0 = 0; i0 < n; i0 += 64) {
      const int64_t i = i0 + lane;
      int s = 0;   // the last lane whose first row is <= i
#pragma unroll
      for (int step = 32; step; step >>= 1) {
        const int64_t pc = __shfl(pre, s + step, 64);
        if (s + step < 64 && pc <= i) s += step;
      }
      const int64_t ps = __shfl(pre, s, 64), so = __shfl(soff, s, 64), dof = __shfl(doff, s, 64);
      if (i < n) {
        uint64_t kx[W], kz[W];
        double c;
        load_key<W>(src, so + (i - ps), kx, kz, c);
        store_key<W>(dst, dof + (i - ps), kx, kz, c);
      }
    }
  }
}

void launch_store_copy_regions(int W, const StoreDev& src, StoreDev dst, int m, int64_t R, int64_t* scratch,
                               hipStream_t s, bool same_m) {
  const int64_t B = 1ll << m;
  int64_t* reg = scratch;               // B
  int64_t* scan_tmp = scratch + B;      // ceil(B/1024)+1
  if (same_m) {
    int64_t lb = (B + kBlock - 1) / kBlock;
    if (lb > 4096) lb = 4096;
    hipLaunchKernelGGL(k_copy_counts_same, dim3((unsigned)lb), dim3(kBlock), 0, s, src, dst, B);
    regions_from_counts(dst, B, m, R, -1, src, reg, scan_tmp, s);
    int64_t wb = (B / 64 + kWaves - 1) / kWaves;
    if (wb < 1) wb = 1;
    if (wb > 8192) wb = 8192;
    switch (W) {
      case 1: hipLaunchKernelGGL(k_copy_rows_same<1>, dim3((unsigned)wb), dim3(kBlock), 0, s, src, dst, B); break;
      case 2: hipLaunchKernelGGL(k_copy_rows_same<2>, dim3((unsigned)wb), dim3(kBlock), 0, s, src, dst, B); break;
      case 3: hipLaunchKernelGGL(k_copy_rows_same<3>, dim3((unsigned)wb), dim3(kBlock), 0, s, src, dst, B); break;
      default: hipLaunchKernelGGL(k_copy_rows_same<4>, dim3((unsigned)wb), dim3(kBlock), 0, s, src, dst, B); break;
    }
    return;
  }
  int64_t blocks = (B + kWaves - 1) / kWaves;
  if (blocks > 16384) blocks = 16384;
  switch (W) {
    case 1: hipLaunchKernelGGL((k_copy_regions<1, true>), dim3(blocks), dim3(kBlock), 0, s, src, dst, m); break;
    case 2: hipLaunchKernelGGL((k_copy_regions<2, true>), dim3(blocks), dim3(kBlock), 0, s, src, dst, m); break;
    case 3: hipLaunchKernelGGL((k_copy_regions<3, true>), dim3(blocks), dim3(kBlock), 0, s, src, dst, m); break;
    default: hipLaunchKernelGGL((k_copy_regions<4, true>), dim3(blocks), dim3(kBlock), 0, s, src, dst, m); break;
  }
  regions_from_counts(dst, B, m, R, -1, src, reg, scan_tmp, s);
  switch (W) {
    case 1: hipLaunchKernelGGL((k_copy_regions<1, false>), dim3(blocks), dim3(kBlock), 0, s, src, dst, m); break;
    case 2: hipLaunchKernelGGL((k_copy_regions<2, false>), dim3(blocks), dim3(kBlock), 0, s, src, dst, m); break;
    case 3: hipLaunchKernelGGL((k_copy_regions<3, false>), dim3(blocks), dim3(kBlock), 0, s, src, dst, m); break;
    default: hipLaunchKernelGGL((k_copy_regions<4, false>), dim3(blocks), dim3(kBlock), 0, s, src, dst, m); break;
  }
}

// ---------------------------------------------------------------------------
// Export: bucketed store -> flat rows grouped by bucket.
// ---------------------------------------------------------------------------
template <int W>
__global__ void k_export(StoreDev st, int64_t B, const int64_t* dest_off, uint64_t* x,
                         uint64_t* z, double* c, int64_t ld) {
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = st.cnt[b], src = st.off[b], dst = dest_off[b];
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        x[w * ld + dst + i] = st.x[w * st.cap + src + i];
        z[w * ld + dst + i] = st.z[w * st.cap + src + i];
      }
      c[dst + i] = st.c[src + i];
    }
  }
}

void launch_store_export(int W, StoreDev st, int m, uint64_t* x, uint64_t* z, double* c,
                         int64_t ld, int64_t* dest_off, int64_t* scratch, hipStream_t s) {
  const int64_t B = 1ll << m;
  launch_scan_i64(st.cnt, dest_off, B, scratch, s);
  int64_t blocks = B < 8192 ? B : 8192;
  switch (W) {
    case 1: hipLaunchKernelGGL(k_export<1>, dim3(blocks), dim3(kBlock), 0, s, st, B, dest_off, x, z, c, ld); break;
    case 2: hipLaunchKernelGGL(k_export<2>, dim3(blocks), dim3(kBlock), 0, s, st, B, dest_off, x, z, c, ld); break;
    case 3: hipLaunchKernelGGL(k_export<3>, dim3(blocks), dim3(kBlock), 0, s, st, B, dest_off, x, z, c, ld); break;
    default: hipLaunchKernelGGL(k_export<4>, dim3(blocks), dim3(kBlock), 0, s, st, B, dest_off, x, z, c, ld); break;
  }
}

// ---------------------------------------------------------------------------
// Lookup: for each query key, scan its bucket (one wave per query).
// ---------------------------------------------------------------------------
template <int W>
__global__ void k_lookup(StoreDev st, const uint64_t* qx, const uint64_t* qz, int64_t nq_,
                         int64_t ld, int8_t* found, double* val) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const uint32_t mask = (uint32_t)((1ull << *st.m) - 1);
  for (int64_t q = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); q < nq_; q += waves) {
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      kx[w] = qx[w * ld + q];
      kz[w] = qz[w * ld + q];
    }
    const uint32_t b = bucket_hash<W>(kx, kz) & mask;
    const int64_t n = st.cnt[b], off = st.off[b];
    int64_t hit = -1;
    for (int64_t i0 = 0; i0 < n; i0 += 64) {
      const int64_t i = i0 + lane;
      bool eq = i < n;
#pragma unroll
      for (int w = 0; w < W; ++w)
        eq = eq && st.x[w * st.cap + off + i] == kx[w] && st.z[w * st.cap + off + i] == kz[w];
      const uint64_t ball = __ballot(eq);
      if (ball) {
        hit = off + i0 + __ffsll((unsigned long long)ball) - 1;
        break;
      }
    }
    if (lane == 0) {
      found[q] = hit >= 0 ? 1 : 0;
      val[q] = hit >= 0 ? st.c[hit] : 0.0;
    }
  }
}

void launch_lookup(int W, const StoreDev& st, const uint64_t* qx, const uint64_t* qz, int64_t n,
                   int64_t ld, int8_t* found, double* val, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + kWaves - 1) / kWaves;
  if (blocks > 8192) blocks = 8192;
  switch (W) {
    case 1: hipLaunchKernelGGL(k_lookup<1>, dim3(blocks), dim3(kBlock), 0, s, st, qx, qz, n, ld, found, val); break;
    case 2: hipLaunchKernelGGL(k_lookup<2>, dim3(blocks), dim3(kBlock), 0, s, st, qx, qz, n, ld, found, val); break;
    case 3: hipLaunchKernelGGL(k_lookup<3>, dim3(blocks), dim3(kBlock), 0, s, st, qx, qz, n, ld, found, val); break;
    default: hipLaunchKernelGGL(k_lookup<4>, dim3(blocks), dim3(kBlock), 0, s, st, qx, qz, n, ld, found, val); break;
  }
}

// Sum of c^2 over the live rows (the squared Frobenius norm of the Pauli sum
// up to 2^n, which a dressing step keeps and compression lowers).  Workgroup g
// takes buckets g, g + grid, ...; per-workgroup sums are reduced in a fixed
// order by launch_finalize_sum.
__global__ void k_sum_squares(StoreDev st, double* partial) {
  __shared__ double red[kWaves];
  const int64_t B = 1ll << *st.m;
  double acc = 0.0;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = st.cnt[b], off = st.off[b];
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
      const double c = st.c[off + i];
      acc += c * c;
    }
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

void launch_sum_squares(const StoreDev& st, int grid, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_squares, dim3(grid), dim3(kBlock), 0, s, st, partial);
}

}  // namespace iqcc
