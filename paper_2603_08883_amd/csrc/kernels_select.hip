// Term-limit compression: keep the M terms of largest |c| (the maximum-terms
// limit of the paper's Ru-catalyst runs, Results, next to the coefficient
// cutoff; ties broken by the smaller canonical key so that the kept set is
// unique).
//
// Radix selection on the IEEE bits of |c|, which order non-negative doubles
// like their values: six digit passes (11, 11, 11, 11, 11, 9 bits, most
// significant first) each build a histogram of the digit over the terms whose
// higher digits equal the prefix chosen so far, and a one-thread kernel picks
// the digit where the running count from the top reaches the number still
// needed.  After the first digit only the terms that share it can matter, so
// the second pass copies their |c| bits aside and the later passes read those
// alone.  That fixes the threshold T (the M-th largest |c|), the number of
// terms above it and the number to take among the terms equal to T.  When not
// all ties are taken, the tie keys are collected and the same selection runs
// on their canonical key words (x words, then z words, most significant
// first), from the bottom.  A last pass copies every bucket's kept terms, in
// input order, to the same rows of the output arena.
#include "iqcc_internal.h"

namespace iqcc {

constexpr int kSelBins = 2048;

__device__ __forceinline__ uint64_t abs_bits(double c) {
  return (uint64_t)__double_as_longlong(c) & 0x7fffffffffffffffull;
}

// |c| digit histogram over the live terms of st whose bits above `shift + width`
// equal `prefix` (all terms when `first`).
template <int W>
__global__ __launch_bounds__(kBlock) void k_abs_hist(StoreDev st, const SelState* ss, int shift,
                                                     int width, int first, unsigned* hist) {
  __shared__ unsigned h[kSelBins];
  for (int i = threadIdx.x; i < kSelBins; i += kBlock) h[i] = 0;
  __syncthreads();
  const uint64_t prefix = ss->prefix;
  const int64_t B = 1ll << *st.m;
  const uint64_t dmask = (1ull << width) - 1;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = st.cnt[b], off = st.off[b];
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
      const uint64_t u = abs_bits(st.c[off + i]);
      if (first || (u >> (shift + width)) == prefix) atomicAdd(&h[(u >> shift) & dmask], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kSelBins; i += kBlock)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Second digit pass: the histogram of k_abs_hist, and the |c| bits of every
// term that matches the prefix appended to cand.  Matches are staged in LDS
// and flushed with one global atomic per ~kCandStage values, so the append
// counter is not a point of contention.
constexpr int kCandStage = 2048;

template <int W>
__global__ __launch_bounds__(kBlock) void k_abs_hist_collect(StoreDev st, const SelState* ss,
                                                             int shift, int width, unsigned* hist,
                                                             uint64_t* cand, int64_t cap,
                                                             unsigned long long* count) {
  __shared__ unsigned h[kSelBins];
  __shared__ uint64_t stage[kCandStage];
  __shared__ uint64_t scan_tmp[kWaves];
  __shared__ unsigned long long gbase;
  for (int i = threadIdx.x; i < kSelBins; i += kBlock) h[i] = 0;
  __syncthreads();
  const uint64_t prefix = ss->prefix;
  const int64_t B = 1ll << *st.m;
  const uint64_t dmask = (1ull << width) - 1;
  int nst = 0;   // staged values (block-uniform)
  auto flush = [&]() {
    if (threadIdx.x == 0) gbase = atomicAdd(count, (unsigned long long)nst);
    __syncthreads();
    for (int k = threadIdx.x; k < nst; k += kBlock)
      if ((int64_t)(gbase + k) < cap) cand[gbase + k] = stage[k];
    __syncthreads();
    nst = 0;
  };
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = st.cnt[b], off = st.off[b];
    for (int64_t i0 = 0; i0 < n; i0 += kBlock) {   // block-uniform
      const int64_t i = i0 + threadIdx.x;
      uint64_t u = 0;
      bool match = false;
      if (i < n) {
        u = abs_bits(st.c[off + i]);
        match = (u >> (shift + width)) == prefix;
      }
      if (match) atomicAdd(&h[(u >> shift) & dmask], 1u);
      uint64_t tot;
      const uint64_t pos = block_exclusive_scan(match ? 1ull : 0ull, scan_tmp, tot);
      if (nst + (int)tot > kCandStage) flush();
      if (match) stage[nst + (int)pos] = u;
      nst += (int)tot;
    }
  }
  __syncthreads();
  if (nst) flush();
  for (int i = threadIdx.x; i < kSelBins; i += kBlock)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Later digit passes over the collected |c| bits only.
__global__ __launch_bounds__(kBlock) void k_cand_hist(const uint64_t* cand, int64_t cap,
                                                      const unsigned long long* count,
                                                      const SelState* ss, int shift, int width,
                                                      unsigned* hist) {
  __shared__ unsigned h[kSelBins];
  for (int i = threadIdx.x; i < kSelBins; i += kBlock) h[i] = 0;
  __syncthreads();
  const uint64_t prefix = ss->prefix;
  const uint64_t dmask = (1ull << width) - 1;
  const int64_t n = (int64_t)*count < cap ? (int64_t)*count : cap;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const uint64_t u = cand[i];
    if ((u >> (shift + width)) == prefix) atomicAdd(&h[(u >> shift) & dmask], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kSelBins; i += kBlock)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Pick the digit at which the count reaches ss->need, scanning from the
// largest digit down (descending) or from 0 up, and clear the histogram.  Each
// thread owns 8 consecutive digits in scan order; a block scan of the per-thread
// sums finds the thread whose digits contain the crossing, and that thread
// resolves it.
__global__ __launch_bounds__(kBlock) void k_pick_digit(SelState* ss, unsigned* hist, int width,
                                                       int descending, int last, int key_word) {
  __shared__ uint64_t scan_tmp[kWaves];
  const int nb = 1 << width;
  constexpr int kPer = kSelBins / kBlock;   // 8 digits per thread
  unsigned v[kPer];
  uint64_t mine = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int r = threadIdx.x * kPer + k;   // rank in scan order
    const int d = descending ? nb - 1 - r : r;
    v[k] = r < nb ? hist[d] : 0u;
    if (r < nb) hist[d] = 0u;
    mine += v[k];
  }
  uint64_t total;
  const uint64_t before_mine = block_exclusive_scan(mine, scan_tmp, total);
  const int64_t need = ss->need;
  __syncthreads();
  // the thread whose range holds the crossing (need >= 1 and need <= total)
  if ((int64_t)before_mine < need && (int64_t)(before_mine + mine) >= need) {
    int64_t before = (int64_t)before_mine;
    int pick_r = threadIdx.x * kPer + kPer - 1;
    unsigned at = v[kPer - 1];
    for (int k = 0; k < kPer; ++k) {
      if (before + (int64_t)v[k] >= need) {
        pick_r = threadIdx.x * kPer + k;
        at = v[k];
        break;
      }
      before += v[k];
    }
    const int pick = descending ? nb - 1 - pick_r : pick_r;
    ss->need = need - before;
    ss->passed += before;
    ss->at = at;
    ss->prefix = (ss->prefix << width) | (uint64_t)pick;
    if (last) {
      if (key_word < 0) {
        ss->T = ss->prefix;
        ss->ties = at;
      } else {
        ss->kthr[key_word] = ss->prefix;
      }
      ss->prefix = 0;
    }
  }
}

// Canonical key word q of a term: x[W-1], ..., x[0], z[W-1], ..., z[0].
template <int W>
__device__ __forceinline__ uint64_t canon_word(const StoreDev& st, int64_t row, int q) {
  return q < W ? st.x[(W - 1 - q) * st.cap + row] : st.z[(2 * W - 1 - q) * st.cap + row];
}

// Keys of the terms with |c| bits == T, as rows of 2W canonical words.
template <int W>
__global__ __launch_bounds__(kBlock) void k_collect_ties(StoreDev st, const SelState* ss,
                                                         uint64_t* keys, int64_t cap,
                                                         unsigned long long* count) {
  const uint64_t T = ss->T;
  const int64_t B = 1ll << *st.m;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = st.cnt[b], off = st.off[b];
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
      if (abs_bits(st.c[off + i]) != T) continue;
      const int64_t r = (int64_t)atomicAdd(count, 1ull);
      if (r < cap)
        for (int q = 0; q < 2 * W; ++q) keys[r * 2 * W + q] = canon_word<W>(st, off + i, q);
    }
  }
}

// Digit histogram of key word q over the tie keys whose earlier words equal
// kthr[0..q) and whose bits of word q above shift + width equal the prefix.
__global__ __launch_bounds__(kBlock) void k_key_hist(const uint64_t* keys, int64_t n, int nw,
                                                     const SelState* ss, int q, int shift,
                                                     int width, int first, unsigned* hist) {
  __shared__ unsigned h[kSelBins];
  for (int i = threadIdx.x; i < kSelBins; i += kBlock) h[i] = 0;
  __syncthreads();
  const uint64_t dmask = (1ull << width) - 1;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const uint64_t* k = keys + i * nw;
    bool match = true;
    for (int p = 0; p < q; ++p) match = match && k[p] == ss->kthr[p];
    if (match && (first || (k[q] >> (shift + width)) == ss->prefix))
      atomicAdd(&h[(k[q] >> shift) & dmask], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kSelBins; i += kBlock)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Copy the kept terms of every bucket, in input order, to the same rows of
// the output arena; the output keeps the input's bucket table shape.
template <int W>
__global__ __launch_bounds__(kBlock) void k_select_compact(StoreDev in, StoreDev out,
                                                           const SelState* ss, int keep_all) {
  __shared__ uint64_t scan_tmp[kWaves];
  const uint64_t T = ss->T;
  const int key_mode = ss->key_mode;
  const int m = *in.m;
  const int64_t B = 1ll << m;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *out.m = m;
    *out.top = *in.top;
  }
  int64_t kept = 0;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = in.cnt[b], off = in.off[b];
    int64_t w = 0;
    for (int64_t i0 = 0; i0 < n; i0 += kBlock) {
      const int64_t i = i0 + threadIdx.x;
      bool keep = false;
      if (i < n && keep_all >= 0) {
        if (keep_all) {
          keep = true;
        } else {
          const uint64_t u = abs_bits(in.c[off + i]);
          keep = u > T;
          if (u == T) {
            keep = true;
            if (key_mode) {
              // keep ties whose canonical key is <= kthr
              for (int q = 0; q < 2 * W; ++q) {
                const uint64_t v = canon_word<W>(in, off + i, q);
                if (v != ss->kthr[q]) {
                  keep = v < ss->kthr[q];
                  break;
                }
              }
            }
          }
        }
      }
      uint64_t tot;
      const uint64_t pos = block_exclusive_scan(keep ? 1ull : 0ull, scan_tmp, tot);
      if (keep) {
        const int64_t r = off + w + (int64_t)pos;
#pragma unroll
        for (int q = 0; q < W; ++q) {
          out.x[q * out.cap + r] = in.x[q * in.cap + off + i];
          out.z[q * out.cap + r] = in.z[q * in.cap + off + i];
        }
        out.c[r] = in.c[off + i];
      }
      w += (int64_t)tot;
    }
    if (threadIdx.x == 0) {
      out.off[b] = off;
      out.cnt[b] = w;
      out.lim[b] = off + n;   // the input bucket's rows
    }
    kept += w;
  }
  if (threadIdx.x == 0 && kept) atomicAdd((unsigned long long*)out.total, (unsigned long long)kept);
}

static const int kDigitWidth[6] = {11, 11, 11, 11, 11, 9};
static const int kDigitShift[6] = {53, 42, 31, 20, 9, 0};

void launch_abs_select_first(int W, const StoreDev& st, SelState* ss, unsigned* hist, int grid,
                             hipStream_t s) {
  const int sh = kDigitShift[0], wd = kDigitWidth[0];
  switch (W) {
    case 1: hipLaunchKernelGGL(k_abs_hist<1>, dim3(grid), dim3(kBlock), 0, s, st, ss, sh, wd, 1, hist); break;
    case 2: hipLaunchKernelGGL(k_abs_hist<2>, dim3(grid), dim3(kBlock), 0, s, st, ss, sh, wd, 1, hist); break;
    case 3: hipLaunchKernelGGL(k_abs_hist<3>, dim3(grid), dim3(kBlock), 0, s, st, ss, sh, wd, 1, hist); break;
    default: hipLaunchKernelGGL(k_abs_hist<4>, dim3(grid), dim3(kBlock), 0, s, st, ss, sh, wd, 1, hist); break;
  }
  hipLaunchKernelGGL(k_pick_digit, dim3(1), dim3(kBlock), 0, s, ss, hist, wd, 1, 0, -1);
}

void launch_abs_select_rest(int W, const StoreDev& st, SelState* ss, unsigned* hist, int grid,
                            uint64_t* cand, int64_t cand_cap, unsigned long long* cand_count,
                            hipStream_t s) {
  {
    const int sh = kDigitShift[1], wd = kDigitWidth[1];
    switch (W) {
      case 1: hipLaunchKernelGGL(k_abs_hist_collect<1>, dim3(grid), dim3(kBlock), 0, s, st, ss, sh, wd, hist, cand, cand_cap, cand_count); break;
      case 2: hipLaunchKernelGGL(k_abs_hist_collect<2>, dim3(grid), dim3(kBlock), 0, s, st, ss, sh, wd, hist, cand, cand_cap, cand_count); break;
      case 3: hipLaunchKernelGGL(k_abs_hist_collect<3>, dim3(grid), dim3(kBlock), 0, s, st, ss, sh, wd, hist, cand, cand_cap, cand_count); break;
      default: hipLaunchKernelGGL(k_abs_hist_collect<4>, dim3(grid), dim3(kBlock), 0, s, st, ss, sh, wd, hist, cand, cand_cap, cand_count); break;
    }
    hipLaunchKernelGGL(k_pick_digit, dim3(1), dim3(kBlock), 0, s, ss, hist, wd, 1, 0, -1);
  }
  int64_t g = (cand_cap + kBlock - 1) / kBlock;
  const int cgrid = (int)(g < 1 ? 1 : g > grid ? grid : g);
  for (int p = 2; p < 6; ++p) {
    hipLaunchKernelGGL(k_cand_hist, dim3(cgrid), dim3(kBlock), 0, s, cand, cand_cap, cand_count, ss,
                       kDigitShift[p], kDigitWidth[p], hist);
    hipLaunchKernelGGL(k_pick_digit, dim3(1), dim3(kBlock), 0, s, ss, hist, kDigitWidth[p], 1, p == 5, -1);
  }
}

void launch_collect_ties(int W, const StoreDev& st, const SelState* ss, uint64_t* keys, int64_t cap,
                         unsigned long long* count, int grid, hipStream_t s) {
  switch (W) {
    case 1: hipLaunchKernelGGL(k_collect_ties<1>, dim3(grid), dim3(kBlock), 0, s, st, ss, keys, cap, count); break;
    case 2: hipLaunchKernelGGL(k_collect_ties<2>, dim3(grid), dim3(kBlock), 0, s, st, ss, keys, cap, count); break;
    case 3: hipLaunchKernelGGL(k_collect_ties<3>, dim3(grid), dim3(kBlock), 0, s, st, ss, keys, cap, count); break;
    default: hipLaunchKernelGGL(k_collect_ties<4>, dim3(grid), dim3(kBlock), 0, s, st, ss, keys, cap, count); break;
  }
}

void launch_key_select(int W, const uint64_t* keys, int64_t n, SelState* ss, unsigned* hist,
                       hipStream_t s) {
  int64_t g = (n + kBlock - 1) / kBlock;
  const int grid = (int)(g < 1 ? 1 : g > 1024 ? 1024 : g);
  for (int q = 0; q < 2 * W; ++q)
    for (int p = 0; p < 6; ++p) {
      hipLaunchKernelGGL(k_key_hist, dim3(grid), dim3(kBlock), 0, s, keys, n, 2 * W, ss, q,
                         kDigitShift[p], kDigitWidth[p], p == 0, hist);
      hipLaunchKernelGGL(k_pick_digit, dim3(1), dim3(kBlock), 0, s, ss, hist, kDigitWidth[p], 0, p == 5, q);
    }
}

void launch_select_compact(int W, const StoreDev& in, const StoreDev& out, const SelState* ss,
                           int keep_all, int grid, hipStream_t s) {
  switch (W) {
    case 1: hipLaunchKernelGGL(k_select_compact<1>, dim3(grid), dim3(kBlock), 0, s, in, out, ss, keep_all); break;
    case 2: hipLaunchKernelGGL(k_select_compact<2>, dim3(grid), dim3(kBlock), 0, s, in, out, ss, keep_all); break;
    case 3: hipLaunchKernelGGL(k_select_compact<3>, dim3(grid), dim3(kBlock), 0, s, in, out, ss, keep_all); break;
    default: hipLaunchKernelGGL(k_select_compact<4>, dim3(grid), dim3(kBlock), 0, s, in, out, ss, keep_all); break;
  }
}

}  // namespace iqcc
