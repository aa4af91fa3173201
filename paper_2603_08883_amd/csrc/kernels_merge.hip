// Merge of an arbitrary multiset of Pauli rows into unique keys (D = H + I of
// App. D) followed by compression |c| < eps (App. A, iterative procedure).
//
// Rows are first partitioned into buckets by the linear key hash (equal keys
// share a bucket), carrying their original row index.  Each bucket is then
// sorted by (key, row) -- bitonic sort of an index permutation in LDS, or in
// global scratch for a bucket larger than the LDS tile -- and each run of equal
// keys is summed left to right in increasing row order, which reproduces the
// order in which a stable sort followed by a left-to-right sum adds them.
#include "iqcc_internal.h"

#pragma clang fp contract(off)

namespace iqcc {

constexpr int kMergeTile = 1024;   // rows of a bucket sorted in LDS

template <int W>
struct Staging {
  uint64_t* x;   // [W][cap]
  uint64_t* z;
  double* c;
  int64_t* row;
  int64_t cap;
};

template <int W>
__global__ void k_merge_hist(const uint64_t* __restrict__ x, const uint64_t* __restrict__ z,
                             int64_t n, int64_t ld, uint32_t mask, int64_t* cnt) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      kx[w] = x[w * ld + i];
      kz[w] = z[w * ld + i];
    }
    atomicAdd((unsigned long long*)&cnt[bucket_hash<W>(kx, kz) & mask], 1ull);
  }
}

template <int W>
__global__ void k_merge_scatter(const uint64_t* __restrict__ x, const uint64_t* __restrict__ z,
                                const double* __restrict__ c, int64_t n, int64_t ld, uint32_t mask,
                                const int64_t* off, int64_t* fill, Staging<W> st) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      kx[w] = x[w * ld + i];
      kz[w] = z[w * ld + i];
    }
    const uint32_t b = bucket_hash<W>(kx, kz) & mask;
    const int64_t pos = off[b] + (int64_t)atomicAdd((unsigned long long*)&fill[b], 1ull);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      st.x[w * st.cap + pos] = kx[w];
      st.z[w * st.cap + pos] = kz[w];
    }
    st.c[pos] = c[i];
    st.row[pos] = i;
  }
}

// a < b in (key, row) order; keys compared as (x[W-1..0], z[W-1..0]) unsigned
template <int W>
__device__ __forceinline__ bool row_less(const Staging<W>& st, int64_t a, int64_t b) {
#pragma unroll
  for (int w = W - 1; w >= 0; --w) {
    const uint64_t u = st.x[w * st.cap + a], v = st.x[w * st.cap + b];
    if (u != v) return u < v;
  }
#pragma unroll
  for (int w = W - 1; w >= 0; --w) {
    const uint64_t u = st.z[w * st.cap + a], v = st.z[w * st.cap + b];
    if (u != v) return u < v;
  }
  return st.row[a] < st.row[b];
}

template <int W>
__device__ __forceinline__ bool same_key(const Staging<W>& st, int64_t a, int64_t b) {
  bool eq = true;
#pragma unroll
  for (int w = 0; w < W; ++w)
    eq = eq && st.x[w * st.cap + a] == st.x[w * st.cap + b] && st.z[w * st.cap + a] == st.z[w * st.cap + b];
  return eq;
}

// Bitonic sort of idx[0..P) (P a power of two); entries >= n are padding that
// sorts last.  idx lives in LDS or global memory.
template <int W, typename IdxT>
__device__ void bitonic(IdxT* idx, int64_t P, int64_t n, int64_t base, const Staging<W>& st) {
  for (int64_t k = 2; k <= P; k <<= 1) {
    for (int64_t j = k >> 1; j > 0; j >>= 1) {
      for (int64_t i = threadIdx.x; i < P; i += blockDim.x) {
        const int64_t l = i ^ j;
        if (l > i) {
          const IdxT a = idx[i], b = idx[l];
          const bool a_pad = (int64_t)a >= n, b_pad = (int64_t)b >= n;
          bool greater;  // a > b
          if (a_pad || b_pad) greater = a_pad && !b_pad;
          else greater = row_less<W>(st, base + b, base + a);
          const bool up = (i & k) == 0;
          if (greater == up) {
            idx[i] = b;
            idx[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_merge_buckets(Staging<W> st, const int64_t* boff,
                                                          const int64_t* bcnt, int64_t B,
                                                          StoreDev out, double eps,
                                                          uint32_t* gidx) {
  __shared__ uint32_t sidx[kMergeTile];
  __shared__ uint64_t scan_tmp[kWaves];
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = bcnt[b], base = boff[b];
    int64_t P = 1;
    while (P < n) P <<= 1;
    uint32_t* idx;
    if (P <= kMergeTile) {
      idx = sidx;
    } else {
      idx = gidx + 2 * base;   // 2*(base + n) <= 2 * total rows
    }
    for (int64_t i = threadIdx.x; i < P; i += blockDim.x) idx[i] = (uint32_t)i;
    __syncthreads();
    if (n > 1) bitonic<W>(idx, P, n, base, st);
    // runs of equal keys: the head sums its run left to right
    int64_t written = 0;
    for (int64_t i0 = 0; i0 < n; i0 += blockDim.x) {
      const int64_t i = i0 + threadIdx.x;
      bool keep = false;
      double sum = 0.0;
      int64_t head_row = 0;
      if (i < n) {
        head_row = base + idx[i];
        const bool head = i == 0 || !same_key<W>(st, base + idx[i - 1], head_row);
        if (head) {
          sum = st.c[head_row];
          for (int64_t j = i + 1; j < n && same_key<W>(st, base + idx[j], head_row); ++j)
            sum = __dadd_rn(sum, st.c[base + idx[j]]);
          keep = !(fabs(sum) < eps);
        }
      }
      uint64_t total;
      const uint64_t ex = block_exclusive_scan(keep ? 1ull : 0ull, scan_tmp, total);
      if (keep) {
        const int64_t r = base + written + (int64_t)ex;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          out.x[w * out.cap + r] = st.x[w * st.cap + head_row];
          out.z[w * out.cap + r] = st.z[w * st.cap + head_row];
        }
        out.c[r] = sum;
      }
      written += (int64_t)total;
    }
    if (threadIdx.x == 0) {
      out.off[b] = base;
      out.cnt[b] = written;
      out.lim[b] = base + n;   // the rows reserved for the bucket's input
      if (written) atomicAdd((unsigned long long*)out.total, (unsigned long long)written);
    }
    __syncthreads();
  }
}

__global__ void k_merge_finish(StoreDev out, int m, int64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *out.m = m;
    *out.top = n;
  }
}

template <int W>
static void merge_t(StoreDev out, const uint64_t* x, const uint64_t* z, const double* c,
                    int64_t n, int64_t ld, int m, double eps, int64_t* scratch,
                    hipStream_t s) {
  const int64_t B = 1ll << m;
  const uint32_t mask = (uint32_t)(B - 1);
  // scratch layout (int64 units): fill[B], scan[B/1024+16], staging x/z (W*n each),
  // c (n), row (n), gidx (2n uint32 = n int64)
  int64_t* fill = scratch;
  int64_t* scan_tmp = fill + B;
  Staging<W> st;
  st.cap = n > 0 ? n : 1;
  st.x = (uint64_t*)(scan_tmp + B / 1024 + 16);
  st.z = st.x + W * st.cap;
  st.c = (double*)(st.z + W * st.cap);
  st.row = (int64_t*)(st.c + st.cap);
  uint32_t* gidx = (uint32_t*)(st.row + st.cap);
  launch_zero_counters(out, s);
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipMemsetAsync(out.cnt, 0, sizeof(int64_t) * B, s);
  hipMemsetAsync(fill, 0, sizeof(int64_t) * B, s);
  if (n > 0) hipLaunchKernelGGL(k_merge_hist<W>, dim3(blocks), dim3(kBlock), 0, s, x, z, n, ld, mask, out.cnt);
  launch_scan_i64(out.cnt, out.off, B, scan_tmp, s);
  if (n > 0)
    hipLaunchKernelGGL(k_merge_scatter<W>, dim3(blocks), dim3(kBlock), 0, s, x, z, c, n, ld, mask,
                       out.off, fill, st);
  // fill[] now holds the bucket sizes and out.off the bucket starts
  int64_t g = B < 4096 ? B : 4096;
  hipLaunchKernelGGL(k_merge_buckets<W>, dim3((unsigned)g), dim3(kBlock), 0, s, st, out.off, fill,
                     B, out, eps, gidx);
  hipLaunchKernelGGL(k_merge_finish, dim3(1), dim3(64), 0, s, out, m, n);
}

int64_t merge_scratch_len(int W, int64_t n, int m) {
  const int64_t B = 1ll << m;
  const int64_t cap = n > 0 ? n : 1;
  return B + B / 1024 + 16 + 2 * W * cap + cap + cap + cap;
}

void launch_merge_buckets(int W, StoreDev st, const uint64_t* x, const uint64_t* z,
                          const double* c, int64_t n, int64_t ld, int m, double eps,
                          int64_t* scratch, int64_t scratch_len, hipStream_t s) {
  (void)scratch_len;
  switch (W) {
    case 1: merge_t<1>(st, x, z, c, n, ld, m, eps, scratch, s); break;
    case 2: merge_t<2>(st, x, z, c, n, ld, m, eps, scratch, s); break;
    case 3: merge_t<3>(st, x, z, c, n, ld, m, eps, scratch, s); break;
    default: merge_t<4>(st, x, z, c, n, ld, m, eps, scratch, s); break;
  }
}

}  // namespace iqcc
