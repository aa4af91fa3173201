// The paper's sortless dressing (App. D), as a second dressing path next to the
// bucket-pair kernel, for comparison.  H is a flat list kept globally sorted in
// canonical order (x words, then z words, most significant word first).
//
//  1. Partition H by the key bits the entangler flips (the x bits under P's x
//     part and the z bits under P's z part): within a partition those bits are
//     equal, so K -> K ^ P preserves order.  The partition is stable (a binary
//     sort of the small label only), so every partition stays sorted.
//  2. Local dressing: rotate the anticommuting terms in place (cos tau) and
//     write their images K ^ P (+-sin tau, sign from the product phase); the
//     images of partition i are sorted and all land in partition i ^ (all
//     label bits).
//  3. Merge per destination partition: the rotated partition and the images
//     that land there are merged by rank (each element finds its place in the
//     other sorted list by binary search); equal keys meet as neighbours and are
//     combined (one IEEE addition), then |c| < eps is dropped.
//  4. Rebuild the global order by a deterministic multiway merge: pairs of
//     sorted runs are merged by rank, log2(#partitions) rounds.
#include <vector>

#include "iqcc_internal.h"

#pragma clang fp contract(off)

namespace iqcc {

// Flat sorted Hamiltonian: word planes x[W][ld], z[W][ld] and c[ld].
struct Flat {
  uint64_t* x;
  uint64_t* z;
  double* c;
  int64_t ld;
};

template <int W>
__device__ __forceinline__ int canon_cmp(const Flat& a, int64_t i, const Flat& b, int64_t j) {
#pragma unroll
  for (int w = W - 1; w >= 0; --w) {
    const uint64_t u = a.x[w * a.ld + i], v = b.x[w * b.ld + j];
    if (u != v) return u < v ? -1 : 1;
  }
#pragma unroll
  for (int w = W - 1; w >= 0; --w) {
    const uint64_t u = a.z[w * a.ld + i], v = b.z[w * b.ld + j];
    if (u != v) return u < v ? -1 : 1;
  }
  return 0;
}

// Number of elements of b[lo, hi) that precede a[i] (strictly smaller when
// !inclusive, smaller or equal when inclusive).
template <int W>
__device__ __forceinline__ int64_t rank_in(const Flat& a, int64_t i, const Flat& b, int64_t lo,
                                           int64_t hi, bool inclusive) {
  int64_t l = lo, r = hi;
  while (l < r) {
    const int64_t mid = (l + r) >> 1;
    const int c = canon_cmp<W>(b, mid, a, i);
    if (c < 0 || (inclusive && c == 0)) l = mid + 1;
    else r = mid;
  }
  return l - lo;
}

// Label: the key bits at P's flipped positions, packed (x plane first).
template <int W>
__global__ void k_sl_labels(Flat h, int64_t n, PauliKey P, uint32_t* label, uint32_t* idx) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t l = 0;
    int b = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint64_t kx = h.x[w * h.ld + i], kz = h.z[w * h.ld + i];
      for (uint64_t m = P.x[w]; m; m &= m - 1, ++b) l |= (uint32_t)((kx >> __builtin_ctzll(m)) & 1ull) << b;
      for (uint64_t m = P.z[w]; m; m &= m - 1, ++b) l |= (uint32_t)((kz >> __builtin_ctzll(m)) & 1ull) << b;
    }
    label[i] = l;
    idx[i] = (uint32_t)i;
  }
}

// start[l] = first position of label l in the sorted labels (start[npart] = n).
__global__ void k_sl_bounds(const uint32_t* label, int64_t n, int64_t npart, int64_t* start) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t prev = i == 0 ? -1 : (int64_t)label[i - 1];
    const int64_t cur = i == n ? npart : (int64_t)label[i];
    for (int64_t l = prev + 1; l <= cur; ++l) start[l] = i;
  }
}

// Stable partition by the label, one label bit per pass (least significant
// first): flag = bit b, then every element moves to (zeros before it) or
// (all zeros + ones before it), which keeps the order within each side.
__global__ void k_sl_bitflag(const uint32_t* label, int64_t n, int b, int64_t* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    flag[i] = (int64_t)((label[i] >> b) & 1u);
}

__global__ void k_sl_split(const uint32_t* label, const uint32_t* idx, int64_t n, const int64_t* flag,
                           const int64_t* ones_before, uint32_t* label_out, uint32_t* idx_out) {
  const int64_t zeros = n - (ones_before[n - 1] + flag[n - 1]);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = ones_before[i];
    const int64_t dst = flag[i] ? zeros + o : i - o;
    label_out[dst] = label[i];
    idx_out[dst] = idx[i];
  }
}

// Gather H into partition order, rotate the anticommuting terms, flag them.
template <int W>
__global__ void k_sl_gather(Flat h, const uint32_t* perm, int64_t n, PauliKey P, double C,
                            Flat g, int64_t* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = perm[i];
    uint64_t kx[W], kz[W];
    uint64_t t = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      kx[w] = h.x[w * h.ld + r];
      kz[w] = h.z[w * h.ld + r];
      g.x[w * g.ld + i] = kx[w];
      g.z[w * g.ld + i] = kz[w];
      t ^= (kx[w] & P.z[w]) ^ (kz[w] & P.x[w]);
    }
    const bool anti = __popcll(t) & 1;
    const double c = h.c[r];
    g.c[i] = anti ? __dmul_rn(C, c) : c;
    flag[i] = anti ? 1 : 0;
  }
}

// Images K ^ P of the anticommuting terms, in partition order.
template <int W>
__global__ void k_sl_images(Flat h, const uint32_t* perm, const uint32_t* label, int64_t n,
                            PauliKey P, double S, const int64_t* flag, const int64_t* pos,
                            Flat im, uint32_t* im_label) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!flag[i]) continue;
    const int64_t r = perm[i], q = pos[i];
    uint64_t kx[W], kz[W], qx[W], qz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      kx[w] = h.x[w * h.ld + r];
      kz[w] = h.z[w * h.ld + r];
      qx[w] = kx[w] ^ P.x[w];
      qz[w] = kz[w] ^ P.z[w];
      im.x[w * im.ld + q] = qx[w];
      im.z[w * im.ld + q] = qz[w];
    }
    const int e = product_phase<W>(P.x, P.z, kx, kz);
    const double s = __dmul_rn(S, h.c[r]);
    im.c[q] = e == 3 ? s : -s;
    im_label[q] = label[i];
  }
}

// Per destination partition j: sizes of (rotated part, arriving images).
__global__ void k_sl_sizes(const int64_t* start, const int64_t* istart, int64_t npart,
                           uint32_t fullmask, int64_t* size) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < npart; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = (int64_t)((uint32_t)j ^ fullmask);
    size[j] = (start[j + 1] - start[j]) + (istart[i + 1] - istart[i]);
  }
}

// Merge by rank: rotated terms (side A) go before equal images (side B).
template <int W>
__global__ void k_sl_merge_a(Flat g, const uint32_t* label, int64_t n, const int64_t* start,
                             Flat im, const int64_t* istart, const int64_t* mstart,
                             uint32_t fullmask, Flat m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t j = label[i];
    const uint32_t src = j ^ fullmask;
    const int64_t p = mstart[j] + (i - start[j]) + rank_in<W>(g, i, im, istart[src], istart[src + 1], false);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      m.x[w * m.ld + p] = g.x[w * g.ld + i];
      m.z[w * m.ld + p] = g.z[w * g.ld + i];
    }
    m.c[p] = g.c[i];
  }
}

template <int W>
__global__ void k_sl_merge_b(Flat im, const uint32_t* im_label, int64_t nimg, const int64_t* istart,
                             Flat g, const int64_t* start, const int64_t* mstart, uint32_t fullmask,
                             Flat m) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nimg; q += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t src = im_label[q];
    const uint32_t j = src ^ fullmask;
    const int64_t p = mstart[j] + (q - istart[src]) + rank_in<W>(im, q, g, start[j], start[j + 1], true);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      m.x[w * m.ld + p] = im.x[w * im.ld + q];
      m.z[w * m.ld + p] = im.z[w * im.ld + q];
    }
    m.c[p] = im.c[q];
  }
}

// Equal neighbours are one key's two contributions: the first keeps their
// sum, the second is dropped; then |c| < eps is dropped.
template <int W>
__global__ void k_sl_combine(Flat m, int64_t total, double eps, double* value, int64_t* keep) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
    const bool second = p > 0 && canon_cmp<W>(m, p, m, p - 1) == 0;
    const bool pair = p + 1 < total && canon_cmp<W>(m, p, m, p + 1) == 0;
    const double v = pair ? __dadd_rn(m.c[p], m.c[p + 1]) : m.c[p];
    value[p] = v;
    keep[p] = (!second && !(fabs(v) < eps)) ? 1 : 0;
  }
}

template <int W>
__global__ void k_sl_compact(Flat m, const double* value, int64_t total, const int64_t* keep,
                             const int64_t* pos, Flat d) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
    if (!keep[p]) continue;
    const int64_t q = pos[p];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      d.x[w * d.ld + q] = m.x[w * m.ld + p];
      d.z[w * d.ld + q] = m.z[w * m.ld + p];
    }
    d.c[q] = value[p];
  }
}

// Run boundaries after compaction: dstart[j] = compacted position of mstart[j].
__global__ void k_sl_dstart(const int64_t* mstart, const int64_t* pos, const int64_t* keep,
                            int64_t total, int64_t npart, int64_t* dstart) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= npart; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = mstart[j];
    dstart[j] = p < total ? pos[p] : (total > 0 ? pos[total - 1] + keep[total - 1] : 0);
  }
}

// One multiway-merge round: run r (elements [rs[r], rs[r+1])) merges with run
// r ^ 1 into run r >> 1 of the next round.
template <int W>
__global__ void k_sl_round(Flat a, int64_t n, const int64_t* rs, int64_t nruns, Flat b) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    // run of element i: last r with rs[r] <= i
    int64_t lo = 0, hi = nruns - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (rs[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const int64_t r = lo;
    const int64_t partner = r ^ 1;
    int64_t rank = 0;
    if (partner < nruns) rank = rank_in<W>(a, i, a, rs[partner], rs[partner + 1], (r & 1) != 0);
    const int64_t p = rs[r & ~1ll] + (i - rs[r]) + rank;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      b.x[w * b.ld + p] = a.x[w * a.ld + i];
      b.z[w * b.ld + p] = a.z[w * a.ld + i];
    }
    b.c[p] = a.c[i];
  }
}

__global__ void k_sl_next_runs(const int64_t* rs, int64_t nruns, int64_t* out) {
  const int64_t nn = (nruns + 1) >> 1;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k <= nn; k += (int64_t)gridDim.x * blockDim.x)
    out[k] = k < nn ? rs[2 * k] : rs[nruns];
}

namespace {

struct DevMem {
  std::vector<void*> p;
  ~DevMem() {
    for (void* q : p) (void)hipFree(q);
  }
  template <class T>
  T* get(size_t count, hipError_t& e) {
    void* q = nullptr;
    if (e == hipSuccess) e = hipMalloc(&q, count ? count * sizeof(T) : sizeof(T));
    if (e == hipSuccess) p.push_back(q);
    return (T*)q;
  }
  Flat flat(int W, int64_t rows, hipError_t& e) {
    Flat f{};
    f.ld = rows > 0 ? rows : 1;
    f.x = get<uint64_t>((size_t)W * f.ld, e);
    f.z = get<uint64_t>((size_t)W * f.ld, e);
    f.c = get<double>((size_t)f.ld, e);
    return f;
  }
};

int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : g > 8192 ? 8192 : g);
}

template <int W>
hipError_t sortless_w(const Flat& h, int64_t n, const PauliKey& P, int nbits, double C, double S,
                      double eps, const Flat& out, int64_t cap, int64_t* n_out, hipStream_t s) {
  hipError_t e = hipSuccess;
  DevMem mem;
  const int64_t npart = 1ll << nbits;
  const uint32_t fullmask = (uint32_t)(npart - 1);
  // 1. stable partition by the flipped bits
  uint32_t* label = mem.get<uint32_t>(n, e);
  uint32_t* idx = mem.get<uint32_t>(n, e);
  uint32_t* label_s = mem.get<uint32_t>(n, e);
  uint32_t* perm = mem.get<uint32_t>(n, e);
  int64_t* start = mem.get<int64_t>(npart + 1, e);
  if (e != hipSuccess) return e;
  int64_t* flag = mem.get<int64_t>(n, e);
  int64_t* pos = mem.get<int64_t>(n, e);
  int64_t* sc = mem.get<int64_t>((n + 1023) / 1024 + 2, e);
  if (e != hipSuccess) return e;
  // nbits stable binary splits between the buffers (label, idx) and
  // (label_s, perm); the labels start in the one that makes the last split
  // land in (label_s, perm)
  const int passes = nbits > 0 ? nbits : 1;
  uint32_t* cur_l = (passes & 1) ? label : label_s;
  uint32_t* cur_i = (passes & 1) ? idx : perm;
  uint32_t* oth_l = (passes & 1) ? label_s : label;
  uint32_t* oth_i = (passes & 1) ? perm : idx;
  hipLaunchKernelGGL(k_sl_labels<W>, dim3(grid_for(n)), dim3(kBlock), 0, s, h, n, P, cur_l, cur_i);
  if (n > 0) {
    for (int b = 0; b < passes; ++b) {
      hipLaunchKernelGGL(k_sl_bitflag, dim3(grid_for(n)), dim3(kBlock), 0, s, cur_l, n, b, flag);
      launch_scan_i64(flag, pos, n, sc, s);
      hipLaunchKernelGGL(k_sl_split, dim3(grid_for(n)), dim3(kBlock), 0, s, cur_l, cur_i, n, flag, pos, oth_l,
                         oth_i);
      uint32_t* t = cur_l; cur_l = oth_l; oth_l = t;
      t = cur_i; cur_i = oth_i; oth_i = t;
    }
  }
  hipLaunchKernelGGL(k_sl_bounds, dim3(grid_for(n + 1)), dim3(kBlock), 0, s, label_s, n, npart, start);
  // 2. rotate in place (partition order) and write the images
  Flat g = mem.flat(W, n, e);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sl_gather<W>, dim3(grid_for(n)), dim3(kBlock), 0, s, h, perm, n, P, C, g, flag);
  launch_scan_i64(flag, pos, n, sc, s);
  int64_t nimg = 0;
  if (n > 0) {
    int64_t last[2];
    e = hipMemcpyAsync(&last[0], pos + n - 1, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&last[1], flag + n - 1, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    nimg = last[0] + last[1];
  }
  Flat im = mem.flat(W, nimg, e);
  uint32_t* im_label = mem.get<uint32_t>(nimg, e);
  int64_t* istart = mem.get<int64_t>(npart + 1, e);
  int64_t* size = mem.get<int64_t>(npart + 1, e);
  int64_t* mstart = mem.get<int64_t>(npart + 1, e);
  int64_t* sc2 = mem.get<int64_t>((npart + 1023) / 1024 + 2, e);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sl_images<W>, dim3(grid_for(n)), dim3(kBlock), 0, s, h, perm, label_s, n, P, S,
                     flag, pos, im, im_label);
  hipLaunchKernelGGL(k_sl_dstart, dim3(grid_for(npart + 1)), dim3(kBlock), 0, s, start, pos, flag, n,
                     npart, istart);
  // 3. merge per destination partition, combine equal neighbours, compress
  hipLaunchKernelGGL(k_sl_sizes, dim3(grid_for(npart)), dim3(kBlock), 0, s, start, istart, npart,
                     fullmask, size);
  launch_scan_i64(size, mstart, npart, sc2, s);
  const int64_t total = n + nimg;
  e = hipMemcpyAsync(mstart + npart, &total, 8, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  Flat m = mem.flat(W, total, e);
  double* value = mem.get<double>(total, e);
  int64_t* keep = mem.get<int64_t>(total, e);
  int64_t* kpos = mem.get<int64_t>(total, e);
  int64_t* sc3 = mem.get<int64_t>((total + 1023) / 1024 + 2, e);
  int64_t* rs = mem.get<int64_t>(npart + 1, e);
  int64_t* rs2 = mem.get<int64_t>(npart + 1, e);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sl_merge_a<W>, dim3(grid_for(n)), dim3(kBlock), 0, s, g, label_s, n, start, im,
                     istart, mstart, fullmask, m);
  hipLaunchKernelGGL(k_sl_merge_b<W>, dim3(grid_for(nimg)), dim3(kBlock), 0, s, im, im_label, nimg,
                     istart, g, start, mstart, fullmask, m);
  hipLaunchKernelGGL(k_sl_combine<W>, dim3(grid_for(total)), dim3(kBlock), 0, s, m, total, eps, value,
                     keep);
  launch_scan_i64(keep, kpos, total, sc3, s);
  int64_t nd = 0;
  if (total > 0) {
    int64_t last[2];
    e = hipMemcpyAsync(&last[0], kpos + total - 1, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&last[1], keep + total - 1, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    nd = last[0] + last[1];
  }
  *n_out = nd;
  if (nd > cap) return hipErrorInvalidValue;
  // runs of the compacted list: one per partition
  Flat d = mem.flat(W, nd, e);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sl_compact<W>, dim3(grid_for(total)), dim3(kBlock), 0, s, m, value, total, keep,
                     kpos, d);
  hipLaunchKernelGGL(k_sl_dstart, dim3(grid_for(npart + 1)), dim3(kBlock), 0, s, mstart, kpos, keep,
                     total, npart, rs);
  // 4. multiway merge: pairs of sorted runs, log2(npart) rounds, ending in `out`
  int rounds = 0;
  for (int64_t r = npart; r > 1; r = (r + 1) >> 1) ++rounds;
  Flat a = d, b = out;
  if (rounds % 2 == 0) {
    // an even number of rounds ends where it starts: start from a copy in `out`
    for (int w = 0; w < W && nd > 0; ++w) {
      e = hipMemcpyAsync(out.x + w * out.ld, d.x + w * d.ld, 8 * nd, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(out.z + w * out.ld, d.z + w * d.ld, 8 * nd, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return e;
    }
    if (nd > 0) e = hipMemcpyAsync(out.c, d.c, 8 * nd, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    a = out;
    b = d;
  }
  int64_t* cur = rs;
  int64_t* nxt = rs2;
  int64_t nruns = npart;
  while (nruns > 1) {
    if (nd > 0)
      hipLaunchKernelGGL(k_sl_round<W>, dim3(grid_for(nd)), dim3(kBlock), 0, s, a, nd, cur, nruns, b);
    hipLaunchKernelGGL(k_sl_next_runs, dim3(grid_for(nruns / 2 + 2)), dim3(kBlock), 0, s, cur, nruns, nxt);
    nruns = (nruns + 1) >> 1;
    std::swap(cur, nxt);
    std::swap(a, b);
  }
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

}  // namespace

hipError_t sortless_dress_run(int W, const uint64_t* x, const uint64_t* z, const double* c, int64_t n,
                              int64_t ld, const PauliKey& P, int nbits, double C, double S, double eps,
                              uint64_t* ox, uint64_t* oz, double* oc, int64_t cap, int64_t ld_out,
                              int64_t* n_out, hipStream_t s) {
  Flat h{(uint64_t*)x, (uint64_t*)z, (double*)c, ld};
  Flat out{ox, oz, oc, ld_out};
  switch (W) {
    case 1: return sortless_w<1>(h, n, P, nbits, C, S, eps, out, cap, n_out, s);
    case 2: return sortless_w<2>(h, n, P, nbits, C, S, eps, out, cap, n_out, s);
    case 3: return sortless_w<3>(h, n, P, nbits, C, S, eps, out, cap, n_out, s);
    default: return sortless_w<4>(h, n, P, nbits, C, S, eps, out, cap, n_out, s);
  }
}

}  // namespace iqcc
