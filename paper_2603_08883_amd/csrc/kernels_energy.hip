// QMF energy (Sec. II, Eq. 3; energy functional of App. A) and its gradient
// with respect to the Bloch angles.
//
// <K> of the product state is prod_j b_j(sigma_j) with b(I) = 1,
// b(X) = sin t cos f, b(Y) = sin t sin f, b(Z) = cos t.  Terms are streamed
// once; the product uses a 3-qubit-group table in LDS and skips identity
// groups.  Partial sums are per workgroup and reduced in a fixed order.
#include <cfloat>

#include "iqcc_internal.h"

#pragma clang fp contract(off)

namespace iqcc {

__global__ void k_build_lut(int W, int nq, const double* theta, const double* phi, double* lut) {
  const int n = W * kGroupsPerWord * kLutEntries;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int idx = e % kLutEntries;
    const int gi = e / kLutEntries;
    const int h = gi / kGroupsPerHalf, g = gi % kGroupsPerHalf;
    double p = 1.0;
    for (int i = 0; i < 3; ++i) {
      const int bitpos = 3 * g + i;          // bit within the 32-bit half
      const int q = 32 * h + bitpos;
      if (bitpos >= 32 || q >= nq) continue;
      const int op = ((idx >> i) & 1) | (((idx >> (3 + i)) & 1) << 1);
      if (op == 0) continue;
      double st, ct, sp, cp;
      sincos(theta[q], &st, &ct);
      sincos(phi[q], &sp, &cp);
      p *= bloch_factor(op, st, ct, sp, cp);
    }
    lut[e] = p;
  }
}

void launch_build_lut(int W, int nq, const double* theta, const double* phi, double* lut,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_build_lut, dim3(16), dim3(kBlock), 0, s, W, nq, theta, phi, lut);
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of per-workgroup partials: out = scale * sum.
// ---------------------------------------------------------------------------
__global__ void k_finalize_sum(const double* partial, int n, const double* scale,
                               const double* base, double* out) {
  __shared__ double red[kWaves];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += partial[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    if (scale) s *= *scale;
    *out = base ? *base + s : s;
  }
}

void launch_finalize_sum(const double* partial, int n, const double* scale, double* out,
                         hipStream_t s, const double* base) {
  hipLaunchKernelGGL(k_finalize_sum, dim3(1), dim3(kBlock), 0, s, partial, n, scale, base, out);
}

// Exact sum of FixedSum parts (hi, lo, mag as three 8-byte words each).
__global__ void k_finalize_fixed(const double* parts, int n, double* out) {
  __shared__ long long red_hi[kWaves], red_lo[kWaves];
  __shared__ double red_mag[kWaves];
  FixedSum f;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    f.hi += __double_as_longlong(parts[3 * i]);
    f.lo += __double_as_longlong(parts[3 * i + 1]);
    f.mag += parts[3 * i + 2];
  }
  const FixedSum t = block_fixed_sum<kWaves>(f, red_hi, red_lo, red_mag);
  if (threadIdx.x == 0) *out = fixed_value(t.hi, t.lo, t.mag);
}

void launch_finalize_fixed(const double* parts, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_fixed, dim3(1), dim3(kBlock), 0, s, parts, n, out);
}

// <K> from every 3-qubit group of every half word, identity groups included
// (their table entry 0 is 1.0): a fixed, branch-free sequence of independent
// lookups whose addresses take two VALU operations each.
template <int W>
__device__ __forceinline__ double expect_dense(const double* lut, const uint64_t* x,
                                               const uint64_t* z) {
  double p[4] = {1.0, 1.0, 1.0, 1.0};
#pragma unroll
  for (int h = 0; h < 2 * W; ++h) {
    const uint32_t xh = (uint32_t)(x[h >> 1] >> (32 * (h & 1)));
    const uint32_t zh = (uint32_t)(z[h >> 1] >> (32 * (h & 1)));
    const double* lh = lut + h * kGroupsPerHalf * kLutEntries;
#pragma unroll
    for (int g = 0; g < kGroupsPerHalf; ++g) {
      const uint32_t code = __builtin_amdgcn_ubfe(xh, 3 * g, 3) | (__builtin_amdgcn_ubfe(zh, 3 * g, 3) << 3);
      p[g & 3] *= lh[g * kLutEntries + code];
    }
  }
  return (p[0] * p[1]) * (p[2] * p[3]);
}

// ---------------------------------------------------------------------------
// Energy of a store.  Workgroup g takes the groups of G consecutive buckets
// g, g + grid, ... (G = 1 .. 256 so that every workgroup has a group); the
// rows of a group's buckets are streamed as one flat range, kEItems terms per
// thread and pass, so small buckets do not each cost a round trip.
// ---------------------------------------------------------------------------
constexpr int kEItems = 4;

template <int W>
__global__ __launch_bounds__(kBlock) void k_energy(StoreDev st, const double* lut_g, double* partial) {
  __shared__ double lut[W * kGroupsPerWord * kLutEntries];
  __shared__ double red[kWaves];
  __shared__ uint64_t scan_tmp[kWaves];
  __shared__ int64_t s_pre[kBlock + 1];
  __shared__ int64_t s_off[kBlock];
  for (int i = threadIdx.x; i < W * kGroupsPerWord * kLutEntries; i += kBlock) lut[i] = lut_g[i];
  const int64_t B = 1ll << *st.m;
  int64_t G = B / gridDim.x;
  G = G < 1 ? 1 : (G > kBlock ? kBlock : G);
  const int64_t ngroups = (B + G - 1) / G;
  double acc = 0.0;
  __syncthreads();
  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t b = grp * G + threadIdx.x;
    const bool mine = threadIdx.x < G && b < B;
    const int64_t cnt = mine ? st.cnt[b] : 0;
    const int64_t off = mine ? st.off[b] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan((uint64_t)cnt, scan_tmp, total);
    s_pre[threadIdx.x] = (int64_t)ex;
    s_off[threadIdx.x] = off;
    if (threadIdx.x == 0) s_pre[kBlock] = (int64_t)total;
    __syncthreads();
    const int64_t n = (int64_t)total;
    for (int64_t i0 = 0; i0 < n; i0 += kBlock * kEItems) {
      uint64_t kx[kEItems][W], kz[kEItems][W];
      double kc[kEItems];
#pragma unroll
      for (int r = 0; r < kEItems; ++r) {
        const int64_t i = i0 + r * kBlock + threadIdx.x;
        kc[r] = 0.0;
#pragma unroll
        for (int w = 0; w < W; ++w) kx[r][w] = kz[r][w] = 0;
        if (i < n) {
          int lo = 0;   // the last bucket of the group whose first row is <= i
#pragma unroll
          for (int step = kBlock / 2; step; step >>= 1)
            if (s_pre[lo + step] <= i) lo += step;
          const int64_t row = s_off[lo] + (i - s_pre[lo]);
#pragma unroll
          for (int w = 0; w < W; ++w) {
            kx[r][w] = __builtin_nontemporal_load(&st.x[w * st.cap + row]);
            kz[r][w] = __builtin_nontemporal_load(&st.z[w * st.cap + row]);
          }
          kc[r] = __builtin_nontemporal_load(&st.c[row]);
        }
      }
#pragma unroll
      for (int r = 0; r < kEItems; ++r) acc += kc[r] * expect_dense<W>(lut, kx[r], kz[r]);
    }
    __syncthreads();
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

void launch_energy(int W, const StoreDev& st, int grid, const double* lut, double* e_partial,
                   hipStream_t s) {
  switch (W) {
    case 1: hipLaunchKernelGGL(k_energy<1>, dim3(grid), dim3(kBlock), 0, s, st, lut, e_partial); break;
    case 2: hipLaunchKernelGGL(k_energy<2>, dim3(grid), dim3(kBlock), 0, s, st, lut, e_partial); break;
    case 3: hipLaunchKernelGGL(k_energy<3>, dim3(grid), dim3(kBlock), 0, s, st, lut, e_partial); break;
    default: hipLaunchKernelGGL(k_energy<4>, dim3(grid), dim3(kBlock), 0, s, st, lut, e_partial); break;
  }
}

// ---------------------------------------------------------------------------
// Stand-alone energy with a table per 4-qubit group ("nibble"): 16 groups per
// key word, 256 entries each (4 x bits, 4 z bits), 32 KB per word in LDS, so
// keys of up to two words.  A byte of x and the same byte of z hold two
// nibbles; two bit-field inserts per 32-bit half word put the codes of its
// eight groups into the bytes of two registers, and each lookup takes one byte
// extraction: 32 lookups per two-word term instead of 44, at about a third of
// the address arithmetic.
// ---------------------------------------------------------------------------
constexpr int kNibbleEntries = 256;
constexpr int kNibblesPerWord = 16;
constexpr int kE4Block = 512;

__global__ void k_build_lut4(int W, int nq, const double* theta, const double* phi, double* lut) {
  const int n = W * kNibblesPerWord * kNibbleEntries;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int code = e % kNibbleEntries;
    const int gi = e / kNibbleEntries;   // qubits 4 gi .. 4 gi + 3
    double p = 1.0;
    for (int r = 0; r < 4; ++r) {
      const int q = 4 * gi + r;
      if (q >= nq) continue;
      const int op = ((code >> r) & 1) | (((code >> (4 + r)) & 1) << 1);
      if (op == 0) continue;
      double st, ct, sp, cp;
      sincos(theta[q], &st, &ct);
      sincos(phi[q], &sp, &cp);
      p *= bloch_factor(op, st, ct, sp, cp);
    }
    lut[e] = p;
  }
}

template <int W>
__device__ __forceinline__ double expect_nibble(const double* lut, const uint64_t* x, const uint64_t* z) {
  double p[4] = {1.0, 1.0, 1.0, 1.0};
#pragma unroll
  for (int h = 0; h < 2 * W; ++h) {
    const uint32_t xh = (uint32_t)(x[h >> 1] >> (32 * (h & 1)));
    const uint32_t zh = (uint32_t)(z[h >> 1] >> (32 * (h & 1)));
    // byte k: code of nibble 2k (lo) and of nibble 2k + 1 (hi), x bits low
    const uint32_t lo = ((zh << 4) & 0xF0F0F0F0u) | (xh & 0x0F0F0F0Fu);
    const uint32_t hi = ((xh >> 4) & 0x0F0F0F0Fu) | (zh & 0xF0F0F0F0u);
    const double* lh = lut + 8 * h * kNibbleEntries;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      p[k] *= lh[(2 * k) * kNibbleEntries + ((lo >> (8 * k)) & 0xFFu)];
      p[k] *= lh[(2 * k + 1) * kNibbleEntries + ((hi >> (8 * k)) & 0xFFu)];
    }
  }
  return (p[0] * p[1]) * (p[2] * p[3]);
}

template <int W>
__global__ __launch_bounds__(kE4Block) void k_energy4(StoreDev st, const double* lut_g, double* partial) {
  constexpr int NE = W * kNibblesPerWord * kNibbleEntries;
  extern __shared__ __align__(16) unsigned char smem_e4[];
  double* lut = (double*)smem_e4;
  int64_t* s_pre = (int64_t*)(lut + NE);     // [kE4Block + 1]
  int64_t* s_off = s_pre + kE4Block + 1;     // [kE4Block]
  __shared__ double red[kE4Block / 64];
  __shared__ uint64_t scan_tmp[kE4Block / 64];
  for (int i = threadIdx.x; i < NE; i += kE4Block) lut[i] = lut_g[i];
  const int64_t B = 1ll << *st.m;
  int64_t G = B / gridDim.x;
  G = G < 1 ? 1 : (G > kE4Block ? kE4Block : G);
  const int64_t ngroups = (B + G - 1) / G;
  double acc = 0.0;
  __syncthreads();
  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t b = grp * G + threadIdx.x;
    const bool mine = threadIdx.x < G && b < B;
    const int64_t cnt = mine ? st.cnt[b] : 0;
    const int64_t off = mine ? st.off[b] : 0;
    uint64_t total;
    // (the scan's barriers also order the previous group's reads of s_pre)
    const uint64_t ex = block_exclusive_scan_n<kE4Block / 64>((uint64_t)cnt, scan_tmp, total);
    s_pre[threadIdx.x] = (int64_t)ex;
    s_off[threadIdx.x] = off;
    if (threadIdx.x == 0) s_pre[kE4Block] = (int64_t)total;
    __syncthreads();
    const int64_t n = (int64_t)total;
    for (int64_t i0 = 0; i0 < n; i0 += kE4Block * kEItems) {
      uint64_t kx[kEItems][W], kz[kEItems][W];
      double kc[kEItems];
#pragma unroll
      for (int r = 0; r < kEItems; ++r) {
        const int64_t i = i0 + r * kE4Block + threadIdx.x;
        kc[r] = 0.0;
#pragma unroll
        for (int w = 0; w < W; ++w) kx[r][w] = kz[r][w] = 0;
        if (i < n) {
          int lo = 0;   // the last bucket of the group whose first row is <= i
#pragma unroll
          for (int step = kE4Block / 2; step; step >>= 1)
            if (s_pre[lo + step] <= i) lo += step;
          const int64_t row = s_off[lo] + (i - s_pre[lo]);
#pragma unroll
          for (int w = 0; w < W; ++w) {
            kx[r][w] = __builtin_nontemporal_load(&st.x[w * st.cap + row]);
            kz[r][w] = __builtin_nontemporal_load(&st.z[w * st.cap + row]);
          }
          kc[r] = __builtin_nontemporal_load(&st.c[row]);
        }
      }
#pragma unroll
      for (int r = 0; r < kEItems; ++r) acc += kc[r] * expect_nibble<W>(lut, kx[r], kz[r]);
    }
  }
  const double s = block_sum_n<kE4Block / 64>(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

int energy_lut_doubles(int W) {
  return W <= 2 ? W * kNibblesPerWord * kNibbleEntries : W * kGroupsPerWord * kLutEntries;
}

void launch_energy_table(int W, int nq, const StoreDev& st, int grid, const double* theta,
                         const double* phi, double* lut, double* partial, hipStream_t s) {
  if (W > 2) {
    launch_build_lut(W, nq, theta, phi, lut, s);
    launch_energy(W, st, grid, lut, partial, s);
    return;
  }
  hipLaunchKernelGGL(k_build_lut4, dim3(16), dim3(kBlock), 0, s, W, nq, theta, phi, lut);
  const size_t lds = (size_t)W * kNibblesPerWord * kNibbleEntries * 8 + (size_t)(2 * kE4Block + 1) * 8;
  if (W == 1) {
    (void)hipFuncSetAttribute((const void*)k_energy4<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_energy4<1>, dim3(grid), dim3(kE4Block), lds, s, st, lut, partial);
  } else {
    (void)hipFuncSetAttribute((const void*)k_energy4<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_energy4<2>, dim3(grid), dim3(kE4Block), lds, s, st, lut, partial);
  }
}

// ---------------------------------------------------------------------------
// Backward w.r.t. the Bloch angles (derivative of the Eq. 3 energy).
// dE/dtheta_q = sum_sigma S[q][sigma] db_sigma/dtheta (likewise phi), where
// S[q][sigma] adds, over the terms with sigma on qubit q, c times the product
// of the term's other factors.
//
// The product of a term runs over its 3-qubit groups (the energy table L), so
// the derivative is first formed per group table entry:
//   T[g][e] = sum over the terms whose group g has code e != 0 of
//             c * prod_{g' != g} L_g',
// and once per workgroup S[q][sigma] = sum over the codes e of q's group with
// sigma at q's position of T[g][e] * (product of the group's other qubit
// factors of that code).  The product of a term's other groups comes from
// prefix and suffix products -- inside each 32-bit half word over its 11
// groups, and across the half words over their products -- with no division,
// so vanishing factors need no special case.
//
// Summation order does not change the result.  Each value is split into two
// integers, round(v * 2^20) and round((v - that * 2^-20) * 2^60), and added
// to two 64-bit integer tables with LDS atomics, which are exact; per
// workgroup the two sums turn into one double, and the per-workgroup S are
// reduced in a fixed order, so dE/dtheta and dE/dphi are the same on every
// run.  The split is exact for |v| < 2^31 and the sums cannot overflow while
// (largest |c| of the workgroup's terms) * (its term count) < 2^42 and the
// count is below 2^23; a workgroup past these bounds, or one that meets a
// non-finite coefficient or angle, writes NaN instead of its S.  Resolution:
// 2^-61 per added value.
// acc layout per workgroup: [3 * nq] with sigma order X, Z, Y.
// ---------------------------------------------------------------------------
constexpr int kBwdBlock = 512;
constexpr int kBwdGroup = 256;   // most buckets per group of one flat range
// LDS tables of the backward hold each 3-qubit group's 64 entries at a stride
// of 65, so that equal codes of different groups fall in different banks.
constexpr int kBwdStride = kLutEntries + 1;

size_t energy_bwd_lds_bytes(int W) {
  // energy table, the two integer tables (the per-qubit factors of the
  // epilogue reuse the first), bucket-group scan
  return (size_t)3 * W * kGroupsPerWord * kBwdStride * 8 + (size_t)(2 * kBwdGroup + 1) * 8;
}

// Workgroups per CU that the LDS of one CU holds (160 KiB), at most 2048
// threads (32 waves) in all.
int energy_bwd_blocks_per_cu(int W) {
  const int k = (int)((size_t)160 * 1024 / (energy_bwd_lds_bytes(W) + 512));
  const int kmax = 2048 / kBwdBlock;
  return k < 1 ? 1 : k > kmax ? kmax : k;
}

// v as round(v * 2^20) * 2^-20 + round(r * 2^60) * 2^-60 (r the remainder),
// both added to their integer tables.  Adding 1.5 * 2^32 (resp. 1.5 * 2^-8)
// rounds to a multiple of 2^-20 (2^-60), and the difference of the bit
// patterns is that multiple as an integer (both sums stay in the binade of the
// constant, whose low 32 bits are zero).
__device__ __forceinline__ void add_fixed(unsigned long long* hi, unsigned long long* lo, int e, double v) {
  const double k1 = 0x1.8p32, k0 = 0x1.8p-8;
  const double a1 = v + k1;
  const double r = v - (a1 - k1);
  const double a0 = r + k0;
  atomicAdd(&hi[e], (unsigned long long)(__double_as_longlong(a1) - __double_as_longlong(k1)));
  atomicAdd(&lo[e], (unsigned long long)(__double_as_longlong(a0) - __double_as_longlong(k0)));
}

// One term of the backward: T contributions of its non-identity groups and,
// when lam is given, its cotangent.
template <int W>
__device__ __forceinline__ void bwd_term(const double* lut, unsigned long long* thi,
                                         unsigned long long* tlo, const uint64_t* kx,
                                         const uint64_t* kz, double c, double* lam_row,
                                         double scale) {
  constexpr int NH = kGroupsPerHalf * kBwdStride;
  // products of the 2W half words (identity groups read entry 0 = 1.0)
  double hp[2 * W];
#pragma unroll
  for (int h = 0; h < 2 * W; ++h) {
    const uint32_t xh = (uint32_t)(kx[h >> 1] >> (32 * (h & 1)));
    const uint32_t zh = (uint32_t)(kz[h >> 1] >> (32 * (h & 1)));
    const double* lh = lut + h * NH;
    double p0 = 1.0, p1 = 1.0;
#pragma unroll
    for (int g = 0; g < kGroupsPerHalf; ++g) {
      const uint32_t code = __builtin_amdgcn_ubfe(xh, 3 * g, 3) | (__builtin_amdgcn_ubfe(zh, 3 * g, 3) << 3);
      if (g & 1) p1 *= lh[g * kBwdStride + code]; else p0 *= lh[g * kBwdStride + code];
    }
    hp[h] = p0 * p1;
  }
  // <K> for the coefficient cotangent
  if (lam_row) {
    double all = hp[0];
#pragma unroll
    for (int h = 1; h < 2 * W; ++h) all *= hp[h];
    *lam_row = scale * all;
  }
  // c times the product of the other half words, per half word
  double ho[2 * W];
  double pre = c;
#pragma unroll
  for (int h = 0; h < 2 * W; ++h) { ho[h] = pre; pre *= hp[h]; }
  double suf = 1.0;
#pragma unroll
  for (int h = 2 * W - 1; h >= 0; --h) { ho[h] *= suf; suf *= hp[h]; }
  // each half word: prefix and suffix over its groups.  A term visits its
  // half words, and the groups of each, starting at ones picked from its own
  // key bits, so that the lanes of a wave add into different groups' tables
  // at a time (fewer lanes on one LDS address or bank); the values do not
  // depend on where the term sits in the store.
  const uint32_t mix = ((uint32_t)kx[0] ^ (uint32_t)(kz[0] >> 29) ^ (uint32_t)(kx[W - 1] >> 35)) * 0x9E3779B1u;
  const int rot = (int)__umulhi(mix, 2u * W);
#pragma unroll 1
  for (int j = 0; j < 2 * W; ++j) {
    int h = rot + j;
    h = h >= 2 * W ? h - 2 * W : h;
    uint64_t xw = kx[0], zw = kz[0];
    double oh = ho[0];
#pragma unroll
    for (int u = 1; u < 2 * W; ++u) {
      if (u == h) oh = ho[u];
      if ((u & 1) == 0 && u == (h & ~1)) { xw = kx[u >> 1]; zw = kz[u >> 1]; }
    }
    const uint32_t xh = (uint32_t)(xw >> (32 * (h & 1)));
    const uint32_t zh = (uint32_t)(zw >> (32 * (h & 1)));
    const int rg = (int)__umulhi(mix * 0x85EBCA6Bu, (uint32_t)kGroupsPerHalf);
    const uint64_t xr = ((uint64_t)xh | ((uint64_t)xh << 33)) >> (3 * rg);
    const uint64_t zr = ((uint64_t)zh | ((uint64_t)zh << 33)) >> (3 * rg);
    double L[kGroupsPerHalf];
    uint32_t code[kGroupsPerHalf];
    int idx[kGroupsPerHalf];
    // group rg + g of the half, wrapped: the base before and after the wrap
    const int base_lo = h * NH + rg * kBwdStride;
    const int base_hi = base_lo - kGroupsPerHalf * kBwdStride;
#pragma unroll
    for (int g = 0; g < kGroupsPerHalf; ++g) {
      code[g] = (uint32_t)((xr >> (3 * g)) & 7) | ((uint32_t)((zr >> (3 * g)) & 7) << 3);
      idx[g] = (rg < kGroupsPerHalf - g ? base_lo : base_hi) + g * kBwdStride + (int)code[g];
      L[g] = lut[idx[g]];
    }
    double sf[kGroupsPerHalf];
    sf[kGroupsPerHalf - 1] = 1.0;
#pragma unroll
    for (int g = kGroupsPerHalf - 1; g > 0; --g) sf[g - 1] = sf[g] * L[g];
    double pg = oh;
#pragma unroll
    for (int g = 0; g < kGroupsPerHalf; ++g) {
      if (code[g] != 0) add_fixed(thi, tlo, idx[g], pg * sf[g]);
      pg *= L[g];
    }
  }
}

template <int W>
__global__ __launch_bounds__(kBwdBlock, 4) void k_energy_bwd(StoreDev st, int nq, const double* theta,
                                                             const double* phi, const double* lut_g,
                                                             const double* dE, double* lam,
                                                             double* acc_g) {
  constexpr int NE = W * kGroupsPerWord * kBwdStride;
  constexpr int NH = kGroupsPerHalf * kBwdStride;   // entries per half word
  extern __shared__ __align__(16) unsigned char smem_bwd[];
  double* lut = (double*)smem_bwd;                                     // [NE] L per group entry
  unsigned long long* thi = (unsigned long long*)(lut + NE);           // [NE] sums of round(v 2^20)
  unsigned long long* tlo = thi + NE;                                  // [NE] sums of the remainders
  double* fac = (double*)thi;   // epilogue: per qubit, factor of I, X, Z, Y (4 * 64W <= NE)
  int64_t* s_pre = (int64_t*)(tlo + NE);                               // [kBwdGroup + 1] group scan
  int64_t* s_off = s_pre + kBwdGroup + 1;                              // [kBwdGroup] first rows
  __shared__ double s_cmax[kBwdBlock / 64];
  __shared__ long long s_cnt[kBwdBlock / 64];
  __shared__ uint64_t scan_tmp[kBwdBlock / 64];
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < NE; i += kBwdBlock) {
    const int k = i % kBwdStride;
    lut[i] = k < kLutEntries ? lut_g[i / kBwdStride * kLutEntries + k] : 0.0;
    thi[i] = tlo[i] = 0ull;
  }
  for (int q = threadIdx.x; q < nq; q += kBwdBlock)
    if (!(fabs(theta[q]) <= DBL_MAX && fabs(phi[q]) <= DBL_MAX)) s_bad = 1;
  const double scale = dE ? *dE : 1.0;
  bool ok = true;   // every coefficient finite and below 2^31 in magnitude
  double cmax = 0.0;
  long long nmine = 0;
  // Workgroup g takes the groups of G consecutive buckets g, g + grid, ...;
  // a group's rows are one flat range, one term per thread and pass, the next
  // pass's term loaded while this one is processed.
  const int64_t B = 1ll << *st.m;
  int64_t G = B / gridDim.x;
  G = G < 1 ? 1 : (G > kBwdGroup ? kBwdGroup : G);
  const int64_t ngroups = (B + G - 1) / G;
  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t b = grp * G + threadIdx.x;
    const bool mine = threadIdx.x < G && b < B;
    const int64_t cnt = mine ? st.cnt[b] : 0;
    const int64_t off = mine ? st.off[b] : 0;
    uint64_t total;
    // (the scan's barriers also order the previous group's reads of s_pre)
    const uint64_t ex = block_exclusive_scan_n<kBwdBlock / 64>((uint64_t)cnt, scan_tmp, total);
    if (threadIdx.x < kBwdGroup) {
      s_pre[threadIdx.x] = (int64_t)ex;
      s_off[threadIdx.x] = off;
    }
    if (threadIdx.x == 0) s_pre[kBwdGroup] = (int64_t)total;
    __syncthreads();
    const int64_t n = (int64_t)total;
    auto row_of = [&](int64_t i) {
      int lo = 0;   // the last bucket of the group whose first row is <= i
#pragma unroll
      for (int step = kBwdGroup / 2; step; step >>= 1)
        if (s_pre[lo + step] <= i) lo += step;
      return s_off[lo] + (i - s_pre[lo]);
    };
    uint64_t cx[W], cz[W], nx[W], nz[W];
    double cc = 0.0, nc = 0.0;
    int64_t crow = 0, nrow = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) cx[w] = cz[w] = 0;
    if (threadIdx.x < n) {
      crow = row_of(threadIdx.x);
#pragma unroll
      for (int w = 0; w < W; ++w) {
        cx[w] = __builtin_nontemporal_load(&st.x[w * st.cap + crow]);
        cz[w] = __builtin_nontemporal_load(&st.z[w * st.cap + crow]);
      }
      cc = __builtin_nontemporal_load(&st.c[crow]);
    }
    for (int64_t i0 = 0; i0 < n; i0 += kBwdBlock) {
      const int64_t in = i0 + kBwdBlock + threadIdx.x;
#pragma unroll
      for (int w = 0; w < W; ++w) nx[w] = nz[w] = 0;
      nc = 0.0;
      if (in < n) {
        nrow = row_of(in);
#pragma unroll
        for (int w = 0; w < W; ++w) {
          nx[w] = __builtin_nontemporal_load(&st.x[w * st.cap + nrow]);
          nz[w] = __builtin_nontemporal_load(&st.z[w * st.cap + nrow]);
        }
        nc = __builtin_nontemporal_load(&st.c[nrow]);
      }
      if (i0 + threadIdx.x < n) {
        ++nmine;
        ok = ok && fabs(cc) < 0x1p31;
        cmax = fmax(cmax, fabs(cc));
        bwd_term<W>(lut, thi, tlo, cx, cz, cc, lam ? lam + crow : nullptr, scale);
      }
#pragma unroll
      for (int w = 0; w < W; ++w) { cx[w] = nx[w]; cz[w] = nz[w]; }
      cc = nc;
      crow = nrow;
    }
  }
  // bounds of the exact integer sums (see above), over the workgroup
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    cmax = fmax(cmax, __shfl_xor(cmax, d, 64));
    nmine += __shfl_xor(nmine, d, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_cmax[threadIdx.x >> 6] = cmax;
    s_cnt[threadIdx.x >> 6] = nmine;
  }
  if (!ok) s_bad = 1;
  __syncthreads();
  double cm = 0.0;
  long long nwg = 0;
  for (int k = 0; k < kBwdBlock / 64; ++k) {
    cm = fmax(cm, s_cmax[k]);
    nwg += s_cnt[k];
  }
  const bool in_range = s_bad == 0 && nwg < (1ll << 23) && cm * (double)nwg < 0x1p42;
  // the sums as doubles, over the energy table (no longer needed), then the
  // per-qubit factors over the first integer table
  for (int i = threadIdx.x; i < NE; i += kBwdBlock)
    lut[i] = (double)(long long)thi[i] * 0x1p-20 + (double)(long long)tlo[i] * 0x1p-60;
  __syncthreads();
  for (int q = threadIdx.x; q < 64 * W; q += kBwdBlock) {
    double st_ = 0, ct = 1, sp = 0, cp = 1;
    if (q < nq) {
      sincos(theta[q], &st_, &ct);
      sincos(phi[q], &sp, &cp);
    }
    for (int op = 0; op < 4; ++op) fac[4 * q + op] = bloch_factor(op, st_, ct, sp, cp);
  }
  __syncthreads();
  // S[q][sigma] from T: the codes of q's group with sigma at q's position,
  // each weighted by the product of the group's other factors of that code
  for (int k = threadIdx.x; k < 3 * nq; k += kBwdBlock) {
    const int q = k / 3, op = k % 3 + 1;   // op: 1 = X, 2 = Z, 3 = Y
    const int h = q >> 5, bit = q & 31;
    const int g = (int)div3_small((uint32_t)bit), r = bit - 3 * g;
    const double* tg = lut + h * NH + g * kBwdStride;
    double s = 0.0;
    for (int code = 1; code < kLutEntries; ++code) {
      if ((((code >> r) & 1) | (((code >> (3 + r)) & 1) << 1)) != op) continue;
      double other = 1.0;
      bool valid = true;
      for (int r2 = 0; r2 < 3; ++r2) {
        if (r2 == r) continue;
        const int o2 = ((code >> r2) & 1) | (((code >> (3 + r2)) & 1) << 1);
        if (3 * g + r2 >= 32) {   // position past the half word: no qubit
          valid = valid && o2 == 0;
          continue;
        }
        other *= fac[4 * (32 * h + 3 * g + r2) + o2];
      }
      if (valid) s += tg[code] * other;
    }
    acc_g[(int64_t)blockIdx.x * 3 * nq + k] = in_range ? s : __builtin_nan("");
  }
}

template <int W>
static void launch_bwd_w(int nq, const StoreDev& st, int grid, const double* theta,
                         const double* phi, const double* lut, const double* dE, double* lam,
                         double* acc, hipStream_t s) {
  const size_t lds = energy_bwd_lds_bytes(W);
  (void)hipFuncSetAttribute((const void*)k_energy_bwd<W>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL(k_energy_bwd<W>, dim3(grid), dim3(kBwdBlock), lds, s, st, nq, theta, phi,
                     lut, dE, lam, acc);
}

void launch_energy_backward(int W, int nq, const StoreDev& st, int grid, const double* theta,
                            const double* phi, const double* lut, const double* dE, double* lam,
                            double* acc, hipStream_t s) {
  switch (W) {
    case 1: launch_bwd_w<1>(nq, st, grid, theta, phi, lut, dE, lam, acc, s); break;
    case 2: launch_bwd_w<2>(nq, st, grid, theta, phi, lut, dE, lam, acc, s); break;
    case 3: launch_bwd_w<3>(nq, st, grid, theta, phi, lut, dE, lam, acc, s); break;
    default: launch_bwd_w<4>(nq, st, grid, theta, phi, lut, dE, lam, acc, s); break;
  }
}

// One workgroup per qubit: S[q][sigma] summed over the per-workgroup
// partials in a fixed order, then the chain rule through the Bloch factors.
__global__ void k_backward_finalize(int nq, int grid, const double* acc, const double* theta,
                                    const double* phi, const double* dE, double* dtheta,
                                    double* dphi) {
  __shared__ double red[kWaves];
  const int q = blockIdx.x;
  double S[3];
  for (int k = 0; k < 3; ++k) {
    double v = 0.0;
    for (int g = threadIdx.x; g < grid; g += kBlock) v += acc[(int64_t)g * 3 * nq + 3 * q + k];
    S[k] = block_sum(v, red);   // valid in thread 0
  }
  if (threadIdx.x == 0) {
    double st, ct, sp, cp;
    sincos(theta[q], &st, &ct);
    sincos(phi[q], &sp, &cp);
    // sigma order X, Z, Y
    const double dt = S[0] * (ct * cp) + S[1] * (-st) + S[2] * (ct * sp);
    const double dp = S[0] * (-st * sp) + S[2] * (st * cp);
    const double sc = dE ? *dE : 1.0;
    dtheta[q] = sc * dt;
    dphi[q] = sc * dp;
  }
}

void launch_backward_finalize(int nq, int grid, const double* acc, const double* theta,
                              const double* phi, const double* dE, double* dtheta, double* dphi,
                              hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(k_backward_finalize, dim3(nq), dim3(kBlock), 0, s, nq, grid, acc, theta, phi,
                     dE, dtheta, dphi);
}

}  // namespace iqcc
