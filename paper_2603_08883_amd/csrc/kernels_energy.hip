// QMF energy (Sec. II, Eq. 3; energy functional of App. A) and its gradient
// with respect to the Bloch angles.
//
// <K> of the product state is prod_j b_j(sigma_j) with b(I) = 1,
// b(X) = sin t cos f, b(Y) = sin t sin f, b(Z) = cos t.  Terms are streamed
// once; the product uses a 3-qubit-group table in LDS and skips identity
// groups.  Partial sums are per workgroup and reduced in a fixed order.
#include "iqcc_internal.h"

#pragma clang fp contract(off)

namespace iqcc {

__device__ __forceinline__ double bloch_factor(int op, double st, double ct, double sp,
                                               double cp) {
  // op: 0 = I, 1 = X, 2 = Z, 3 = Y (bit0 = x, bit1 = z)
  return op == 0 ? 1.0 : op == 1 ? st * cp : op == 2 ? ct : st * sp;
}

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
// Energy of a store: workgroup g takes buckets g, g + grid, ...
// ---------------------------------------------------------------------------
constexpr int kEItems = 4;

template <int W>
__global__ __launch_bounds__(kBlock) void k_energy(StoreDev st, const double* lut_g,
                                                   double* partial) {
  __shared__ double lut[W * kGroupsPerWord * kLutEntries];
  __shared__ double red[kWaves];
  for (int i = threadIdx.x; i < W * kGroupsPerWord * kLutEntries; i += kBlock) lut[i] = lut_g[i];
  __syncthreads();
  const int64_t B = 1ll << *st.m;
  double acc = 0.0;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = st.cnt[b], off = st.off[b];
    for (int64_t i0 = 0; i0 < n; i0 += kBlock * kEItems) {
      uint64_t kx[kEItems][W], kz[kEItems][W];
      double kc[kEItems];
#pragma unroll
      for (int r = 0; r < kEItems; ++r) {
        const int64_t i = i0 + r * kBlock + threadIdx.x;
        kc[r] = 0.0;
        if (i < n) {
#pragma unroll
          for (int w = 0; w < W; ++w) {
            kx[r][w] = __builtin_nontemporal_load(&st.x[w * st.cap + off + i]);
            kz[r][w] = __builtin_nontemporal_load(&st.z[w * st.cap + off + i]);
          }
          kc[r] = __builtin_nontemporal_load(&st.c[off + i]);
        } else {
#pragma unroll
          for (int w = 0; w < W; ++w) kx[r][w] = kz[r][w] = 0;
        }
      }
#pragma unroll
      for (int r = 0; r < kEItems; ++r) acc += kc[r] * expect_dense<W>(lut, kx[r], kz[r]);
    }
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
// Backward w.r.t. the Bloch angles.
// dE/dtheta_q = sum_sigma S[q][sigma] db_sigma/dtheta (likewise phi), where
// S[q][sigma] adds, over the terms with sigma on qubit q, c times the product
// of the term's other factors.
//
// The product of a term is taken over its 3-qubit groups (the energy table),
// so the derivative is first formed per group table entry:
//   T[e] = sum over the terms whose group g has code e of c * prod_{g' != g} L_g',
// then, once per workgroup, S[q][sigma] = sum over the codes e of q's group
// with sigma at q's position of T[e] * (product of the other qubits' factors
// of that code).  Per term: ZK, the number of zero group factors, and PK, the
// product of the non-zero ones, formed as one division by the product of
// their tabulated reciprocals (the term's <K> is PK when ZK = 0, else 0; it
// is written per row when the caller asks for the coefficient cotangents).  The other groups of group g then multiply to
// PK * (1 / L_g) when L_g != 0 and ZK = 0, to PK when L_g = 0 and ZK = 1, and
// to 0 otherwise (exact zeros never divide).  Only the term's non-identity
// groups are visited for T.  T lives in LDS and takes FP64 atomics (one per
// non-identity group of a term); per-workgroup S are reduced in a fixed
// order.  acc layout per workgroup: [3 * nq] with sigma order X, Z, Y.
// ---------------------------------------------------------------------------
constexpr int kBwdBlock = 512;

// LDS tables of the backward hold one pad entry after every group's 64
// entries, so that the same code of different groups falls in different
// banks (entry e sits at e + e / 64).
__host__ __device__ constexpr int bwd_padded(int n) { return n + n / kLutEntries; }

size_t energy_bwd_lds_bytes(int W) {
  return (size_t)2 * bwd_padded(W * kGroupsPerWord * kLutEntries) * 8 + (size_t)W * 64 * 4 * 8;
}

// Workgroups per CU that the LDS of one CU holds (160 KiB), at most four
// 512-thread workgroups (32 waves).
int energy_bwd_blocks_per_cu(int W) {
  const int k = (int)((size_t)160 * 1024 / energy_bwd_lds_bytes(W));
  return k < 1 ? 1 : k > 4 ? 4 : k;
}

template <int W>
__global__ __launch_bounds__(kBwdBlock) void k_energy_bwd(StoreDev st, int nq, const double* theta,
                                                          const double* phi, const double* lut_g,
                                                          const double* dE, double* lam,
                                                          double* acc_g) {
  constexpr int NE = W * kGroupsPerWord * kLutEntries;
  constexpr int NP = bwd_padded(NE);
  constexpr int HP = bwd_padded(kGroupsPerHalf * kLutEntries);   // padded entries per half word
  extern __shared__ __align__(16) unsigned char smem_bwd[];
  double* rec = (double*)smem_bwd;     // 1 / L per table entry (0 where L is 0)
  double* tg = rec + NP;               // T per table entry
  double* fac = tg + NP;               // per qubit: factor of I, X, Z, Y
  for (int i = threadIdx.x; i < NP; i += kBwdBlock) {
    const int g = i / (kLutEntries + 1), k = i % (kLutEntries + 1);
    const double l = k < kLutEntries ? lut_g[g * kLutEntries + k] : 1.0;
    const double r = 1.0 / l;
    // a factor whose reciprocal overflows (|L| below 2^-1024) counts as a zero
    rec[i] = (l != 0.0 && r - r == 0.0) ? r : 0.0;
    tg[i] = 0.0;
  }
  for (int q = threadIdx.x; q < 64 * W; q += kBwdBlock) {
    double st_ = 0, ct = 1, sp = 0, cp = 1;
    if (q < nq) {
      sincos(theta[q], &st_, &ct);
      sincos(phi[q], &sp, &cp);
    }
    for (int op = 0; op < 4; ++op) fac[4 * q + op] = bloch_factor(op, st_, ct, sp, cp);
  }
  __syncthreads();
  const double scale = dE ? *dE : 1.0;
  const int64_t B = 1ll << *st.m;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = st.cnt[b], off = st.off[b];
    for (int64_t i = threadIdx.x; i < n; i += kBwdBlock) {
      uint64_t kx[W], kz[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        kx[w] = __builtin_nontemporal_load(&st.x[w * st.cap + off + i]);
        kz[w] = __builtin_nontemporal_load(&st.z[w * st.cap + off + i]);
      }
      const double c = __builtin_nontemporal_load(&st.c[off + i]);
      // ZK, the number of zero group factors, and R, the product of the
      // reciprocals of the others: every group of every half word in a fixed
      // order (identity groups read 1.0), the same group in every lane at a time
      double r[4] = {1.0, 1.0, 1.0, 1.0};
      int zk = 0;
#pragma unroll 1
      for (int w = 0; w < W; ++w) {
        uint64_t xw = kx[0], zw = kz[0];
#pragma unroll
        for (int u = 1; u < W; ++u) {
          xw = u == w ? kx[u] : xw;
          zw = u == w ? kz[u] : zw;
        }
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const uint32_t xh = (uint32_t)(xw >> (32 * hh));
          const uint32_t zh = (uint32_t)(zw >> (32 * hh));
          const double* rh = rec + (2 * w + hh) * HP;
#pragma unroll
          for (int g = 0; g < kGroupsPerHalf; ++g) {
            const uint32_t code = __builtin_amdgcn_ubfe(xh, 3 * g, 3) | (__builtin_amdgcn_ubfe(zh, 3 * g, 3) << 3);
            const double v = rh[g * (kLutEntries + 1) + code];
            zk += v == 0.0;
            r[g & 3] *= v == 0.0 ? 1.0 : v;
          }
        }
      }
      const double pk = 1.0 / ((r[0] * r[1]) * (r[2] * r[3]));   // PK
      // dE/dc of the term: <K> = PK without zero factors, else 0
      if (lam) lam[off + i] = zk == 0 ? scale * pk : 0.0;
      if (zk > 1) continue;   // every group's other factors include a zero
      const double cpk = c * pk;
      const bool one_zero = zk == 1;
      // T over the term's non-identity groups only
#pragma unroll
      for (int h = 0; h < 2 * W; ++h) {
        const uint32_t xh = (uint32_t)(kx[h >> 1] >> (32 * (h & 1)));
        const uint32_t zh = (uint32_t)(kz[h >> 1] >> (32 * (h & 1)));
        const double* rh = rec + h * HP;
        double* th = tg + h * HP;
        uint32_t t = group_starts(xh | zh);
        while (t) {
          // entry 0 (code 0 of group 0) only comes from an exhausted t
          const uint32_t e0 = next_group_entry(t, xh, zh);
          const uint32_t e1 = next_group_entry(t, xh, zh);
          const uint32_t p0 = e0 + (e0 >> 6), p1 = e1 + (e1 >> 6);
          const double v0 = rh[p0], v1 = rh[p1];
          const bool z0 = v0 == 0.0, z1 = v1 == 0.0;
          const double o0 = z0 ? cpk : cpk * v0;
          const double o1 = z1 ? cpk : cpk * v1;
          if (e0 != 0 && z0 == one_zero) atomicAdd(&th[p0], o0);
          if (e1 != 0 && z1 == one_zero) atomicAdd(&th[p1], o1);
        }
      }
    }
  }
  __syncthreads();
  // S[q][sigma] from T: the codes of q's group with sigma at q's position,
  // each weighted by the product of the group's other factors of that code
  for (int k = threadIdx.x; k < 3 * nq; k += kBwdBlock) {
    const int q = k / 3, op = k % 3 + 1;   // op: 1 = X, 2 = Z, 3 = Y
    const int h = q >> 5, bit = q & 31;
    const int g = (int)div3_small((uint32_t)bit), r = bit - 3 * g;
    const double* th = tg + h * HP + g * (kLutEntries + 1);
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
      if (valid) s += th[code] * other;
    }
    acc_g[(int64_t)blockIdx.x * 3 * nq + k] = s;
  }
}

template <int W>
static void launch_bwd_w(int nq, const StoreDev& st, int grid, const double* theta,
                         const double* phi, const double* lut, const double* dE, double* lam,
                         double* acc, hipStream_t s) {
  const size_t lds = energy_bwd_lds_bytes(W);
  hipFuncSetAttribute((const void*)k_energy_bwd<W>, hipFuncAttributeMaxDynamicSharedMemorySize,
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
