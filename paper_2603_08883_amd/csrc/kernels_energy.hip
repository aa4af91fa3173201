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
// of the term's other factors.  Each term forms PK, the product of its
// non-zero qubit factors, and ZK, the number of zero ones; the other factors
// of qubit q then multiply to PK / b_q when b_q != 0 and ZK = 0, to PK when
// b_q = 0 and ZK = 1, and to 0 otherwise (exact zeros never divide).  The
// division is a multiplication by a tabulated 1 / b_q.  Contributions go to
// S in LDS with FP64 atomics; per-workgroup S are reduced in a fixed order.
// acc layout per workgroup: [3 * nq] with sigma order X, Z, Y.
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kBlock) void k_energy_bwd(StoreDev st, int nq, const double* theta,
                                                       const double* phi, const double* lut_g,
                                                       double* acc_g) {
  (void)lut_g;
  __shared__ double fac[kMaxWords * 64 * 4];   // per qubit: factor of I, X, Z, Y
  __shared__ double inv[kMaxWords * 64 * 4];   // 1 / factor (0 where the factor is 0)
  __shared__ double acc[kMaxWords * 64 * 3];
  for (int q = threadIdx.x; q < 64 * W; q += kBlock) {
    double st_ = 0, ct = 1, sp = 0, cp = 1;
    if (q < nq) {
      sincos(theta[q], &st_, &ct);
      sincos(phi[q], &sp, &cp);
    }
    for (int op = 0; op < 4; ++op) {
      const double f = bloch_factor(op, st_, ct, sp, cp);
      fac[4 * q + op] = f;
      inv[4 * q + op] = f != 0.0 ? 1.0 / f : 0.0;
    }
    for (int k = 0; k < 3; ++k) acc[3 * q + k] = 0.0;
  }
  __syncthreads();
  const int64_t B = 1ll << *st.m;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = st.cnt[b], off = st.off[b];
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
      uint64_t kx[W], kz[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        kx[w] = st.x[w * st.cap + off + i];
        kz[w] = st.z[w * st.cap + off + i];
      }
      const double c = st.c[off + i];
      double pk = 1.0;
      int zk = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        for (uint64_t t = kx[w] | kz[w]; t; t &= t - 1) {
          const int bq = __builtin_ctzll(t);
          const int op = (int)((kx[w] >> bq) & 1) | (int)(((kz[w] >> bq) & 1) << 1);
          const double f = fac[4 * (64 * w + bq) + op];
          if (f == 0.0) ++zk; else pk *= f;
        }
      }
      if (zk > 1) continue;   // every qubit's other factors include a zero
      const double cpk = c * pk;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        for (uint64_t t = kx[w] | kz[w]; t; t &= t - 1) {
          const int bq = __builtin_ctzll(t);
          const int op = (int)((kx[w] >> bq) & 1) | (int)(((kz[w] >> bq) & 1) << 1);
          const int q4 = 4 * (64 * w + bq) + op;
          const bool zero = fac[q4] == 0.0;
          if (zero != (zk == 1)) continue;   // a zero elsewhere, or a zero here and not alone
          const double others = zero ? cpk : cpk * inv[q4];
          atomicAdd(&acc[3 * (64 * w + bq) + (op - 1)], others);
        }
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 3 * nq; k += kBlock) acc_g[(int64_t)blockIdx.x * 3 * nq + k] = acc[k];
}

void launch_energy_backward(int W, int nq, const StoreDev& st, int grid, const double* theta,
                            const double* phi, const double* lut, double* acc, hipStream_t s) {
  switch (W) {
    case 1: hipLaunchKernelGGL(k_energy_bwd<1>, dim3(grid), dim3(kBlock), 0, s, st, nq, theta, phi, lut, acc); break;
    case 2: hipLaunchKernelGGL(k_energy_bwd<2>, dim3(grid), dim3(kBlock), 0, s, st, nq, theta, phi, lut, acc); break;
    case 3: hipLaunchKernelGGL(k_energy_bwd<3>, dim3(grid), dim3(kBlock), 0, s, st, nq, theta, phi, lut, acc); break;
    default: hipLaunchKernelGGL(k_energy_bwd<4>, dim3(grid), dim3(kBlock), 0, s, st, nq, theta, phi, lut, acc); break;
  }
}

__global__ void k_backward_finalize(int nq, int grid, const double* acc, const double* theta,
                                    const double* phi, const double* dE, double* dtheta,
                                    double* dphi) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
    double S[3] = {0.0, 0.0, 0.0};
    for (int g = 0; g < grid; ++g)
      for (int k = 0; k < 3; ++k) S[k] += acc[(int64_t)g * 3 * nq + 3 * q + k];
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
  hipLaunchKernelGGL(k_backward_finalize, dim3(1), dim3(kBlock), 0, s, nq, grid, acc, theta, phi,
                     dE, dtheta, dphi);
}

}  // namespace iqcc
