// DIS gradient screening (Sec. II, Eq. 7; App. A):
//   g_a = Im <Omega| H P_a |Omega> = sum_k c_k Im(i^e) <Q_k>,  P_k P_a = i^e Q_k,
// so only terms that anticommute with P_a contribute, with +<Q_k> for e = 1
// and -<Q_k> for e = 3.
//
// Batched form: one launch; a workgroup holds a tile of up to 256 candidates,
// one per thread, and streams a share of the terms through LDS; every lane of
// a wave reads the same staged term (LDS broadcast).  Q = K P_a differs from K
// only on the 3-qubit groups P_a touches, so with <K> formed once per staged
// term, <Q> = <K> * prod_{g of P_a} f_g(Q) / prod_{g of P_a} f_g(K): a few
// lookups per (term, candidate) pair instead of the whole product.  When a
// factor of K on those groups is exactly zero the full product of Q is used.
// Per-workgroup partial sums are reduced over term shares in a fixed order.
// Plain form: one launch per candidate streaming all terms (reference form).
#include "iqcc_internal.h"

#pragma clang fp contract(off)

namespace iqcc {

template <int W>
__global__ __launch_bounds__(kBlock) void k_dis_batched(StoreDev st, const double* lut_g,
                                                        const uint64_t* cx, const uint64_t* cz,
                                                        int64_t n_cand, int64_t ld_cand,
                                                        double* partial) {
  __shared__ double lut[W * kGroupsPerWord * kLutEntries];
  __shared__ uint64_t tx[W][kBlock], tz[W][kBlock];
  __shared__ double tc[kBlock], tk[kBlock];
  for (int i = threadIdx.x; i < W * kGroupsPerWord * kLutEntries; i += kBlock) lut[i] = lut_g[i];
  const int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = a < n_cand;
  uint64_t ax[W], az[W];
  uint32_t pg[2 * W];   // start bits of the groups P_a touches, per 32-bit half
#pragma unroll
  for (int w = 0; w < W; ++w) {
    ax[w] = active ? cx[w * ld_cand + a] : 0;
    az[w] = active ? cz[w * ld_cand + a] : 0;
    pg[2 * w] = group_starts((uint32_t)(ax[w] | az[w]));
    pg[2 * w + 1] = group_starts((uint32_t)((ax[w] | az[w]) >> 32));
  }
  __syncthreads();
  const int64_t B = 1ll << *st.m;
  double acc = 0.0;
  for (int64_t b = blockIdx.y; b < B; b += gridDim.y) {
    const int64_t n = st.cnt[b], off = st.off[b];
    for (int64_t i0 = 0; i0 < n; i0 += kBlock) {
      const int64_t i = i0 + threadIdx.x;
      if (i < n) {
        uint64_t kx[W], kz[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
          kx[w] = st.x[w * st.cap + off + i];
          kz[w] = st.z[w * st.cap + off + i];
          tx[w][threadIdx.x] = kx[w];
          tz[w][threadIdx.x] = kz[w];
        }
        tc[threadIdx.x] = st.c[off + i];
        tk[threadIdx.x] = expect_lut<W>(lut, kx, kz);   // <K>, shared by the whole tile
      }
      __syncthreads();
      const int cnt = (int)((n - i0) < kBlock ? (n - i0) : kBlock);
      if (active) {
        for (int j0 = 0; j0 < cnt; j0 += 64) {
          // which of the next 64 staged terms anticommute with this lane's
          // candidate (every lane reads the same term: LDS broadcast)
          const int jn = (cnt - j0) < 64 ? (cnt - j0) : 64;
          uint64_t mask = 0;
          for (int j = 0; j < jn; ++j) {
            uint64_t t = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) t ^= (tx[w][j0 + j] & az[w]) ^ (tz[w][j0 + j] & ax[w]);
            mask |= (uint64_t)(__popcll(t) & 1) << j;
          }
          // only the anticommuting terms of this lane
          while (mask) {
            const int j = j0 + __builtin_ctzll(mask);
            mask &= mask - 1;
            uint64_t kx[W], kz[W], qx[W], qz[W];
#pragma unroll
            for (int w = 0; w < W; ++w) {
              kx[w] = tx[w][j];
              kz[w] = tz[w][j];
              qx[w] = kx[w] ^ ax[w];
              qz[w] = kz[w] ^ az[w];
            }
            const int e = product_phase<W>(kx, kz, ax, az);
            // factors of K and of Q on the groups of P_a
            double fk = 1.0, fq = 1.0;
#pragma unroll
            for (int h = 0; h < 2 * W; ++h) {
              const uint32_t kxh = (uint32_t)(kx[h >> 1] >> (32 * (h & 1)));
              const uint32_t kzh = (uint32_t)(kz[h >> 1] >> (32 * (h & 1)));
              const uint32_t qxh = (uint32_t)(qx[h >> 1] >> (32 * (h & 1)));
              const uint32_t qzh = (uint32_t)(qz[h >> 1] >> (32 * (h & 1)));
              const double* lh = lut + h * kGroupsPerHalf * kLutEntries;
              for (uint32_t t = pg[h]; t; t &= t - 1) {
                const uint32_t sh = (uint32_t)__builtin_ctz(t);
                const uint32_t base = div3_small(sh) * kLutEntries;
                fk *= lh[base + (__builtin_amdgcn_ubfe(kxh, sh, 3) | (__builtin_amdgcn_ubfe(kzh, sh, 3) << 3))];
                fq *= lh[base + (__builtin_amdgcn_ubfe(qxh, sh, 3) | (__builtin_amdgcn_ubfe(qzh, sh, 3) << 3))];
              }
            }
            const double q = fk != 0.0 ? (tk[j] / fk) * fq : expect_lut<W>(lut, qx, qz);
            const double v = tc[j] * q;
            acc += (e == 1) ? v : -v;
          }
        }
      }
      __syncthreads();
    }
  }
  if (active) partial[(int64_t)blockIdx.y * n_cand + a] = acc;
}

__global__ void k_dis_reduce(const double* partial, int rows, int64_t n_cand, double* g) {
  for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n_cand;
       a += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += partial[(int64_t)r * n_cand + a];
    g[a] = s;
  }
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_dis_one(StoreDev st, const double* lut_g,
                                                    const uint64_t* cx, const uint64_t* cz,
                                                    int64_t ld_cand, int64_t a, double* partial) {
  constexpr int R = 4;   // terms per thread per load round
  __shared__ double lut[W * kGroupsPerWord * kLutEntries];
  __shared__ double red[kWaves];
  for (int i = threadIdx.x; i < W * kGroupsPerWord * kLutEntries; i += kBlock) lut[i] = lut_g[i];
  uint64_t px[W], pz[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    px[w] = cx[w * ld_cand + a];
    pz[w] = cz[w * ld_cand + a];
  }
  __syncthreads();
  const int64_t B = 1ll << *st.m;
  double acc = 0.0;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = st.cnt[b], off = st.off[b];
    for (int64_t i0 = 0; i0 < n; i0 += kBlock * R) {
      uint64_t kx[R][W], kz[R][W];
      bool ok[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t i = i0 + r * kBlock + threadIdx.x;
        ok[r] = i < n;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          kx[r][w] = ok[r] ? st.x[w * st.cap + off + i] : 0;
          kz[r][w] = ok[r] ? st.z[w * st.cap + off + i] : 0;
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (ok[r] && anticommutes<W>(kx[r], kz[r], px, pz)) {
          const int e = product_phase<W>(kx[r], kz[r], px, pz);
          uint64_t qx[W], qz[W];
#pragma unroll
          for (int w = 0; w < W; ++w) {
            qx[w] = kx[r][w] ^ px[w];
            qz[w] = kz[r][w] ^ pz[w];
          }
          const double v = st.c[off + i0 + r * kBlock + threadIdx.x] * expect_lut<W>(lut, qx, qz);
          acc += (e == 1) ? v : -v;
        }
      }
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

void launch_dis(int W, const StoreDev& st, const double* lut, const uint64_t* cx,
                const uint64_t* cz, int64_t n_cand, int64_t ld_cand, int mode, int tile,
                int grid, double* partial, int grid_terms, double* g, hipStream_t s) {
  (void)tile;
  if (n_cand <= 0) return;
  if (mode == 0) {
    const int64_t tiles = (n_cand + kBlock - 1) / kBlock;
    dim3 gr((unsigned)tiles, (unsigned)grid_terms);
    switch (W) {
      case 1: hipLaunchKernelGGL(k_dis_batched<1>, gr, dim3(kBlock), 0, s, st, lut, cx, cz, n_cand, ld_cand, partial); break;
      case 2: hipLaunchKernelGGL(k_dis_batched<2>, gr, dim3(kBlock), 0, s, st, lut, cx, cz, n_cand, ld_cand, partial); break;
      case 3: hipLaunchKernelGGL(k_dis_batched<3>, gr, dim3(kBlock), 0, s, st, lut, cx, cz, n_cand, ld_cand, partial); break;
      default: hipLaunchKernelGGL(k_dis_batched<4>, gr, dim3(kBlock), 0, s, st, lut, cx, cz, n_cand, ld_cand, partial); break;
    }
    int64_t blocks = (n_cand + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_dis_reduce, dim3((unsigned)blocks), dim3(kBlock), 0, s, partial, grid_terms, n_cand, g);
  } else {
    for (int64_t a = 0; a < n_cand; ++a) {
      switch (W) {
        case 1: hipLaunchKernelGGL(k_dis_one<1>, dim3(grid), dim3(kBlock), 0, s, st, lut, cx, cz, ld_cand, a, partial); break;
        case 2: hipLaunchKernelGGL(k_dis_one<2>, dim3(grid), dim3(kBlock), 0, s, st, lut, cx, cz, ld_cand, a, partial); break;
        case 3: hipLaunchKernelGGL(k_dis_one<3>, dim3(grid), dim3(kBlock), 0, s, st, lut, cx, cz, ld_cand, a, partial); break;
        default: hipLaunchKernelGGL(k_dis_one<4>, dim3(grid), dim3(kBlock), 0, s, st, lut, cx, cz, ld_cand, a, partial); break;
      }
      launch_finalize_sum(partial, grid, nullptr, g + a, s);
    }
  }
}

}  // namespace iqcc
