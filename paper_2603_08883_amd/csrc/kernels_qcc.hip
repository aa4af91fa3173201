// Kernels of one iQCC iteration (Sec. II, iterative procedure) beyond the
// dressing step itself:
//   * the flip sets of a Hamiltonian (x parts of its terms, App. A: DIS
//     candidates must share the flip set of some term), gathered as rows for
//     the merge, which makes them unique;
//   * the anticommuting part of the QMF energy, sum over terms K with
//     {K, P} = 0 of c_K <Omega|K|Omega> (Eq. 3 restricted), which fixes the
//     cos(tau) coefficient of the single-generator energy
//     E(tau) = a + b cos(tau) + c sin(tau) implied by Eq. 5.
#include "iqcc_internal.h"

#pragma clang fp contract(off)

namespace iqcc {

template <int W>
__global__ __launch_bounds__(kBlock) void k_flip_rows(StoreDev st, int w_max, uint64_t* ox,
                                                      uint64_t* oz, double* oc, int64_t ld,
                                                      unsigned long long* count) {
  const int lane = threadIdx.x & 63;
  const int64_t B = 1ll << *st.m;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = st.cnt[b], off = st.off[b];
    for (int64_t i0 = (threadIdx.x & ~63); i0 < n; i0 += kBlock) {   // wave-uniform
      const int64_t i = i0 + lane;
      uint64_t kx[W];
      int wt = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        kx[w] = i < n ? st.x[w * st.cap + off + i] : 0ull;
        wt += __popcll(kx[w]);
      }
      const bool keep = wt >= 1 && wt <= w_max;
      const uint64_t mask = __ballot(keep);
      if (mask == 0) continue;
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(count, (unsigned long long)__popcll(mask));
      base = __shfl(base, 0, 64);
      if (keep) {
        const int64_t r = (int64_t)base + __popcll(mask & ((1ull << lane) - 1));
        if (r < ld) {
#pragma unroll
          for (int w = 0; w < W; ++w) {
            ox[w * ld + r] = kx[w];
            oz[w * ld + r] = 0ull;
          }
          oc[r] = 1.0;
        }
      }
    }
  }
}

void launch_flip_rows(int W, const StoreDev& st, int w_max, uint64_t* ox, uint64_t* oz, double* oc,
                      int64_t ld, unsigned long long* count, int grid, hipStream_t s) {
  switch (W) {
    case 1: hipLaunchKernelGGL(k_flip_rows<1>, dim3(grid), dim3(kBlock), 0, s, st, w_max, ox, oz, oc, ld, count); break;
    case 2: hipLaunchKernelGGL(k_flip_rows<2>, dim3(grid), dim3(kBlock), 0, s, st, w_max, ox, oz, oc, ld, count); break;
    case 3: hipLaunchKernelGGL(k_flip_rows<3>, dim3(grid), dim3(kBlock), 0, s, st, w_max, ox, oz, oc, ld, count); break;
    default: hipLaunchKernelGGL(k_flip_rows<4>, dim3(grid), dim3(kBlock), 0, s, st, w_max, ox, oz, oc, ld, count); break;
  }
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_energy_anti(StoreDev st, const double* lut_g,
                                                        PauliKey P, double* partial) {
  __shared__ double lut[W * kGroupsPerWord * kLutEntries];
  __shared__ double red[kWaves];
  for (int i = threadIdx.x; i < W * kGroupsPerWord * kLutEntries; i += kBlock) lut[i] = lut_g[i];
  __syncthreads();
  const int64_t B = 1ll << *st.m;
  double acc = 0.0;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = st.cnt[b], off = st.off[b];
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
      uint64_t kx[W], kz[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        kx[w] = st.x[w * st.cap + off + i];
        kz[w] = st.z[w * st.cap + off + i];
      }
      if (anticommutes<W>(kx, kz, P.x, P.z)) acc += st.c[off + i] * expect_lut<W>(lut, kx, kz);
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

void launch_energy_anti(int W, const StoreDev& st, const PauliKey& P, int grid, const double* lut,
                        double* partial, hipStream_t s) {
  switch (W) {
    case 1: hipLaunchKernelGGL(k_energy_anti<1>, dim3(grid), dim3(kBlock), 0, s, st, lut, P, partial); break;
    case 2: hipLaunchKernelGGL(k_energy_anti<2>, dim3(grid), dim3(kBlock), 0, s, st, lut, P, partial); break;
    case 3: hipLaunchKernelGGL(k_energy_anti<3>, dim3(grid), dim3(kBlock), 0, s, st, lut, P, partial); break;
    default: hipLaunchKernelGGL(k_energy_anti<4>, dim3(grid), dim3(kBlock), 0, s, st, lut, P, partial); break;
  }
}

}  // namespace iqcc
