// Reverse mode through the iterated dressing (Sec. II, Eqs. 4 and 6) with the
// compression decisions of the forward pass held fixed.
//
// Forward step j maps input coefficients c to outputs
//   c'[A]     += cos(t) c[A]                 (every anticommuting A)
//   c'[A^P]   += s_A sin(t) c[A]             (s_A = +1 if P A = i^3 Q, -1 if i^1)
//   c'[A]      = c[A]                        (commuting A)
// followed by dropping small outputs.  With lambda' = dE/dc' on the output
// rows (0 on dropped keys) the cotangent of the input is
//   lambda[A] = cos(t) lambda'[A] + s_A sin(t) lambda'[A^P]   (anticommuting)
//   lambda[A] = lambda'[A]                                    (commuting)
// and the step's amplitude receives
//   dE/dt += sum_A  -sin(t) c[A] lambda'[A] + s_A cos(t) c[A] lambda'[A^P].
// The tape recorded by the forward kernel gives, for every input row, the
// output rows of A and A^P and the sign s_A, so no key is read or looked up
// here.  The step's dE/dt is an exact fixed-point sum, so it has the same
// bits for any order of the rows.
#include "iqcc_internal.h"

#pragma clang fp contract(off)

namespace iqcc {

template <int W>
__global__ __launch_bounds__(kBlock) void k_dress_backward(StoreDev in, double C,
                                                           double S, const int32_t* tape_self,
                                                           const int32_t* tape_partner,
                                                           const double* lam_out, double* lam_in,
                                                           double* partial) {
  __shared__ long long red_hi[kWaves], red_lo[kWaves];
  __shared__ double red_mag[kWaves];
  const int64_t B = 1ll << *in.m;
  // dE/dt as an exact fixed-point sum: the same bits for any row order
  FixedSum acc;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t n = in.cnt[b], off = in.off[b];
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
      const int64_t row = off + i;
      const int32_t ts = tape_self[row], enc = tape_partner[row];
      const double la = ts >= 0 ? lam_out[ts] : 0.0;
      if (enc < 0) {   // commuting
        lam_in[row] = la;
        continue;
      }
      // anticommuting: enc = 2 * (output row of K^P + 1) + [s_K = +1]
      const int32_t tp = (enc >> 1) - 1;
      const double lp = tp >= 0 ? lam_out[tp] : 0.0;
      const double s = (enc & 1) ? 1.0 : -1.0;
      const double c = in.c[row];
      lam_in[row] = __dadd_rn(__dmul_rn(C, la), s * __dmul_rn(S, lp));
      fixed_add(acc, __dadd_rn(-__dmul_rn(__dmul_rn(S, c), la), s * __dmul_rn(__dmul_rn(C, c), lp)));
    }
  }
  const FixedSum t = block_fixed_sum<kWaves>(acc, red_hi, red_lo, red_mag);
  if (threadIdx.x == 0) {
    partial[3 * blockIdx.x] = __longlong_as_double(t.hi);
    partial[3 * blockIdx.x + 1] = __longlong_as_double(t.lo);
    partial[3 * blockIdx.x + 2] = t.mag;
  }
}

void launch_dress_backward(int W, const StoreDev& in, double C, double S,
                           const int32_t* tape_self, const int32_t* tape_partner,
                           const double* lam_out, double* lam_in, double* partial, int grid,
                           hipStream_t s) {
  switch (W) {
    case 1: hipLaunchKernelGGL(k_dress_backward<1>, dim3(grid), dim3(kBlock), 0, s, in, C, S, tape_self, tape_partner, lam_out, lam_in, partial); break;
    case 2: hipLaunchKernelGGL(k_dress_backward<2>, dim3(grid), dim3(kBlock), 0, s, in, C, S, tape_self, tape_partner, lam_out, lam_in, partial); break;
    case 3: hipLaunchKernelGGL(k_dress_backward<3>, dim3(grid), dim3(kBlock), 0, s, in, C, S, tape_self, tape_partner, lam_out, lam_in, partial); break;
    default: hipLaunchKernelGGL(k_dress_backward<4>, dim3(grid), dim3(kBlock), 0, s, in, C, S, tape_self, tape_partner, lam_out, lam_in, partial); break;
  }
}

// out[row] = scale * <K_row> for every live row of the store.
template <int W>
__global__ __launch_bounds__(kBlock) void k_expectations(StoreDev st, const double* lut_g,
                                                         const double* scale, double* out) {
  __shared__ double lut[W * kGroupsPerWord * kLutEntries];
  for (int i = threadIdx.x; i < W * kGroupsPerWord * kLutEntries; i += kBlock) lut[i] = lut_g[i];
  __syncthreads();
  const double sc = scale ? *scale : 1.0;
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
      out[off + i] = sc * expect_lut<W>(lut, kx, kz);
    }
  }
}

void launch_expectations(int W, const StoreDev& st, const double* lut, const double* scale,
                         double* out, int grid, hipStream_t s) {
  switch (W) {
    case 1: hipLaunchKernelGGL(k_expectations<1>, dim3(grid), dim3(kBlock), 0, s, st, lut, scale, out); break;
    case 2: hipLaunchKernelGGL(k_expectations<2>, dim3(grid), dim3(kBlock), 0, s, st, lut, scale, out); break;
    case 3: hipLaunchKernelGGL(k_expectations<3>, dim3(grid), dim3(kBlock), 0, s, st, lut, scale, out); break;
    default: hipLaunchKernelGGL(k_expectations<4>, dim3(grid), dim3(kBlock), 0, s, st, lut, scale, out); break;
  }
}

}  // namespace iqcc
