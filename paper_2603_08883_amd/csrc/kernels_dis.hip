// DIS gradient screening (Sec. II, Eq. 7; App. A):
//   g_a = Im <Omega| H P_a |Omega> = sum_k c_k Im(i^e) <Q_k>,  P_k P_a = i^e Q_k,
// so only terms that anticommute with P_a contribute, with +<Q_k> for e = 1
// and -<Q_k> for e = 3.
//
// Batched form: the QMF state is a product state, so for a term K and a
// candidate P_a the ratio <Q>/<K> (Q = K P_a) only involves the qubits in the
// support of P_a, and so does the phase e (a sum of per-qubit parts).  A table
// per (qubit, Pauli of P_a there, Pauli of K there) gives the factor ratio
// b_q(Q)/b_q(K), the qubit's share of e and whether b_q(K) is exactly zero.
// Each term carries PK = product of its non-zero qubit factors and ZK = the
// number of zero factors; then <Q> = PK * prod(ratios) when every zero factor
// of K lies in the support of P_a, else 0.  One table lookup per support qubit
// and term, no division in the loop and no special case at zero factors.
// A workgroup holds a tile of candidates and a contiguous range of buckets;
// lanes hold terms (kR per lane, pre-split into 2-bit qubit codes) and the
// candidate loop is uniform, so the support of P_a is walked in scalar
// registers.  Sums over lanes and waves, then over bucket ranges, are taken in
// a fixed order.
// Plain form: one launch per candidate streaming all terms (reference form).
#include "iqcc_internal.h"

#pragma clang fp contract(off)

namespace iqcc {

constexpr int kDisB = 512;          // threads per workgroup of the batched kernel
constexpr int kDisWaves = kDisB / 64;
constexpr int kDisR = 4;            // terms per lane
constexpr int kDisTile = 256;       // candidates per workgroup
constexpr int kDisChunk = kDisB;    // buckets whose prefix sums are staged at once

// Per-qubit tables for the batched kernel, q < 64 W:
//   ent[(q * 4 + p) * 4 + k] = {ratio, meta} for the Pauli k of K and p of P
//   (bit 0 = x, bit 1 = z): ratio = b_q(k ^ p) / b_q(k) (b_q(k ^ p) when
//   b_q(k) = 0), meta = [b_q(k) == 0] | (phase part << 12);
//   fac[q * 4 + k] = b_q(k).
struct DisEnt {
  double ratio;
  uint32_t meta;
  uint32_t pad;
};

__global__ void k_dis_tables(int W, int nq, const double* theta, const double* phi,
                             DisEnt* ent, double* fac) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 64 * W) return;
  double b[4] = {1.0, 1.0, 1.0, 1.0};
  if (q < nq) {
    double st, ct, sp, cp;
    sincos(theta[q], &st, &ct);
    sincos(phi[q], &sp, &cp);
    b[1] = st * cp;   // X
    b[2] = ct;        // Z
    b[3] = st * sp;   // Y
  }
  for (int k = 0; k < 4; ++k) fac[q * 4 + k] = b[k];
  for (int p = 0; p < 4; ++p) {
    for (int k = 0; k < 4; ++k) {
      const int x1 = k & 1, z1 = k >> 1, x2 = p & 1, z2 = p >> 1;
      const int ph = (x1 * z1 + x2 * z2 + 2 * z1 * x2 - (x1 ^ x2) * (z1 ^ z2)) & 3;
      const bool zero = b[k] == 0.0;
      DisEnt e;
      e.ratio = zero ? b[k ^ p] : b[k ^ p] / b[k];
      e.meta = (zero ? 1u : 0u) | ((uint32_t)ph << 12);
      e.pad = 0;
      ent[(q * 4 + p) * 4 + k] = e;
    }
  }
}

// Spread the 16 bits of v to the even bits of a 32-bit word.
__device__ __forceinline__ uint32_t spread16(uint32_t v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

// Sum over the 64 lanes of a wave with DPP moves (no LDS traffic); the total
// lands in lane 63.  Fixed pairing order, so the result is reproducible.
__device__ __forceinline__ double dpp_f64(double v, int ctrl_sel) {
  const uint64_t u = __double_as_longlong(v);
  int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
  switch (ctrl_sel) {   // constant after inlining
    case 0: lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
            hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false); break;
    case 1: lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
            hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false); break;
    case 2: lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false);  // row_half_mirror
            hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false); break;
    case 3: lo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false);  // row_mirror
            hi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false); break;
    case 4: lo = __builtin_amdgcn_update_dpp(0, lo, 0x142, 0xA, 0xF, false);  // row_bcast:15 -> rows 1, 3
            hi = __builtin_amdgcn_update_dpp(0, hi, 0x142, 0xA, 0xF, false); break;
    default: lo = __builtin_amdgcn_update_dpp(0, lo, 0x143, 0xC, 0xF, false); // row_bcast:31 -> rows 2, 3
             hi = __builtin_amdgcn_update_dpp(0, hi, 0x143, 0xC, 0xF, false); break;
  }
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ double wave_sum_to_lane63(double v) {
  v += dpp_f64(v, 0);   // pairs within quads
  v += dpp_f64(v, 1);   // quads: every lane holds its quad's sum
  v += dpp_f64(v, 2);   // half rows
  v += dpp_f64(v, 3);   // rows of 16
  v += dpp_f64(v, 4);   // rows 1 and 3 add rows 0 and 2 (other rows add +0)
  v += dpp_f64(v, 5);   // rows 2 and 3 add rows 0..1
  return v;
}

template <int W>
__global__ __launch_bounds__(kDisB) void k_dis_batched(StoreDev st, const DisEnt* __restrict__ ent_g,
                                                       const double* __restrict__ fac_g,
                                                       const uint64_t* __restrict__ cx,
                                                       const uint64_t* __restrict__ cz,
                                                       int64_t n_cand, int64_t ld_cand,
                                                       int tile_size,
                                                       double* __restrict__ partial) {
  constexpr int R = kDisR;
  constexpr int NQ = 64 * W;
  constexpr int NS = 4 * W;   // 16-qubit slots
  __shared__ DisEnt ent[NQ * 16];
  __shared__ double fac[NQ * 4];
  __shared__ double acc[kDisWaves][kDisTile];
  __shared__ int64_t pre[kDisChunk + 1];
  __shared__ int64_t boff[kDisChunk];
  __shared__ uint64_t scan_tmp[kDisWaves];
  for (int i = threadIdx.x; i < NQ * 16; i += kDisB) ent[i] = ent_g[i];
  for (int i = threadIdx.x; i < NQ * 4; i += kDisB) fac[i] = fac_g[i];
  for (int i = threadIdx.x; i < kDisWaves * kDisTile; i += kDisB) (&acc[0][0])[i] = 0.0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t a0 = (int64_t)blockIdx.x * tile_size;   // tile_size <= kDisTile
  const int tile = (int)((n_cand - a0) < tile_size ? (n_cand - a0) : tile_size);
  const int64_t B = 1ll << *st.m;
  const int64_t b_lo = B * blockIdx.y / gridDim.y, b_hi = B * (blockIdx.y + 1) / gridDim.y;
  const char* ent_base = reinterpret_cast<const char*>(ent);

  for (int64_t cb = b_lo; cb < b_hi; cb += kDisChunk) {
    const int nb = (int)((b_hi - cb) < kDisChunk ? (b_hi - cb) : kDisChunk);
    __syncthreads();   // tables ready / previous chunk done with pre, boff
    uint64_t total;
    const uint64_t n_b = threadIdx.x < nb ? (uint64_t)st.cnt[cb + threadIdx.x] : 0ull;
    const uint64_t ex = block_exclusive_scan_n<kDisWaves>(n_b, scan_tmp, total);
    if (threadIdx.x < nb) {
      pre[threadIdx.x] = (int64_t)ex;
      boff[threadIdx.x] = st.off[cb + threadIdx.x];
    }
    if (threadIdx.x == 0) pre[nb] = (int64_t)total;
    __syncthreads();
    const int64_t n_chunk = (int64_t)total;
    for (int64_t j0 = 0; j0 < n_chunk; j0 += (int64_t)kDisB * R) {
      // --- stage R terms per lane: 2-bit qubit codes, c * PK and ZK ---
      uint32_t code[R][NS];
      double cpk[R];
      uint32_t zk[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t j = j0 + (int64_t)r * kDisB + threadIdx.x;
        uint64_t kx[W], kz[W];
        double c = 0.0;
        if (j < n_chunk) {
          int lo = 0, hi = nb - 1;   // last bucket with pre <= j (pre[0] = 0)
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= j) lo = mid; else hi = mid - 1;
          }
          const int64_t i = boff[lo] + (j - pre[lo]);
#pragma unroll
          for (int w = 0; w < W; ++w) {
            kx[w] = st.x[w * st.cap + i];
            kz[w] = st.z[w * st.cap + i];
          }
          c = st.c[i];
        } else {
#pragma unroll
          for (int w = 0; w < W; ++w) kx[w] = kz[w] = 0ull;
        }
        double pk = 1.0;
        uint32_t nz = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          for (uint64_t t = kx[w] | kz[w]; t; t &= t - 1) {
            const int bq = __builtin_ctzll(t);
            const int k = (int)((kx[w] >> bq) & 1) | (int)(((kz[w] >> bq) & 1) << 1);
            const double f = fac[(64 * w + bq) * 4 + k];
            if (f == 0.0) ++nz; else pk *= f;
          }
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const uint32_t xs = (uint32_t)(kx[w] >> (16 * s4)), zs = (uint32_t)(kz[w] >> (16 * s4));
            code[r][4 * w + s4] = spread16(xs) | (spread16(zs) << 1);
          }
        }
        cpk[r] = c * pk;
        zk[r] = nz | (1u << 12);   // meta sum of a live pair with e = 1; e = 3 adds 2 << 12
      }
      // --- candidates of the tile (uniform loop) ---
      for (int t = 0; t < tile; ++t) {
        const int64_t a = a0 + t;
        double prod[R];
        uint32_t msum[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          prod[r] = 1.0;
          msum[r] = 0;
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const uint64_t ax = cx[w * ld_cand + a], az = cz[w * ld_cand + a];
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const uint32_t xs = (uint32_t)(ax >> (16 * s4)) & 0xffffu;
            const uint32_t zs = (uint32_t)(az >> (16 * s4)) & 0xffffu;
            for (uint32_t m = xs | zs; m; m &= m - 1) {
              const uint32_t qb = (uint32_t)__builtin_ctz(m);
              const uint32_t q = 64 * w + 16 * s4 + qb;
              const uint32_t p = ((xs >> qb) & 1u) | (((zs >> qb) & 1u) << 1);
              const char* row = ent_base + (size_t)((q * 4 + p) * 4) * sizeof(DisEnt);
#pragma unroll
              for (int r = 0; r < R; ++r) {
                const uint32_t k = __builtin_amdgcn_ubfe(code[r][4 * w + s4], 2 * qb, 2);
                const DisEnt e = *reinterpret_cast<const DisEnt*>(row + k * sizeof(DisEnt));
                prod[r] *= e.ratio;
                msum[r] += e.meta;
              }
            }
          }
        }
        double v = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          // live: every zero factor of K in the support, and e odd (+ for 1, - for 3)
          const uint32_t m = msum[r] & 0x3fffu;
          const double f = m == zk[r] ? 1.0 : (m == zk[r] + (2u << 12) ? -1.0 : 0.0);
          v = fma(f, cpk[r] * prod[r], v);   // exact product by +-1 or 0
        }
        v = wave_sum_to_lane63(v);
        if (lane == 63) acc[wid][t] += v;
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < tile; t += kDisB) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kDisWaves; ++w) s += acc[w][t];
    partial[(int64_t)blockIdx.y * n_cand + a0 + t] = s;
  }
}

int64_t dis_tables_doubles(int W) { return 64 * W * 16 * 2 + 64 * W * 4; }

int64_t dis_tile() { return kDisTile; }   // the largest tile the batched kernel holds

__global__ void k_dis_reduce(const double* partial, int rows, int64_t n_cand, double* g) {
  for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n_cand;
       a += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += partial[(int64_t)r * n_cand + a];
    g[a] = s;
  }
}

// Plain form: one candidate per launch.  Workgroup g takes the groups of G
// consecutive buckets g, g + grid, ... and streams each group's rows as one
// flat range, four terms per thread and pass, so short buckets keep every lane
// busy.  About half the terms anticommute with a candidate; their products
// Q = K P_a go to a per-wavefront ring in LDS, and the expectation of Q is
// formed on full wavefronts of 64 ring entries, so the 44-lookup product is
// not issued for lanes whose term commutes.  The last workgroup to finish
// sums the per-workgroup partials in a fixed order and writes g[a], so a
// candidate costs one launch.
constexpr int kDisOneR = 8;
constexpr int kDisRing = 128;   // ring entries per wavefront (< 64 left + 64 added)

template <int W>
struct DisRing {
  uint64_t x[W][kDisRing], z[W][kDisRing];
  double v[kDisRing];   // +-c: the sign of Im(i^e) for the product phase e
};

template <int W>
__global__ __launch_bounds__(kBlock) void k_dis_one(StoreDev st, const double* lut_g,
                                                    const uint64_t* cx, const uint64_t* cz,
                                                    int64_t ld_cand, int64_t a, double* partial,
                                                    unsigned int* done, double* g) {
  constexpr int R = kDisOneR;
  __shared__ double lut[W * kGroupsPerWord * kLutEntries];
  __shared__ double red[kWaves];
  __shared__ uint64_t scan_tmp[kWaves];
  __shared__ int64_t s_pre[kBlock + 1];
  __shared__ int64_t s_off[kBlock];
  __shared__ DisRing<W> ring_all[kWaves];
  __shared__ int s_last;
  for (int i = threadIdx.x; i < W * kGroupsPerWord * kLutEntries; i += kBlock) lut[i] = lut_g[i];
  uint64_t px[W], pz[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    px[w] = cx[w * ld_cand + a];
    pz[w] = cz[w * ld_cand + a];
  }
  const int lane = threadIdx.x & 63;
  DisRing<W>& ring = ring_all[threadIdx.x >> 6];
  int head = 0, fill = 0;   // wave-uniform ring state
  double acc = 0.0;
  // <Q> of 64 ring entries from the head (lanes past `count` add nothing)
  auto drain = [&](int count) {
    // the ring entries were written by other lanes of this wavefront
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int k = (head + lane) & (kDisRing - 1);
    if (lane < count) {
      uint64_t qx[W], qz[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        qx[w] = ring.x[w][k];
        qz[w] = ring.z[w][k];
      }
      acc += ring.v[k] * expect_lut<W>(lut, qx, qz);
    }
    head = (head + count) & (kDisRing - 1);
    fill -= count;
    // the drained entries are read before later entries overwrite them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  const int64_t B = 1ll << *st.m;
  int64_t G = B / gridDim.x;
  G = G < 1 ? 1 : (G > kBlock ? kBlock : G);
  const int64_t ngroups = (B + G - 1) / G;
  __syncthreads();
  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t b = grp * G + threadIdx.x;
    const bool mine = threadIdx.x < G && b < B;
    const int64_t cnt = mine ? st.cnt[b] : 0;
    const int64_t off = mine ? st.off[b] : 0;
    uint64_t total;
    // (the scan's barriers also order the previous group's reads of s_pre)
    const uint64_t ex = block_exclusive_scan((uint64_t)cnt, scan_tmp, total);
    s_pre[threadIdx.x] = (int64_t)ex;
    s_off[threadIdx.x] = off;
    if (threadIdx.x == 0) s_pre[kBlock] = (int64_t)total;
    __syncthreads();
    // the group's rows are one range when every bucket starts where the one
    // before it ends (a loaded store); then row = base + i, the row the
    // search below would find (thread 0 holds the group's first bucket)
    const int64_t base = s_off[0];
    const bool contig = __syncthreads_and(!mine || off - (int64_t)ex == base) != 0;
    const int64_t n = (int64_t)total;
    for (int64_t i0 = 0; i0 < n; i0 += kBlock * R) {
      uint64_t kx[R][W], kz[R][W];
      double kc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t i = i0 + r * kBlock + threadIdx.x;
        kc[r] = 0.0;
#pragma unroll
        for (int w = 0; w < W; ++w) kx[r][w] = kz[r][w] = 0;
        if (i < n) {
          int64_t row = base + i;
          if (!contig) {
            int lo = 0;   // the last bucket of the group whose first row is <= i
#pragma unroll
            for (int step = kBlock / 2; step; step >>= 1)
              if (s_pre[lo + step] <= i) lo += step;
            row = s_off[lo] + (i - s_pre[lo]);
          }
#pragma unroll
          for (int w = 0; w < W; ++w) {
            kx[r][w] = __builtin_nontemporal_load(&st.x[w * st.cap + row]);
            kz[r][w] = __builtin_nontemporal_load(&st.z[w * st.cap + row]);
          }
          kc[r] = __builtin_nontemporal_load(&st.c[row]);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // padding lanes (key 0) commute
        const bool anti = anticommutes<W>(kx[r], kz[r], px, pz);
        const uint64_t mask = __ballot(anti);
        if (anti) {
          const int e = product_phase<W>(kx[r], kz[r], px, pz);
          const int k = (head + fill + lanes_below(mask)) & (kDisRing - 1);
#pragma unroll
          for (int w = 0; w < W; ++w) {
            ring.x[w][k] = kx[r][w] ^ px[w];
            ring.z[w][k] = kz[r][w] ^ pz[w];
          }
          ring.v[k] = (e == 1) ? kc[r] : -kc[r];
        }
        fill += __popcll(mask);
        if (fill >= 64) drain(64);   // LDS operations of one wavefront complete in order
      }
    }
  }
  if (fill > 0) drain(fill);
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s;
    __threadfence();
    s_last = atomicAdd(done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (s_last) {   // every partial is written: sum them in a fixed order
    __threadfence();
    const volatile double* vp = partial;
    double t = 0.0;
    for (int k = threadIdx.x; k < (int)gridDim.x; k += kBlock) t += vp[k];
    t = block_sum(t, red);
    if (threadIdx.x == 0) {
      g[a] = t;
      *done = 0u;   // ready for the next candidate
    }
  }
}

__global__ void k_zero_u32(unsigned int* p) { *p = 0u; }

// Workgroups of k_dis_one that one CU holds at once (its LDS bounds it): the
// plain launch uses exactly that many per CU, so every workgroup is resident
// and takes one bucket group.
int dis_one_blocks_per_cu(int W) {
  int nb = 0;
  hipError_t e;
  switch (W) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_dis_one<1>, kBlock, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_dis_one<2>, kBlock, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_dis_one<3>, kBlock, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_dis_one<4>, kBlock, 0); break;
  }
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

void launch_dis(int W, const StoreDev& st, const double* lut, const uint64_t* cx,
                const uint64_t* cz, int64_t n_cand, int64_t ld_cand, int mode, int tile,
                int grid, double* partial, int grid_terms, double* g, hipStream_t s,
                const double* theta, const double* phi, int nq, double* tables) {
  if (n_cand <= 0) return;
  if (tile < 1 || tile > kDisTile) tile = kDisTile;
  if (mode == 0) {
    DisEnt* ent = reinterpret_cast<DisEnt*>(tables);
    double* fac = tables + dis_tables_doubles(W) - 64 * W * 4;
    hipLaunchKernelGGL(k_dis_tables, dim3((64 * W + 255) / 256), dim3(256), 0, s, W, nq, theta, phi,
                       ent, fac);
    const int64_t tiles = (n_cand + tile - 1) / tile;
    dim3 gr((unsigned)tiles, (unsigned)grid_terms);
    switch (W) {
      case 1: hipLaunchKernelGGL(k_dis_batched<1>, gr, dim3(kDisB), 0, s, st, ent, fac, cx, cz, n_cand, ld_cand, tile, partial); break;
      case 2: hipLaunchKernelGGL(k_dis_batched<2>, gr, dim3(kDisB), 0, s, st, ent, fac, cx, cz, n_cand, ld_cand, tile, partial); break;
      case 3: hipLaunchKernelGGL(k_dis_batched<3>, gr, dim3(kDisB), 0, s, st, ent, fac, cx, cz, n_cand, ld_cand, tile, partial); break;
      default: hipLaunchKernelGGL(k_dis_batched<4>, gr, dim3(kDisB), 0, s, st, ent, fac, cx, cz, n_cand, ld_cand, tile, partial); break;
    }
    int64_t blocks = (n_cand + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_dis_reduce, dim3((unsigned)blocks), dim3(kBlock), 0, s, partial, grid_terms, n_cand, g);
  } else {
    // partial[0, grid) per-workgroup sums, then the finish counter
    unsigned int* done = reinterpret_cast<unsigned int*>(partial + grid);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, done);
    for (int64_t a = 0; a < n_cand; ++a) {
      switch (W) {
        case 1: hipLaunchKernelGGL(k_dis_one<1>, dim3(grid), dim3(kBlock), 0, s, st, lut, cx, cz, ld_cand, a, partial, done, g); break;
        case 2: hipLaunchKernelGGL(k_dis_one<2>, dim3(grid), dim3(kBlock), 0, s, st, lut, cx, cz, ld_cand, a, partial, done, g); break;
        case 3: hipLaunchKernelGGL(k_dis_one<3>, dim3(grid), dim3(kBlock), 0, s, st, lut, cx, cz, ld_cand, a, partial, done, g); break;
        default: hipLaunchKernelGGL(k_dis_one<4>, dim3(grid), dim3(kBlock), 0, s, st, lut, cx, cz, ld_cand, a, partial, done, g); break;
      }
    }
  }
}

}  // namespace iqcc
