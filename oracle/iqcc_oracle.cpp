// Plain, slow, FP64 CPU oracle for the iQCC hot path.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
// this file; only the test-suite, the smoke check and the CPU-baseline leg of
// the benchmark do.  It shares no code, header or table with the HIP library.
//
// Conventions (one reading of the paper, stated once here):
//  * Pauli word of n qubits: words x[0..W-1], z[0..W-1]; qubit j is bit j%64 of
//    word j/64.  Local operator: I (x=0,z=0), X (1,0), Z (0,1), Y (1,1), Y the
//    Hermitian Pauli-Y; coefficients real (Eq. 2, H = sum_k C_k P_k).
//  * Products are formed qubit by qubit from the single-qubit multiplication
//    table (XY = iZ, YZ = iX, ZX = iY, reverses with -i, squares = I).
//  * Dressing (Eq. 5): H_d = e^{i tau P/2} H e^{-i tau P/2}.  A term A that
//    commutes with P is unchanged; an anticommuting A becomes
//    cos(tau) A + i sin(tau) P A, and with P A = i^e Q (e odd) the new term is
//    -sin(tau) a Q for e = 1 and +sin(tau) a Q for e = 3.
//  * Merge (sortless-dressing appendix, D = H + I): equal words are combined by
//    adding coefficients, in input order after a stable sort on the canonical
//    key (x[W-1..0], z[W-1..0] compared as unsigned words).
//  * Compression (the optional compression step of the iterative procedure): drop a term
//    when |c| < eps (strict).
//  * QMF energy (Eq. 3 and the energy functional of App. A):
//    E = sum_k C_k prod_j <sigma_kj>_j with <X> = sin t cos f, <Y> = sin t sin f,
//    <Z> = cos t, product taken in ascending qubit order, Neumaier summation.
//  * DIS gradient (Eq. 7): g_a = Im <Omega| H P_a |Omega> = sum_k C_k Im(i^e) <Q_k>
//    with P_k P_a = i^e Q_k.
//  * Angle gradients: analytic derivative of each single-qubit factor, product of
//    the other factors by explicit prefix/suffix loops (no division).
//  * tau tangents (iterated dressing, Eq. 6): forward-mode derivative of the chain
//    with every step's truncation decision frozen at the forward pass.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fopenmp -fPIC -shared (no -ffast-math).

#include <algorithm>
#include <map>
#include <string>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

namespace {

// single-qubit operator codes: 0 = I, 1 = X, 2 = Y, 3 = Z
inline int op_of(const uint64_t* x, const uint64_t* z, int q) {
  int bx = (int)((x[q / 64] >> (q % 64)) & 1u);
  int bz = (int)((z[q / 64] >> (q % 64)) & 1u);
  if (bx && bz) return 2;
  if (bx) return 1;
  if (bz) return 3;
  return 0;
}

inline void set_op(uint64_t* x, uint64_t* z, int q, int op) {
  uint64_t b = (uint64_t)1 << (q % 64);
  if (op == 1 || op == 2) x[q / 64] |= b;
  if (op == 3 || op == 2) z[q / 64] |= b;
}

// a * b = i^k * r  for single-qubit Paulis.
struct Mul { int r; int k; };
const Mul kMul[4][4] = {
    /* I* */ {{0, 0}, {1, 0}, {2, 0}, {3, 0}},
    /* X* */ {{1, 0}, {0, 0}, {3, 1}, {2, 3}},   // XY = iZ, XZ = -iY
    /* Y* */ {{2, 0}, {3, 3}, {0, 0}, {1, 1}},   // YX = -iZ, YZ = iX
    /* Z* */ {{3, 0}, {2, 1}, {1, 3}, {0, 0}},   // ZX = iY, ZY = -iX
};

// P1 * P2 = i^e * P3 ; returns e in 0..3
int product(int nq, int W, const uint64_t* x1, const uint64_t* z1, const uint64_t* x2,
            const uint64_t* z2, uint64_t* x3, uint64_t* z3) {
  for (int w = 0; w < W; ++w) { x3[w] = 0; z3[w] = 0; }
  int e = 0;
  for (int q = 0; q < nq; ++q) {
    Mul m = kMul[op_of(x1, z1, q)][op_of(x2, z2, q)];
    e = (e + m.k) & 3;
    set_op(x3, z3, q, m.r);
  }
  return e;
}

// canonical order: x[W-1] .. x[0], then z[W-1] .. z[0], unsigned
inline bool key_less(int W, const uint64_t* xa, const uint64_t* za, const uint64_t* xb,
                     const uint64_t* zb) {
  for (int w = W - 1; w >= 0; --w)
    if (xa[w] != xb[w]) return xa[w] < xb[w];
  for (int w = W - 1; w >= 0; --w)
    if (za[w] != zb[w]) return za[w] < zb[w];
  return false;
}

inline bool key_eq(int W, const uint64_t* xa, const uint64_t* za, const uint64_t* xb,
                   const uint64_t* zb) {
  for (int w = 0; w < W; ++w)
    if (xa[w] != xb[w] || za[w] != zb[w]) return false;
  return true;
}

struct Neumaier {
  double s = 0.0, comp = 0.0;
  void add(double v) {
    double t = s + v;
    if (std::fabs(s) >= std::fabs(v)) comp += (s - t) + v;
    else comp += (v - t) + s;
    s = t;
  }
  double value() const { return s + comp; }
};

// <sigma>_q of the product state, sigma in {I, X, Y, Z}
struct Bloch {
  std::vector<double> b;  // 4 per qubit
  explicit Bloch(int nq, const double* th, const double* ph) : b(4 * (size_t)nq) {
    for (int q = 0; q < nq; ++q) {
      double st = std::sin(th[q]), ct = std::cos(th[q]);
      double sp = std::sin(ph[q]), cp = std::cos(ph[q]);
      b[4 * q + 0] = 1.0;
      b[4 * q + 1] = st * cp;
      b[4 * q + 2] = st * sp;
      b[4 * q + 3] = ct;
    }
  }
  double expect(int nq, const uint64_t* x, const uint64_t* z) const {
    double p = 1.0;
    for (int q = 0; q < nq; ++q) p *= b[4 * q + op_of(x, z, q)];
    return p;
  }
};

}  // namespace

extern "C" {

int oracle_abi_version() { return 1; }

// Product of two Pauli words; returns the phase exponent e (P1 P2 = i^e P3).
int oracle_pauli_product(int nq, int W, const uint64_t* x1, const uint64_t* z1,
                         const uint64_t* x2, const uint64_t* z2, uint64_t* x3, uint64_t* z3) {
  return product(nq, W, x1, z1, x2, z2, x3, z3);
}

// Raw dressing (Eq. 5), no merge: emits, for every input term, itself (commuting),
// or itself scaled by cos(tau) plus P*A scaled by +-sin(tau) (anticommuting).
// Output rows are written in input order (commuting/rotated row first, then the
// new row).  Arrays are row-major: x[i*W + w].  Returns the number of rows.
int64_t oracle_dress_raw(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z,
                         const double* c, const uint64_t* px, const uint64_t* pz, double tau,
                         uint64_t* ox, uint64_t* oz, double* oc) {
  const double C = std::cos(tau), S = std::sin(tau);
  std::vector<uint64_t> qx(W), qz(W);
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t* xi = x + i * W;
    const uint64_t* zi = z + i * W;
    int e = product(nq, W, px, pz, xi, zi, qx.data(), qz.data());  // P * A
    if ((e & 1) == 0) {
      std::memcpy(ox + m * W, xi, W * 8);
      std::memcpy(oz + m * W, zi, W * 8);
      oc[m++] = c[i];
    } else {
      std::memcpy(ox + m * W, xi, W * 8);
      std::memcpy(oz + m * W, zi, W * 8);
      oc[m++] = C * c[i];
      double s = (e == 3) ? 1.0 : -1.0;
      std::memcpy(ox + m * W, qx.data(), W * 8);
      std::memcpy(oz + m * W, qz.data(), W * 8);
      oc[m++] = s * (S * c[i]);
    }
  }
  return m;
}

// Merge of a multiset (D = H + I) and compression |c| < eps.  Stable sort on the
// canonical key, left-to-right sums of equal keys.  Optional second channel dc
// (nullable) is merged the same way and dropped with its row.
int64_t oracle_merge_truncate(int W, int64_t n, const uint64_t* x, const uint64_t* z,
                              const double* c, const double* dc, double eps, uint64_t* ox,
                              uint64_t* oz, double* oc, double* odc) {
  std::vector<int64_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    return key_less(W, x + a * W, z + a * W, x + b * W, z + b * W);
  });
  int64_t m = 0;
  int64_t i = 0;
  while (i < n) {
    int64_t j = i;
    double s = 0.0, ds = 0.0;
    bool first = true;
    while (j < n && key_eq(W, x + idx[i] * W, z + idx[i] * W, x + idx[j] * W, z + idx[j] * W)) {
      if (first) {
        s = c[idx[j]];
        ds = dc ? dc[idx[j]] : 0.0;
        first = false;
      } else {
        s = s + c[idx[j]];
        if (dc) ds = ds + dc[idx[j]];
      }
      ++j;
    }
    if (!(std::fabs(s) < eps)) {
      std::memcpy(ox + m * W, x + idx[i] * W, W * 8);
      std::memcpy(oz + m * W, z + idx[i] * W, W * 8);
      oc[m] = s;
      if (odc) odc[m] = ds;
      ++m;
    }
    i = j;
  }
  return m;
}

// Dressing with a tangent channel: (c, dc) -> (c', dc').  When `active` is
// non-zero this step's amplitude is the one being differentiated, so the
// derivatives of cos/sin enter; otherwise dc is rotated like c.
int64_t oracle_dress_raw_tangent(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z,
                                 const double* c, const double* dc, const uint64_t* px,
                                 const uint64_t* pz, double tau, int active, uint64_t* ox,
                                 uint64_t* oz, double* oc, double* odc) {
  const double C = std::cos(tau), S = std::sin(tau);
  const double dC = active ? -S : 0.0, dS = active ? C : 0.0;
  std::vector<uint64_t> qx(W), qz(W);
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t* xi = x + i * W;
    const uint64_t* zi = z + i * W;
    int e = product(nq, W, px, pz, xi, zi, qx.data(), qz.data());
    std::memcpy(ox + m * W, xi, W * 8);
    std::memcpy(oz + m * W, zi, W * 8);
    if ((e & 1) == 0) {
      oc[m] = c[i];
      odc[m++] = dc[i];
    } else {
      double s = (e == 3) ? 1.0 : -1.0;
      oc[m] = C * c[i];
      odc[m++] = C * dc[i] + dC * c[i];
      std::memcpy(ox + m * W, qx.data(), W * 8);
      std::memcpy(oz + m * W, qz.data(), W * 8);
      oc[m] = s * (S * c[i]);
      odc[m++] = s * (S * dc[i] + dS * c[i]);
    }
  }
  return m;
}

// QMF energy.
double oracle_qmf_energy(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z,
                         const double* c, const double* theta, const double* phi) {
  Bloch B(nq, theta, phi);
  Neumaier acc;
  for (int64_t i = 0; i < n; ++i) acc.add(c[i] * B.expect(nq, x + i * W, z + i * W));
  return acc.value();
}

// Per-term expectation values <P_k> (for sampled checks).
void oracle_expectations(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z,
                         const double* theta, const double* phi, double* out) {
  Bloch B(nq, theta, phi);
  for (int64_t i = 0; i < n; ++i) out[i] = B.expect(nq, x + i * W, z + i * W);
}

// DIS gradients for n_cand candidate generators (row-major cx, cz).
void oracle_dis_gradients(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z,
                          const double* c, const double* theta, const double* phi,
                          int64_t n_cand, const uint64_t* cx, const uint64_t* cz, double* g) {
  Bloch B(nq, theta, phi);
  std::vector<uint64_t> qx(W), qz(W);
  for (int64_t a = 0; a < n_cand; ++a) {
    Neumaier acc;
    for (int64_t k = 0; k < n; ++k) {
      int e = product(nq, W, x + k * W, z + k * W, cx + a * W, cz + a * W, qx.data(), qz.data());
      if (e == 1) acc.add(c[k] * B.expect(nq, qx.data(), qz.data()));
      else if (e == 3) acc.add(-(c[k] * B.expect(nq, qx.data(), qz.data())));
    }
    g[a] = acc.value();
  }
}

// dE/dtheta_j and dE/dphi_j.
void oracle_qmf_grad_angles(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z,
                            const double* c, const double* theta, const double* phi,
                            double* dtheta, double* dphi) {
  Bloch B(nq, theta, phi);
  std::vector<double> dbt(4 * (size_t)nq), dbp(4 * (size_t)nq);
  for (int q = 0; q < nq; ++q) {
    double st = std::sin(theta[q]), ct = std::cos(theta[q]);
    double sp = std::sin(phi[q]), cp = std::cos(phi[q]);
    dbt[4 * q + 0] = 0.0; dbt[4 * q + 1] = ct * cp; dbt[4 * q + 2] = ct * sp; dbt[4 * q + 3] = -st;
    dbp[4 * q + 0] = 0.0; dbp[4 * q + 1] = -st * sp; dbp[4 * q + 2] = st * cp; dbp[4 * q + 3] = 0.0;
  }
  std::vector<Neumaier> at(nq), ap(nq);
  std::vector<int> ops(nq);
  std::vector<double> pre(nq + 1), suf(nq + 1);
  for (int64_t k = 0; k < n; ++k) {
    for (int q = 0; q < nq; ++q) ops[q] = op_of(x + k * W, z + k * W, q);
    pre[0] = 1.0;
    for (int q = 0; q < nq; ++q) pre[q + 1] = pre[q] * B.b[4 * q + ops[q]];
    suf[nq] = 1.0;
    for (int q = nq - 1; q >= 0; --q) suf[q] = suf[q + 1] * B.b[4 * q + ops[q]];
    for (int q = 0; q < nq; ++q) {
      if (ops[q] == 0) continue;
      double others = pre[q] * suf[q + 1];
      at[q].add(c[k] * dbt[4 * q + ops[q]] * others);
      ap[q].add(c[k] * dbp[4 * q + ops[q]] * others);
    }
  }
  for (int q = 0; q < nq; ++q) { dtheta[q] = at[q].value(); dphi[q] = ap[q].value(); }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Point query of the iterated dressing (Eq. 6 applied to one key at a time).
//
// The coefficient of key K after step j depends only on the coefficients of K
// and K^P_j after step j-1 (Eq. 5: a commuting K keeps its value; an
// anticommuting K receives cos(t) c[K] from itself and s sin(t) c[K^P] from its
// partner), followed by the compression rule |c| < eps.  Evaluated
// recursively with memoisation; H0 is given sorted in the canonical order.
// Returns 1 and the value if K is present after the last step, else 0.
// ---------------------------------------------------------------------------
namespace {

struct PointChain {
  int nq, W, K;
  int64_t n0;
  const uint64_t *x0, *z0;
  const double* c0;
  const uint64_t *px, *pz;   // [K][W]
  const double* taus;
  double eps;
  std::map<std::string, std::pair<int, double>> memo;

  std::string key(int j, const uint64_t* x, const uint64_t* z) const {
    std::string k((const char*)&j, sizeof j);
    k.append((const char*)x, 8 * W);
    k.append((const char*)z, 8 * W);
    return k;
  }

  int lookup0(const uint64_t* x, const uint64_t* z, double* v) const {
    int64_t lo = 0, hi = n0;
    while (lo < hi) {
      int64_t mid = (lo + hi) / 2;
      if (key_less(W, x0 + mid * W, z0 + mid * W, x, z)) lo = mid + 1;
      else hi = mid;
    }
    if (lo < n0 && key_eq(W, x0 + lo * W, z0 + lo * W, x, z)) {
      *v = c0[lo];
      return 1;
    }
    return 0;
  }

  // present after step j (j = 0: H0)?
  int value(int j, const uint64_t* x, const uint64_t* z, double* v) {
    if (j == 0) return lookup0(x, z, v);
    std::string k = key(j, x, z);
    auto it = memo.find(k);
    if (it != memo.end()) {
      *v = it->second.second;
      return it->second.first;
    }
    const uint64_t* ex = px + (size_t)(j - 1) * W;
    const uint64_t* ez = pz + (size_t)(j - 1) * W;
    std::vector<uint64_t> qx(W), qz(W);
    int e = product(nq, W, ex, ez, x, z, qx.data(), qz.data());   // P * K
    double a = 0.0;
    int have = value(j - 1, x, z, &a);
    double out = 0.0;
    int present = 0;
    if ((e & 1) == 0) {
      present = have;
      out = a;
    } else {
      const double C = std::cos(taus[j - 1]), S = std::sin(taus[j - 1]);
      double b = 0.0;
      int have_p = value(j - 1, qx.data(), qz.data(), &b);
      std::vector<uint64_t> rx(W), rz(W);
      int ep = product(nq, W, ex, ez, qx.data(), qz.data(), rx.data(), rz.data());  // P * (K^P)
      double from_p = (ep == 3 ? 1.0 : -1.0) * (S * b);
      if (have && have_p) { out = C * a + from_p; present = 1; }
      else if (have) { out = C * a; present = 1; }
      else if (have_p) { out = from_p; present = 1; }
    }
    if (present && std::fabs(out) < eps) present = 0;
    memo[k] = {present, out};
    *v = out;
    return present;
  }
};

}  // namespace

extern "C" {

// H0 sorted canonically (row-major x0/z0 [n0][W]); entanglers px/pz [K][W].
// For each of n_q query keys: found[i] = present after all K steps, val[i].
void oracle_chain_point(int nq, int W, int64_t n0, const uint64_t* x0, const uint64_t* z0,
                        const double* c0, int K, const uint64_t* px, const uint64_t* pz,
                        const double* taus, double eps, int64_t n_q, const uint64_t* qx,
                        const uint64_t* qz, int8_t* found, double* val) {
  PointChain pc{nq, W, K, n0, x0, z0, c0, px, pz, taus, eps, {}};
  for (int64_t i = 0; i < n_q; ++i) {
    double v = 0.0;
    found[i] = (int8_t)pc.value(K, qx + i * W, qz + i * W, &v);
    val[i] = v;
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The same step on several host threads (the CPU baseline on all cores).
// Arithmetic and summation order are those of oracle_dress_raw,
// oracle_merge_truncate and oracle_qmf_energy; only the work is split, so the
// result does not depend on the thread count:
//  * raw dressing of input slices, concatenated in input order;
//  * the raw rows partitioned by a hash of the key (every copy of a key in one
//    partition, in input order), each partition merged and compressed exactly
//    as oracle_merge_truncate treats a whole list;
//  * energy: per-term products in parallel, the Neumaier sum in input order.
// Output rows come partition by partition, canonical inside a partition.
// ---------------------------------------------------------------------------
namespace {

constexpr int kParts = 256;

inline uint32_t part_of(int W, const uint64_t* x, const uint64_t* z) {
  uint64_t h = 0x9E3779B97F4A7C15ull;
  for (int w = 0; w < W; ++w) {
    h = (h ^ x[w]) * 0xBF58476D1CE4E5B9ull;
    h = (h ^ z[w]) * 0x94D049BB133111EBull;
  }
  h ^= h >> 31;
  return (uint32_t)(h % kParts);
}

}  // namespace

extern "C" {

int64_t oracle_dress_step_par(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z,
                              const double* c, const uint64_t* px, const uint64_t* pz, double tau,
                              double eps, int nthreads, uint64_t* ox, uint64_t* oz, double* oc) {
  const int T = nthreads > 0 ? nthreads : 1;
  const int S = 4 * T;   // input slices
  std::vector<std::vector<uint64_t>> sx(S), sz(S);
  std::vector<std::vector<double>> sc(S);
  std::vector<std::vector<int64_t>> cnt(S, std::vector<int64_t>(kParts, 0));
#pragma omp parallel for schedule(dynamic) num_threads(T)
  for (int s = 0; s < S; ++s) {
    const int64_t lo = n * s / S, hi = n * (s + 1) / S;
    sx[s].resize((size_t)(2 * (hi - lo)) * W);
    sz[s].resize((size_t)(2 * (hi - lo)) * W);
    sc[s].resize((size_t)(2 * (hi - lo)));
    const int64_t m = oracle_dress_raw(nq, W, hi - lo, x + lo * W, z + lo * W, c + lo, px, pz, tau,
                                       sx[s].data(), sz[s].data(), sc[s].data());
    sc[s].resize((size_t)m);
    for (int64_t i = 0; i < m; ++i) ++cnt[s][part_of(W, &sx[s][i * W], &sz[s][i * W])];
  }
  // partition-major layout; inside a partition the slices (input order) follow each other
  std::vector<int64_t> poff(kParts + 1, 0);
  std::vector<std::vector<int64_t>> at(S, std::vector<int64_t>(kParts, 0));
  for (int p = 0; p < kParts; ++p) {
    int64_t o = poff[p];
    for (int s = 0; s < S; ++s) { at[s][p] = o; o += cnt[s][p]; }
    poff[p + 1] = o;
  }
  const int64_t nraw = poff[kParts];
  std::vector<uint64_t> qx((size_t)nraw * W), qz((size_t)nraw * W);
  std::vector<double> qc((size_t)nraw);
#pragma omp parallel for schedule(dynamic) num_threads(T)
  for (int s = 0; s < S; ++s) {
    std::vector<int64_t> pos = at[s];
    for (int64_t i = 0; i < (int64_t)sc[s].size(); ++i) {
      const uint32_t p = part_of(W, &sx[s][i * W], &sz[s][i * W]);
      const int64_t r = pos[p]++;
      std::memcpy(&qx[(size_t)r * W], &sx[s][i * W], W * 8);
      std::memcpy(&qz[(size_t)r * W], &sz[s][i * W], W * 8);
      qc[(size_t)r] = sc[s][i];
    }
    std::vector<uint64_t>().swap(sx[s]);
    std::vector<uint64_t>().swap(sz[s]);
    std::vector<double>().swap(sc[s]);
  }
  // merge + compression of each partition into its own slice of the output
  std::vector<int64_t> kept(kParts, 0);
#pragma omp parallel for schedule(dynamic) num_threads(T)
  for (int p = 0; p < kParts; ++p) {
    const int64_t b = poff[p], len = poff[p + 1] - poff[p];
    kept[p] = oracle_merge_truncate(W, len, &qx[(size_t)b * W], &qz[(size_t)b * W], &qc[(size_t)b],
                                    nullptr, eps, ox + b * W, oz + b * W, oc + b, nullptr);
  }
  int64_t m = 0;
  for (int p = 0; p < kParts; ++p) {
    const int64_t b = poff[p];
    if (m != b) {
      std::memmove(ox + m * W, ox + b * W, (size_t)kept[p] * W * 8);
      std::memmove(oz + m * W, oz + b * W, (size_t)kept[p] * W * 8);
      std::memmove(oc + m, oc + b, (size_t)kept[p] * 8);
    }
    m += kept[p];
  }
  return m;
}

double oracle_qmf_energy_par(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z,
                             const double* c, const double* theta, const double* phi, int nthreads) {
  const int T = nthreads > 0 ? nthreads : 1;
  Bloch B(nq, theta, phi);
  std::vector<double> t((size_t)n);
#pragma omp parallel for schedule(static) num_threads(T)
  for (int64_t i = 0; i < n; ++i) t[(size_t)i] = c[i] * B.expect(nq, x + i * W, z + i * W);
  Neumaier acc;
  for (int64_t i = 0; i < n; ++i) acc.add(t[(size_t)i]);
  return acc.value();
}

}  // extern "C"
