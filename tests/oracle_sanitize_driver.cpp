// Runs every entry point of the oracle (oracle/iqcc_oracle.cpp) on small
// seeded inputs; tests/test_oracle_sanitized.py compiles it together with the
// oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code only)
// and checks that it finishes cleanly.  Prints "ok" at the end.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

extern "C" {
int oracle_pauli_product(int nq, int W, const uint64_t* x1, const uint64_t* z1, const uint64_t* x2,
                         const uint64_t* z2, uint64_t* x3, uint64_t* z3);
int64_t oracle_dress_raw(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z, const double* c,
                         const uint64_t* px, const uint64_t* pz, double tau, uint64_t* ox, uint64_t* oz,
                         double* oc);
int64_t oracle_merge_truncate(int W, int64_t n, const uint64_t* x, const uint64_t* z, const double* c,
                              const double* dc, double eps, uint64_t* ox, uint64_t* oz, double* oc,
                              double* odc);
int64_t oracle_dress_raw_tangent(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z,
                                 const double* c, const double* dc, const uint64_t* px, const uint64_t* pz,
                                 double tau, int active, uint64_t* ox, uint64_t* oz, double* oc, double* odc);
double oracle_qmf_energy(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z, const double* c,
                         const double* theta, const double* phi);
void oracle_expectations(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z,
                         const double* theta, const double* phi, double* out);
void oracle_dis_gradients(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z, const double* c,
                          const double* theta, const double* phi, int64_t n_cand, const uint64_t* cx,
                          const uint64_t* cz, double* g);
void oracle_qmf_grad_angles(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z, const double* c,
                            const double* theta, const double* phi, double* dtheta, double* dphi);
void oracle_chain_point(int nq, int W, int64_t n0, const uint64_t* x0, const uint64_t* z0, const double* c0,
                        int K, const uint64_t* px, const uint64_t* pz, const double* taus, double eps,
                        int64_t n_q, const uint64_t* qx, const uint64_t* qz, int8_t* found, double* val);
int64_t oracle_dress_step_par(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z, const double* c,
                              const uint64_t* px, const uint64_t* pz, double tau, double eps, int nthreads,
                              uint64_t* ox, uint64_t* oz, double* oc);
double oracle_qmf_energy_par(int nq, int W, int64_t n, const uint64_t* x, const uint64_t* z, const double* c,
                             const double* theta, const double* phi, int nthreads);
}

static int fail(const char* what) {
  std::printf("FAIL %s\n", what);
  return 1;
}

static int run(int nq, int n, unsigned seed) {
  const int W = (nq + 63) / 64;
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  auto key_word = [&](int w) {
    const int bits = nq - 64 * w < 64 ? nq - 64 * w : 64;
    const uint64_t mask = bits == 64 ? ~0ull : ((1ull << bits) - 1);
    return rng() & rng() & mask;   // sparse keys
  };
  std::vector<uint64_t> x((size_t)n * W), z((size_t)n * W);
  std::vector<double> c(n), dc(n);
  for (int i = 0; i < n; ++i) {
    for (int w = 0; w < W; ++w) {
      x[(size_t)i * W + w] = key_word(w);
      z[(size_t)i * W + w] = key_word(w);
    }
    c[i] = U(rng);
    dc[i] = U(rng);
  }
  std::vector<double> th(nq), ph(nq);
  for (int q = 0; q < nq; ++q) {
    th[q] = 3.0 * U(rng);
    ph[q] = 3.0 * U(rng);
  }
  // a canonical, duplicate-free H0 from the merge
  std::vector<uint64_t> hx((size_t)n * W), hz((size_t)n * W);
  std::vector<double> hc(n), hdc(n);
  const int64_t n0 = oracle_merge_truncate(W, n, x.data(), z.data(), c.data(), dc.data(), 0.0, hx.data(),
                                           hz.data(), hc.data(), hdc.data());
  if (n0 <= 0 || n0 > n) return fail("merge size");
  // an entangler with odd Y count
  std::vector<uint64_t> px(W, 0), pz(W, 0);
  px[0] = 0x5ull;
  pz[0] = 0x1ull;
  std::vector<uint64_t> qx(W), qz(W);
  oracle_pauli_product(nq, W, px.data(), pz.data(), hx.data(), hz.data(), qx.data(), qz.data());
  // raw dressing, merge, tangent
  std::vector<uint64_t> rx((size_t)2 * n0 * W), rz((size_t)2 * n0 * W);
  std::vector<double> rc(2 * n0), rdc(2 * n0);
  const int64_t nr = oracle_dress_raw(nq, W, n0, hx.data(), hz.data(), hc.data(), px.data(), pz.data(), 0.3,
                                      rx.data(), rz.data(), rc.data());
  if (nr < n0 || nr > 2 * n0) return fail("raw size");
  const int64_t nt = oracle_dress_raw_tangent(nq, W, n0, hx.data(), hz.data(), hc.data(), hdc.data(), px.data(),
                                              pz.data(), 0.3, 1, rx.data(), rz.data(), rc.data(), rdc.data());
  if (nt != nr) return fail("tangent size");
  std::vector<uint64_t> mx((size_t)nr * W), mz((size_t)nr * W);
  std::vector<double> mc(nr), mdc(nr);
  const int64_t nm = oracle_merge_truncate(W, nr, rx.data(), rz.data(), rc.data(), rdc.data(), 1e-3, mx.data(),
                                           mz.data(), mc.data(), mdc.data());
  std::vector<uint64_t> sx((size_t)2 * n0 * W), sz((size_t)2 * n0 * W);
  std::vector<double> sc(2 * n0);
  const int64_t ns = oracle_dress_step_par(nq, W, n0, hx.data(), hz.data(), hc.data(), px.data(), pz.data(), 0.3,
                                           1e-3, 3, sx.data(), sz.data(), sc.data());
  if (ns != nm) return fail("parallel step size");
  // energy, expectations, DIS gradients, angle gradients
  const double e = oracle_qmf_energy(nq, W, nm, mx.data(), mz.data(), mc.data(), th.data(), ph.data());
  const double ep = oracle_qmf_energy_par(nq, W, nm, mx.data(), mz.data(), mc.data(), th.data(), ph.data(), 3);
  if (e != e || ep != ep) return fail("energy");
  std::vector<double> ex(nm), g(5), dth(nq), dph(nq);
  oracle_expectations(nq, W, nm, mx.data(), mz.data(), th.data(), ph.data(), ex.data());
  oracle_dis_gradients(nq, W, nm, mx.data(), mz.data(), mc.data(), th.data(), ph.data(), 5, hx.data(), hz.data(),
                       g.data());
  oracle_qmf_grad_angles(nq, W, nm, mx.data(), mz.data(), mc.data(), th.data(), ph.data(), dth.data(), dph.data());
  // point queries of a two-step chain
  std::vector<uint64_t> pxs((size_t)2 * W, 0), pzs((size_t)2 * W, 0);
  pxs[0] = 0x5ull; pzs[0] = 0x1ull;
  pxs[W] = 0x6ull; pzs[W] = 0x4ull;
  const double taus[2] = {0.3, -0.2};
  std::vector<int8_t> found(8);
  std::vector<double> val(8);
  oracle_chain_point(nq, W, n0, hx.data(), hz.data(), hc.data(), 2, pxs.data(), pzs.data(), taus, 1e-8, 8,
                     mx.data(), mz.data(), found.data(), val.data());
  return 0;
}

int main() {
  if (run(40, 300, 1)) return 1;
  if (run(100, 300, 2)) return 1;
  if (run(200, 200, 3)) return 1;
  std::printf("ok\n");
  return 0;
}
