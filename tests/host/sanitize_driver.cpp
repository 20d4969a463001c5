// Host-only driver for the sanitizer test: exercises the C ABI calls that
// need no GPU (basis enumeration, Hamiltonian triplets, FP64 Taylor
// propagator, argument validation) on several systems, checking sizes,
// symmetry and unitarity.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py; exits
// non-zero on the first failed check.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "qme.h"

static int failures = 0;
#define CHECK(cond)                                                    \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

struct Sys {
  std::vector<int32_t> atoms, caps;
  std::vector<double> oc, oa, g;
  std::vector<qme_hop> hops;
  std::vector<qme_jump> jumps;
  qme_system sys{};
  qme_params par{};
  void finish(int32_t exc_min, int32_t exc_max, double dt) {
    int n_atoms = 0;
    for (int32_t a : atoms) n_atoms += a;
    oc.assign(atoms.size(), 1.0);
    oa.assign(n_atoms > 0 ? n_atoms : 1, 1.0);
    g.resize(n_atoms > 0 ? n_atoms : 1);
    for (size_t k = 0; k < g.size(); ++k) g[k] = 0.01 * (1.0 + 0.1 * double(k));
    sys = {int32_t(atoms.size()), atoms.data(), caps.data(), exc_min, exc_max};
    par = {oc.data(), oa.data(), g.data(), int32_t(hops.size()), hops.data(),
           int32_t(jumps.size()), jumps.data(), dt};
  }
};

static void run(Sys &s, int64_t expect_n, bool propagator) {
  int64_t n = 0;
  CHECK(qme_basis(&s.sys, &n, nullptr, 0) == QME_OK);
  CHECK(n == expect_n);
  int n_modes = int(s.atoms.size());
  for (int32_t a : s.atoms) n_modes += a;
  std::vector<int32_t> occ(size_t(n) * n_modes);
  CHECK(qme_basis(&s.sys, &n, occ.data(), n - 1) == QME_E_SIZE);   // too small a table
  CHECK(qme_basis(&s.sys, &n, occ.data(), n) == QME_OK);
  int64_t nnz = 0;
  CHECK(qme_hamiltonian_coo(&s.sys, &s.par, &nnz, nullptr, nullptr, nullptr, 0) == QME_OK);
  std::vector<int32_t> r(nnz), c(nnz);
  std::vector<double> v(nnz);
  if (nnz > 1)
    CHECK(qme_hamiltonian_coo(&s.sys, &s.par, &nnz, r.data(), c.data(), v.data(), nnz - 1) ==
          QME_E_SIZE);
  CHECK(qme_hamiltonian_coo(&s.sys, &s.par, &nnz, r.data(), c.data(), v.data(), nnz) == QME_OK);
  std::vector<double> h(size_t(n) * n, 0.0);
  for (int64_t e = 0; e < nnz; ++e) {
    CHECK(r[e] >= 0 && r[e] < n && c[e] >= 0 && c[e] < n);
    h[size_t(r[e]) * n + c[e]] += v[e];
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) CHECK(h[size_t(i) * n + j] == h[size_t(j) * n + i]);
  if (!propagator) return;
  std::vector<double> dre(size_t(n) * n), dim(size_t(n) * n);
  CHECK(qme_propagator_host(&s.sys, &s.par, dre.data(), dim.data(), n) == QME_OK);
  // U = I + dU is unitary: |U^dag U - I| small
  double worst = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double sr = 0.0, si = 0.0;
      for (int64_t k = 0; k < n; ++k) {
        const double ar = dre[size_t(k) * n + i] + (k == i), ai = -dim[size_t(k) * n + i];
        const double br = dre[size_t(k) * n + j] + (k == j), bi = dim[size_t(k) * n + j];
        sr += ar * br - ai * bi;
        si += ar * bi + ai * br;
      }
      worst = std::fmax(worst, std::hypot(sr - (i == j), si));
    }
  CHECK(worst < 1e-12);
}

int main() {
  {   // Jaynes-Cummings: one cavity, one atom, photon cap 3 (N = 8)
    Sys s;
    s.atoms = {1};
    s.caps = {3};
    s.jumps = {{QME_JUMP_PHOTON_LEAK, 0, 0, 0.001}};
    s.finish(0, -1, 0.01);
    run(s, 8, true);
  }
  {   // 2 x 2 Tavis-Cummings-Hubbard, cap 2 (N = 144)
    Sys s;
    s.atoms = {2, 2};
    s.caps = {2, 2};
    s.hops = {{0, 1, 0.005}};
    s.jumps = {{QME_JUMP_PHOTON_LEAK, 0, 0, 0.001}, {QME_JUMP_PHOTON_LEAK, 1, 0, 0.001}};
    s.finish(0, -1, 0.01);
    run(s, 144, true);
  }
  {   // three-cavity chain, cap 5 (N = 1728): basis and Hamiltonian only
    Sys s;
    s.atoms = {1, 1, 1};
    s.caps = {5, 5, 5};
    s.hops = {{0, 1, 0.005}, {1, 2, 0.005}};
    s.jumps = {{QME_JUMP_ATOM_DEPHASE, 1, 0, 0.0005}};
    s.finish(0, -1, 0.005);
    run(s, 1728, false);
  }
  {   // 8 x 8 lattice, one atom per site, single excitation (N = 128)
    Sys s;
    s.atoms.assign(64, 1);
    s.caps.assign(64, 1);
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j) {
        if (i + 1 < 8) s.hops.push_back({i * 8 + j, (i + 1) * 8 + j, 0.01});
        if (j + 1 < 8) s.hops.push_back({i * 8 + j, i * 8 + j + 1, 0.01});
      }
    s.finish(1, 1, 0.01);
    run(s, 128, true);
  }
  {   // argument errors
    Sys s;
    s.atoms = {1};
    s.caps = {-1};
    s.finish(0, -1, 0.01);
    int64_t n = 0;
    CHECK(qme_basis(&s.sys, &n, nullptr, 0) == QME_E_ARG);             // negative cap
    CHECK(qme_basis(nullptr, &n, nullptr, 0) == QME_E_ARG);
    s.caps = {3};
    s.finish(5, 4, 0.01);
    CHECK(qme_basis(&s.sys, &n, nullptr, 0) != QME_OK);                // empty window
    s.finish(0, -1, 0.0);
    int64_t nnz = 0;
    CHECK(qme_hamiltonian_coo(&s.sys, &s.par, &nnz, nullptr, nullptr, nullptr, 0) == QME_E_ARG);
    s.finish(0, -1, 0.01);
    s.g[0] = std::nan("");
    CHECK(qme_hamiltonian_coo(&s.sys, &s.par, &nnz, nullptr, nullptr, nullptr, 0) == QME_E_ARG);
    s.g[0] = 0.01;
    s.jumps = {{QME_JUMP_PHOTON_LEAK, 0, 0, -1.0}};
    s.finish(0, -1, 0.01);
    CHECK(qme_hamiltonian_coo(&s.sys, &s.par, &nnz, nullptr, nullptr, nullptr, 0) == QME_E_ARG);
    CHECK(qme_last_error() != nullptr && qme_last_error()[0] != '\0');
  }
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
