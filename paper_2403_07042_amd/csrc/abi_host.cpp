// Host-only entry points of the C ABI (no device needed): basis, Hamiltonian
// COO, FP64 propagator, error text, version.
#include <cstring>
#include <exception>
#include <string>

#include "model.hpp"
#include "qme.h"

namespace qme {
static thread_local std::string tl_error;
void set_error(const std::string &s) { tl_error = s; }
}  // namespace qme

using namespace qme;

#define QME_GUARD_BEGIN try {
#define QME_GUARD_END                                   \
  }                                                     \
  catch (const std::bad_alloc &) {                      \
    set_error("out of host memory");                    \
    return QME_E_SIZE;                                  \
  }                                                     \
  catch (const std::exception &e) {                     \
    set_error(std::string("internal error: ") + e.what()); \
    return QME_E_STATE;                                 \
  }

extern "C" const char *qme_last_error(void) { return tl_error.c_str(); }

extern "C" const char *qme_version(void) { return "qme-mi355x 0.1 (gfx950)"; }

extern "C" qme_status qme_basis(const qme_system *sys, int64_t *n_states, int32_t *occ,
                                int64_t occ_rows) {
  QME_GUARD_BEGIN
  set_error("");
  if (!n_states) { set_error("n_states is NULL"); return QME_E_ARG; }
  Model m;
  std::string err;
  if (!build_model(sys, nullptr, m, err)) { set_error(err); return QME_E_ARG; }
  if (!enumerate_basis(m, err)) { set_error(err); return QME_E_SIZE; }
  *n_states = m.n;
  if (!occ) return QME_OK;
  if (occ_rows < m.n) { set_error("occ buffer has fewer rows than the basis"); return QME_E_SIZE; }
  std::memcpy(occ, m.occ.data(), m.occ.size() * sizeof(int32_t));
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_hamiltonian_coo(const qme_system *sys, const qme_params *par,
                                          int64_t *nnz, int32_t *rows, int32_t *cols,
                                          double *vals, int64_t capacity) {
  QME_GUARD_BEGIN
  set_error("");
  if (!nnz) { set_error("nnz is NULL"); return QME_E_ARG; }
  if (!par) { set_error("params is NULL"); return QME_E_ARG; }
  Model m;
  std::string err;
  if (!build_model(sys, par, m, err)) { set_error(err); return QME_E_ARG; }
  if (!enumerate_basis(m, err)) { set_error(err); return QME_E_SIZE; }
  std::vector<int32_t> r, c;
  std::vector<double> v;
  hamiltonian_coo(m, r, c, v);
  *nnz = int64_t(v.size());
  if (!rows && !cols && !vals) return QME_OK;
  if (!rows || !cols || !vals) { set_error("rows / cols / vals must all be given"); return QME_E_ARG; }
  if (capacity < int64_t(v.size())) { set_error("COO capacity below nnz"); return QME_E_SIZE; }
  std::memcpy(rows, r.data(), r.size() * sizeof(int32_t));
  std::memcpy(cols, c.data(), c.size() * sizeof(int32_t));
  std::memcpy(vals, v.data(), v.size() * sizeof(double));
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_propagator_host(const qme_system *sys, const qme_params *par,
                                          double *du_re, double *du_im, int64_t n) {
  QME_GUARD_BEGIN
  set_error("");
  if (!par || !du_re || !du_im) { set_error("NULL argument"); return QME_E_ARG; }
  Model m;
  std::string err;
  if (!build_model(sys, par, m, err)) { set_error(err); return QME_E_ARG; }
  if (!enumerate_basis(m, err)) { set_error(err); return QME_E_SIZE; }
  if (n != m.n) { set_error("n does not match the basis size"); return QME_E_SIZE; }
  std::vector<int32_t> r, c;
  std::vector<double> v;
  hamiltonian_coo(m, r, c, v);
  Csr h = to_csr(m.n, r, c, v);
  std::vector<double> re, im;
  if (!propagator_increment(m, h, re, im, err)) { set_error(err); return QME_E_NUMERIC; }
  std::memcpy(du_re, re.data(), re.size() * sizeof(double));
  std::memcpy(du_im, im.data(), im.size() * sizeof(double));
  return QME_OK;
  QME_GUARD_END
}
