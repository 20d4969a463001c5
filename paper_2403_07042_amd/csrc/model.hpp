// Host-side model of a cavity-QED system: basis, Hamiltonian, decoherence
// tables and the FP64 propagator (the "Taylor approximation" stage).
//
// Everything here runs on the CPU and is independent of HIP, so it can be
// checked without a GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "qme.h"

namespace qme {

// Copy of a validated system + parameters, with the mode layout derived.
struct Model {
  int n_cav = 0;
  std::vector<int> atoms, cap;
  int exc_lo = 0, exc_hi = 0;      // effective window
  int n_modes = 0;
  std::vector<int> photon_mode;     // per cavity
  std::vector<int> atom_mode;       // per atom (cavity-major)
  std::vector<int> atom_cavity;     // cavity of each atom
  std::vector<int> mode_cap;
  std::vector<int> first_atom;      // per cavity, index of its first atom

  // parameters
  std::vector<double> omega_c, omega_a, g;
  std::vector<qme_hop> hops;
  std::vector<qme_jump> jumps;
  double dt = 0.0;
  bool has_params = false;

  // basis
  int64_t n = 0;
  std::vector<int32_t> occ;         // n x n_modes, lexicographic order
  // cnt[m * (exc_hi + 1) + s]: completions of modes m.. given prefix sum s
  // that land in the window; rank() sums it over the levels below a tuple's
  std::vector<uint64_t> cnt;
  // general form (qme_hamiltonian_general): H given as sorted, merged,
  // symmetric COO and each decoherence operator as moves (A |src> has the
  // component c |dst>; moves with one (src, dst) add up); jumps[j].gamma holds
  // the rates.  dst = -1: a component outside the basis, orthogonal to every
  // other one; dst <= -2: a state removed by a restriction (qme_subspace),
  // shared by every move onto it, so A^dag A keeps its cross terms.  No
  // occupation table; the parameter terms are H's symmetric entries.
  struct Move {
    int32_t src;
    int64_t dst;
    double c;
  };
  int64_t next_outside = 0;               // first unused removed-state id (-2 - id)
  std::vector<int32_t> h_in_row, h_in_col;   // H's pattern as given (before merging)
  bool general = false;
  std::vector<int32_t> h_row, h_col;
  std::vector<double> h_val;
  std::vector<std::vector<Move>> moves;   // per jump
  // selected subset of the window basis (state-space selection): remap[f]
  // is the index of window state f in this basis, -1 if it was removed;
  // empty when the basis is the whole window
  std::vector<int32_t> remap;

  int64_t rank(const int32_t *levels) const;   // index in basis or -1
};

// Sparse real matrix, CSR.
struct Csr {
  int64_t n = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

// Per-parameter derivative terms dH/dtheta_p (for gradients), as COO.
struct TermCoo {
  std::vector<int32_t> row, col;
  std::vector<double> val;
};

// Decoherence tables in the gather form used by the dissipator:
//   (A_j rho A_j^dag)[u,v] = c_j[u] c_j[v] rho[pi_j[u], pi_j[v]],
// with pi_j[u] the basis state that A_j maps onto u (-1 if none).
// Only channels with at least one arrival inside the basis are kept in
// pi/cg ("gather channels").  cg = sqrt(gamma_j) c_j.
struct JumpTables {
  int n_gather = 0;
  std::vector<int32_t> gather_channel;   // original jump index of each gather channel
  std::vector<int32_t> pi;               // n_gather x n
  std::vector<double> cg;                // n_gather x n
  std::vector<double> d;                 // sum_j gamma_j (A_j^dag A_j)_uu
  std::vector<double> leak;              // sum_j gamma_j |a_j(u)|^2 [A_j u leaves the basis]
  // forward maps of the gather channels (adjoint decoherence):
  //   (A_j^dag L A_j)[u,v] = a_j[u] a_j[v] L[tau_j[u], tau_j[v]],
  // tau_j[u] = basis index of A_j u (-1 if zero or outside), ca = sqrt(gamma) a
  std::vector<int32_t> tau;              // n_gather x n
  std::vector<double> ca;                // n_gather x n
  // per original jump, unit-rate tables (for rate gradients)
  std::vector<int32_t> unit_pi;          // n_jumps x n
  std::vector<double> unit_c;            // n_jumps x n (c_j, not scaled)
  std::vector<double> unit_ada;          // n_jumps x n diag of A^dag A
  // channels with an arrival inside the basis, whatever their rate
  std::vector<int32_t> arrival_channel;  // original jump index
  std::vector<int32_t> arrival_of;       // per jump: index into arrival_channel or -1

  // General-form channels that are not monomial (a state with several images
  // or several preimages), in sparse form.  Per such channel j (index q):
  //   (A Z A^dag)[u,v] = sum_{(k,a) in row u} sum_{(l,b) in row v} a b Z[k,l]
  // over the rows of A restricted to the basis (row u: the preimages k of
  // image u with their unit-rate coefficients), csr_ptr[q * (n + 1) + u]
  // indexing csr_col / csr_val; the transposed rows (row k: images u of
  // preimage k) in csrt_*; csr_sg[q] = sqrt(gamma_j).  koff: the off-diagonal
  // part of K = sum over these channels of gamma_j A_j^dag A_j (A^dag A formed
  // from the whole operator, before any restriction), CSR over rows u; its
  // diagonal is in d.  kj: the same per channel at unit rate (rate
  // gradients).  loff: the off-diagonal entries (k, l, value) of
  // sum_j gamma_j (A_j^dag A_j - A_Pj^T A_Pj), non-zero only where two kept
  // states move onto one removed state (the lost probability's cross terms;
  // the diagonal part is in leak).  arrive: sum_j gamma_j (A_Pj^T A_Pj)[w,w],
  // the probability each state w sends into the basis (trace weights).
  int n_csr = 0;
  std::vector<int32_t> csr_channel;      // original jump index
  std::vector<int64_t> csr_ptr, csrt_ptr, kj_ptr;   // n_csr x (n + 1)
  std::vector<int32_t> csr_col, csrt_col, kj_col;
  std::vector<double> csr_val, csrt_val, kj_val;
  std::vector<double> csr_sg;
  std::vector<int64_t> koff_ptr;         // n + 1
  std::vector<int32_t> koff_col;
  std::vector<double> koff_val;
  std::vector<int32_t> loff_row, loff_col;
  std::vector<double> loff_val;
  std::vector<double> arrive;            // n
};

bool build_model(const qme_system *sys, const qme_params *par, Model &m,
                 std::string &err);
bool enumerate_basis(Model &m, std::string &err);
// Keep only basis states keep[0..n_keep) (strictly increasing indices into
// the current basis), in that order.
bool restrict_basis(Model &m, const int32_t *keep, int64_t n_keep, std::string &err);
// A model in the general form (validates: symmetric H, monomial jumps).
bool build_general_model(int64_t n, int64_t h_nnz, const int32_t *h_rows, const int32_t *h_cols,
                         const double *h_vals, int32_t n_jumps, const qme_general_jump *jumps,
                         double dt, Model &m, std::string &err, bool &unsupported);
void hamiltonian_coo(const Model &m, std::vector<int32_t> &r,
                     std::vector<int32_t> &c, std::vector<double> &v);
Csr to_csr(int64_t n, const std::vector<int32_t> &r,
           const std::vector<int32_t> &c, const std::vector<double> &v);
// dH/dtheta for each parameter in the gradient order (g per atom, mu per hop).
std::vector<TermCoo> hamiltonian_terms(const Model &m);
JumpTables jump_tables(const Model &m);
// dU = exp(-i H dt) - I, row-major n x n planes; exactly symmetric.
// When scaling and squaring was needed, levels receives the increments
// V_i - I of V_i = exp(-i H dt / 2^i) for i = 1..s (level i-1 in the vector)
// so that the adjoint can undo the squarings.
bool propagator_increment(const Model &m, const Csr &h, std::vector<double> &re,
                          std::vector<double> &im, std::string &err,
                          std::vector<std::vector<double>> *levels = nullptr,
                          int *squarings = nullptr);

// W = L(A, G), the Frechet derivative of exp at A = -i H dt applied to G
// in its adjoint form tr(G L(A, E)) = tr(L(A, G) E); G and W are complex
// planar n x n (FP64, row-major).
bool frechet_adjoint(const Model &m, const Csr &h, const std::vector<double> &g_re,
                     const std::vector<double> &g_im, std::vector<double> &w_re,
                     std::vector<double> &w_im, std::string &err);

// Thread-local error text of the ABI.
void set_error(const std::string &s);

}  // namespace qme
