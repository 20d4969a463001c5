// Host-side model: validation, basis enumeration, Hamiltonian assembly,
// decoherence gather tables and the FP64 Taylor propagator.
//
// Basis (Sec. II first point; Sec. IV.B Eqs. 10-11): occupation tuples with
// total excitation in a window, lexicographic order, mode 0 most significant.
// Hamiltonian (Sec. IV.A Eq. 8b, Sec. IV.B Eq. 12): RWA Jaynes-/Tavis-
// Cummings-Hubbard form, hbar = 1.  Propagator ("Taylor approximation"
// stage, Sec. IV.B / Table III): truncated Taylor series of exp(-i H dt)
// with scaling and squaring, in FP64.
#include "model.hpp"

#include <algorithm>
#include <map>
#include <cmath>
#include <thread>

namespace qme {

static constexpr int64_t kMaxStates = int64_t(1) << 20;

namespace {
struct Trip {
  int32_t r, c;
  double v;
};
}  // namespace
static constexpr int kMaxLevel = 64;

static bool finite(double x) { return std::isfinite(x); }

bool build_model(const qme_system *sys, const qme_params *par, Model &m,
                 std::string &err) {
  if (!sys) { err = "system is NULL"; return false; }
  if (sys->n_cavities < 1 || sys->n_cavities > (1 << 20)) {
    err = "n_cavities must be in [1, 2^20]"; return false;
  }
  if (!sys->atoms || !sys->photon_cap) { err = "atoms / photon_cap is NULL"; return false; }
  m = Model();
  m.n_cav = sys->n_cavities;
  int total_cap = 0;
  for (int c = 0; c < m.n_cav; ++c) {
    int a = sys->atoms[c], p = sys->photon_cap[c];
    if (a < 0 || a > kMaxLevel) { err = "atoms[c] must be in [0, 64]"; return false; }
    if (p < 0 || p > kMaxLevel) { err = "photon_cap[c] must be in [0, 64]"; return false; }
    m.atoms.push_back(a);
    m.cap.push_back(p);
    m.first_atom.push_back(int(m.atom_mode.size()));
    m.photon_mode.push_back(int(m.mode_cap.size()));
    m.mode_cap.push_back(p);
    total_cap += p;
    for (int k = 0; k < a; ++k) {
      m.atom_mode.push_back(int(m.mode_cap.size()));
      m.atom_cavity.push_back(c);
      m.mode_cap.push_back(1);
      total_cap += 1;
    }
  }
  m.n_modes = int(m.mode_cap.size());
  if (sys->exc_min < 0) { err = "exc_min must be >= 0"; return false; }
  m.exc_lo = sys->exc_min;
  m.exc_hi = sys->exc_max < 0 ? total_cap : std::min(sys->exc_max, total_cap);
  if (sys->exc_max >= 0 && sys->exc_max < sys->exc_min) {
    err = "empty excitation window (exc_max < exc_min)"; return false;
  }
  if (m.exc_lo > m.exc_hi) { err = "empty excitation window (exc_min above the largest excitation)"; return false; }

  if (!par) return true;
  const int n_atoms = int(m.atom_mode.size());
  if (!par->omega_c || (n_atoms > 0 && (!par->omega_a || !par->g))) {
    err = "omega_c / omega_a / g is NULL"; return false;
  }
  if (!finite(par->dt) || !(par->dt > 0.0)) { err = "dt must be finite and > 0"; return false; }
  for (int c = 0; c < m.n_cav; ++c) {
    if (!finite(par->omega_c[c])) { err = "omega_c is not finite"; return false; }
    m.omega_c.push_back(par->omega_c[c]);
  }
  for (int k = 0; k < n_atoms; ++k) {
    if (!finite(par->omega_a[k]) || !finite(par->g[k])) { err = "omega_a / g is not finite"; return false; }
    m.omega_a.push_back(par->omega_a[k]);
    m.g.push_back(par->g[k]);
  }
  if (par->n_hops < 0 || (par->n_hops > 0 && !par->hops)) { err = "bad hops"; return false; }
  for (int h = 0; h < par->n_hops; ++h) {
    qme_hop hp = par->hops[h];
    if (hp.a < 0 || hp.a >= m.n_cav || hp.b < 0 || hp.b >= m.n_cav || hp.a == hp.b) {
      err = "hop cavities must be two distinct valid cavities"; return false;
    }
    if (!finite(hp.mu)) { err = "hop mu is not finite"; return false; }
    m.hops.push_back(hp);
  }
  if (par->n_jumps < 0 || (par->n_jumps > 0 && !par->jumps)) { err = "bad jumps"; return false; }
  for (int j = 0; j < par->n_jumps; ++j) {
    qme_jump jp = par->jumps[j];
    if (jp.kind < QME_JUMP_PHOTON_LEAK || jp.kind > QME_JUMP_ATOM_DEPHASE) {
      err = "unknown jump kind"; return false;
    }
    if (jp.cavity < 0 || jp.cavity >= m.n_cav) { err = "jump cavity out of range"; return false; }
    if (jp.kind != QME_JUMP_PHOTON_LEAK && (jp.atom < 0 || jp.atom >= m.atoms[jp.cavity])) {
      err = "jump atom out of range"; return false;
    }
    if (!finite(jp.gamma) || jp.gamma < 0.0) { err = "jump gamma must be finite and >= 0"; return false; }
    m.jumps.push_back(jp);
  }
  m.dt = par->dt;
  m.has_params = true;
  return true;
}

// ---------------------------------------------------------------- basis
// cnt[m][s]: number of completions of modes m..M-1 given prefix sum s whose
// total lies in [lo, hi]; saturates at 2^62.

static std::vector<uint64_t> count_table(const Model &m) {
  const int M = m.n_modes, H = m.exc_hi;
  std::vector<uint64_t> cnt(size_t(M + 1) * (H + 1), 0);
  const uint64_t sat = uint64_t(1) << 62;
  for (int s = 0; s <= H; ++s) cnt[size_t(M) * (H + 1) + s] = (s >= m.exc_lo) ? 1 : 0;
  for (int md = M - 1; md >= 0; --md) {
    for (int s = 0; s <= H; ++s) {
      uint64_t acc = 0;
      for (int l = 0; l <= m.mode_cap[md] && s + l <= H; ++l) {
        acc += cnt[size_t(md + 1) * (H + 1) + s + l];
        if (acc > sat) acc = sat;
      }
      cnt[size_t(md) * (H + 1) + s] = acc;
    }
  }
  return cnt;
}

int64_t Model::rank(const int32_t *x) const {
  const int H = exc_hi;
  int64_t r = 0;
  int s = 0;
  for (int md = 0; md < n_modes; ++md) {
    int l = x[md];
    if (l < 0 || l > mode_cap[md]) return -1;
    for (int t = 0; t < l; ++t) {
      if (s + t > H) break;
      r += int64_t(cnt[size_t(md + 1) * (H + 1) + s + t]);
    }
    s += l;
  }
  if (s < exc_lo || s > exc_hi) return -1;
  return remap.empty() ? r : int64_t(remap[size_t(r)]);
}

bool build_general_model(int64_t n, int64_t h_nnz, const int32_t *h_rows, const int32_t *h_cols,
                         const double *h_vals, int32_t n_jumps, const qme_general_jump *jumps,
                         double dt, Model &m, std::string &err, bool &unsupported) {
  unsupported = false;
  if (n < 1 || n > kMaxStates) { err = "n must be in [1, 2^20]"; return false; }
  if (h_nnz < 0 || (h_nnz > 0 && (!h_rows || !h_cols || !h_vals))) { err = "H arrays are NULL"; return false; }
  if (n_jumps < 0 || (n_jumps > 0 && !jumps)) { err = "jumps is NULL"; return false; }
  if (!(dt > 0.0) || !std::isfinite(dt)) { err = "dt must be finite and > 0"; return false; }
  m = Model();
  m.general = true;
  m.n = n;
  m.dt = dt;
  m.has_params = true;
  std::vector<Trip> t;
  t.reserve(size_t(h_nnz));
  for (int64_t e = 0; e < h_nnz; ++e) {
    if (h_rows[e] < 0 || h_rows[e] >= n || h_cols[e] < 0 || h_cols[e] >= n) {
      err = "H index out of range"; return false;
    }
    if (!std::isfinite(h_vals[e])) { err = "H value is not finite"; return false; }
    t.push_back({h_rows[e], h_cols[e], h_vals[e]});
  }
  std::sort(t.begin(), t.end(), [](const Trip &a, const Trip &b) {
    return a.r != b.r ? a.r < b.r : a.c < b.c;
  });
  for (const Trip &x : t) {
    if (!m.h_row.empty() && m.h_row.back() == x.r && m.h_col.back() == x.c) {
      m.h_val.back() += x.v;
    } else {
      m.h_row.push_back(x.r); m.h_col.push_back(x.c); m.h_val.push_back(x.v);
    }
  }
  // symmetric: the transpose, sorted the same way, must match entry for entry
  {
    std::vector<size_t> idx(m.h_val.size());
    for (size_t e = 0; e < idx.size(); ++e) idx[e] = e;
    std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
      return m.h_col[a] != m.h_col[b] ? m.h_col[a] < m.h_col[b] : m.h_row[a] < m.h_row[b];
    });
    for (size_t e = 0; e < idx.size(); ++e) {
      const size_t q = idx[e];
      if (m.h_col[q] != m.h_row[e] || m.h_row[q] != m.h_col[e] || m.h_val[q] != m.h_val[e]) {
        err = "H must be symmetric (real Hermitian)";
        return false;
      }
    }
  }
  m.moves.resize(size_t(n_jumps));
  for (int32_t j = 0; j < n_jumps; ++j) {
    const qme_general_jump &jp = jumps[j];
    if (!(jp.gamma >= 0.0) || !std::isfinite(jp.gamma)) { err = "gamma must be finite and >= 0"; return false; }
    if (jp.n_moves < 0 || (jp.n_moves > 0 && (!jp.source || !jp.target || !jp.coef))) {
      err = "jump arrays are NULL"; return false;
    }
    qme_jump q{-1, 0, 0, jp.gamma};
    m.jumps.push_back(q);
    for (int64_t e = 0; e < jp.n_moves; ++e) {
      const int32_t a = jp.source[e], b = jp.target[e];
      if (a < 0 || a >= n || b < -1 || b >= n) { err = "jump index out of range"; return false; }
      if (!std::isfinite(jp.coef[e])) { err = "jump coefficient is not finite"; return false; }
      if (jp.coef[e] != 0.0) m.moves[size_t(j)].push_back({a, int64_t(b), jp.coef[e]});
    }
  }
  // the gradient parameters: H's symmetric entries (one per pair r <= c of
  // the merged pattern)
  for (size_t e = 0; e < m.h_val.size(); ++e)
    if (m.h_row[e] <= m.h_col[e]) {
      m.h_in_row.push_back(m.h_row[e]);
      m.h_in_col.push_back(m.h_col[e]);
    }
  return true;
}

bool restrict_basis(Model &m, const int32_t *keep, int64_t n_keep, std::string &err) {
  if (n_keep < 1 || n_keep > m.n) { err = "n_keep must be in [1, N]"; return false; }
  if (!keep) { err = "keep is NULL"; return false; }
  std::vector<int32_t> pos(size_t(m.n), -1);
  for (int64_t i = 0; i < n_keep; ++i) {
    if (keep[i] < 0 || keep[i] >= m.n || (i > 0 && keep[i] <= keep[i - 1])) {
      err = "keep must be strictly increasing basis indices";
      return false;
    }
    pos[size_t(keep[i])] = int32_t(i);
  }
  if (m.general) {
    std::vector<int32_t> r, c;
    std::vector<double> v;
    for (size_t e = 0; e < m.h_val.size(); ++e) {
      const int32_t a = pos[size_t(m.h_row[e])], b = pos[size_t(m.h_col[e])];
      if (a >= 0 && b >= 0) { r.push_back(a); c.push_back(b); v.push_back(m.h_val[e]); }
    }
    m.h_row.swap(r);
    m.h_col.swap(c);
    m.h_val.swap(v);
    // a move onto a removed state keeps that state's identity (an id below
    // -1, unique over all restrictions of this model), so moves of two kept
    // states onto it still share it in A^dag A
    for (auto &mv : m.moves) {
      std::vector<Model::Move> kept;
      for (const Model::Move &x : mv) {
        if (pos[size_t(x.src)] < 0) continue;
        int64_t d = x.dst;
        if (d >= 0) d = pos[size_t(d)] >= 0 ? int64_t(pos[size_t(d)]) : -2 - (m.next_outside + d);
        kept.push_back({pos[size_t(x.src)], d, x.c});
      }
      mv.swap(kept);
    }
    m.next_outside += m.n;
    // the parameters keep their identity on the kept states
    {
      std::vector<int32_t> r, c;
      for (size_t e = 0; e < m.h_in_row.size(); ++e) {
        r.push_back(pos[size_t(m.h_in_row[e])]);
        c.push_back(pos[size_t(m.h_in_col[e])]);
      }
      m.h_in_row.swap(r);
      m.h_in_col.swap(c);
    }
    m.n = n_keep;
    return true;
  }
  // window index -> current index -> new index
  if (m.remap.empty()) {
    m.remap = pos;
  } else {
    for (int32_t &f : m.remap)
      if (f >= 0) f = pos[size_t(f)];
  }
  const int M = m.n_modes;
  std::vector<int32_t> occ(size_t(n_keep) * M);
  for (int64_t i = 0; i < n_keep; ++i)
    std::copy(m.occ.begin() + size_t(keep[i]) * M, m.occ.begin() + size_t(keep[i] + 1) * M,
              occ.begin() + size_t(i) * M);
  m.occ.swap(occ);
  m.n = n_keep;
  return true;
}

bool enumerate_basis(Model &m, std::string &err) {
  const int M = m.n_modes, H = m.exc_hi;
  if (double(M + 1) * double(H + 1) > double(1 << 26)) {
    err = "basis too large (modes x excitation window)"; return false;
  }
  m.cnt = count_table(m);
  uint64_t n = m.cnt[0];
  if (n > uint64_t(kMaxStates)) { err = "basis has more than 2^20 states"; return false; }
  if (n == 0) { err = "empty basis"; return false; }
  m.n = int64_t(n);
  m.occ.assign(size_t(n) * M, 0);
  // remaining capacity after mode md
  std::vector<int> rem(M + 1, 0);
  for (int md = M - 1; md >= 0; --md) rem[md] = rem[md + 1] + m.mode_cap[md];
  std::vector<int> lvl(M, -1), pre(M + 1, 0);
  int64_t row = 0;
  int md = 0;
  // iterative depth-first search, levels ascending: emits tuples in
  // lexicographic order
  while (md >= 0) {
    int s = pre[md];
    int l = lvl[md] + 1;
    bool found = false;
    for (; l <= m.mode_cap[md] && s + l <= H; ++l) {
      if (s + l + rem[md + 1] >= m.exc_lo) { found = true; break; }
    }
    if (!found) { lvl[md] = -1; --md; continue; }
    lvl[md] = l;
    if (md == M - 1) {
      if (row >= m.n) { err = "internal: basis enumeration overran its count"; return false; }
      std::copy(lvl.begin(), lvl.end(), m.occ.begin() + size_t(row) * M);
      ++row;
      continue;
    }
    pre[md + 1] = s + l;
    ++md;
    lvl[md] = -1;
  }
  if (row != m.n) { err = "internal: basis enumeration count mismatch"; return false; }
  return true;
}

// ------------------------------------------------------------ Hamiltonian


// Visit every off-diagonal move of the coupling/hopping terms from source
// state u: fn(param_index, target, amplitude).  param_index follows the
// gradient order (atoms, then hops).
template <class Fn>
static void for_each_move(const Model &m, int64_t u, std::vector<int32_t> &buf,
                          Fn &&fn) {
  const int M = m.n_modes;
  const int32_t *src = m.occ.data() + size_t(u) * M;
  const int n_atoms = int(m.atom_mode.size());
  for (int k = 0; k < n_atoms; ++k) {
    int am = m.atom_mode[k], pm = m.photon_mode[m.atom_cavity[k]];
    int n = src[pm], s = src[am];
    if (s == 1 && n < m.mode_cap[pm]) {           // a^dag sigma
      std::copy(src, src + M, buf.begin());
      buf[pm] = n + 1; buf[am] = 0;
      int64_t t = m.rank(buf.data());
      if (t >= 0) fn(k, t, std::sqrt(double(n + 1)));
    } else if (s == 0 && n >= 1) {                 // a sigma^dag
      std::copy(src, src + M, buf.begin());
      buf[pm] = n - 1; buf[am] = 1;
      int64_t t = m.rank(buf.data());
      if (t >= 0) fn(k, t, std::sqrt(double(n)));
    }
  }
  for (size_t h = 0; h < m.hops.size(); ++h) {
    int pa = m.photon_mode[m.hops[h].a], pb = m.photon_mode[m.hops[h].b];
    for (int dir = 0; dir < 2; ++dir) {
      int to = dir ? pb : pa, from = dir ? pa : pb;   // a_to^dag a_from
      int nf = src[from], nt = src[to];
      if (nf >= 1 && nt < m.mode_cap[to]) {
        std::copy(src, src + M, buf.begin());
        buf[from] = nf - 1; buf[to] = nt + 1;
        int64_t t = m.rank(buf.data());
        if (t >= 0) fn(n_atoms + int(h), t, std::sqrt(double(nf)) * std::sqrt(double(nt + 1)));
      }
    }
  }
}

void hamiltonian_coo(const Model &m, std::vector<int32_t> &r,
                     std::vector<int32_t> &c, std::vector<double> &v) {
  if (m.general) {   // already sorted by (row, col) and merged; a subset keeps the order
    r = m.h_row;
    c = m.h_col;
    v = m.h_val;
    return;
  }
  const int M = m.n_modes;
  const int n_atoms = int(m.atom_mode.size());
  std::vector<Trip> t;
  t.reserve(size_t(m.n) * 4);
  std::vector<int32_t> buf(M);
  for (int64_t u = 0; u < m.n; ++u) {
    const int32_t *src = m.occ.data() + size_t(u) * M;
    double diag = 0.0;
    for (int cv = 0; cv < m.n_cav; ++cv) diag += m.omega_c[cv] * double(src[m.photon_mode[cv]]);
    for (int k = 0; k < n_atoms; ++k) diag += m.omega_a[k] * double(src[m.atom_mode[k]]);
    t.push_back({int32_t(u), int32_t(u), diag});
    for_each_move(m, u, buf, [&](int p, int64_t tgt, double amp) {
      double coef = p < n_atoms ? m.g[p] : m.hops[p - n_atoms].mu;
      t.push_back({int32_t(tgt), int32_t(u), coef * amp});
    });
  }
  std::sort(t.begin(), t.end(), [](const Trip &a, const Trip &b) {
    return a.r != b.r ? a.r < b.r : a.c < b.c;
  });
  r.clear(); c.clear(); v.clear();
  for (const Trip &x : t) {
    if (!r.empty() && r.back() == x.r && c.back() == x.c) {
      v.back() += x.v;
    } else {
      r.push_back(x.r); c.push_back(x.c); v.push_back(x.v);
    }
  }
}

std::vector<TermCoo> hamiltonian_terms(const Model &m) {
  if (m.general) {
    // one parameter per symmetric entry h = H[r][c] = H[c][r] (r <= c) of the
    // model as given; an entry whose state a restriction removed acts on
    // nothing (empty term, zero gradient)
    std::vector<TermCoo> terms(m.h_in_row.size());
    for (size_t e = 0; e < m.h_in_row.size(); ++e) {
      const int32_t r = m.h_in_row[e], c = m.h_in_col[e];
      if (r < 0 || c < 0) continue;
      terms[e].row.push_back(r);
      terms[e].col.push_back(c);
      terms[e].val.push_back(1.0);
      if (r != c) {
        terms[e].row.push_back(c);
        terms[e].col.push_back(r);
        terms[e].val.push_back(1.0);
      }
    }
    return terms;
  }
  const int n_atoms = int(m.atom_mode.size());
  std::vector<TermCoo> terms(n_atoms + m.hops.size());
  std::vector<int32_t> buf(m.n_modes);
  for (int64_t u = 0; u < m.n; ++u) {
    for_each_move(m, u, buf, [&](int p, int64_t tgt, double amp) {
      terms[p].row.push_back(int32_t(tgt));
      terms[p].col.push_back(int32_t(u));
      terms[p].val.push_back(amp);
    });
  }
  return terms;
}

Csr to_csr(int64_t n, const std::vector<int32_t> &r, const std::vector<int32_t> &c,
           const std::vector<double> &v) {
  Csr a;
  a.n = n;
  a.ptr.assign(n + 1, 0);
  for (int32_t x : r) a.ptr[x + 1]++;
  for (int64_t i = 0; i < n; ++i) a.ptr[i + 1] += a.ptr[i];
  a.col.resize(c.size());
  a.val.resize(v.size());
  std::vector<int64_t> pos(a.ptr.begin(), a.ptr.end() - 1);
  for (size_t e = 0; e < r.size(); ++e) {
    int64_t p = pos[r[e]]++;
    a.col[p] = c[e];
    a.val[p] = v[e];
  }
  return a;
}

// ---------------------------------------------------------- decoherence

JumpTables jump_tables(const Model &m) {
  const int64_t n = m.n;
  const int M = m.n_modes;
  const int nj = int(m.jumps.size());
  JumpTables jt;
  jt.d.assign(n, 0.0);
  jt.leak.assign(n, 0.0);
  jt.unit_pi.assign(size_t(nj) * n, -1);
  jt.unit_c.assign(size_t(nj) * n, 0.0);
  jt.unit_ada.assign(size_t(nj) * n, 0.0);
  std::vector<int32_t> buf(M);
  std::vector<char> has_arrival(nj, 0);
  jt.arrive.assign(n, 0.0);
  jt.koff_ptr.assign(n + 1, 0);
  std::vector<std::vector<std::pair<int32_t, double>>> koff_rows(m.general ? size_t(n) : 0);
  std::vector<std::vector<std::pair<int32_t, double>>> loff_rows(m.general ? size_t(n) : 0);
  for (int j = 0; m.general && j < nj; ++j) {
    const double gamma = m.jumps[j].gamma;
    const std::vector<Model::Move> &mv = m.moves[j];
    // monomial: every state has at most one move and every target (other
    // than the private outside one, -1) at most one source
    bool monomial = true;
    {
      std::vector<char> src_seen(size_t(n), 0);
      std::map<int64_t, int> dst_seen;
      for (const Model::Move &x : mv) {
        if (src_seen[size_t(x.src)]++ || (x.dst != -1 && dst_seen[x.dst]++)) {
          monomial = false;
          break;
        }
      }
    }
    if (monomial) {
      for (const Model::Move &x : mv) {
        const double a2 = x.c * x.c;
        jt.unit_ada[size_t(j) * n + x.src] = a2;
        jt.d[x.src] += gamma * a2;
        if (x.dst >= 0) {
          jt.unit_pi[size_t(j) * n + x.dst] = x.src;
          jt.unit_c[size_t(j) * n + x.dst] = x.c;
          has_arrival[j] = 1;
        } else {
          jt.leak[x.src] += gamma * a2;
        }
      }
      continue;
    }
    // sparse channel: A's entries per image key (basis state, removed state
    // id, or a private outside row per move onto -1), duplicates summed
    std::map<int64_t, std::map<int32_t, double>> rows;   // key -> (preimage -> coefficient)
    int64_t private_key = -(int64_t(1) << 62);
    for (const Model::Move &x : mv) {
      const int64_t key = x.dst == -1 ? private_key++ : x.dst;
      rows[key][x.src] += x.c;
    }
    // K = A^dag A over every row; M = the same over the basis rows only
    std::map<std::pair<int32_t, int32_t>, double> kmat, mmat;
    for (const auto &kv : rows)
      for (const auto &a : kv.second)
        for (const auto &b : kv.second) {
          const double prod = a.second * b.second;
          kmat[{a.first, b.first}] += prod;
          if (kv.first >= 0) mmat[{a.first, b.first}] += prod;
        }
    const int q = jt.n_csr++;
    jt.csr_channel.push_back(j);
    jt.csr_sg.push_back(std::sqrt(gamma));
    // A on the basis, rows = images, and its transpose
    std::vector<std::vector<std::pair<int32_t, double>>> arow(static_cast<size_t>(n)), atrow(static_cast<size_t>(n));
    for (const auto &kv : rows) {
      if (kv.first < 0) continue;
      for (const auto &a : kv.second) {
        if (a.second == 0.0) continue;
        arow[size_t(kv.first)].push_back({a.first, a.second});
        atrow[size_t(a.first)].push_back({int32_t(kv.first), a.second});
      }
    }
    auto append = [&](std::vector<int64_t> &ptr, std::vector<int32_t> &col, std::vector<double> &val,
                      const std::vector<std::vector<std::pair<int32_t, double>>> &r) {
      for (int64_t u = 0; u < n; ++u) {
        ptr.push_back(int64_t(col.size()));
        for (const auto &e : r[size_t(u)]) {
          col.push_back(e.first);
          val.push_back(e.second);
        }
      }
      ptr.push_back(int64_t(col.size()));
    };
    append(jt.csr_ptr, jt.csr_col, jt.csr_val, arow);
    append(jt.csrt_ptr, jt.csrt_col, jt.csrt_val, atrow);
    std::vector<std::vector<std::pair<int32_t, double>>> krow(static_cast<size_t>(n));
    for (const auto &kv : kmat) {
      const int32_t k = kv.first.first, l = kv.first.second;
      const double mv_kl = mmat.count(kv.first) ? mmat[kv.first] : 0.0;
      if (k == l) {
        jt.unit_ada[size_t(j) * n + k] = kv.second;
        jt.d[k] += gamma * kv.second;
        jt.arrive[k] += gamma * mv_kl;
        jt.leak[k] += gamma * (kv.second - mv_kl);
      } else if (kv.second != 0.0) {
        krow[size_t(k)].push_back({l, kv.second});
        koff_rows[size_t(k)].push_back({l, gamma * kv.second});
        if (kv.second - mv_kl != 0.0) loff_rows[size_t(k)].push_back({l, gamma * (kv.second - mv_kl)});
      }
    }
    append(jt.kj_ptr, jt.kj_col, jt.kj_val, krow);
  }
  if (m.general) {
    // K's off-diagonal part summed over the sparse channels (entries of one
    // (k, l) added in channel order), and the lost probability's cross terms
    for (int64_t k = 0; k < n; ++k) {
      std::map<int32_t, double> acc;
      for (const auto &e : koff_rows[size_t(k)]) acc[e.first] += e.second;
      for (const auto &e : acc) {
        jt.koff_col.push_back(e.first);
        jt.koff_val.push_back(e.second);
      }
      jt.koff_ptr[size_t(k) + 1] = int64_t(jt.koff_col.size());
      std::map<int32_t, double> lacc;
      for (const auto &e : loff_rows[size_t(k)]) lacc[e.first] += e.second;
      for (const auto &e : lacc) {
        jt.loff_row.push_back(int32_t(k));
        jt.loff_col.push_back(e.first);
        jt.loff_val.push_back(e.second);
      }
    }
  }
  for (int j = 0; !m.general && j < nj; ++j) {
    const qme_jump &jp = m.jumps[j];
    int mode = jp.kind == QME_JUMP_PHOTON_LEAK
                   ? m.photon_mode[jp.cavity]
                   : m.atom_mode[m.first_atom[jp.cavity] + jp.atom];
    for (int64_t w = 0; w < n; ++w) {
      const int32_t *src = m.occ.data() + size_t(w) * M;
      int lv = src[mode];
      if (lv == 0) continue;
      double amp = jp.kind == QME_JUMP_PHOTON_LEAK ? std::sqrt(double(lv)) : 1.0;
      std::copy(src, src + M, buf.begin());
      if (jp.kind != QME_JUMP_ATOM_DEPHASE) buf[mode] = lv - 1;
      int64_t t = m.rank(buf.data());
      double a2 = amp * amp;
      jt.unit_ada[size_t(j) * n + w] = a2;
      jt.d[w] += jp.gamma * a2;
      if (t >= 0) {
        jt.unit_pi[size_t(j) * n + t] = int32_t(w);
        jt.unit_c[size_t(j) * n + t] = amp;
        has_arrival[j] = 1;
      } else {
        jt.leak[w] += jp.gamma * a2;
      }
    }
  }
  jt.arrival_of.assign(nj, -1);
  for (int j = 0; j < nj; ++j) {
    if (!has_arrival[j]) continue;
    jt.arrival_of[j] = int(jt.arrival_channel.size());
    jt.arrival_channel.push_back(j);
    if (m.jumps[j].gamma == 0.0) continue;
    jt.gather_channel.push_back(j);
    double sg = std::sqrt(m.jumps[j].gamma);
    size_t base = jt.tau.size();
    jt.tau.resize(base + n, -1);
    jt.ca.resize(base + n, 0.0);
    for (int64_t u = 0; u < n; ++u) {
      int32_t w = jt.unit_pi[size_t(j) * n + u];
      jt.pi.push_back(w);
      jt.cg.push_back(sg * jt.unit_c[size_t(j) * n + u]);
      if (w >= 0) {   // A_j maps w onto u
        jt.tau[base + w] = int32_t(u);
        jt.ca[base + w] = sg * jt.unit_c[size_t(j) * n + u];
      }
    }
  }
  jt.n_gather = int(jt.gather_channel.size());
  return jt;
}

// ------------------------------------------------------------ propagator

// out = a * x (sparse real times dense real, row-major n x n), threaded.
static void spmm(const Csr &a, const std::vector<double> &x, std::vector<double> &out,
                 double scale) {
  const int64_t n = a.n;
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  auto work = [&](int64_t r0, int64_t r1) {
    for (int64_t i = r0; i < r1; ++i) {
      double *o = out.data() + size_t(i) * n;
      std::fill(o, o + n, 0.0);
      for (int64_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
        const double hv = a.val[p] * scale;
        const double *xr = x.data() + size_t(a.col[p]) * n;
        for (int64_t j = 0; j < n; ++j) o[j] += hv * xr[j];
      }
    }
  };
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    int64_t r0 = t * chunk, r1 = std::min(n, r0 + chunk);
    if (r0 < r1) th.emplace_back(work, r0, r1);
  }
  for (auto &t : th) t.join();
}

// c = a * b for complex planar dense n x n (host, threaded; squaring only).
static void zgemm_host(int64_t n, const std::vector<double> &ar, const std::vector<double> &ai,
                       const std::vector<double> &br, const std::vector<double> &bi,
                       std::vector<double> &cr, std::vector<double> &ci) {
  cr.assign(size_t(n) * n, 0.0);
  ci.assign(size_t(n) * n, 0.0);
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  auto work = [&](int64_t r0, int64_t r1) {
    for (int64_t i = r0; i < r1; ++i) {
      double *orr = cr.data() + size_t(i) * n, *oi = ci.data() + size_t(i) * n;
      for (int64_t k = 0; k < n; ++k) {
        double xr = ar[size_t(i) * n + k], xi = ai[size_t(i) * n + k];
        if (xr == 0.0 && xi == 0.0) continue;
        const double *yr = br.data() + size_t(k) * n, *yi = bi.data() + size_t(k) * n;
        for (int64_t j = 0; j < n; ++j) {
          orr[j] += xr * yr[j] - xi * yi[j];
          oi[j] += xr * yi[j] + xi * yr[j];
        }
      }
    }
  };
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    int64_t r0 = t * chunk, r1 = std::min(n, r0 + chunk);
    if (r0 < r1) th.emplace_back(work, r0, r1);
  }
  for (auto &t : th) t.join();
}

bool propagator_increment(const Model &m, const Csr &h, std::vector<double> &re,
                          std::vector<double> &im, std::string &err,
                          std::vector<std::vector<double>> *levels, int *nsq) {
  const int64_t n = m.n;
  // theta = |H dt|_1 (largest absolute column sum; H is symmetric, so rows)
  double norm1 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t p = h.ptr[i]; p < h.ptr[i + 1]; ++p) s += std::fabs(h.val[p]);
    norm1 = std::max(norm1, s);
  }
  double theta = norm1 * m.dt;
  int squarings = 0;
  while (theta > 0.5 && squarings < 60) { theta *= 0.5; ++squarings; }
  const double tau = m.dt / std::ldexp(1.0, squarings);

  // dU(tau) = sum_{k>=1} (-i tau H)^k / k!.  (-i)^k cycles -i, -1, +i, +1:
  // odd k feed the imaginary plane, even k the real plane, and every power
  // P_k = (tau H)^k / k! is real.
  re.assign(size_t(n) * n, 0.0);
  im.assign(size_t(n) * n, 0.0);
  std::vector<double> p(size_t(n) * n, 0.0), q(size_t(n) * n, 0.0);
  for (int64_t i = 0; i < n; ++i) p[size_t(i) * n + i] = 1.0;
  for (int k = 1; k <= 60; ++k) {
    spmm(h, p, q, tau / double(k));
    p.swap(q);
    double mx = 0.0;
    for (double x : p) mx = std::max(mx, std::fabs(x));
    const double sign = (k % 4 == 1 || k % 4 == 2) ? -1.0 : 1.0;
    std::vector<double> &dst = (k % 2 == 1) ? im : re;
    for (size_t e = 0; e < p.size(); ++e) dst[e] += sign * p[e];
    if (mx < 1e-18 && double(k) > theta) break;
    if (k == 60) { err = "Taylor series did not converge"; return false; }
  }
  if (nsq) *nsq = squarings;
  if (levels) levels->clear();
  // squaring in increment form: (I + D)^2 - I = 2 D + D D
  for (int s = 0; s < squarings; ++s) {
    if (levels) {   // V_{squarings - s} - I, stored re plane then im plane
      std::vector<double> lv(re);
      lv.insert(lv.end(), im.begin(), im.end());
      levels->push_back(std::move(lv));
    }
    std::vector<double> cr, ci;
    zgemm_host(n, re, im, re, im, cr, ci);
    for (size_t e = 0; e < re.size(); ++e) {
      re[e] = 2.0 * re[e] + cr[e];
      im[e] = 2.0 * im[e] + ci[e];
    }
  }
  // U = exp(-i H dt) is symmetric for real symmetric H; remove the rounding
  // asymmetry so that the device products may read dU by rows or columns.
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = i + 1; j < n; ++j) {
      size_t a = size_t(i) * n + j, b = size_t(j) * n + i;
      double r = 0.5 * (re[a] + re[b]), x = 0.5 * (im[a] + im[b]);
      re[a] = re[b] = r;
      im[a] = im[b] = x;
    }
  }
  return true;
}

// ------------------------------------------------------------ Frechet

// y = (-i tau H) x for complex planar dense x (rows), H sparse real symmetric.
static void apply_left(const Csr &h, double tau, const std::vector<double> &xr,
                       const std::vector<double> &xi, std::vector<double> &yr,
                       std::vector<double> &yi) {
  // (-i tau) (H xr + i H xi) = tau H xi - i tau H xr
  spmm(h, xi, yr, tau);
  spmm(h, xr, yi, -tau);
}

// y = x (-i tau H) = (-i tau) (x H); with H symmetric, (x H)^T = H x^T.
static void apply_right(const Csr &h, double tau, const std::vector<double> &xr,
                        const std::vector<double> &xi, std::vector<double> &yr,
                        std::vector<double> &yi) {
  const int64_t n = h.n;
  std::vector<double> tr(size_t(n) * n), ti(size_t(n) * n), ur, ui;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      tr[size_t(j) * n + i] = xr[size_t(i) * n + j];
      ti[size_t(j) * n + i] = xi[size_t(i) * n + j];
    }
  ur.resize(tr.size());
  ui.resize(ti.size());
  apply_left(h, tau, tr, ti, ur, ui);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      yr[size_t(i) * n + j] = ur[size_t(j) * n + i];
      yi[size_t(i) * n + j] = ui[size_t(j) * n + i];
    }
}

// L(B, G) for B = -i tau H by its power series
//   L(B, G) = sum_{k>=1} (1/k!) sum_{j=0}^{k-1} B^j G B^{k-1-j},
// accumulated with M_1 = G, R_1 = G B, M_{k+1} = (B M_k + R_k) / (k+1),
// R_{k+1} = R_k B / (k+1); every product is sparse x dense.
static bool frechet_series(const Csr &h, double tau, const std::vector<double> &g_re,
                           const std::vector<double> &g_im, std::vector<double> &w_re,
                           std::vector<double> &w_im, std::string &err) {
  const size_t nn = g_re.size();
  std::vector<double> mr(g_re), mi(g_im), rr(nn), ri(nn), tr(nn), ti(nn);
  apply_right(h, tau, g_re, g_im, rr, ri);
  w_re = mr;
  w_im = mi;
  double gmax = 0.0;
  for (size_t e = 0; e < nn; ++e) gmax = std::max(gmax, std::fabs(g_re[e]) + std::fabs(g_im[e]));
  if (gmax == 0.0) return true;
  for (int k = 1; k < 80; ++k) {
    apply_left(h, tau, mr, mi, tr, ti);
    double mx = 0.0;
    for (size_t e = 0; e < nn; ++e) {
      mr[e] = (tr[e] + rr[e]) / double(k + 1);
      mi[e] = (ti[e] + ri[e]) / double(k + 1);
      w_re[e] += mr[e];
      w_im[e] += mi[e];
      mx = std::max(mx, std::fabs(mr[e]) + std::fabs(mi[e]));
    }
    if (mx < 1e-18 * gmax) return true;
    apply_right(h, tau, rr, ri, tr, ti);
    for (size_t e = 0; e < nn; ++e) {
      rr[e] = tr[e] / double(k + 1);
      ri[e] = ti[e] / double(k + 1);
    }
  }
  err = "Frechet series did not converge";
  return false;
}

bool frechet_adjoint(const Model &m, const Csr &h, const std::vector<double> &g_re,
                     const std::vector<double> &g_im, std::vector<double> &w_re,
                     std::vector<double> &w_im, std::string &err) {
  // Undo the squarings: L(2B, G) = L(B, G V + V G) / 2 with V = exp(B), so
  // L(A, G) = 2^{-s} L(A / 2^s, G_s),  G_i = G_{i-1} V_i + V_i G_{i-1},
  // V_i = exp(A / 2^i), i = 1..s.
  std::vector<double> re, im;
  std::vector<std::vector<double>> levels;
  int s = 0;
  if (!propagator_increment(m, h, re, im, err, &levels, &s)) return false;
  const int64_t n = m.n;
  const size_t nn = size_t(n) * n;
  std::vector<double> gr(g_re), gi(g_im);
  for (int i = 1; i <= s; ++i) {
    // levels[s - i] holds V_i - I (the squaring loop stores V_s first)
    const std::vector<double> &lv = levels[size_t(s - i)];
    std::vector<double> vr(lv.begin(), lv.begin() + nn), vi(lv.begin() + nn, lv.end());
    for (int64_t d = 0; d < n; ++d) vr[size_t(d) * n + d] += 1.0;
    std::vector<double> ar, ai, br, bi;
    zgemm_host(n, gr, gi, vr, vi, ar, ai);
    zgemm_host(n, vr, vi, gr, gi, br, bi);
    for (size_t e = 0; e < nn; ++e) {
      gr[e] = ar[e] + br[e];
      gi[e] = ai[e] + bi[e];
    }
  }
  const double tau = m.dt / std::ldexp(1.0, s);
  if (!frechet_series(h, tau, gr, gi, w_re, w_im, err)) return false;
  const double f = std::ldexp(1.0, -s);
  for (size_t e = 0; e < nn; ++e) {
    w_re[e] *= f;
    w_im[e] *= f;
  }
  return true;
}

}  // namespace qme
