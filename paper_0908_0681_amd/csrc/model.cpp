// Host side of libhyb: bit-encoded Fock basis, (n_up, n_dn) blocks, the
// Kanamori H_loc of Eq.(4) as per-block CSR, the block spectra and the
// retained set (initialisation steps 1-2 of Sec. III).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <thread>
#include <vector>

#include "hyb_internal.h"

namespace hyb {

static thread_local std::string g_err;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

namespace {

inline int popc(uint32_t x) { return __builtin_popcount(x); }

// Applies c_f (dagger = 0) or c_f^dag (dagger = 1) to basis state s.  Returns false
// if the result vanishes; otherwise sets t and multiplies sign by the Jordan-Wigner
// factor (-1)^{number of occupied flavors below f}.
inline bool apply_one(uint32_t s, int f, int dagger, uint32_t& t, int& sign) {
  const uint32_t bit = 1u << f;
  const bool occ = (s & bit) != 0;
  if (dagger ? occ : !occ) return false;
  if (popc(s & (bit - 1u)) & 1) sign = -sign;
  t = s ^ bit;
  return true;
}

// Applies the product O_1 O_2 O_3 O_4 (rightmost first) to s.
inline bool apply_four(uint32_t s, const int (&f)[4], const int (&dg)[4], uint32_t& t, int& sign) {
  sign = 1;
  uint32_t cur = s;
  for (int k = 3; k >= 0; --k) {
    uint32_t nxt;
    if (!apply_one(cur, f[k], dg[k], nxt, sign)) return false;
    cur = nxt;
  }
  t = cur;
  return true;
}

// Diagonal (density-density) part of Eq.(4) for state s.
double diag_energy(const hyb_model& m, uint32_t s) {
  const int n = m.n_orb;
  auto occ = [&](int a, int sg) -> int { return (s >> (a + n * sg)) & 1u; };
  double e = 0.0;
  for (int a = 0; a < n; ++a) {
    e += m.eps[a] * (occ(a, 0) + occ(a, 1));
    e += m.p.U * occ(a, 0) * occ(a, 1);
  }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < a; ++b) {
      e += m.p.Up * (occ(a, 0) * occ(b, 1) + occ(a, 1) * occ(b, 0));
      e += (m.p.Up - m.p.J) * (occ(a, 0) * occ(b, 0) + occ(a, 1) * occ(b, 1));
    }
  return e;
}

int build_basis(hyb_model& m) {
  const int n = m.n_orb;
  m.F = 2 * n;
  m.n_states = int64_t(1) << m.F;
  m.n_blocks = (n + 1) * (n + 1);
  std::vector<int32_t> dims(m.n_blocks, 0);
  m.block_of.assign(m.n_states, 0);
  m.rank.assign(m.n_states, 0);
  const uint32_t lowmask = (1u << n) - 1u;
  for (int64_t s = 0; s < m.n_states; ++s) {
    const int nu = popc(uint32_t(s) & lowmask), nd = popc(uint32_t(s) >> n);
    const int b = nd * (n + 1) + nu;
    m.block_of[s] = b;
    m.rank[s] = dims[b]++;  // ascending state integer inside the block
  }
  m.blocks.assign(m.n_blocks, BlockDev{});
  int32_t off = 0;
  m.max_dim = 0;
  for (int b = 0; b < m.n_blocks; ++b) {
    m.blocks[b].dim = dims[b];
    m.blocks[b].state_off = off;
    m.blocks[b].n_up = b % (n + 1);
    m.blocks[b].n_dn = b / (n + 1);
    off += dims[b];
    m.max_dim = std::max(m.max_dim, dims[b]);
  }
  m.states.assign(m.n_states, 0);
  for (int64_t s = 0; s < m.n_states; ++s)
    m.states[m.blocks[m.block_of[s]].state_off + m.rank[s]] = uint32_t(s);
  // one spin's patterns ranked among those of equal popcount; blocks list states by
  // ascending integer up | dn << n, so a state's index is rank(dn) * C(n, n_up) + rank(up)
  m.rank_half.assign(size_t(1) << n, 0);
  std::vector<int16_t> seen(n + 1, 0);
  for (uint32_t x = 0; x < (1u << n); ++x) m.rank_half[x] = seen[popc(x)]++;
  for (int b = 0; b < m.n_blocks; ++b) m.blocks[b].up_states = seen[m.blocks[b].n_up];
  return 0;
}

// H_loc of Eq.(4): diagonal density-density part plus, for every ordered orbital
// pair a != b taken once, spin-flip -J_sf c+_{a dn} c+_{b up} c_{b dn} c_{a up} and
// pair hopping -J_ph c+_{b up} c+_{b dn} c_{a up} c_{a dn}.  H is real symmetric,
// so the entries of packed row s are the coefficients of H|s>.
int build_hamiltonian(hyb_model& m) {
  const int n = m.n_orb;
  m.diag.assign(m.n_states, 0.0);
  m.rowptr.assign(m.n_states + 1, 0);
  m.col.clear();
  m.val.clear();
  std::map<int32_t, double> row;
  for (int b = 0; b < m.n_blocks; ++b) {
    const BlockDev& B = m.blocks[b];
    for (int i = 0; i < B.dim; ++i) {
      const int64_t g = B.state_off + i;
      const uint32_t s = m.states[g];
      m.diag[g] = diag_energy(m, s);
      row.clear();
      for (int a = 0; a < n; ++a)
        for (int c = 0; c < n; ++c) {
          if (a == c) continue;
          const int up_a = a, dn_a = a + n, up_c = c, dn_c = c + n;
          uint32_t t;
          int sg;
          if (m.p.J_sf != 0.0) {
            const int f[4] = {dn_a, up_c, dn_c, up_a};
            const int dg[4] = {1, 1, 0, 0};
            if (apply_four(s, f, dg, t, sg)) row[m.rank[t]] += -m.p.J_sf * sg;
          }
          if (m.p.J_ph != 0.0) {
            const int f[4] = {up_c, dn_c, up_a, dn_a};
            const int dg[4] = {1, 1, 0, 0};
            if (apply_four(s, f, dg, t, sg)) row[m.rank[t]] += -m.p.J_ph * sg;
          }
        }
      for (auto& kv : row) {
        if (kv.second == 0.0) continue;
        if (kv.first == i) {
          m.diag[g] += kv.second;  // never happens for Kanamori, kept for safety
          continue;
        }
        m.col.push_back(kv.first);
        m.val.push_back(kv.second);
      }
      m.rowptr[g + 1] = int32_t(m.col.size());
    }
  }
  return 0;
}

void block_dense(const hyb_model& m, int b, double* h) {
  const BlockDev& B = m.blocks[b];
  std::fill(h, h + size_t(B.dim) * B.dim, 0.0);
  for (int i = 0; i < B.dim; ++i) {
    const int64_t g = B.state_off + i;
    h[size_t(i) * B.dim + i] = m.diag[g];
    for (int k = m.rowptr[g]; k < m.rowptr[g + 1]; ++k) h[size_t(i) * B.dim + m.col[k]] += m.val[k];
  }
}

int build_spectrum(hyb_model& m) {
  const double w = m.p.retain_window;
  m.evals.assign(m.n_blocks, {});
  std::vector<std::vector<double>> vecs(m.n_blocks);
  std::vector<int> nvec(m.n_blocks, 0);
  std::atomic<int> next{0}, err{0};
  // largest blocks first for load balance
  std::vector<int> order(m.n_blocks);
  for (int b = 0; b < m.n_blocks; ++b) order[b] = b;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return m.blocks[x].dim > m.blocks[y].dim; });
  auto worker = [&]() {
    std::vector<double> h;
    for (;;) {
      const int j = next.fetch_add(1);
      if (j >= m.n_blocks) return;
      const int b = order[j];
      const int d = m.blocks[b].dim;
      if (d == 0) continue;
      h.resize(size_t(d) * d);
      block_dense(m, b, h.data());
      m.evals[b].resize(d);
      // eigenvectors of every level within the window of the block's own minimum;
      // the retained set is selected against the global E0 afterwards
      int rc = sym_eig(d, h.data(), m.evals[b].data(), 0, nullptr);
      if (rc) {
        err = rc;
        return;
      }
      int nv = d;
      if (w >= 0.0) {
        nv = 0;
        while (nv < d && m.evals[b][nv] - m.evals[b][0] <= w) ++nv;
      }
      nvec[b] = nv;
      vecs[b].resize(size_t(d) * nv);
      rc = sym_eig(d, h.data(), m.evals[b].data(), nv, vecs[b].data());
      if (rc) {
        err = rc;
        return;
      }
    }
  };
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) th.emplace_back(worker);
  for (auto& t : th) t.join();
  if (err) return set_error(err, "block eigensolver did not converge");
  m.E0 = INFINITY;
  for (int b = 0; b < m.n_blocks; ++b) {
    if (m.blocks[b].dim == 0) continue;
    m.E0 = std::min(m.E0, m.evals[b][0]);
    m.blocks[b].shift = m.evals[b][0];
  }
  m.ret_block.clear();
  m.ret_index.clear();
  m.ret_energy.clear();
  m.ret_off.clear();
  m.ret_vec.clear();
  for (int b = 0; b < m.n_blocks; ++b) {
    const int d = m.blocks[b].dim;
    for (int j = 0; j < nvec[b]; ++j) {
      if (w >= 0.0 && m.evals[b][j] - m.E0 > w) break;
      m.ret_block.push_back(b);
      m.ret_index.push_back(j);
      m.ret_energy.push_back(m.evals[b][j]);
      m.ret_off.push_back(int64_t(m.ret_vec.size()));
      for (int i = 0; i < d; ++i) m.ret_vec.push_back(vecs[b][size_t(i) * nvec[b] + j]);
    }
  }
  return 0;
}

}  // namespace
}  // namespace hyb

using namespace hyb;

extern "C" {

const char* hyb_last_error(void) { return g_err.c_str(); }
const char* hyb_version(void) { return "libhyb 0.1 gfx950"; }

int hyb_model_create(const hyb_model_params* p, hyb_model** out) {
  if (!p || !out) return set_error(HYB_E_ARG, "NULL argument");
  *out = nullptr;
  if (p->n_orb < 1 || p->n_orb > 7) return set_error(HYB_E_ARG, "n_orb must be in 1..7 (got %d)", p->n_orb);
  if (!p->eps) return set_error(HYB_E_ARG, "eps is NULL");
  if (p->storage != HYB_CSR && p->storage != HYB_MATRIX_FREE)
    return set_error(HYB_E_ARG, "unsupported storage %d", p->storage);
  if (p->precision != HYB_FP64 && p->precision != HYB_MIXED)
    return set_error(HYB_E_ARG, "unknown precision %d", p->precision);
  if (p->krylov_max < 2 || p->krylov_max > 20) return set_error(HYB_E_ARG, "krylov_max must be in 2..20");
  if (p->spectrum != HYB_SPECTRUM_HOST && p->spectrum != HYB_SPECTRUM_DEVICE)
    return set_error(HYB_E_ARG, "unknown spectrum mode %d", p->spectrum);
  if (!(p->krylov_tol > 0.0) || !(p->krylov_tol < 1.0)) return set_error(HYB_E_ARG, "krylov_tol must be in (0,1)");
  const double vals[] = {p->U, p->Up, p->J, p->J_sf, p->J_ph, p->retain_window};
  for (double v : vals)
    if (!std::isfinite(v)) return set_error(HYB_E_NONFINITE, "non-finite model parameter");
  for (int a = 0; a < p->n_orb; ++a)
    if (!std::isfinite(p->eps[a])) return set_error(HYB_E_NONFINITE, "non-finite eps[%d]", a);
  hyb_model* m = new (std::nothrow) hyb_model();
  if (!m) return set_error(HYB_E_OOM, "out of host memory");
  m->p = *p;
  m->eps.assign(p->eps, p->eps + p->n_orb);
  m->p.eps = m->eps.data();
  m->n_orb = p->n_orb;
  int rc = build_basis(*m);
  if (!rc) rc = build_hamiltonian(*m);
  if (!rc && p->spectrum == HYB_SPECTRUM_HOST) rc = build_spectrum(*m);
  if (!rc && p->spectrum == HYB_SPECTRUM_DEVICE) m->E0 = NAN;  // hyb_init_lanczos supplies it
  if (rc) {
    delete m;
    return rc;
  }
  *out = m;
  return HYB_OK;
}

void hyb_model_destroy(hyb_model* m) {
  if (!m) return;
  hyb::free_device(m);
  delete m;
}

int hyb_model_info(const hyb_model* m, hyb_model_info_t* o) {
  if (!m || !o) return set_error(HYB_E_ARG, "NULL argument");
  o->n_orb = m->n_orb;
  o->n_flavors = m->F;
  o->n_blocks = m->n_blocks;
  o->max_dim = m->max_dim;
  o->n_retained = int32_t(m->ret_block.size());
  o->precision = m->p.precision;
  o->n_states = m->n_states;
  o->nnz_offdiag = int64_t(m->col.size());
  o->E0 = m->E0;
  return HYB_OK;
}

int hyb_block_info(const hyb_model* m, int32_t b, int32_t* dim, int32_t* nnz, double* emin) {
  if (!m) return set_error(HYB_E_ARG, "NULL model");
  if (b < 0 || b >= m->n_blocks) return set_error(HYB_E_ARG, "block %d out of range", b);
  const BlockDev& B = m->blocks[b];
  if (dim) *dim = B.dim;
  if (nnz) *nnz = m->rowptr[B.state_off + B.dim] - m->rowptr[B.state_off];
  if (emin) {
    if (!B.dim)
      *emin = 0.0;
    else if (!m->evals.empty())
      *emin = m->evals[b][0];
    else  // device spectrum: the lowest Ritz value, once computed
      *emin = m->ret_block.empty() ? NAN : B.shift;
  }
  return HYB_OK;
}

int hyb_block_eigenvalues(const hyb_model* m, int32_t b, double* e) {
  if (!m || !e) return set_error(HYB_E_ARG, "NULL argument");
  if (b < 0 || b >= m->n_blocks) return set_error(HYB_E_ARG, "block %d out of range", b);
  if (m->evals.empty()) return set_error(HYB_E_STATE, "spectrum computed on the device: only retained levels are known");
  std::copy(m->evals[b].begin(), m->evals[b].end(), e);
  return HYB_OK;
}

int hyb_basis_state(const hyb_model* m, int32_t b, int32_t idx, uint32_t* bits) {
  if (!m || !bits) return set_error(HYB_E_ARG, "NULL argument");
  if (b < 0 || b >= m->n_blocks) return set_error(HYB_E_ARG, "block %d out of range", b);
  if (idx < 0 || idx >= m->blocks[b].dim) return set_error(HYB_E_ARG, "index %d out of range", idx);
  *bits = m->states[m->blocks[b].state_off + idx];
  return HYB_OK;
}

int hyb_basis_index(const hyb_model* m, uint32_t bits, int32_t* b, int32_t* idx) {
  if (!m || !b || !idx) return set_error(HYB_E_ARG, "NULL argument");
  if (int64_t(bits) >= m->n_states) return set_error(HYB_E_ARG, "state 0x%x out of range", bits);
  *b = m->block_of[bits];
  *idx = m->rank[bits];
  return HYB_OK;
}

int hyb_block_dense(const hyb_model* m, int32_t b, double* h) {
  if (!m || !h) return set_error(HYB_E_ARG, "NULL argument");
  if (b < 0 || b >= m->n_blocks) return set_error(HYB_E_ARG, "block %d out of range", b);
  block_dense(*m, b, h);
  return HYB_OK;
}

int hyb_retained(const hyb_model* m, int32_t* blk, double* energy, double* vec) {
  if (!m) return set_error(HYB_E_ARG, "NULL model");
  if (blk) std::copy(m->ret_block.begin(), m->ret_block.end(), blk);
  if (energy) std::copy(m->ret_energy.begin(), m->ret_energy.end(), energy);
  if (vec) std::copy(m->ret_vec.begin(), m->ret_vec.end(), vec);
  return HYB_OK;
}

int hyb_apply_op(const hyb_model* m, int32_t f, int32_t dagger, int32_t bin, const double* x,
                 int32_t* bout, double* y) {
  if (!m || !x || !bout || !y) return set_error(HYB_E_ARG, "NULL argument");
  if (f < 0 || f >= m->F || (dagger != 0 && dagger != 1)) return set_error(HYB_E_FLAVOR, "bad operator");
  if (bin < 0 || bin >= m->n_blocks) return set_error(HYB_E_ARG, "block %d out of range", bin);
  const BlockDev& B = m->blocks[bin];
  int nu = B.n_up, nd = B.n_dn;
  const int step = dagger ? 1 : -1;
  if (f < m->n_orb) nu += step; else nd += step;
  if (nu < 0 || nu > m->n_orb || nd < 0 || nd > m->n_orb) {
    *bout = -1;
    return HYB_OK;
  }
  const int bt = nd * (m->n_orb + 1) + nu;
  *bout = bt;
  const BlockDev& T = m->blocks[bt];
  std::fill(y, y + T.dim, 0.0);
  for (int i = 0; i < B.dim; ++i) {
    uint32_t t;
    int sg = 1;
    if (!apply_one(m->states[B.state_off + i], f, dagger, t, sg)) continue;
    y[m->rank[t]] = sg * x[i];
  }
  return HYB_OK;
}

}  // extern "C"
