// Initialisation on the device (Sec. III step 1): the lowest eigenstates of every
// (n_up, n_dn) block by band (block) Lanczos, which resolves a degenerate level up to
// the block size, and the retained set of step 2 from them (an energy window above the
// ground state, Sec. IV.C).
//
// Per block of dimension d, block size p, T the projection of H_b on Q = [Q_1 Q_2 ...]:
//   Q_1   = p orthonormal pseudo-random vectors;
//   W     = H_b Q_j   (FP64 SpMM over the block's ELL rows and its diagonal);
//   A_j   = Q_j^T W;  W -= Q_j A_j + Q_{j-1} B_{j-1}^T;
//   Q_{j+1} from the columns of W by Gram-Schmidt against every earlier vector, two
//           passes per column (full reorthogonalisation); a column that keeps no new
//           direction (norm below 1e-14 ||H_b||) is dropped, and a block left short is
//           filled with pseudo-random vectors orthogonalised the same way;
//   B_j   = Q_{j+1}^T W  (so that H_b Q_j = Q_{j-1} B_{j-1}^T + Q_j A_j + Q_{j+1} B_j).
// Fill vectors keep T block tridiagonal: W lies in span(Q_{j+1}) whichever vectors
// complete it.  The Ritz pairs (theta_i, Q s_i) of T have residual
// ||H_b x_i - theta_i x_i|| = ||B_j s_i[last block]||.
//
// Two phases: every block first runs until its lowest Ritz value has converged, which
// gives E0 = min over blocks; blocks whose lowest value lies within the window of E0
// then continue until every Ritz value up to E0 + window and the first one above it
// have converged (or Q spans the block).  The Ritz vectors up to E0 + window form the
// retained set.  In exact arithmetic block Lanczos holds at most p copies of a
// degenerate level, so a wanted level found p times (without Q spanning the block)
// is an error: the block size must exceed every wanted multiplicity.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "hyb_internal.h"

namespace hyb {

// Y = H_b X for w column-major vectors of length d: the diagonal plus the ELL slots
// (slot q of row r at q d + r; padding has value 0 and the row's own index).
__global__ void k_lz_spmm(int d, int w, int ek, const int32_t* __restrict__ ecol, const double* __restrict__ eval,
                          const double* __restrict__ diag, const double* __restrict__ X, double* __restrict__ Y) {
  const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= int64_t(d) * w) return;
  const int v = int(id / d), r = int(id - int64_t(v) * d);
  const double* x = X + int64_t(v) * d;
  double acc = diag[r] * x[r];
  for (int q = 0; q < ek; ++q) {
    const int64_t at = int64_t(q) * d + r;
    acc += eval[at] * x[ecol[at]];
  }
  Y[id] = acc;
}

namespace {

// Pseudo-random numbers in [-1, 1) (splitmix64).
double prand(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return double(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

struct Lz {
  // problem
  int b = 0, d = 0, p = 0, ek = 0;
  double hnorm = 0.0;  // Gershgorin bound on ||H_b||
  uint64_t seed = 0;
  // device
  int32_t* ecol = nullptr;
  double *eval = nullptr, *diag = nullptr;
  double* Q = nullptr;  // d x cap, column-major
  int cap = 0;
  double *W = nullptr, *W0 = nullptr, *h = nullptr, *S = nullptr;
  // recurrence
  std::vector<int> off, wid;               // offset and width of Q_1, Q_2, ...
  std::vector<std::vector<double>> A, Bm;  // A_j (w_j x w_j), B_j (w_{j+1} x w_j), row-major
  int n = 0;                               // columns of Q inside T
  int nq = 0;                              // columns of Q written
  // the last Ritz step
  std::vector<double> theta, Sv;           // Ritz values; eigenvectors of T, row-major n x n
  std::vector<double> res;                 // residual of each Ritz pair
  bool spans = false;
  int steps = 0;

  ~Lz() {
    for (void* q : {(void*)ecol, (void*)eval, (void*)diag, (void*)Q, (void*)W, (void*)W0, (void*)h, (void*)S})
      if (q) (void)hipFree(q);
  }
};

struct Ctx {
  hyb_model* m;
  rocblas_handle h;
  hipStream_t s;
};

#define LZ_HIP(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return set_error(HYB_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)
#define LZ_BLAS(expr)                                                                                    \
  do {                                                                                                   \
    if ((expr) != rocblas_status_success) return set_error(HYB_E_HIP, "rocBLAS call failed: %s", #expr); \
  } while (0)

const double kOne = 1.0, kZero = 0.0, kMinusOne = -1.0;

int grow_q(Ctx& c, Lz& z, int need) {
  if (need <= z.cap) return 0;
  const int cap = std::min(z.d, std::max(need, std::max(2 * z.cap, 8 * z.p)));
  double* q = nullptr;
  LZ_HIP(hipMalloc(&q, sizeof(double) * size_t(z.d) * cap));
  if (z.Q) {
    LZ_HIP(hipMemcpyAsync(q, z.Q, sizeof(double) * size_t(z.d) * z.nq, hipMemcpyDeviceToDevice, c.s));
    LZ_HIP(hipStreamSynchronize(c.s));
    (void)hipFree(z.Q);
  }
  z.Q = q;
  z.cap = cap;
  return 0;
}

// v (device, length d) against Q[:, 0:k], two passes; returns ||v|| afterwards.
double orth(Ctx& c, Lz& z, double* v, int k, int& rc) {
  for (int pass = 0; pass < 2 && k > 0 && !rc; ++pass) {
    if (rocblas_dgemv(c.h, rocblas_operation_transpose, z.d, k, &kOne, z.Q, z.d, v, 1, &kZero, z.h, 1) !=
            rocblas_status_success ||
        rocblas_dgemv(c.h, rocblas_operation_none, z.d, k, &kMinusOne, z.Q, z.d, z.h, 1, &kOne, v, 1) !=
            rocblas_status_success)
      rc = set_error(HYB_E_HIP, "rocblas_dgemv (reorthogonalisation)");
  }
  double r = 0.0;
  if (!rc && rocblas_dnrm2(c.h, z.d, v, 1, &r) != rocblas_status_success) rc = set_error(HYB_E_HIP, "rocblas_dnrm2");
  return r;
}

// Q[:, at] = a pseudo-random unit vector orthogonal to Q[:, 0:at].
int fill(Ctx& c, Lz& z, int at) {
  std::vector<double> r(z.d);
  for (int tries = 0; tries < 4; ++tries) {
    for (double& x : r) x = prand(z.seed);
    double* v = z.Q + size_t(at) * z.d;
    LZ_HIP(hipMemcpyAsync(v, r.data(), sizeof(double) * z.d, hipMemcpyHostToDevice, c.s));
    int rc = 0;
    const double nv = orth(c, z, v, at, rc);  // dnrm2 returns to the host: r may be reused
    if (rc) return rc;
    if (nv > 1e-8) {
      const double inv = 1.0 / nv;
      LZ_BLAS(rocblas_dscal(c.h, z.d, &inv, v, 1));
      return 0;
    }
  }
  return set_error(HYB_E_NOCONV, "band Lanczos: no direction left to fill block %d", z.b);
}

// Columns 0..wc-1 of src -> orthonormal Q[:, n0 : n0 + w] with w = min(p, d - n0): the
// columns that keep a new direction first, fill vectors after them.
int extend(Ctx& c, Lz& z, const double* src, int wc, int n0, int& w_out) {
  const int w = std::min(z.p, z.d - n0);
  int rc = grow_q(c, z, n0 + w);
  if (rc) return rc;
  int k = 0;
  for (int col = 0; col < wc && k < w; ++col) {
    double* v = z.Q + size_t(n0 + k) * z.d;
    LZ_HIP(hipMemcpyAsync(v, src + size_t(col) * z.d, sizeof(double) * z.d, hipMemcpyDeviceToDevice, c.s));
    const double nv = orth(c, z, v, n0 + k, rc);
    if (rc) return rc;
    if (nv > 1e-14 * z.hnorm) {
      const double inv = 1.0 / nv;
      LZ_BLAS(rocblas_dscal(c.h, z.d, &inv, v, 1));
      ++k;
    }
  }
  for (; k < w; ++k)
    if ((rc = fill(c, z, n0 + k))) return rc;
  w_out = w;
  z.nq = n0 + w;
  return 0;
}

int setup(Ctx& c, Lz& z, int b, int p) {
  const hyb_model* m = c.m;
  const BlockDev& B = m->blocks[b];
  z.b = b;
  z.d = B.dim;
  z.p = std::min(p, B.dim);
  z.seed = 0x243F6A8885A308D3ull ^ (uint64_t(b + 1) * 0x9E3779B97F4A7C15ull);
  // the block's rows as ELL (natural order), its diagonal and a Gershgorin bound
  int ek = 0;
  double hn = 0.0;
  for (int r = 0; r < z.d; ++r) {
    const int g = B.state_off + r;
    ek = std::max(ek, m->rowptr[g + 1] - m->rowptr[g]);
    double row = std::fabs(m->diag[g]);
    for (int q = m->rowptr[g]; q < m->rowptr[g + 1]; ++q) row += std::fabs(m->val[q]);
    hn = std::max(hn, row);
  }
  z.ek = ek;
  z.hnorm = std::max(hn, 1e-300);
  std::vector<int32_t> col(std::max<size_t>(size_t(ek) * z.d, 1), 0);
  std::vector<double> val(std::max<size_t>(size_t(ek) * z.d, 1), 0.0);
  for (int r = 0; r < z.d; ++r) {
    const int g = B.state_off + r, len = m->rowptr[g + 1] - m->rowptr[g];
    for (int q = 0; q < ek; ++q) {
      col[size_t(q) * z.d + r] = q < len ? m->col[m->rowptr[g] + q] : r;
      val[size_t(q) * z.d + r] = q < len ? m->val[m->rowptr[g] + q] : 0.0;
    }
  }
  LZ_HIP(hipMalloc(&z.ecol, sizeof(int32_t) * col.size()));
  LZ_HIP(hipMalloc(&z.eval, sizeof(double) * val.size()));
  LZ_HIP(hipMalloc(&z.diag, sizeof(double) * z.d));
  LZ_HIP(hipMalloc(&z.W, sizeof(double) * size_t(z.d) * z.p));
  LZ_HIP(hipMalloc(&z.W0, sizeof(double) * size_t(z.d) * z.p));
  LZ_HIP(hipMalloc(&z.h, sizeof(double) * size_t(z.d)));
  LZ_HIP(hipMalloc(&z.S, sizeof(double) * size_t(z.p) * z.p));
  LZ_HIP(hipMemcpyAsync(z.ecol, col.data(), sizeof(int32_t) * col.size(), hipMemcpyHostToDevice, c.s));
  LZ_HIP(hipMemcpyAsync(z.eval, val.data(), sizeof(double) * val.size(), hipMemcpyHostToDevice, c.s));
  LZ_HIP(hipMemcpyAsync(z.diag, m->diag.data() + B.state_off, sizeof(double) * z.d, hipMemcpyHostToDevice, c.s));
  // Q_1: p pseudo-random vectors, orthonormalised
  std::vector<double> r0(size_t(z.d) * z.p);
  for (double& x : r0) x = prand(z.seed);
  LZ_HIP(hipMemcpyAsync(z.W, r0.data(), sizeof(double) * r0.size(), hipMemcpyHostToDevice, c.s));
  int w = 0;
  const int rc = extend(c, z, z.W, z.p, 0, w);
  if (rc) return rc;
  z.off.assign(1, 0);
  z.wid.assign(1, w);
  z.n = 0;
  LZ_HIP(hipStreamSynchronize(c.s));  // the pageable staging vectors go out of scope
  return 0;
}

// One block step on the newest block of Q: A_j, B_j and Q_{j+1}; T grows by A_j.
int step(Ctx& c, Lz& z) {
  const int j = int(z.off.size()) - 1;
  const int o = z.off[j], w = z.wid[j];
  const int64_t nt = int64_t(z.d) * w;
  k_lz_spmm<<<unsigned((nt + 255) / 256), 256, 0, c.s>>>(z.d, w, z.ek, z.ecol, z.eval, z.diag, z.Q + size_t(o) * z.d,
                                                        z.W);
  LZ_HIP(hipGetLastError());
  // A_j = Q_j^T W, symmetrised on the host
  LZ_BLAS(rocblas_dgemm(c.h, rocblas_operation_transpose, rocblas_operation_none, w, w, z.d, &kOne,
                        z.Q + size_t(o) * z.d, z.d, z.W, z.d, &kZero, z.S, w));
  std::vector<double> Ac(size_t(w) * w);
  LZ_HIP(hipMemcpyAsync(Ac.data(), z.S, sizeof(double) * Ac.size(), hipMemcpyDeviceToHost, c.s));
  LZ_HIP(hipStreamSynchronize(c.s));
  std::vector<double> A(size_t(w) * w);
  for (int a = 0; a < w; ++a)
    for (int e = 0; e < w; ++e) A[size_t(a) * w + e] = 0.5 * (Ac[size_t(e) * w + a] + Ac[size_t(a) * w + e]);
  // W -= Q_j A_j + Q_{j-1} B_{j-1}^T (the Gram-Schmidt in extend removes what rounding
  // leaves of both)
  LZ_BLAS(rocblas_dgemm(c.h, rocblas_operation_none, rocblas_operation_none, z.d, w, w, &kMinusOne,
                        z.Q + size_t(o) * z.d, z.d, z.S, w, &kOne, z.W, z.d));
  if (j > 0) {
    const int wp = z.wid[j - 1];
    // B_{j-1} is w x wp row-major, which is B_{j-1}^T column-major (wp x w)
    LZ_HIP(hipMemcpyAsync(z.S, z.Bm[j - 1].data(), sizeof(double) * size_t(w) * wp, hipMemcpyHostToDevice, c.s));
    LZ_BLAS(rocblas_dgemm(c.h, rocblas_operation_none, rocblas_operation_none, z.d, w, wp, &kMinusOne,
                          z.Q + size_t(z.off[j - 1]) * z.d, z.d, z.S, wp, &kOne, z.W, z.d));
  }
  LZ_HIP(hipMemcpyAsync(z.W0, z.W, sizeof(double) * size_t(z.d) * w, hipMemcpyDeviceToDevice, c.s));
  z.A.push_back(A);
  z.n = o + w;
  z.steps = j + 1;
  z.spans = z.n >= z.d;
  if (z.spans) {
    LZ_HIP(hipStreamSynchronize(c.s));
    z.Bm.push_back({});
    return 0;
  }
  int wn = 0;
  int rc = extend(c, z, z.W0, w, z.n, wn);
  if (rc) return rc;
  // B_j = Q_{j+1}^T W  (wn x w)
  LZ_BLAS(rocblas_dgemm(c.h, rocblas_operation_transpose, rocblas_operation_none, wn, w, z.d, &kOne,
                        z.Q + size_t(z.n) * z.d, z.d, z.W0, z.d, &kZero, z.S, wn));
  std::vector<double> Bc(size_t(wn) * w), Br(size_t(wn) * w);
  LZ_HIP(hipMemcpyAsync(Bc.data(), z.S, sizeof(double) * Bc.size(), hipMemcpyDeviceToHost, c.s));
  LZ_HIP(hipStreamSynchronize(c.s));
  for (int a = 0; a < wn; ++a)
    for (int e = 0; e < w; ++e) Br[size_t(a) * w + e] = Bc[size_t(e) * wn + a];
  z.Bm.push_back(Br);
  z.off.push_back(z.n);
  z.wid.push_back(wn);
  return 0;
}

// Ritz values of T_n, its eigenvectors and the residual of each pair.
int ritz(Lz& z) {
  const int n = z.n;
  std::vector<double> T(size_t(n) * n, 0.0);
  for (size_t j = 0; j < z.A.size(); ++j) {
    const int o = z.off[j], w = z.wid[j];
    for (int a = 0; a < w; ++a)
      for (int e = 0; e < w; ++e) T[size_t(o + a) * n + o + e] = z.A[j][size_t(a) * w + e];
    if (j + 1 < z.A.size()) {
      const int o2 = z.off[j + 1], w2 = z.wid[j + 1];
      for (int a = 0; a < w2; ++a)
        for (int e = 0; e < w; ++e) {
          T[size_t(o2 + a) * n + o + e] = z.Bm[j][size_t(a) * w + e];
          T[size_t(o + e) * n + o2 + a] = z.Bm[j][size_t(a) * w + e];
        }
    }
  }
  z.theta.assign(n, 0.0);
  z.Sv.assign(size_t(n) * n, 0.0);
  const int rc = sym_eig(n, T.data(), z.theta.data(), n, z.Sv.data());
  if (rc) return set_error(rc, "band Lanczos: eigensolver of T did not converge");
  z.res.assign(n, 0.0);
  if (z.spans) return 0;
  const int jl = int(z.A.size()) - 1;
  const int o = z.off[jl], w = z.wid[jl];
  const std::vector<double>& B = z.Bm[jl];
  const int wn = int(B.size()) / w;
  for (int i = 0; i < n; ++i) {
    double r2 = 0.0;
    for (int a = 0; a < wn; ++a) {
      double t = 0.0;
      for (int e = 0; e < w; ++e) t += B[size_t(a) * w + e] * z.Sv[size_t(o + e) * n + i];
      r2 += t * t;
    }
    z.res[i] = std::sqrt(r2);
  }
  return 0;
}

// Block steps until the Ritz values up to `upto` and the first one above it have
// residuals <= tol ||H_b|| (lowest_only: theta_0 alone), or Q spans the block.
int run(Ctx& c, Lz& z, bool lowest_only, double upto, double tol) {
  for (;;) {
    int rc = 0;
    if (z.A.size() < z.off.size() && (rc = step(c, z))) return rc;  // a block of Q not yet in T
    if ((rc = ritz(z))) return rc;
    if (z.spans) return 0;
    const double lim = tol * z.hnorm;
    bool conv = true;
    if (lowest_only) {
      conv = z.res[0] <= lim;
    } else {
      int k = 0;
      while (k < z.n && z.theta[k] <= upto) ++k;
      if (k >= z.n) conv = false;  // nothing seen above the window yet
      for (int i = 0; i <= std::min(k, z.n - 1); ++i) conv = conv && z.res[i] <= lim;
    }
    if (conv) return 0;
  }
}

}  // namespace
}  // namespace hyb

using namespace hyb;

extern "C" {

int hyb_init_lanczos(hyb_model* m, int32_t block_size, double tol, int32_t* steps, double* resid, void* stream) {
  if (!m) return set_error(HYB_E_ARG, "NULL model");
  if (!m->uploaded) return set_error(HYB_E_STATE, "model not uploaded to a device");
  const double window = m->p.retain_window;
  if (!(window >= 0.0)) return set_error(HYB_E_ARG, "the device initialisation needs retain_window >= 0");
  if (block_size < 2 || block_size > 64) return set_error(HYB_E_ARG, "block size must be in 2..64");
  if (!(tol >= 1e-15 && tol <= 1e-4)) return set_error(HYB_E_ARG, "tol must be in [1e-15, 1e-4]");
  int dev = -1;
  LZ_HIP(hipGetDevice(&dev));
  if (dev != m->dev.device) return set_error(HYB_E_STATE, "model lives on device %d, current is %d", m->dev.device, dev);
  Ctx c{m, nullptr, reinterpret_cast<hipStream_t>(stream)};
  if (rocblas_create_handle(&c.h) != rocblas_status_success) return set_error(HYB_E_HIP, "rocblas_create_handle");
  std::unique_ptr<_rocblas_handle, rocblas_status (*)(rocblas_handle)> guard(c.h, rocblas_destroy_handle);
  LZ_BLAS(rocblas_set_stream(c.h, c.s));
  std::vector<std::unique_ptr<Lz>> z(m->n_blocks);
  int rc = 0;
  // phase 1: the lowest level of every block
  double E0 = INFINITY;
  std::vector<double> lowest(m->n_blocks, 0.0);
  for (int b = 0; b < m->n_blocks; ++b) {
    if (m->blocks[b].dim == 0) continue;
    z[b].reset(new Lz());
    if ((rc = setup(c, *z[b], b, block_size))) return rc;
    if ((rc = run(c, *z[b], true, 0.0, tol))) return rc;
    lowest[b] = z[b]->theta[0];
    E0 = std::min(E0, lowest[b]);
  }
  // phase 2: every level within the window of E0
  const double upto = E0 + window;
  std::vector<int32_t> rb, ri;
  std::vector<double> re, rv;
  std::vector<int64_t> ro;
  for (int b = 0; b < m->n_blocks; ++b) {
    if (!z[b] || z[b]->theta[0] > upto) continue;
    Lz& L = *z[b];
    if ((rc = run(c, L, false, upto, tol))) return rc;
    int k = 0;
    while (k < L.n && L.theta[k] <= upto) ++k;
    // a wanted level found p times may have more copies than the block Krylov space holds
    if (!L.spans)
      for (int i = 0; i < k;) {
        int e = i;
        while (e + 1 < L.n && L.theta[e + 1] - L.theta[i] <= 1e-9 * L.hnorm) ++e;
        if (e - i + 1 >= L.p)
          return set_error(HYB_E_ARG,
                           "block %d: a retained level appears %d times; the band Lanczos block size (%d) must "
                           "exceed its multiplicity",
                           b, e - i + 1, L.p);
        i = e + 1;
      }
    if (k == 0) continue;
    // Ritz vectors X = Q[:, 0:n] S[:, 0:k]
    const int n = L.n;
    std::vector<double> Sc(size_t(n) * k);
    for (int i = 0; i < k; ++i)
      for (int a = 0; a < n; ++a) Sc[size_t(i) * n + a] = L.Sv[size_t(a) * n + i];
    double *dS = nullptr, *dX = nullptr;
    LZ_HIP(hipMalloc(&dS, sizeof(double) * Sc.size()));
    if (hipMalloc(&dX, sizeof(double) * size_t(L.d) * k) != hipSuccess) {
      (void)hipFree(dS);
      return set_error(HYB_E_OOM, "Ritz vectors of block %d", b);
    }
    std::vector<double> X(size_t(L.d) * k);
    const bool ok =
        hipMemcpyAsync(dS, Sc.data(), sizeof(double) * Sc.size(), hipMemcpyHostToDevice, c.s) == hipSuccess &&
        rocblas_dgemm(c.h, rocblas_operation_none, rocblas_operation_none, L.d, k, n, &kOne, L.Q, L.d, dS, n, &kZero,
                      dX, L.d) == rocblas_status_success &&
        hipMemcpyAsync(X.data(), dX, sizeof(double) * X.size(), hipMemcpyDeviceToHost, c.s) == hipSuccess &&
        hipStreamSynchronize(c.s) == hipSuccess;
    (void)hipFree(dS);
    (void)hipFree(dX);
    if (!ok) return set_error(HYB_E_HIP, "Ritz vectors of block %d", b);
    for (int i = 0; i < k; ++i) {
      double nrm = 0.0;
      for (int r = 0; r < L.d; ++r) nrm += X[size_t(i) * L.d + r] * X[size_t(i) * L.d + r];
      nrm = 1.0 / std::sqrt(nrm);
      rb.push_back(b);
      ri.push_back(i);
      re.push_back(L.theta[i]);
      ro.push_back(int64_t(rv.size()));
      for (int r = 0; r < L.d; ++r) rv.push_back(X[size_t(i) * L.d + r] * nrm);
    }
  }
  for (int b = 0; b < m->n_blocks; ++b) {
    if (steps) steps[b] = z[b] ? z[b]->steps : 0;
    if (resid) {
      double worst = 0.0;
      if (z[b])
        for (int i = 0; i < z[b]->n && (i == 0 || z[b]->theta[i] <= upto); ++i) worst = std::max(worst, z[b]->res[i]);
      resid[b] = worst;
    }
  }
  z.clear();
  // install E0, each block's lowest Ritz value as its shift c_b and the retained set;
  // hyb_model_upload then writes the device copies (shifted diagonal, retained vectors)
  m->E0 = E0;
  for (int b = 0; b < m->n_blocks; ++b)
    if (m->blocks[b].dim > 0) m->blocks[b].shift = lowest[b];
  m->ret_block = rb;
  m->ret_index = ri;
  m->ret_energy = re;
  m->ret_off = ro;
  m->ret_vec = rv;
  return hyb_model_upload(m, stream);
}

}  // extern "C"
