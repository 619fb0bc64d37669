// Dense symmetric eigensolver for the (n_up, n_dn) blocks of H_loc (host, float64).
//
// Initialisation step 1 of the Krylov method (Sec. III) asks for the low
// spectrum and eigenvectors of H_loc; the paper allows full diagonalisation.
// This file does it per block with textbook dense linear algebra:
//   1. Householder reduction to tridiagonal form  A = Q T Q^T,
//   2. implicit symmetric QR sweeps with the Wilkinson shift on T (eigenvalues;
//      for small blocks also the accumulated eigenvectors),
//   3. for larger blocks, eigenvectors of the requested eigenvalues by inverse
//      iteration on T (tridiagonal LU with partial pivoting), orthogonalised
//      inside clusters of close eigenvalues, then mapped back with Q.
// References: Golub & Van Loan, Matrix Computations, Alg. 8.3.1 (tridiagonal
// reduction) and 8.3.2 (implicit symmetric QR step); inverse iteration as in
// Sec. 8.2.2 there.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

#include "hyb_internal.h"

namespace hyb {
namespace {

// Householder tridiagonalisation of the symmetric row-major matrix a (n x n, overwritten).
// On return diag[n], off[n-1] hold T; reflector k (acting on indices k+1..n-1) is
// stored as v = hv[k*n + (k+1..n-1)] with v[k+1] = 1 and coefficient hb[k].
void householder_tridiag(int n, std::vector<double>& a, std::vector<double>& diag,
                         std::vector<double>& off, std::vector<double>& hv,
                         std::vector<double>& hb) {
  diag.assign(n, 0.0);
  off.assign(std::max(n - 1, 0), 0.0);
  hv.assign(static_cast<size_t>(n) * n, 0.0);
  hb.assign(n, 0.0);
  std::vector<double> v(n), p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    // x = a[k+1:, k]
    const int m = n - k - 1;
    double x0 = a[static_cast<size_t>(k + 1) * n + k];
    double sigma = 0.0;
    for (int i = 1; i < m; ++i) {
      double xi = a[static_cast<size_t>(k + 1 + i) * n + k];
      sigma += xi * xi;
    }
    double beta = 0.0, mu = std::fabs(x0);
    v[0] = 1.0;
    if (sigma == 0.0) {
      // already tridiagonal in this column
      for (int i = 1; i < m; ++i) v[i] = 0.0;
      mu = x0;
    } else {
      mu = std::sqrt(x0 * x0 + sigma);
      double v0 = (x0 <= 0.0) ? (x0 - mu) : (-sigma / (x0 + mu));
      beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
      for (int i = 1; i < m; ++i) v[i] = a[static_cast<size_t>(k + 1 + i) * n + k] / v0;
      // P x = mu e_1 with this choice of v0
    }
    hb[k] = beta;
    for (int i = 0; i < m; ++i) hv[static_cast<size_t>(k) * n + k + 1 + i] = v[i];
    // column/row k of the reduced matrix
    a[static_cast<size_t>(k + 1) * n + k] = mu;
    a[static_cast<size_t>(k) * n + k + 1] = mu;
    for (int i = 1; i < m; ++i) {
      a[static_cast<size_t>(k + 1 + i) * n + k] = 0.0;
      a[static_cast<size_t>(k) * n + k + 1 + i] = 0.0;
    }
    if (beta == 0.0) continue;
    // p = beta * A22 v ; w = p - (beta/2)(p.v) v ; A22 -= v w^T + w v^T
    for (int i = 0; i < m; ++i) {
      const double* row = &a[static_cast<size_t>(k + 1 + i) * n + k + 1];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = beta * s;
    }
    double pv = 0.0;
    for (int i = 0; i < m; ++i) pv += p[i] * v[i];
    const double c = 0.5 * beta * pv;
    for (int i = 0; i < m; ++i) w[i] = p[i] - c * v[i];
    for (int i = 0; i < m; ++i) {
      double* row = &a[static_cast<size_t>(k + 1 + i) * n + k + 1];
      const double vi = v[i], wi = w[i];
      for (int j = 0; j < m; ++j) row[j] -= vi * w[j] + wi * v[j];
    }
  }
  for (int i = 0; i < n; ++i) diag[i] = a[static_cast<size_t>(i) * n + i];
  for (int i = 0; i + 1 < n; ++i) off[i] = a[static_cast<size_t>(i + 1) * n + i];
}

// Implicit symmetric QR with Wilkinson shift on the tridiagonal (d, e).  If z is
// non-null it is an n x n row-major matrix that receives the accumulated rotations
// (z <- z G^T), so that starting from the identity its columns are eigenvectors of T.
int tridiag_qr(int n, std::vector<double>& d, std::vector<double>& e, double* z) {
  const double eps = 2.220446049250313e-16;
  int q = n - 1;
  long guard = 60L * n + 100;
  while (q > 0) {
    if (--guard < 0) return HYB_E_NOCONV;
    for (int i = 0; i < q; ++i)
      if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
    if (e[q - 1] == 0.0) {
      --q;
      continue;
    }
    int p = q - 1;
    while (p > 0 && e[p - 1] != 0.0) --p;
    // Wilkinson shift from the trailing 2x2 of T[p..q]
    const double dd = 0.5 * (d[q - 1] - d[q]);
    const double bq = e[q - 1];
    const double den = dd + (dd >= 0.0 ? 1.0 : -1.0) * std::hypot(dd, bq);
    const double mu = d[q] - bq * bq / den;
    double x = d[p] - mu, zz = e[p];
    for (int k = p; k < q; ++k) {
      double r = std::hypot(x, zz);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = x / r;
        s = zz / r;
      }
      if (k > p) e[k - 1] = r;
      const double ak = d[k], ak1 = d[k + 1], bk = e[k];
      d[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
      d[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
      e[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
      double bulge = 0.0;
      if (k + 1 < q) {
        bulge = s * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      if (z) {
        for (int row = 0; row < n; ++row) {
          double* zr = z + static_cast<size_t>(row) * n;
          const double zk = zr[k], zk1 = zr[k + 1];
          zr[k] = c * zk + s * zk1;
          zr[k + 1] = -s * zk + c * zk1;
        }
      }
      x = e[k];
      zz = bulge;
    }
  }
  return 0;
}

// Solves (T - sigma I) x = b for the tridiagonal T (d, e) by Gaussian elimination with
// partial pivoting; b is overwritten by x.  Zero pivots are replaced by a tiny value
// (standard for inverse iteration, where sigma is an eigenvalue).
void tridiag_solve_shifted(int n, const std::vector<double>& d, const std::vector<double>& e,
                           double sigma, double tiny, std::vector<double>& b) {
  // U has up to two super-diagonals after pivoting
  std::vector<double> u0(n), u1(n, 0.0), u2(n, 0.0);
  std::vector<double> l(n, 0.0);
  std::vector<char> swapped(n, 0);
  double cur_diag = d[0] - sigma;
  double cur_sup = (n > 1) ? e[0] : 0.0;
  double cur_sup2 = 0.0;
  for (int i = 0; i < n - 1; ++i) {
    const double sub = e[i];
    const double nd = d[i + 1] - sigma;
    const double ns = (i + 2 < n) ? e[i + 1] : 0.0;
    if (std::fabs(cur_diag) >= std::fabs(sub)) {
      double piv = (cur_diag == 0.0) ? tiny : cur_diag;
      const double m = sub / piv;
      l[i] = m;
      u0[i] = piv;
      u1[i] = cur_sup;
      u2[i] = cur_sup2;
      cur_diag = nd - m * cur_sup;
      cur_sup = ns - m * cur_sup2;
      cur_sup2 = 0.0;
    } else {
      // swap rows i and i+1
      swapped[i] = 1;
      const double m = cur_diag / sub;
      l[i] = m;
      u0[i] = sub;
      u1[i] = nd;
      u2[i] = ns;
      const double new_diag = cur_sup - m * nd;
      const double new_sup = cur_sup2 - m * ns;
      cur_diag = new_diag;
      cur_sup = new_sup;
      cur_sup2 = 0.0;
    }
  }
  u0[n - 1] = (cur_diag == 0.0) ? tiny : cur_diag;
  // forward: apply the row operations to b
  for (int i = 0; i < n - 1; ++i) {
    if (swapped[i]) std::swap(b[i], b[i + 1]);
    b[i + 1] -= l[i] * b[i];
  }
  // backward
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    if (i + 1 < n) s -= u1[i] * b[i + 1];
    if (i + 2 < n) s -= u2[i] * b[i + 2];
    b[i] = s / u0[i];
  }
}

inline uint64_t lcg_next(uint64_t& s) {
  s = s * 6364136223846793005ULL + 1442695040888963407ULL;
  return s;
}

}  // namespace

int sym_eig(int n, const double* a_in, double* evals, int n_vec, double* vec) {
  if (n <= 0) return 0;
  if (n == 1) {
    evals[0] = a_in[0];
    if (n_vec > 0) vec[0] = 1.0;
    return 0;
  }
  std::vector<double> a(a_in, a_in + static_cast<size_t>(n) * n);
  std::vector<double> d, e, hv, hb;
  householder_tridiag(n, a, d, e, hv, hb);
  double tnorm = 0.0;
  for (int i = 0; i < n; ++i) {
    double r = std::fabs(d[i]) + (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    tnorm = std::max(tnorm, r);
  }
  const bool full_accumulate = (n_vec > 0) && (n <= 256 || n_vec * 4 > n);
  std::vector<double> z;
  std::vector<double> d0 = d, e0 = e;
  if (full_accumulate) {
    z.assign(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i < n; ++i) z[static_cast<size_t>(i) * n + i] = 1.0;
  }
  int rc = tridiag_qr(n, d, e, full_accumulate ? z.data() : nullptr);
  if (rc) return rc;
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int i = 0; i < n; ++i) evals[i] = d[order[i]];
  if (n_vec <= 0) return 0;
  n_vec = std::min(n_vec, n);

  // eigenvectors of T, columns y_j (j < n_vec) stored as ty[j*n + i]
  std::vector<double> ty(static_cast<size_t>(n_vec) * n);
  if (full_accumulate) {
    for (int j = 0; j < n_vec; ++j)
      for (int i = 0; i < n; ++i) ty[static_cast<size_t>(j) * n + i] = z[static_cast<size_t>(i) * n + order[j]];
  } else {
    const double eps = 2.220446049250313e-16;
    const double ortol = 1e-3 * tnorm;
    const double tiny = eps * std::max(tnorm, 1e-300);
    uint64_t seed = 0x9E3779B97F4A7C15ULL ^ static_cast<uint64_t>(n);
    std::vector<double> x(n);
    int cluster_start = 0;
    double prev_sigma = 0.0;
    for (int j = 0; j < n_vec; ++j) {
      double lam = evals[j];
      if (j > 0 && lam - evals[j - 1] > ortol) cluster_start = j;
      double sigma = lam;
      if (j > cluster_start && sigma <= prev_sigma + 10.0 * eps * std::fabs(sigma))
        sigma = prev_sigma + 10.0 * eps * std::max(std::fabs(sigma), tnorm);
      prev_sigma = sigma;
      for (int i = 0; i < n; ++i) x[i] = static_cast<double>(lcg_next(seed) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
      for (int it = 0; it < 5; ++it) {
        tridiag_solve_shifted(n, d0, e0, sigma, tiny, x);
        // orthogonalise against earlier members of the cluster (twice)
        for (int pass = 0; pass < 2; ++pass)
          for (int k = cluster_start; k < j; ++k) {
            const double* yk = &ty[static_cast<size_t>(k) * n];
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += yk[i] * x[i];
            for (int i = 0; i < n; ++i) x[i] -= s * yk[i];
          }
        double nr = 0.0;
        for (int i = 0; i < n; ++i) nr += x[i] * x[i];
        nr = std::sqrt(nr);
        if (!(nr > 0.0) || !std::isfinite(nr)) return HYB_E_NOCONV;
        for (int i = 0; i < n; ++i) x[i] /= nr;
      }
      std::copy(x.begin(), x.end(), ty.begin() + static_cast<size_t>(j) * n);
    }
  }
  // back-transform with the Householder reflectors: y <- P_0 P_1 ... P_{n-3} y
  for (int j = 0; j < n_vec; ++j) {
    double* y = &ty[static_cast<size_t>(j) * n];
    for (int k = n - 3; k >= 0; --k) {
      if (hb[k] == 0.0) continue;
      const double* v = &hv[static_cast<size_t>(k) * n];
      double s = 0.0;
      for (int i = k + 1; i < n; ++i) s += v[i] * y[i];
      s *= hb[k];
      for (int i = k + 1; i < n; ++i) y[i] -= s * v[i];
    }
    for (int i = 0; i < n; ++i) vec[static_cast<size_t>(i) * n_vec + j] = y[i];
  }
  return 0;
}

}  // namespace hyb
