// The matrix formulation of the trace (Sec. II, Eq.(3)): the comparison path the
// Krylov method is measured against (Sec. IV.B).  In the eigenbasis of every block
// the time evolution is diagonal, exp(-dtau (E_b - E0)), and each operator is a
// dense block U_t^T O U_b.  A trace is then a chain of diagonal scalings and dense
// matrix-vector products over the same retained outer states R as the Krylov path,
// so both give the same Tr_R(c).
//
// Device layout (built once by hyb_matrix_build):
//  - E: every block's eigenvalues, ascending, at the block's state offset;
//  - ops: for every (block b, flavor f, dagger) with a physical target block t the
//    d_t x d_b block of O in the two eigenbases, column-major (entry (t, s) at
//    t + s d_t), so that consecutive threads read consecutive rows of a column;
//  - op_off[(b F + f) 2 + dagger]: the block's offset in ops, -1 without target.
// The operator blocks are U_t^T (O U_b): the signed row gather O U_b on the device
// and one rocBLAS DGEMM per block.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "hyb_internal.h"
#include "trace_kernels.h"

namespace hyb {

#define MAT_HIP_TRY(expr)                                                             \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return set_error(HYB_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

struct MatrixForm {
  double* E = nullptr;          // [n_states] eigenvalues per block, ascending
  double* ops = nullptr;        // operator blocks (column-major), concatenated
  int64_t* op_off = nullptr;    // [n_blocks * F * 2]
  int32_t* ret_index = nullptr; // [n_ret] eigen-index of each retained state in its block
  int64_t op_elems = 0;
  double build_seconds = 0.0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int device = -1;
  uint64_t dev_gen = 0;         // the model upload this form was built against
};

struct MatParams {
  const double* E;
  const double* ops;
  const int64_t* op_off;
  const int32_t* ret_index;
  int32_t F;
};

// O U_b gathered into G (column-major d_t x d_b): G[r][s] = sign * U_b[src(r)][s],
// with U_b row-major (component i of eigenvector s at i d_b + s).
__global__ void k_mat_gather(const uint32_t* states, const int32_t* rank, BlockDev Bs, BlockDev Bt, int f, int dagger,
                             const double* Ub, double* G) {
  const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= int64_t(Bt.dim) * Bs.dim) return;
  const int s = int(id / Bt.dim), r = int(id - int64_t(s) * Bt.dim);
  const uint32_t bit = 1u << f;
  const uint32_t t = states[Bt.state_off + r];
  const bool has = dagger ? ((t & bit) != 0u) : ((t & bit) == 0u);
  double v = 0.0;
  if (has) {
    const uint32_t src = t ^ bit;
    v = Ub[int64_t(rank[src]) * Bs.dim + s];
    if (__popc(src & (bit - 1u)) & 1) v = -v;
  }
  G[id] = v;
}

__global__ void k_mat_init(int32_t* c) {
  if (threadIdx.x < 4) c[threadIdx.x] = 0;
}

__global__ void k_mat_scan(TraceParams P) {
  __shared__ float width[64];  // (n_orb + 1)^2 <= 64 blocks
  const int nb = (P.n_orb + 1) * (P.n_orb + 1);
  for (int i = threadIdx.x; i < nb; i += blockDim.x) width[i] = P.blocks[i].width;
  __syncthreads();
  const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id < int64_t(P.n_configs) * P.n_ret) scan_pair(P, id, width);
}

__global__ void k_mat_reduce(TraceParams P, double* out_log, int8_t* out_sign, int32_t* out_steps, int32_t* out_sub,
                             int32_t* out_feas, int64_t* out_rs, int64_t* out_rw) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < P.n_configs) reduce_config(P, c, out_log, out_sign, out_steps, out_sub, out_feas, out_rs, out_rw);
}

// One workgroup per feasible path: the retained eigenstate e_i enters with the edge
// phase (step 3), every interval scales the eigenbasis vector by exp(-dtau (E - E0))
// (the lowest energy the vector occupies factored into the log-scale), every
// operator is a dense product with its eigenbasis block judged against the norm of
// the vector it acts on, the result is renormalised with its log kept aside, and the
// overlap with e_i closes the path.  rowsteps counts the matrix elements read
// (d_t d_b per operator), rows the target dimensions.
template <int NT, int RPT>
__global__ __launch_bounds__(NT) void k_mat_path(TraceParams P, MatParams M) {
  extern __shared__ double sm[];
  const int w = blockIdx.x;
  if (w >= P.counters[0]) return;
  const int tid = threadIdx.x;
  double* va = sm;
  double* vb = sm + NT * RPT;
  double* red = sm + 2 * NT * RPT;
  const int id = P.work[w];
  const int c = id / P.n_ret, r = id - c * P.n_ret;
  const int64_t o0 = P.offsets[c], o1 = cfg_end(P, c);
  const int b0 = P.ret_block[r], i0 = M.ret_index[r];
  const double Ei = P.ret_energy[r];
  if (o1 == o0) {
    if (tid == 0) {
      P.p_sign[id] = 1;
      P.p_log[id] = -P.beta * Ei;
      P.p_steps[id] = 0;
      P.p_sub[id] = 0;
      P.p_rowsteps[id] = 0;
      P.p_rows[id] = 0;
    }
    return;
  }
  int b = b0;
  BlockDev B = P.blocks[b];
  for (int i = tid; i < B.dim; i += NT) va[i] = (i == i0) ? 1.0 : 0.0;
  double ell = -(P.beta - P.tau[o1 - 1] + P.tau[o0]) * (Ei - P.E0);
  bool zero = false, failed = false;
  int64_t elems = 0, rows = 0;
  __syncthreads();
  for (int64_t k = o0; k < o1; ++k) {
    double n2_in = 1.0;  // squared norm of the vector the operator acts on
    if (k > o0) {
      // diagonal evolution in the eigenbasis, exp(-dt (E_i - e)) with e the lowest
      // energy the (unit) vector occupies above 1e-30, factored into the log-scale
      const double dt = P.tau[k] - P.tau[k - 1];
      double emin = INFINITY;
      for (int i = tid; i < B.dim; i += NT)
        if (fabs(va[i]) > 1e-30) emin = fmin(emin, M.E[B.state_off + i]);
      for (int o = 32; o >= 1; o >>= 1) emin = fmin(emin, shfl_xor_d(emin, o));
      if ((tid & 63) == 0) red[4 + (tid >> 6)] = emin;
      __syncthreads();
      emin = red[4];
#pragma unroll
      for (int q = 1; q < NT / 64; ++q) emin = fmin(emin, red[4 + q]);
      double part = 0.0;
      for (int i = tid; i < B.dim; i += NT) {
        const double x = va[i] * exp(-dt * (M.E[B.state_off + i] - emin));
        va[i] = x;
        part += x * x;
      }
      part = wave_sum(part);
      if ((tid & 63) == 0) red[8 + (tid >> 6)] = part;
      ell += -dt * (emin - P.E0);
      __syncthreads();
      n2_in = 0.0;
#pragma unroll
      for (int q = 0; q < NT / 64; ++q) n2_in += red[8 + q];
    }
    const int f = P.flavor[k];
    const int dg = P.dagger[k] ? 1 : 0;
    const int64_t off = M.op_off[(int64_t(b) * M.F + f) * 2 + dg];
    if (off < 0) {  // excluded by the scan
      failed = true;
      break;
    }
    int nu = B.n_up, nd = B.n_dn;
    if (f < P.n_orb) nu += dg ? 1 : -1; else nd += dg ? 1 : -1;
    const int bt = nd * (P.n_orb + 1) + nu;
    const BlockDev Bt = P.blocks[bt];
    const double* C = M.ops + off;
    double acc[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) acc[q] = 0.0;
    // y_t = sum_s C[t + s d_t] v_s: each thread its rows t, all of them at once so
    // that their loads are in flight together
    for (int s = 0; s < B.dim; ++s) {
      const double vs = va[s];
      const double* col = C + int64_t(s) * Bt.dim;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int t = tid + q * NT;
        if (t < Bt.dim) acc[q] += col[t] * vs;
      }
    }
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) part += acc[q] * acc[q];
    part = wave_sum(part);
    if ((tid & 63) == 0) red[tid >> 6] = part;
    __syncthreads();
    double n2 = 0.0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) n2 += red[q];
    elems += int64_t(Bt.dim) * B.dim;
    rows += Bt.dim;
    // the operator is judged on the unit vector: a result below the threshold of its
    // input's norm is a zero imposed by symmetry
    if (!(n2 > P.zero_tol2 * n2_in) || !isfinite(n2) || !(n2_in > 0.0)) {
      zero = (n2 >= 0.0) && (n2 <= P.zero_tol2 * n2_in);
      failed = !zero;
      break;
    }
    const double inv = 1.0 / sqrt(n2);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int t = tid + q * NT;
      if (t < Bt.dim) vb[t] = acc[q] * inv;
    }
    ell += 0.5 * log(n2);
    double* tmp = va;
    va = vb;
    vb = tmp;
    b = bt;
    B = Bt;
    __syncthreads();  // the new vector is read whole by the next product; red is reused
  }
  if (tid == 0) {
    const double ov = (!zero && !failed && b == b0) ? va[i0] : 0.0;
    if (zero || failed || !(ov * ov > P.zero_tol2)) {
      P.p_sign[id] = 0;
      P.p_log[id] = -INFINITY;
    } else {
      P.p_sign[id] = ov > 0.0 ? 1 : -1;
      P.p_log[id] = ell + log(fabs(ov)) - P.beta * P.E0;
    }
    P.p_steps[id] = 0;
    P.p_sub[id] = 0;
    P.p_rowsteps[id] = elems;
    P.p_rows[id] = rows;
    if (failed) atomicOr(&P.counters[2], ERR_NONFINITE);
  }
}

void matrix_release(hyb_model* m) {
  if (!m || !m->mat) return;
  MatrixForm* F = static_cast<MatrixForm*>(m->mat);
  void* ptrs[] = {F->E, F->ops, F->op_off, F->ret_index, F->ws};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete F;
  m->mat = nullptr;
}

namespace {

// Every eigenvector of every block (host, threads over blocks), row-major per block:
// component i of eigenvector j at i d + j.
int full_eigvecs(const hyb_model* m, std::vector<std::vector<double>>& U, std::vector<std::vector<double>>& E) {
  U.assign(m->n_blocks, {});
  E.assign(m->n_blocks, {});
  std::vector<int> order(m->n_blocks);
  for (int b = 0; b < m->n_blocks; ++b) order[b] = b;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return m->blocks[x].dim > m->blocks[y].dim; });
  std::atomic<int> next{0}, err{0};
  auto worker = [&]() {
    std::vector<double> h;
    for (;;) {
      const int j = next.fetch_add(1);
      if (j >= m->n_blocks) return;
      const int b = order[j];
      const int d = m->blocks[b].dim;
      if (d == 0) continue;
      h.assign(size_t(d) * d, 0.0);
      int rc = hyb_block_dense(m, b, h.data());
      if (rc) {
        err = rc;
        return;
      }
      U[b].resize(size_t(d) * d);
      E[b].resize(d);
      rc = sym_eig(d, h.data(), E[b].data(), d, U[b].data());
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
  return err.load();
}

int target_block(const hyb_model* m, int b, int f, int dg) {
  const BlockDev& B = m->blocks[b];
  int nu = B.n_up, nd = B.n_dn;
  if (f < m->n_orb) nu += dg ? 1 : -1; else nd += dg ? 1 : -1;
  if (nu < 0 || nu > m->n_orb || nd < 0 || nd > m->n_orb) return -1;
  return nd * (m->n_orb + 1) + nu;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace
}  // namespace hyb

using namespace hyb;

extern "C" {

int hyb_matrix_build(hyb_model* m, void* stream) {
  if (!m) return set_error(HYB_E_ARG, "NULL model");
  if (!m->uploaded) return set_error(HYB_E_STATE, "model not uploaded to a device");
  if (int rc0 = require_spectrum(m)) return rc0;
  int dev = -1;
  MAT_HIP_TRY(hipGetDevice(&dev));
  if (dev != m->dev.device) return set_error(HYB_E_STATE, "model lives on device %d, current is %d", m->dev.device, dev);
  const auto t0 = std::chrono::steady_clock::now();
  matrix_release(m);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<std::vector<double>> U, E;
  int rc = full_eigvecs(m, U, E);
  if (rc) return set_error(rc, "block eigensolver did not converge");
  MatrixForm* F = new MatrixForm();
  m->mat = F;
  F->device = dev;
  F->dev_gen = m->dev_gen;
  const int nF = m->F;
  // operator block offsets
  std::vector<int64_t> off(size_t(m->n_blocks) * nF * 2, -1);
  int64_t total = 0, max_g = 0;
  for (int b = 0; b < m->n_blocks; ++b)
    for (int f = 0; f < nF; ++f)
      for (int dg = 0; dg < 2; ++dg) {
        const int t = target_block(m, b, f, dg);
        if (t < 0 || m->blocks[b].dim == 0 || m->blocks[t].dim == 0) continue;
        off[(size_t(b) * nF + f) * 2 + dg] = total;
        const int64_t n = int64_t(m->blocks[t].dim) * m->blocks[b].dim;
        total += n;
        max_g = std::max(max_g, n);
      }
  F->op_elems = total;
  std::vector<double> Eh(m->n_states, 0.0);
  for (int b = 0; b < m->n_blocks; ++b)
    for (int i = 0; i < m->blocks[b].dim; ++i) Eh[m->blocks[b].state_off + i] = E[b][i];
  // retained states are the lowest eigen-indices of their blocks, in order
  std::vector<int32_t> ridx(m->ret_block.size());
  for (size_t q = 0; q < ridx.size(); ++q) ridx[q] = m->ret_index[q];
  int64_t ucount = 0;
  std::vector<int64_t> uoff(m->n_blocks);
  for (int b = 0; b < m->n_blocks; ++b) {
    uoff[b] = ucount;
    ucount += int64_t(m->blocks[b].dim) * m->blocks[b].dim;
  }
  double *dU = nullptr, *dG = nullptr;
  auto fail = [&](int code) {
    if (dU) (void)hipFree(dU);
    if (dG) (void)hipFree(dG);
    matrix_release(m);
    return code;
  };
  if (hipMalloc(&F->E, sizeof(double) * std::max<int64_t>(m->n_states, 1)) != hipSuccess ||
      hipMalloc(&F->ops, sizeof(double) * std::max<int64_t>(total, 1)) != hipSuccess ||
      hipMalloc(&F->op_off, sizeof(int64_t) * off.size()) != hipSuccess ||
      hipMalloc(&F->ret_index, sizeof(int32_t) * std::max<size_t>(ridx.size(), 1)) != hipSuccess ||
      hipMalloc(&dU, sizeof(double) * std::max<int64_t>(ucount, 1)) != hipSuccess ||
      hipMalloc(&dG, sizeof(double) * std::max<int64_t>(max_g, 1)) != hipSuccess)
    return fail(set_error(HYB_E_OOM, "matrix formulation needs %.2f GB of device memory", total * 8e-9));
  if (hipMemcpyAsync(F->E, Eh.data(), sizeof(double) * m->n_states, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(F->op_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      (!ridx.empty() &&
       hipMemcpyAsync(F->ret_index, ridx.data(), sizeof(int32_t) * ridx.size(), hipMemcpyHostToDevice, s) != hipSuccess))
    return fail(set_error(HYB_E_HIP, "upload of the eigenbasis data failed"));
  for (int b = 0; b < m->n_blocks; ++b)
    if (!U[b].empty() &&
        hipMemcpyAsync(dU + uoff[b], U[b].data(), sizeof(double) * U[b].size(), hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(set_error(HYB_E_HIP, "upload of the eigenvectors failed"));
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) return fail(set_error(HYB_E_HIP, "rocblas_create_handle"));
  rocblas_set_stream(h, s);
  const double one = 1.0, zero = 0.0;
  int err = 0;
  for (int b = 0; b < m->n_blocks && !err; ++b)
    for (int f = 0; f < nF && !err; ++f)
      for (int dg = 0; dg < 2 && !err; ++dg) {
        const int64_t o = off[(size_t(b) * nF + f) * 2 + dg];
        if (o < 0) continue;
        const int t = target_block(m, b, f, dg);
        const BlockDev &Bs = m->blocks[b], &Bt = m->blocks[t];
        const int64_t n = int64_t(Bt.dim) * Bs.dim;
        k_mat_gather<<<unsigned((n + 255) / 256), 256, 0, s>>>(m->dev.states, m->dev.rank, Bs, Bt, f, dg, dU + uoff[b],
                                                               dG);
        // ops = U_t^T G: U_t row-major is U_t^T column-major (ld d_t)
        if (rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, Bt.dim, Bs.dim, Bt.dim, &one,
                          dU + uoff[t], Bt.dim, dG, Bt.dim, &zero, F->ops + o, Bt.dim) != rocblas_status_success)
          err = 1;
      }
  rocblas_destroy_handle(h);
  const hipError_t e1 = hipStreamSynchronize(s);
  (void)hipFree(dU);
  (void)hipFree(dG);
  dU = dG = nullptr;
  if (err || e1 != hipSuccess || hipGetLastError() != hipSuccess)
    return fail(set_error(HYB_E_HIP, "building the eigenbasis operator blocks failed"));
  F->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return HYB_OK;
}

int hyb_matrix_info(const hyb_model* m, int64_t* op_bytes, double* build_seconds) {
  if (!m) return set_error(HYB_E_ARG, "NULL model");
  if (!m->mat) return set_error(HYB_E_STATE, "matrix formulation not built");
  const MatrixForm* F = static_cast<const MatrixForm*>(m->mat);
  if (op_bytes) *op_bytes = F->op_elems * int64_t(sizeof(double));
  if (build_seconds) *build_seconds = F->build_seconds;
  return HYB_OK;
}

int hyb_trace_batch_matrix(hyb_model* m, const hyb_config_batch* cfg, double beta, hyb_trace_out* out, void* stream) {
  if (!m || !cfg || !out) return set_error(HYB_E_ARG, "NULL argument");
  if (!m->mat) return set_error(HYB_E_STATE, "matrix formulation not built (hyb_matrix_build)");
  MatrixForm* F = static_cast<MatrixForm*>(m->mat);
  if (!m->uploaded || F->dev_gen != m->dev_gen)
    return set_error(HYB_E_STATE, "the model was uploaded again after hyb_matrix_build");
  if (!(beta > 0.0) || !std::isfinite(beta)) return set_error(HYB_E_ARG, "beta must be positive and finite");
  if (cfg->n_configs < 0) return set_error(HYB_E_ARG, "negative n_configs");
  if (cfg->n_configs == 0) return HYB_OK;
  if (!cfg->offsets || !out->log_abs || !out->sign) return set_error(HYB_E_ARG, "NULL array");
  int dev = -1;
  MAT_HIP_TRY(hipGetDevice(&dev));
  if (dev != F->device) return set_error(HYB_E_STATE, "matrix formulation lives on device %d", F->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int nc = cfg->n_configs, n_ret = int(m->ret_block.size());
  const int64_t npairs = int64_t(nc) * n_ret;
  if (npairs > (int64_t(1) << 31) - 1) return set_error(HYB_E_ARG, "too many (config, state) pairs");
  int64_t n_ops = 0;
  if (!cfg->on_device) {
    if (cfg->offsets[0] != 0) return set_error(HYB_E_ARG, "offsets must start at 0");
    for (int c = 0; c < nc; ++c)
      if (cfg->offsets[c + 1] < cfg->offsets[c]) return set_error(HYB_E_ARG, "offsets must not decrease");
    n_ops = cfg->offsets[nc];
    if (n_ops > 0 && (!cfg->tau || !cfg->flavor || !cfg->dagger)) return set_error(HYB_E_ARG, "NULL operator array");
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t o_cnt = take(16), o_work = take(npairs * 4), o_ps = take(npairs), o_pl = take(npairs * 8),
               o_pst = take(npairs * 4), o_psu = take(npairs * 4), o_prs = take(npairs * 8), o_prw = take(npairs * 8);
  size_t o_offs = 0, o_tau = 0, o_fl = 0, o_dg = 0;
  if (!cfg->on_device) {
    o_offs = take((nc + 1) * 8);
    o_tau = take(std::max<int64_t>(n_ops, 1) * 8);
    o_fl = take(std::max<int64_t>(n_ops, 1) * 2);
    o_dg = take(std::max<int64_t>(n_ops, 1));
  }
  size_t o_out[7] = {0, 0, 0, 0, 0, 0, 0};
  const size_t out_bytes[7] = {8, 1, 4, 4, 4, 8, 8};
  if (!out->on_device)
    for (int q = 0; q < 7; ++q) o_out[q] = take(size_t(nc) * out_bytes[q]);
  if (F->ws_bytes < off) {
    if (F->ws) {
      MAT_HIP_TRY(hipDeviceSynchronize());
      (void)hipFree(F->ws);
      F->ws = nullptr;
      F->ws_bytes = 0;
    }
    if (hipMalloc(&F->ws, off) != hipSuccess) return set_error(HYB_E_OOM, "matrix workspace of %zu bytes", off);
    F->ws_bytes = off;
  }
  char* ws = static_cast<char*>(F->ws);
  TraceParams P{};
  P.states = m->dev.states;
  P.rank = m->dev.rank;
  P.blocks = m->dev.blocks;
  P.ret_block = m->dev.ret_block;
  P.ret_energy = m->dev.ret_energy;
  P.n_orb = m->n_orb;
  P.n_ret = n_ret;
  P.E0 = m->E0;
  P.n_configs = nc;
  P.n_pairs = int32_t(npairs);
  P.beta = beta;
  P.zero_tol2 = 1e-20;
  P.counters = reinterpret_cast<int32_t*>(ws + o_cnt);
  P.work = reinterpret_cast<int32_t*>(ws + o_work);
  P.p_sign = reinterpret_cast<int8_t*>(ws + o_ps);
  P.p_log = reinterpret_cast<double*>(ws + o_pl);
  P.p_steps = reinterpret_cast<int32_t*>(ws + o_pst);
  P.p_sub = reinterpret_cast<int32_t*>(ws + o_psu);
  P.p_rowsteps = reinterpret_cast<int64_t*>(ws + o_prs);
  P.p_rows = reinterpret_cast<int64_t*>(ws + o_prw);
  if (cfg->on_device) {
    P.offsets = cfg->offsets;
    P.tau = cfg->tau;
    P.flavor = cfg->flavor;
    P.dagger = cfg->dagger;
  } else {
    P.offsets = reinterpret_cast<int64_t*>(ws + o_offs);
    P.tau = reinterpret_cast<double*>(ws + o_tau);
    P.flavor = reinterpret_cast<int16_t*>(ws + o_fl);
    P.dagger = reinterpret_cast<int8_t*>(ws + o_dg);
    MAT_HIP_TRY(hipMemcpyAsync(const_cast<int64_t*>(P.offsets), cfg->offsets, (nc + 1) * 8, hipMemcpyHostToDevice, s));
    if (n_ops > 0) {
      MAT_HIP_TRY(hipMemcpyAsync(const_cast<double*>(P.tau), cfg->tau, n_ops * 8, hipMemcpyHostToDevice, s));
      MAT_HIP_TRY(hipMemcpyAsync(const_cast<int16_t*>(P.flavor), cfg->flavor, n_ops * 2, hipMemcpyHostToDevice, s));
      MAT_HIP_TRY(hipMemcpyAsync(const_cast<int8_t*>(P.dagger), cfg->dagger, n_ops, hipMemcpyHostToDevice, s));
    }
  }
  MatParams M{F->E, F->ops, F->op_off, F->ret_index, m->F};
  void* outp[7] = {out->log_abs, out->sign, out->krylov_steps, out->substeps, out->feasible_paths, out->rowsteps,
                   out->rows};
  void* dout[7];
  for (int q = 0; q < 7; ++q) dout[q] = out->on_device ? outp[q] : static_cast<void*>(ws + o_out[q]);
  k_mat_init<<<1, 64, 0, s>>>(P.counters);
  k_mat_scan<<<unsigned((npairs + 255) / 256), 256, 0, s>>>(P);
  int32_t cnt[3] = {0, 0, 0};
  MAT_HIP_TRY(hipMemcpyAsync(cnt, P.counters, sizeof cnt, hipMemcpyDeviceToHost, s));
  MAT_HIP_TRY(hipStreamSynchronize(s));
  if (cnt[2] & ERR_UNSORTED) return set_error(HYB_E_UNSORTED, "operator times not strictly increasing in [0, beta)");
  if (cnt[2] & ERR_FLAVOR) return set_error(HYB_E_FLAVOR, "flavor or dagger out of range");
  const int nwork = cnt[0];
  if (nwork > 0) {
    // rows per thread for the largest block; the two LDS vectors hold max_dim each
    const size_t smem = sizeof(double) * (2 * 256 * 5 + 12);
    if (m->max_dim <= 256)
      k_mat_path<256, 1><<<unsigned(nwork), 256, sizeof(double) * (2 * 256 + 12), s>>>(P, M);
    else if (m->max_dim <= 1280)
      k_mat_path<256, 5><<<unsigned(nwork), 256, smem, s>>>(P, M);
    else
      return set_error(HYB_E_ARG, "blocks of dimension %d exceed the matrix kernel (1280)", m->max_dim);
  }
  k_mat_reduce<<<(nc + 255) / 256, 256, 0, s>>>(P, static_cast<double*>(dout[0]), static_cast<int8_t*>(dout[1]),
                                                static_cast<int32_t*>(dout[2]), static_cast<int32_t*>(dout[3]),
                                                static_cast<int32_t*>(dout[4]), static_cast<int64_t*>(dout[5]),
                                                static_cast<int64_t*>(dout[6]));
  MAT_HIP_TRY(hipGetLastError());
  int32_t flags = 0;
  MAT_HIP_TRY(hipMemcpyAsync(&flags, P.counters + 2, sizeof flags, hipMemcpyDeviceToHost, s));
  if (!out->on_device)
    for (int q = 0; q < 7; ++q)
      if (outp[q]) MAT_HIP_TRY(hipMemcpyAsync(outp[q], dout[q], size_t(nc) * out_bytes[q], hipMemcpyDeviceToHost, s));
  MAT_HIP_TRY(hipStreamSynchronize(s));
  if (flags & ERR_NONFINITE) return set_error(HYB_E_NONFINITE, "non-finite value in the matrix products");
  return HYB_OK;
}

}  // extern "C"
