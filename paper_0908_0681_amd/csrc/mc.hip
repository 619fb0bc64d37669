// Monte Carlo sampling of the hybridization expansion on the device: random pair
// insertion / removal per flavor (Sec. II), determinant ratios and fast inverse
// updates in O(k^2) (Sec. II: fast matrix updates), one truncated Krylov trace per
// chain and move (the batched trace path), Metropolis-Hastings acceptance and
// the binned G(tau) estimator.
//
// Weight of a configuration: w = s_perm * Tr_R(literal time-ordered product)
// * prod_f det A_f, with A_f[i][j] = Delta(tau'_{f,i} - tau_{f,j}) (row i: the
// i-th creator of flavor f, column j: its j-th annihilator).  s_perm is the sign
// of the permutation from the canonical string (flavor by flavor, label by label:
// c_f(tau_{f,i}) c^dag_f(tau'_{f,i})) to descending time order: the fermionic sign
// of the time-ordering operator of Eq.(2).  M_f = A_f^{-1} is kept per flavor.
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) with counter (move low word,
// move high word, chain, call) and key (seed low word, seed high word).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "hyb_internal.h"
#include "trace_kernels.h"
#include "trace_launch.h"

namespace hyb {

#define MC_HIP_TRY(expr)                                                              \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return set_error(HYB_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

}  // namespace hyb (device code in mc_kernels.h)
#include "mc_kernels.h"
namespace hyb {

// The move counter lives on the device: move `off` of a launch sequence is move
// *Q.step_dev + off, and k_mc_advance moves the counter on at the end of the
// sequence.  A captured sweep therefore draws new random numbers on every replay.
__global__ __launch_bounds__(64) void k_mc_propose(MCParams Q, int64_t off) {
  __shared__ double sb[64], sc[64];
  mc_propose(Q, blockIdx.x, *Q.step_dev + off, sb, sc);
}

__global__ __launch_bounds__(64) void k_mc_accept(MCParams Q, int64_t off, int32_t meas_every) {
  extern __shared__ double canon[];
  const int64_t step = *Q.step_dev + off;
  mc_accept(Q, blockIdx.x, step, ((step + 1) % meas_every) == 0 ? 1 : 0, canon);
}

__global__ __launch_bounds__(64) void k_mc_sectors(MCParams Q) { mc_sectors(Q, blockIdx.x); }

__global__ void k_mc_copy(const double* src, double* dst, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ __launch_bounds__(64) void k_mc_choose(MCParams Q, int64_t off) {
  mc_choose(Q, blockIdx.x, *Q.step_dev + off);
}

__global__ void k_mc_set_step(int64_t* step, int64_t value, int64_t add) {
  if (threadIdx.x == 0) step[0] = (add ? step[0] : 0) + value;
}

// Rebuild of M from scratch after every `every`-th move (the kernel reads the move
// counter, so a captured sweep rebuilds on the same moves as direct launches).
// every <= 0: unconditional (checkpoint checks and explicit calls).
__global__ __launch_bounds__(64) void k_mc_rebuild(MCParams Q, int64_t off, int32_t every, int32_t apply, double* ld_f,
                                                   int32_t* sd_f, double* drift_f, int32_t* err) {
  __shared__ double a[64 * RB_LD];
  __shared__ int piv[64];
  if (every > 0 && ((*Q.step_dev + off + 1) % every) != 0) return;
  mc_rebuild(Q, blockIdx.x / Q.F, blockIdx.x % Q.F, apply, a, piv, ld_f, sd_f, drift_f, err);
}

__global__ void k_mc_rebuild_finish(MCParams Q, int64_t off, int32_t every, int32_t apply, const double* ld_f,
                                    const int32_t* sd_f, const double* drift_f, double* drift, double* ld_out,
                                    int32_t* sd_out) {
  if (every > 0 && ((*Q.step_dev + off + 1) % every) != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < Q.n_chains) mc_rebuild_finish(Q, c, apply, ld_f, sd_f, drift_f, drift, ld_out, sd_out);
}

__global__ __launch_bounds__(64) void k_mc_harvest(MCParams Q, int64_t index, __bf16* X, int32_t* T) {
  mc_harvest(Q, blockIdx.x, index, X, T);
}

}  // namespace hyb

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct hyb_mc {
  hyb_model* m = nullptr;
  hyb_mc_params p{};
  int F = 0;
  int64_t step = 0;
  hyb::MCParams Q{};
  double* t_log = nullptr;
  int8_t* t_sign = nullptr;
  int32_t* err = nullptr;
  // rebuild of M from scratch: per (chain, flavor) log|det|, sign and drift, and the
  // largest drift seen per chain
  double* rb_ld = nullptr;
  int32_t* rb_sd = nullptr;
  double* rb_drift_f = nullptr;
  double* drift = nullptr;
  void* trace_ws = nullptr;
  hyb_mlp* mlp = nullptr;      // learned proposal (NULL: uniform)
  __bf16* X = nullptr;         // [C][MLP_IN] features of the proposing configurations
  float* logits = nullptr;     // [C][MLP_OUT]
  std::vector<void*> allocs;
  // sweeps replayed from a captured HIP graph (hyb_mc_set_graphs)
  bool graphs = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<unsigned char> gkey;  // everything the captured launches depend on
};

namespace {

using namespace hyb;

template <typename T>
int mc_alloc(hyb_mc* mc, T*& ptr, size_t n) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
    return set_error(HYB_E_OOM, "device allocation of %zu bytes", n * sizeof(T));
  mc->allocs.push_back(p);
  ptr = static_cast<T*>(p);
  return 0;
}

// In-place LU with partial pivoting of an n x n row-major matrix, then its inverse
// into inv (row-major), log|det| and sign.  Returns false for a singular matrix.
bool lu_inverse(int n, std::vector<double> a, double* inv, int ld, double& logdet, int& sign) {
  std::vector<int> piv(n);
  logdet = 0.0;
  sign = 1;
  for (int col = 0; col < n; ++col) {
    int p = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(a[r * n + col]) > std::fabs(a[p * n + col])) p = r;
    if (a[p * n + col] == 0.0) return false;
    piv[col] = p;
    if (p != col) {
      for (int q = 0; q < n; ++q) std::swap(a[p * n + q], a[col * n + q]);
      sign = -sign;
    }
    const double d = a[col * n + col];
    logdet += std::log(std::fabs(d));
    if (d < 0) sign = -sign;
    for (int r = col + 1; r < n; ++r) {
      const double l = a[r * n + col] / d;
      a[r * n + col] = l;
      for (int q = col + 1; q < n; ++q) a[r * n + q] -= l * a[col * n + q];
    }
  }
  // solve A X = I column by column (P A = L U)
  std::vector<double> x(n);
  for (int e = 0; e < n; ++e) {
    for (int r = 0; r < n; ++r) x[r] = (r == e) ? 1.0 : 0.0;
    for (int col = 0; col < n; ++col) std::swap(x[col], x[piv[col]]);
    for (int r = 0; r < n; ++r)
      for (int q = 0; q < r; ++q) x[r] -= a[r * n + q] * x[q];
    for (int r = n - 1; r >= 0; --r) {
      for (int q = r + 1; q < n; ++q) x[r] -= a[r * n + q] * x[q];
      x[r] /= a[r * n + r];
    }
    for (int r = 0; r < n; ++r) inv[r * ld + e] = x[r];
  }
  return true;
}

double delta_host(const hyb_mc* mc, double tau) {
  double sgn = 1.0;
  if (tau < 0.0) {
    tau += mc->p.beta;
    sgn = -1.0;
  }
  const int n = mc->p.n_delta;
  const double x = tau / mc->p.beta * n;
  int k = int(x);
  if (k > n - 1) k = n - 1;
  const double fr = x - k;
  return sgn * (mc->p.delta[k] + fr * (mc->p.delta[k + 1] - mc->p.delta[k]));
}

int run_traces(hyb_mc* mc, hipStream_t s) {
  return trace_resident(mc->m, mc->p.n_chains, mc->Q.p_begin, mc->Q.p_end, mc->Q.p_tau, mc->Q.p_fl, mc->Q.p_dg,
                        mc->p.nmax_ops, mc->p.beta, mc->trace_ws, mc->t_log, mc->t_sign, mc->err, s);
}

// Enqueues `moves` moves of every chain and the advance of the device move counter
// on s.  Nothing here synchronises with the host, so the sequence can be captured.
int launch_moves(hyb_mc* mc, int64_t moves, hipStream_t s) {
  const int C = mc->p.n_chains;
  const size_t smem = sizeof(double) * std::max(mc->p.nmax_ops, 64);
  for (int64_t mv = 0; mv < moves; ++mv) {
    if (mc->mlp) {
      k_mc_choose<<<C, 64, 0, s>>>(mc->Q, mv);
      MlpActs a = mc->mlp->acts;
      a.z3 = mc->logits;
      int rc0 = mlp_forward(mc->mlp, C, mc->X, a, s);
      if (rc0) return rc0;
    }
    k_mc_propose<<<C, 64, 0, s>>>(mc->Q, mv);
    int rc = run_traces(mc, s);
    if (rc) return rc;
    k_mc_sectors<<<C, 64, 0, s>>>(mc->Q);
    k_mc_accept<<<C, 64, smem, s>>>(mc->Q, mv, mc->p.meas_every);
    if (mc->p.rebuild_every > 0) {
      const int32_t every = mc->p.rebuild_every, apply = 1;
      k_mc_rebuild<<<C * mc->F, 64, 0, s>>>(mc->Q, mv, every, apply, mc->rb_ld, mc->rb_sd, mc->rb_drift_f, mc->err);
      k_mc_rebuild_finish<<<(C + 255) / 256, 256, 0, s>>>(mc->Q, mv, every, apply, mc->rb_ld, mc->rb_sd,
                                                          mc->rb_drift_f, mc->drift, nullptr, nullptr);
    }
    MC_HIP_TRY(hipGetLastError());
  }
  k_mc_set_step<<<1, 64, 0, s>>>(mc->Q.step_dev, moves, 1);
  MC_HIP_TRY(hipGetLastError());
  return 0;
}

// What a captured sweep depends on: the chain parameters (device pointers, learned
// flag, mixture weight), the sweep length, the network's buffers, the model's
// device copy and its kernel variant.  A change of any of them forces a new capture.
std::vector<unsigned char> sweep_key(const hyb_mc* mc) {
  std::vector<unsigned char> k;
  auto put = [&k](const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    k.insert(k.end(), b, b + n);
  };
  put(&mc->Q, sizeof(mc->Q));
  put(&mc->p.moves_per_sweep, sizeof(mc->p.moves_per_sweep));
  put(&mc->p.meas_every, sizeof(mc->p.meas_every));
  put(&mc->p.rebuild_every, sizeof(mc->p.rebuild_every));
  put(&mc->mlp, sizeof(mc->mlp));
  if (mc->mlp) {
    put(&mc->mlp->acts, sizeof(mc->mlp->acts));
    put(mc->mlp->wb, sizeof(mc->mlp->wb));
    put(mc->mlp->bias, sizeof(mc->mlp->bias));
  }
  put(&mc->m->dev_gen, sizeof(mc->m->dev_gen));
  const int v = trace_resident_variant(mc->m);
  put(&v, sizeof(v));
  return k;
}

void drop_graph(hyb_mc* mc) {
  if (mc->gexec) (void)hipGraphExecDestroy(mc->gexec);
  if (mc->graph) (void)hipGraphDestroy(mc->graph);
  mc->gexec = nullptr;
  mc->graph = nullptr;
  mc->gkey.clear();
}

// Captures one sweep (moves_per_sweep moves and the counter advance) on a private
// stream and instantiates it.
int capture_sweep(hyb_mc* mc) {
  drop_graph(mc);
  if (!mc->cap_stream) MC_HIP_TRY(hipStreamCreateWithFlags(&mc->cap_stream, hipStreamNonBlocking));
  MC_HIP_TRY(hipStreamBeginCapture(mc->cap_stream, hipStreamCaptureModeThreadLocal));
  const int rc = launch_moves(mc, mc->p.moves_per_sweep, mc->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(mc->cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess || !g) return set_error(HYB_E_HIP, "capture of a sweep failed: %s", hipGetErrorString(e));
  mc->graph = g;
  MC_HIP_TRY(hipGraphInstantiate(&mc->gexec, g, nullptr, nullptr, 0));
  mc->gkey = sweep_key(mc);
  return 0;
}

// ---- checkpoints ------------------------------------------------------------------

struct CkptHeader {
  char magic[8];  // "HYBMCCK2"
  int32_t n_chains, F, kmax, nmax_ops, n_tau, n_delta, meas_every, moves_per_sweep, rebuild_every, precision;
  double beta;
  uint64_t seed;
  int64_t step;
  uint64_t delta_hash;  // FNV-1a over the bytes of the Delta table
  uint64_t payload;     // bytes after the header
};
constexpr char kCkptMagic[8] = {'H', 'Y', 'B', 'M', 'C', 'C', 'K', '2'};

uint64_t fnv1a(const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

// The device arrays of a checkpoint, in file order: the chain state (pair lists,
// M, the time-ordered operator list, weight factors), the statistics and the
// measurement accumulators.
struct CkptField {
  void* dev;
  size_t bytes;
};
std::vector<CkptField> ckpt_fields(const hyb_mc* mc) {
  const MCParams& Q = mc->Q;
  const size_t C = mc->p.n_chains, F = mc->F, KM = mc->p.kmax, NM = mc->p.nmax_ops, NT = mc->p.n_tau;
  return {{Q.kf, C * F * 4},          {Q.cre, C * F * KM * 8},   {Q.ann, C * F * KM * 8},
          {Q.M, C * F * KM * KM * 8}, {Q.cur_n, C * 4},          {Q.cur_tau, C * NM * 8},
          {Q.cur_fl, C * NM * 2},     {Q.cur_dg, C * NM},        {Q.cur_logtr, C * 8},
          {Q.cur_signtr, C * 4},      {Q.cur_logdet, C * 8},     {Q.cur_signdet, C * 4},
          {Q.cur_sign, C * 4},        {Q.stats, C * ST_N * 8},   {Q.sign_sum, C * 8},
          {Q.gacc, C * F * NT * 8},   {Q.meas_sign, C * 8},      {Q.n_meas, C * 8},
          {mc->drift, C * 8},         {Q.cur_psec, C * size_t(Q.n_blocks) * 8},
          {Q.sec_acc, C * size_t(Q.n_blocks) * 8}};
}

CkptHeader ckpt_header(const hyb_mc* mc) {
  CkptHeader h{};
  std::memcpy(h.magic, kCkptMagic, 8);
  h.n_chains = mc->p.n_chains;
  h.F = mc->F;
  h.kmax = mc->p.kmax;
  h.nmax_ops = mc->p.nmax_ops;
  h.n_tau = mc->p.n_tau;
  h.n_delta = mc->p.n_delta;
  h.meas_every = mc->p.meas_every;
  h.moves_per_sweep = mc->p.moves_per_sweep;
  h.rebuild_every = mc->p.rebuild_every;
  h.precision = mc->m->p.precision;
  h.beta = mc->p.beta;
  h.seed = mc->p.seed;
  h.step = mc->step;
  h.delta_hash = fnv1a(mc->p.delta, sizeof(double) * (mc->p.n_delta + 1));
  h.payload = 0;
  for (const CkptField& f : ckpt_fields(mc)) h.payload += f.bytes;
  return h;
}

}  // namespace

extern "C" {

int hyb_mc_destroy(hyb_mc* mc) {
  if (!mc) return HYB_OK;
  drop_graph(mc);
  if (mc->cap_stream) (void)hipStreamDestroy(mc->cap_stream);
  for (void* p : mc->allocs) (void)hipFree(p);
  delete[] mc->p.delta;
  delete mc;
  return HYB_OK;
}

int hyb_mc_create(hyb_model* m, const hyb_mc_params* p, hyb_mc** out) {
  if (!m || !p || !out) return set_error(HYB_E_ARG, "NULL argument");
  *out = nullptr;
  if (!m->uploaded) return set_error(HYB_E_STATE, "model not uploaded to a device");
  if (int rc0 = require_spectrum(m)) return rc0;
  if (p->n_chains < 1 || p->n_chains > (1 << 20)) return set_error(HYB_E_ARG, "n_chains out of range");
  if (p->kmax < 1 || p->kmax > 63) return set_error(HYB_E_ARG, "kmax must be in 1..63");
  if (p->nmax_ops < 2 || p->nmax_ops > 4096) return set_error(HYB_E_ARG, "nmax_ops must be in 2..4096");
  if (p->n_delta < 2 || !p->delta) return set_error(HYB_E_ARG, "Delta table needs n_delta >= 2 intervals");
  if (!(p->beta > 0.0) || !std::isfinite(p->beta)) return set_error(HYB_E_ARG, "beta must be positive");
  if (p->n_tau < 1 || p->meas_every < 1 || p->moves_per_sweep < 1)
    return set_error(HYB_E_ARG, "n_tau, meas_every and moves_per_sweep must be >= 1");
  if (p->rebuild_every < 0) return set_error(HYB_E_ARG, "rebuild_every must be >= 0");
  for (int i = 0; i <= p->n_delta; ++i)
    if (!std::isfinite(p->delta[i])) return set_error(HYB_E_ARG, "non-finite Delta table entry %d", i);
  hyb_mc* mc = new hyb_mc();
  mc->m = m;
  mc->p = *p;
  double* table = new double[p->n_delta + 1];
  std::memcpy(table, p->delta, sizeof(double) * (p->n_delta + 1));
  mc->p.delta = table;
  mc->F = m->F;
  const int C = p->n_chains, F = m->F, KM = p->kmax, NM = p->nmax_ops;
  MCParams& Q = mc->Q;
  Q.n_chains = C;
  Q.F = F;
  Q.kmax = KM;
  Q.nmax = NM;
  Q.n_delta = p->n_delta;
  Q.n_tau = p->n_tau;
  Q.beta = p->beta;
  Q.key0 = uint32_t(p->seed);
  Q.key1 = uint32_t(p->seed >> 32);
  int rc = 0;
  double* d_delta = nullptr;
  int64_t* d_begin = nullptr;
  auto fail = [&](int code) {
    hyb_mc_destroy(mc);
    return code;
  };
  if ((rc = mc_alloc(mc, d_delta, p->n_delta + 1)) || (rc = mc_alloc(mc, Q.kf, size_t(C) * F)) ||
      (rc = mc_alloc(mc, Q.cre, size_t(C) * F * KM)) || (rc = mc_alloc(mc, Q.ann, size_t(C) * F * KM)) ||
      (rc = mc_alloc(mc, Q.M, size_t(C) * F * KM * KM)) || (rc = mc_alloc(mc, Q.cur_n, C)) ||
      (rc = mc_alloc(mc, Q.cur_tau, size_t(C) * NM)) || (rc = mc_alloc(mc, Q.cur_fl, size_t(C) * NM)) ||
      (rc = mc_alloc(mc, Q.cur_dg, size_t(C) * NM)) || (rc = mc_alloc(mc, d_begin, C)) ||
      (rc = mc_alloc(mc, Q.p_end, C)) || (rc = mc_alloc(mc, Q.p_tau, size_t(C) * NM)) ||
      (rc = mc_alloc(mc, Q.p_fl, size_t(C) * NM)) || (rc = mc_alloc(mc, Q.p_dg, size_t(C) * NM)) ||
      (rc = mc_alloc(mc, Q.mv, C)) || (rc = mc_alloc(mc, Q.uvec, size_t(C) * KM)) ||
      (rc = mc_alloc(mc, Q.vvec, size_t(C) * KM)) || (rc = mc_alloc(mc, Q.cur_logtr, C)) ||
      (rc = mc_alloc(mc, Q.cur_signtr, C)) || (rc = mc_alloc(mc, Q.cur_logdet, C)) ||
      (rc = mc_alloc(mc, Q.cur_signdet, C)) || (rc = mc_alloc(mc, Q.cur_sign, C)) ||
      (rc = mc_alloc(mc, mc->t_log, C)) || (rc = mc_alloc(mc, mc->t_sign, C)) ||
      (rc = mc_alloc(mc, Q.stats, size_t(C) * ST_N)) || (rc = mc_alloc(mc, Q.sign_sum, C)) ||
      (rc = mc_alloc(mc, Q.gacc, size_t(C) * F * p->n_tau)) || (rc = mc_alloc(mc, Q.meas_sign, C)) ||
      (rc = mc_alloc(mc, Q.n_meas, C)) || (rc = mc_alloc(mc, mc->err, 1)) || (rc = mc_alloc(mc, Q.step_dev, 1)) ||
      (rc = mc_alloc(mc, mc->rb_ld, size_t(C) * F)) || (rc = mc_alloc(mc, mc->rb_sd, size_t(C) * F)) ||
      (rc = mc_alloc(mc, mc->rb_drift_f, size_t(C) * F)) || (rc = mc_alloc(mc, mc->drift, C)) ||
      (rc = mc_alloc(mc, Q.psec_prop, size_t(C) * m->n_blocks)) ||
      (rc = mc_alloc(mc, Q.cur_psec, size_t(C) * m->n_blocks)) ||
      (rc = mc_alloc(mc, Q.sec_acc, size_t(C) * m->n_blocks)))
    return fail(rc);
  char* ws = nullptr;
  if ((rc = mc_alloc(mc, ws, trace_ws_bytes(m, C)))) return fail(rc);
  mc->trace_ws = ws;
  {
    const ResidentPairs pr = trace_resident_pairs(m, C, ws);
    Q.pr_sign = pr.sign;
    Q.pr_log = pr.log;
    Q.pr_mid = pr.midblk;
    Q.n_blocks = m->n_blocks;
    Q.n_ret = int32_t(m->ret_block.size());
  }
  Q.delta = d_delta;
  Q.p_begin = d_begin;
  Q.t_log = mc->t_log;
  Q.t_sign = mc->t_sign;
  std::vector<int64_t> begin(C);
  for (int c = 0; c < C; ++c) begin[c] = int64_t(c) * NM;
  if (hipMemcpy(d_delta, table, sizeof(double) * (p->n_delta + 1), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_begin, begin.data(), sizeof(int64_t) * C, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(mc->err, 0, sizeof(int32_t)) != hipSuccess)
    return fail(set_error(HYB_E_HIP, "upload of the Monte Carlo tables failed"));
  *out = mc;
  // every chain starts empty (weight Tr_R of the empty configuration > 0)
  std::vector<int32_t> k0(size_t(C) * F, 0);
  std::vector<double> z(size_t(C) * F * KM, 0.0);
  rc = hyb_mc_set_configs(mc, k0.data(), z.data(), z.data(), nullptr);
  if (rc) {
    hyb_mc_destroy(mc);
    *out = nullptr;
  }
  return rc;
}

int hyb_mc_set_configs(hyb_mc* mc, const int32_t* k, const double* cre, const double* ann, void* stream) {
  if (!mc || !k || !cre || !ann) return set_error(HYB_E_ARG, "NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int C = mc->p.n_chains, F = mc->F, KM = mc->p.kmax, NM = mc->p.nmax_ops;
  const double beta = mc->p.beta;
  std::vector<double> Mh(size_t(C) * F * KM * KM, 0.0), ptau(size_t(C) * NM, 0.0);
  std::vector<int16_t> pfl(size_t(C) * NM, 0);
  std::vector<int8_t> pdg(size_t(C) * NM, 0);
  std::vector<int64_t> pend(C);
  std::vector<int32_t> n_ops(C), signdet(C), sperm(C);
  std::vector<double> logdet(C);
  for (int c = 0; c < C; ++c) {
    struct Op {
      double t;
      int f, dg;
    };
    std::vector<Op> ops;
    std::vector<double> canon;
    double ld = 0.0;
    int sd = 1;
    for (int f = 0; f < F; ++f) {
      const int kf = k[c * F + f];
      if (kf < 0 || kf > KM) return set_error(HYB_E_ARG, "chain %d flavor %d: order %d outside 0..%d", c, f, kf, KM);
      const double* cf = cre + (size_t(c) * F + f) * KM;
      const double* af = ann + (size_t(c) * F + f) * KM;
      for (int i = 0; i < kf; ++i) {
        if (!(cf[i] >= 0.0 && cf[i] < beta && af[i] >= 0.0 && af[i] < beta))
          return set_error(HYB_E_UNSORTED, "chain %d: operator time outside [0, beta)", c);
        ops.push_back({cf[i], f, 1});
        ops.push_back({af[i], f, 0});
        canon.push_back(af[i]);
        canon.push_back(cf[i]);
      }
      if (kf > 0) {
        std::vector<double> A(size_t(kf) * kf);
        for (int i = 0; i < kf; ++i)
          for (int j = 0; j < kf; ++j) A[i * kf + j] = delta_host(mc, cf[i] - af[j]);
        // M = A^{-1}: rows of M follow annihilator labels, columns creator labels
        double l = 0.0;
        int sg = 1;
        if (!lu_inverse(kf, A, Mh.data() + (size_t(c) * F + f) * KM * KM, KM, l, sg))
          return set_error(HYB_E_ARG, "chain %d flavor %d: singular hybridization matrix", c, f);
        ld += l;
        sd *= sg;
      }
    }
    if (int(ops.size()) > NM) return set_error(HYB_E_ARG, "chain %d: %zu operators exceed nmax_ops", c, ops.size());
    std::sort(ops.begin(), ops.end(), [](const Op& a, const Op& b) { return a.t < b.t; });
    for (size_t q = 1; q < ops.size(); ++q)
      if (!(ops[q].t > ops[q - 1].t)) return set_error(HYB_E_UNSORTED, "chain %d: equal operator times", c);
    for (size_t q = 0; q < ops.size(); ++q) {
      ptau[size_t(c) * NM + q] = ops[q].t;
      pfl[size_t(c) * NM + q] = int16_t(ops[q].f);
      pdg[size_t(c) * NM + q] = int8_t(ops[q].dg);
    }
    int64_t inv = 0;
    for (size_t a = 0; a < canon.size(); ++a)
      for (size_t b = a + 1; b < canon.size(); ++b) inv += canon[a] < canon[b];
    n_ops[c] = int(ops.size());
    pend[c] = int64_t(c) * NM + int64_t(ops.size());
    logdet[c] = ld;
    signdet[c] = sd;
    sperm[c] = (inv & 1) ? -1 : 1;
  }
  MCParams& Q = mc->Q;
  const size_t nst = size_t(C) * ST_N;
  std::vector<int64_t> zeros64(std::max(nst, size_t(C)), 0);
  std::vector<double> zerosd(std::max(size_t(C), size_t(C) * F * mc->p.n_tau), 0.0);
  MC_HIP_TRY(hipMemcpyAsync(Q.kf, k, sizeof(int32_t) * C * F, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.cre, cre, sizeof(double) * C * F * KM, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.ann, ann, sizeof(double) * C * F * KM, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.M, Mh.data(), sizeof(double) * Mh.size(), hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.cur_n, n_ops.data(), sizeof(int32_t) * C, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.cur_tau, ptau.data(), sizeof(double) * ptau.size(), hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.cur_fl, pfl.data(), sizeof(int16_t) * pfl.size(), hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.cur_dg, pdg.data(), sizeof(int8_t) * pdg.size(), hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.p_tau, ptau.data(), sizeof(double) * ptau.size(), hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.p_fl, pfl.data(), sizeof(int16_t) * pfl.size(), hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.p_dg, pdg.data(), sizeof(int8_t) * pdg.size(), hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.p_end, pend.data(), sizeof(int64_t) * C, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.cur_logdet, logdet.data(), sizeof(double) * C, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.cur_signdet, signdet.data(), sizeof(int32_t) * C, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.stats, zeros64.data(), sizeof(int64_t) * nst, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.sign_sum, zerosd.data(), sizeof(double) * C, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.gacc, zerosd.data(), sizeof(double) * C * F * mc->p.n_tau, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.meas_sign, zerosd.data(), sizeof(double) * C, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.n_meas, zeros64.data(), sizeof(int64_t) * C, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(mc->drift, zerosd.data(), sizeof(double) * C, hipMemcpyHostToDevice, s));
  // a new state starts without the error of an earlier failed sweep
  MC_HIP_TRY(hipMemcpyAsync(mc->err, zeros64.data(), sizeof(int32_t), hipMemcpyHostToDevice, s));
  // traces of the initial configurations (through the proposal slots) and their
  // sector distributions at beta/2
  int rc = run_traces(mc, s);
  if (rc) return rc;
  {
    const int64_t nsec = int64_t(C) * mc->m->n_blocks;
    k_mc_sectors<<<C, 64, 0, s>>>(Q);
    k_mc_copy<<<unsigned((nsec + 255) / 256), 256, 0, s>>>(Q.psec_prop, Q.cur_psec, nsec);
    MC_HIP_TRY(hipMemsetAsync(Q.sec_acc, 0, sizeof(double) * nsec, s));
  }
  std::vector<double> tl(C);
  std::vector<int8_t> ts(C);
  int32_t err = 0;
  MC_HIP_TRY(hipMemcpyAsync(tl.data(), mc->t_log, sizeof(double) * C, hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipMemcpyAsync(ts.data(), mc->t_sign, sizeof(int8_t) * C, hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipMemcpyAsync(&err, mc->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipStreamSynchronize(s));
  if (err) return set_error(HYB_E_NOCONV, "trace of the initial configurations failed (error bits %d)", err);
  std::vector<int32_t> signtr(C), sign(C);
  for (int c = 0; c < C; ++c) {
    if (ts[c] == 0) return set_error(HYB_E_ARG, "chain %d: initial configuration has zero weight", c);
    signtr[c] = ts[c];
    sign[c] = sperm[c] * signtr[c] * signdet[c];
  }
  MC_HIP_TRY(hipMemcpyAsync(Q.cur_logtr, tl.data(), sizeof(double) * C, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.cur_signtr, signtr.data(), sizeof(int32_t) * C, hipMemcpyHostToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.cur_sign, sign.data(), sizeof(int32_t) * C, hipMemcpyHostToDevice, s));
  k_mc_set_step<<<1, 64, 0, s>>>(Q.step_dev, 0, 0);
  MC_HIP_TRY(hipGetLastError());
  MC_HIP_TRY(hipStreamSynchronize(s));
  mc->step = 0;
  return HYB_OK;
}

int hyb_mc_sweep(hyb_mc* mc, int32_t n_sweeps, void* stream) {
  if (!mc) return set_error(HYB_E_ARG, "NULL argument");
  if (n_sweeps < 0) return set_error(HYB_E_ARG, "negative sweep count");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t moves = int64_t(n_sweeps) * mc->p.moves_per_sweep;
  if (moves > 0) {
    if (mc->graphs) {
      if (!mc->gexec || mc->gkey != sweep_key(mc)) {
        const int rc = capture_sweep(mc);
        if (rc) return rc;
      }
      for (int32_t sw = 0; sw < n_sweeps; ++sw) MC_HIP_TRY(hipGraphLaunch(mc->gexec, s));
    } else {
      const int rc = launch_moves(mc, moves, s);
      if (rc) return rc;
    }
    mc->step += moves;
  }
  int32_t err = 0;
  MC_HIP_TRY(hipMemcpyAsync(&err, mc->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipStreamSynchronize(s));
  if (err) {
    // reported once: the flag is cleared so that later calls report their own errors
    const int32_t zero = 0;
    MC_HIP_TRY(hipMemcpyAsync(mc->err, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
    MC_HIP_TRY(hipStreamSynchronize(s));
  }
  if (err & ERR_NOCONV) return set_error(HYB_E_NOCONV, "Krylov propagation failed inside a move");
  if (err & ERR_NONFINITE) return set_error(HYB_E_NONFINITE, "non-finite value inside a move");
  if (err & ERR_SINGULAR) return set_error(HYB_E_NONFINITE, "singular hybridization matrix at a rebuild of M");
  if (err) return set_error(HYB_E_HIP, "inconsistent proposal (error bits %d)", err);
  return HYB_OK;
}

int hyb_mc_get_state(const hyb_mc* mc, int32_t* k, double* cre, double* ann, double* M, double* logw, int8_t* sign,
                     void* stream) {
  if (!mc) return set_error(HYB_E_ARG, "NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int C = mc->p.n_chains, F = mc->F, KM = mc->p.kmax;
  const MCParams& Q = mc->Q;
  if (k) MC_HIP_TRY(hipMemcpyAsync(k, Q.kf, sizeof(int32_t) * C * F, hipMemcpyDeviceToHost, s));
  if (cre) MC_HIP_TRY(hipMemcpyAsync(cre, Q.cre, sizeof(double) * C * F * KM, hipMemcpyDeviceToHost, s));
  if (ann) MC_HIP_TRY(hipMemcpyAsync(ann, Q.ann, sizeof(double) * C * F * KM, hipMemcpyDeviceToHost, s));
  if (M) MC_HIP_TRY(hipMemcpyAsync(M, Q.M, sizeof(double) * size_t(C) * F * KM * KM, hipMemcpyDeviceToHost, s));
  std::vector<double> lt(C), ld(C);
  std::vector<int32_t> sg(C);
  MC_HIP_TRY(hipMemcpyAsync(lt.data(), Q.cur_logtr, sizeof(double) * C, hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipMemcpyAsync(ld.data(), Q.cur_logdet, sizeof(double) * C, hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipMemcpyAsync(sg.data(), Q.cur_sign, sizeof(int32_t) * C, hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipStreamSynchronize(s));
  for (int c = 0; c < C; ++c) {
    if (logw) logw[c] = lt[c] + ld[c];
    if (sign) sign[c] = int8_t(sg[c]);
  }
  return HYB_OK;
}

int hyb_mc_get_stats(const hyb_mc* mc, hyb_mc_stats* out, void* stream) {
  if (!mc || !out) return set_error(HYB_E_ARG, "NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int C = mc->p.n_chains;
  std::vector<int64_t> st(size_t(C) * ST_N);
  std::vector<double> ss(C), dr(C);
  MC_HIP_TRY(hipMemcpyAsync(st.data(), mc->Q.stats, sizeof(int64_t) * st.size(), hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipMemcpyAsync(ss.data(), mc->Q.sign_sum, sizeof(double) * C, hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipMemcpyAsync(dr.data(), mc->drift, sizeof(double) * C, hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipStreamSynchronize(s));
  *out = hyb_mc_stats{};
  for (int c = 0; c < C; ++c) out->max_drift = std::max(out->max_drift, dr[c]);
  for (int c = 0; c < C; ++c) {
    const int64_t* a = st.data() + size_t(c) * ST_N;
    out->insert_proposed += a[ST_INS_PROP];
    out->insert_accepted += a[ST_INS_ACC];
    out->remove_proposed += a[ST_REM_PROP];
    out->remove_accepted += a[ST_REM_ACC];
    out->impossible += a[ST_IMPOSSIBLE];
    out->zero_weight += a[ST_ZERO];
    out->order_sum += double(a[ST_ORDER]);
    out->moves += a[ST_MOVES];
    out->sign_sum += ss[c];
  }
  return HYB_OK;
}

int hyb_mc_get_accumulators(const hyb_mc* mc, double* gacc, double* meas_sign, int64_t* n_meas, void* stream) {
  if (!mc) return set_error(HYB_E_ARG, "NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int C = mc->p.n_chains, F = mc->F;
  if (gacc)
    MC_HIP_TRY(hipMemcpyAsync(gacc, mc->Q.gacc, sizeof(double) * size_t(C) * F * mc->p.n_tau, hipMemcpyDeviceToHost, s));
  if (meas_sign) MC_HIP_TRY(hipMemcpyAsync(meas_sign, mc->Q.meas_sign, sizeof(double) * C, hipMemcpyDeviceToHost, s));
  if (n_meas) MC_HIP_TRY(hipMemcpyAsync(n_meas, mc->Q.n_meas, sizeof(int64_t) * C, hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipStreamSynchronize(s));
  return HYB_OK;
}

int hyb_mc_measure(const hyb_mc* mc, double* G, double* sign_avg, void* stream) {
  if (!mc || !G) return set_error(HYB_E_ARG, "NULL argument");
  const int C = mc->p.n_chains, F = mc->F, NT = mc->p.n_tau;
  std::vector<double> acc(size_t(C) * F * NT), ms(C);
  std::vector<int64_t> nm(C);
  int rc = hyb_mc_get_accumulators(mc, acc.data(), ms.data(), nm.data(), stream);
  if (rc) return rc;
  double ssum = 0.0;
  int64_t ntot = 0;
  for (int c = 0; c < C; ++c) {
    ssum += ms[c];
    ntot += nm[c];
  }
  if (ntot == 0 || ssum == 0.0) return set_error(HYB_E_STATE, "no measurements (or zero average sign)");
  const double h = mc->p.beta / NT;
  for (int f = 0; f < F; ++f)
    for (int b = 0; b < NT; ++b) {
      double a = 0.0;
      for (int c = 0; c < C; ++c) a += acc[(size_t(c) * F + f) * NT + b];
      G[f * NT + b] = -a / (mc->p.beta * h * ssum);
    }
  if (sign_avg) *sign_avg = ssum / double(ntot);
  return HYB_OK;
}

int hyb_mc_reset_measurements(hyb_mc* mc, void* stream) {
  if (!mc) return set_error(HYB_E_ARG, "NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int C = mc->p.n_chains, F = mc->F;
  MC_HIP_TRY(hipMemsetAsync(mc->Q.gacc, 0, sizeof(double) * size_t(C) * F * mc->p.n_tau, s));
  MC_HIP_TRY(hipMemsetAsync(mc->Q.meas_sign, 0, sizeof(double) * C, s));
  MC_HIP_TRY(hipMemsetAsync(mc->Q.n_meas, 0, sizeof(int64_t) * C, s));
  MC_HIP_TRY(hipMemsetAsync(mc->Q.stats, 0, sizeof(int64_t) * size_t(C) * ST_N, s));
  MC_HIP_TRY(hipMemsetAsync(mc->Q.sign_sum, 0, sizeof(double) * C, s));
  MC_HIP_TRY(hipMemsetAsync(mc->Q.sec_acc, 0, sizeof(double) * size_t(C) * mc->m->n_blocks, s));
  MC_HIP_TRY(hipStreamSynchronize(s));
  return HYB_OK;
}

int hyb_mc_attach_mlp(hyb_mc* mc, hyb_mlp* mlp, double eps) {
  if (!mc) return set_error(HYB_E_ARG, "NULL argument");
  if (mlp && !(eps > 0.0 && eps <= 1.0)) return set_error(HYB_E_ARG, "mixture weight eps must be in (0, 1]");
  if (mlp && mc->F > 10) return set_error(HYB_E_ARG, "the learned proposal takes at most 10 flavors");
  const int C = mc->p.n_chains;
  if (mlp && !mc->X) {
    int rc = 0;
    if ((rc = mc_alloc(mc, mc->X, size_t(C) * MLP_IN)) || (rc = mc_alloc(mc, mc->logits, size_t(C) * MLP_OUT)))
      return rc;
  }
  if (mlp) {
    int rc = mlp_ensure(mlp, C);
    if (rc) return rc;
  }
  mc->mlp = mlp;
  mc->Q.learned = mlp ? 1 : 0;
  mc->Q.eps_mix = eps;
  mc->Q.X = mc->X;
  mc->Q.logits = mc->logits;
  return HYB_OK;
}

int hyb_mc_harvest(hyb_mc* mc, int64_t index, void* X, int32_t* targets, void* stream) {
  if (!mc || !X || !targets) return set_error(HYB_E_ARG, "NULL argument");
  if (mc->F > 10) return set_error(HYB_E_ARG, "the learned proposal takes at most 10 flavors");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  k_mc_harvest<<<mc->p.n_chains, 64, 0, s>>>(mc->Q, index, static_cast<__bf16*>(X), targets);
  MC_HIP_TRY(hipGetLastError());
  return HYB_OK;
}

int hyb_mc_set_graphs(hyb_mc* mc, int32_t enable) {
  if (!mc) return set_error(HYB_E_ARG, "NULL argument");
  mc->graphs = enable != 0;
  if (!mc->graphs) drop_graph(mc);
  return HYB_OK;
}

int hyb_mc_save(const hyb_mc* mc, void* buf, size_t* len, void* stream) {
  if (!mc || !len) return set_error(HYB_E_ARG, "NULL argument");
  const CkptHeader h = ckpt_header(mc);
  const size_t need = sizeof(CkptHeader) + h.payload;
  if (!buf) {
    *len = need;
    return HYB_OK;
  }
  if (*len < need) return set_error(HYB_E_ARG, "checkpoint buffer of %zu bytes, %zu needed", *len, need);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* out = static_cast<char*>(buf);
  std::memcpy(out, &h, sizeof h);
  size_t off = sizeof h;
  for (const CkptField& f : ckpt_fields(mc)) {
    MC_HIP_TRY(hipMemcpyAsync(out + off, f.dev, f.bytes, hipMemcpyDeviceToHost, s));
    off += f.bytes;
  }
  MC_HIP_TRY(hipStreamSynchronize(s));
  *len = need;
  return HYB_OK;
}

int hyb_mc_load(hyb_mc* mc, const void* buf, size_t len, void* stream) {
  if (!mc || !buf) return set_error(HYB_E_ARG, "NULL argument");
  if (len < sizeof(CkptHeader)) return set_error(HYB_E_ARG, "checkpoint shorter than its header");
  CkptHeader h;
  std::memcpy(&h, buf, sizeof h);
  const CkptHeader mine = ckpt_header(mc);
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0) return set_error(HYB_E_ARG, "not a chain checkpoint");
  if (h.n_chains != mine.n_chains || h.F != mine.F || h.kmax != mine.kmax || h.nmax_ops != mine.nmax_ops ||
      h.n_tau != mine.n_tau || h.n_delta != mine.n_delta || h.beta != mine.beta || h.seed != mine.seed ||
      h.delta_hash != mine.delta_hash || h.precision != mine.precision || h.payload != mine.payload)
    return set_error(HYB_E_ARG, "checkpoint of other chains (sizes, beta, seed, bath or precision differ)");
  if (len < sizeof h + h.payload) return set_error(HYB_E_ARG, "truncated checkpoint");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int C = mc->p.n_chains, F = mc->F, NM = mc->p.nmax_ops;
  const char* in = static_cast<const char*>(buf) + sizeof h;
  for (const CkptField& f : ckpt_fields(mc)) {
    MC_HIP_TRY(hipMemcpyAsync(f.dev, in, f.bytes, hipMemcpyHostToDevice, s));
    in += f.bytes;
  }
  MCParams& Q = mc->Q;
  const int32_t zero = 0;
  MC_HIP_TRY(hipMemcpyAsync(mc->err, &zero, sizeof zero, hipMemcpyHostToDevice, s));
  k_mc_set_step<<<1, 64, 0, s>>>(Q.step_dev, h.step, 0);
  MC_HIP_TRY(hipGetLastError());
  mc->step = h.step;
  // Consistency: the stored weight factors against a fresh trace of the stored
  // operator lists and a fresh inverse of the stored pair lists.  The stored M is
  // kept, so the resumed chains continue bit for bit.
  MC_HIP_TRY(hipMemcpyAsync(Q.p_tau, Q.cur_tau, sizeof(double) * size_t(C) * NM, hipMemcpyDeviceToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.p_fl, Q.cur_fl, sizeof(int16_t) * size_t(C) * NM, hipMemcpyDeviceToDevice, s));
  MC_HIP_TRY(hipMemcpyAsync(Q.p_dg, Q.cur_dg, sizeof(int8_t) * size_t(C) * NM, hipMemcpyDeviceToDevice, s));
  std::vector<int32_t> n(C);
  MC_HIP_TRY(hipMemcpyAsync(n.data(), Q.cur_n, sizeof(int32_t) * C, hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipStreamSynchronize(s));
  std::vector<int64_t> pend(C);
  for (int c = 0; c < C; ++c) {
    if (n[c] < 0 || n[c] > NM) return set_error(HYB_E_ARG, "checkpoint: chain %d has %d operators", c, n[c]);
    pend[c] = int64_t(c) * NM + n[c];
  }
  MC_HIP_TRY(hipMemcpyAsync(Q.p_end, pend.data(), sizeof(int64_t) * C, hipMemcpyHostToDevice, s));
  int rc = run_traces(mc, s);
  if (rc) return rc;
  double* tmp = nullptr;
  MC_HIP_TRY(hipMalloc(&tmp, sizeof(double) * 2 * C + sizeof(int32_t) * C));
  double* ld_chk = tmp;
  double* dr_chk = tmp + C;
  int32_t* sd_chk = reinterpret_cast<int32_t*>(tmp + 2 * C);
  MC_HIP_TRY(hipMemsetAsync(dr_chk, 0, sizeof(double) * C, s));
  k_mc_rebuild<<<C * F, 64, 0, s>>>(Q, 0, 0, 0, mc->rb_ld, mc->rb_sd, mc->rb_drift_f, mc->err);
  k_mc_rebuild_finish<<<(C + 255) / 256, 256, 0, s>>>(Q, 0, 0, 0, mc->rb_ld, mc->rb_sd, mc->rb_drift_f, dr_chk, ld_chk,
                                                      sd_chk);
  std::vector<double> tl(C), lt(C), ld(C), lk(C), dr(C);
  std::vector<int8_t> ts(C);
  std::vector<int32_t> st(C), sd(C), sk(C);
  int32_t err = 0;
  hipError_t e = hipSuccess;
  auto d2h = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
  };
  d2h(tl.data(), mc->t_log, sizeof(double) * C);
  d2h(ts.data(), mc->t_sign, sizeof(int8_t) * C);
  d2h(lt.data(), Q.cur_logtr, sizeof(double) * C);
  d2h(st.data(), Q.cur_signtr, sizeof(int32_t) * C);
  d2h(ld.data(), Q.cur_logdet, sizeof(double) * C);
  d2h(sd.data(), Q.cur_signdet, sizeof(int32_t) * C);
  d2h(lk.data(), ld_chk, sizeof(double) * C);
  d2h(sk.data(), sd_chk, sizeof(int32_t) * C);
  d2h(dr.data(), dr_chk, sizeof(double) * C);
  d2h(&err, mc->err, sizeof(int32_t));
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(tmp);
  if (e != hipSuccess) return set_error(HYB_E_HIP, "checkpoint check: %s", hipGetErrorString(e));
  if (err) return set_error(HYB_E_ARG, "checkpoint: trace or determinant of the stored state failed (bits %d)", err);
  const double tol_tr = (mc->m->p.precision == HYB_FP64) ? 1e-8 : 1e-4;
  for (int c = 0; c < C; ++c) {
    if (ts[c] != st[c] || !(std::fabs(tl[c] - lt[c]) <= tol_tr * std::max(1.0, std::fabs(lt[c]))))
      return set_error(HYB_E_ARG, "checkpoint: chain %d stored trace disagrees with its operators", c);
    if (sk[c] != sd[c] || !(std::fabs(lk[c] - ld[c]) <= 1e-8 * std::max(1.0, std::fabs(ld[c]))) || !(dr[c] <= 1e-6))
      return set_error(HYB_E_ARG, "checkpoint: chain %d stored M / determinant disagree with its times", c);
  }
  return HYB_OK;
}

int hyb_mc_set_delta(hyb_mc* mc, const double* delta, void* stream) {
  if (!mc || !delta) return set_error(HYB_E_ARG, "NULL argument");
  const int n = mc->p.n_delta;
  for (int i = 0; i <= n; ++i)
    if (!std::isfinite(delta[i])) return set_error(HYB_E_ARG, "non-finite Delta table entry %d", i);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::memcpy(const_cast<double*>(mc->p.delta), delta, sizeof(double) * (n + 1));
  MC_HIP_TRY(hipMemcpyAsync(const_cast<double*>(mc->Q.delta), mc->p.delta, sizeof(double) * (n + 1),
                            hipMemcpyHostToDevice, s));
  // every chain's A_f changed: M_f, log|det| and the weight's sign from scratch
  const int C = mc->p.n_chains;
  const int32_t zero = 0;
  MC_HIP_TRY(hipMemcpyAsync(mc->err, &zero, sizeof zero, hipMemcpyHostToDevice, s));
  k_mc_rebuild<<<C * mc->F, 64, 0, s>>>(mc->Q, 0, 0, 1, mc->rb_ld, mc->rb_sd, mc->rb_drift_f, mc->err);
  // the drift of this rebuild is the change of Delta, not an error of the updates:
  // fold it into a scratch copy rather than the chains' drift record
  double* scratch_drift = nullptr;
  MC_HIP_TRY(hipMalloc(&scratch_drift, sizeof(double) * C));
  MC_HIP_TRY(hipMemsetAsync(scratch_drift, 0, sizeof(double) * C, s));
  k_mc_rebuild_finish<<<(C + 255) / 256, 256, 0, s>>>(mc->Q, 0, 0, 1, mc->rb_ld, mc->rb_sd, mc->rb_drift_f,
                                                      scratch_drift, nullptr, nullptr);
  int32_t err = 0;
  const hipError_t e1 = hipMemcpyAsync(&err, mc->err, sizeof err, hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipStreamSynchronize(s);
  (void)hipFree(scratch_drift);
  if (e1 != hipSuccess || e2 != hipSuccess) return set_error(HYB_E_HIP, "setting Delta failed");
  if (err) {
    MC_HIP_TRY(hipMemcpyAsync(mc->err, &zero, sizeof zero, hipMemcpyHostToDevice, s));
    MC_HIP_TRY(hipStreamSynchronize(s));
    return set_error(HYB_E_ARG, "a chain's hybridization matrix is singular with the new Delta");
  }
  return HYB_OK;
}

int hyb_mc_bethe_delta(const hyb_mc* mc, double t, double mix, int32_t symmetrize, double* delta_out, void* stream) {
  if (!mc || !delta_out) return set_error(HYB_E_ARG, "NULL argument");
  if (!(mix > 0.0 && mix <= 1.0) || !std::isfinite(t)) return set_error(HYB_E_ARG, "mix must be in (0, 1], t finite");
  const int F = mc->F, NT = mc->p.n_tau, n = mc->p.n_delta;
  if (NT < 2) return set_error(HYB_E_ARG, "the Bethe update needs at least 2 G(tau) bins");
  std::vector<double> G(size_t(F) * NT);
  double sgn = 0.0;
  int rc = hyb_mc_measure(mc, G.data(), &sgn, stream);
  if (rc) return rc;
  // one Delta serves every flavor: average G over the flavors (paramagnetic,
  // orbitally degenerate), then optionally G(tau) = G(beta - tau)
  std::vector<double> g(NT, 0.0);
  for (int b = 0; b < NT; ++b) {
    for (int f = 0; f < F; ++f) g[b] += G[size_t(f) * NT + b];
    g[b] /= F;
  }
  if (symmetrize & 1) {
    std::vector<double> h(g);
    for (int b = 0; b < NT; ++b) g[b] = 0.5 * (h[b] + h[NT - 1 - b]);
  }
  // bin centres (b + 1/2) beta / NT; the ends by linear extrapolation, shifted
  // together so that G(0+) + G(beta-) = -1
  const double beta = mc->p.beta, hb = beta / NT;
  double g0 = g[0] - 0.5 * (g[1] - g[0]), gb = g[NT - 1] + 0.5 * (g[NT - 1] - g[NT - 2]);
  const double shift = 0.5 * (-1.0 - g0 - gb);
  g0 += shift;
  gb += shift;
  for (int k = 0; k <= n; ++k) {
    const double tau = beta * k / n;
    double gv;
    const double x = tau / hb - 0.5;  // position in units of bins from the first centre
    if (x <= 0.0) {
      gv = g0 + (g[0] - g0) * (tau / (0.5 * hb));
    } else if (x >= NT - 1) {
      gv = g[NT - 1] + (gb - g[NT - 1]) * ((tau - (NT - 0.5) * hb) / (0.5 * hb));
    } else {
      const int b = int(x);
      const double fr = x - b;
      gv = g[b] + fr * (g[b + 1] - g[b]);
    }
    delta_out[k] = (1.0 - mix) * mc->p.delta[k] + mix * t * t * gv;
  }
  return HYB_OK;
}

int hyb_dmft_bethe(hyb_mc* mc, const hyb_dmft_params* p, double* g_half, double* sign_avg, void* stream) {
  if (!mc || !p) return set_error(HYB_E_ARG, "NULL argument");
  if (p->n_iter < 1 || p->therm_sweeps < 0 || p->meas_sweeps < 1)
    return set_error(HYB_E_ARG, "n_iter and meas_sweeps must be >= 1, therm_sweeps >= 0");
  const int F = mc->F, NT = mc->p.n_tau;
  std::vector<double> G(size_t(F) * NT), d(mc->p.n_delta + 1);
  for (int it = 0; it < p->n_iter; ++it) {
    int rc = hyb_mc_sweep(mc, p->therm_sweeps, stream);
    if (!rc) rc = hyb_mc_reset_measurements(mc, stream);
    if (!rc) rc = hyb_mc_sweep(mc, p->meas_sweeps, stream);
    double sg = 0.0;
    if (!rc) rc = hyb_mc_measure(mc, G.data(), &sg, stream);
    if (rc) return rc;
    double gh = 0.0;
    for (int f = 0; f < F; ++f) gh += 0.5 * (G[size_t(f) * NT + NT / 2 - 1] + G[size_t(f) * NT + NT / 2]);
    if (g_half) g_half[it] = gh / F;
    if (sign_avg) sign_avg[it] = sg;
    rc = hyb_mc_bethe_delta(mc, p->t, p->mix, p->symmetrize, d.data(), stream);
    if (!rc) rc = hyb_mc_set_delta(mc, d.data(), stream);
    if (rc) return rc;
  }
  return HYB_OK;
}

int hyb_mc_get_delta(const hyb_mc* mc, double* delta) {
  if (!mc || !delta) return set_error(HYB_E_ARG, "NULL argument");
  std::memcpy(delta, mc->p.delta, sizeof(double) * (mc->p.n_delta + 1));
  return HYB_OK;
}

int hyb_mc_sector_weights(const hyb_mc* mc, double* w, double* acc, void* stream) {
  if (!mc || (!w && !acc)) return set_error(HYB_E_ARG, "NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int C = mc->p.n_chains, NB = mc->m->n_blocks;
  std::vector<double> a(size_t(C) * NB), ms(C);
  MC_HIP_TRY(hipMemcpyAsync(a.data(), mc->Q.sec_acc, sizeof(double) * a.size(), hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipMemcpyAsync(ms.data(), mc->Q.meas_sign, sizeof(double) * C, hipMemcpyDeviceToHost, s));
  MC_HIP_TRY(hipStreamSynchronize(s));
  if (acc) std::memcpy(acc, a.data(), sizeof(double) * a.size());
  if (w) {
    double ssum = 0.0;
    for (int c = 0; c < C; ++c) ssum += ms[c];
    if (ssum == 0.0) return set_error(HYB_E_STATE, "no measurements (or zero average sign)");
    for (int b = 0; b < NB; ++b) {
      double t = 0.0;
      for (int c = 0; c < C; ++c) t += a[size_t(c) * NB + b];
      w[b] = t / ssum;
    }
  }
  return HYB_OK;
}

int hyb_mc_step_count(const hyb_mc* mc, int64_t* step) {
  if (!mc || !step) return set_error(HYB_E_ARG, "NULL argument");
  *step = mc->step;
  return HYB_OK;
}

}  // extern "C"
