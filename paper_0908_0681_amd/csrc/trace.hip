// Device side of libhyb: model upload, the batched trace (scan -> path kernels,
// one workgroup per feasible path -> signed log-sum), device parity hooks and
// kernel variants.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "hyb_internal.h"
#include "trace_kernels.h"
#include "trace_launch.h"

namespace hyb {

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return set_error(HYB_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

__global__ void k_init_counters(int32_t* c, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0;
}

__global__ void k_scan(TraceParams P) {
  __shared__ float width[64];  // (n_orb + 1)^2 <= 64 blocks
  const int nb = (P.n_orb + 1) * (P.n_orb + 1);
  for (int i = threadIdx.x; i < nb; i += blockDim.x) width[i] = P.blocks[i].width;
  __syncthreads();
  const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id < int64_t(P.n_configs) * P.n_ret) scan_pair(P, id, width);
}

// First queue slot of every cost bucket, the costliest bucket first (one workgroup
// of ORDER_NB threads).
__global__ void k_order_base(int32_t* c) {
  const int b = threadIdx.x;
  int s = 0;
  for (int q = b + 1; q < ORDER_NB; ++q) s += c[4 + q];
  c[4 + ORDER_NB + b] = s;
}

// Every feasible path into the next slot of its bucket.
__global__ void k_order_place(TraceParams P) {
  const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= int64_t(P.n_configs) * P.n_ret) return;
  const int b = P.p_bucket[id];
  if (b >= 0) P.work[atomicAdd(&P.counters[4 + ORDER_NB + b], 1)] = int32_t(id);
}

template <typename VT, int NT>
__global__ __launch_bounds__(NT) void k_path_init(TraceParams P) {
  if (int(blockIdx.x) >= P.counters[0]) return;  // grids may be sized for every pair
  path_init<VT, NT>(P, blockIdx.x);
}

template <typename VT, int NT, int RPT>
__global__ __launch_bounds__(NT) void k_path_op(TraceParams P, int k) {
  __shared__ double red[NT / 64];
  if (int(blockIdx.x) >= P.counters[0]) return;
  path_op<VT, NT, RPT>(P, blockIdx.x, k, red);
}

template <typename VT, int NT, int RPT, int MAXM, bool MF, bool VL, int OCC>
__global__ __launch_bounds__(NT, OCC) void k_path_prop(TraceParams P, int k) {
  __shared__ typename PathEngine<VT, NT, RPT, MAXM, MF, VL>::Smem S;
  if (int(blockIdx.x) >= P.counters[0]) return;
  path_prop<VT, NT, RPT, MAXM, MF, VL>(P, blockIdx.x, k, S);
}

// Operators [k0, k1) of every path, one workgroup per path: the propagation before
// operator k (k > 0) and the operator itself, with the same arithmetic as the
// single-step kernels; the path's state stays on chip between operators.
template <typename VT, int NT, int RPT, int MAXM, bool MF, bool VL, int OCC>
__global__ __launch_bounds__(NT, OCC) void k_path_chunk(TraceParams P, int k0, int k1) {
  __shared__ typename PathEngine<VT, NT, RPT, MAXM, MF, VL>::Smem S;
  __shared__ double red[NT / 64];
  __shared__ PathCarry carry;
  __shared__ PathTables tables;
  const int w = blockIdx.x;
  if (w >= P.counters[0]) return;
  path_tables_load<NT>(P, tables);
  {
    // stop at this path's own length (uniform over the workgroup)
    const int c = P.work[w] / P.n_ret;
    const int64_t n = cfg_end(P, c) - P.offsets[c];
    if (int64_t(k1) > n) k1 = int(n);
  }
  path_run<VT, NT, RPT, MAXM, MF, VL>(P, w, k0, k1, S, red, carry, tables);
}

template <typename VT, int NT, int RPT>
__global__ __launch_bounds__(NT) void k_path_final(TraceParams P) {
  __shared__ double red[NT / 64];
  if (int(blockIdx.x) >= P.counters[0]) return;
  path_final<VT, NT, RPT>(P, blockIdx.x, red);
}

__global__ void k_fold_errors(const int32_t* counters, int32_t* acc) {
  if (threadIdx.x == 0 && counters[2] != 0) atomicOr(acc, counters[2]);
}

__global__ void k_reduce(TraceParams P, double* out_log, int8_t* out_sign, int32_t* out_steps,
                         int32_t* out_sub, int32_t* out_feas, int64_t* out_rowsteps, int64_t* out_rows) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < P.n_configs)
    reduce_config(P, c, out_log, out_sign, out_steps, out_sub, out_feas, out_rowsteps, out_rows);
}

// Operator application on a batch of vectors (parity hook): the whole-path trace
// kernel's own gather (gather_tab on the LDS tables), one thread per output component.
__global__ __launch_bounds__(256) void k_apply_op(TraceParams P, BlockDev Bin, BlockDev Bout, int f, int dagger,
                                                  int n_vec, const double* x, double* y) {
  __shared__ PathTables tables;
  path_tables_load<256>(P, tables);
  const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= int64_t(n_vec) * Bout.dim) return;
  const int v = int(id / Bout.dim), r = int(id - int64_t(v) * Bout.dim);
  y[id] = gather_tab<double>(tables, P.n_orb, Bin, Bout, r, f, dagger, x + int64_t(v) * Bin.dim);
}

// Krylov propagation of a batch of vectors of one block (parity hook): one
// workgroup per vector, same engine as the trace kernel.
template <typename VT, int NT, int RPT, int MAXM, bool MF, bool VL, int OCC>
__global__ __launch_bounds__(NT, OCC) void k_propagate(TraceParams P, int block, const VT* x, const double* dtau,
                                                       VT* y, double* log_scale, int32_t* steps_out) {
  using E = PathEngine<VT, NT, RPT, MAXM, MF, VL>;
  __shared__ typename E::Smem S;
  E eng(P, S);
  const BlockDev B = P.blocks[block];
  const int v = blockIdx.x;
  VT xr[RPT];
  double part = 0.0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = eng.row(k);
    xr[k] = (r < B.dim) ? x[int64_t(v) * B.dim + r] : VT(0);
    part += to_d(xr[k]) * to_d(xr[k]);
  }
  const double n2 = eng.block_sum1(part);
  double ell = 0.5 * log(n2);
  const double inv = 1.0 / sqrt(n2);
#pragma unroll
  for (int k = 0; k < RPT; ++k) xr[k] = static_cast<VT>(to_d(xr[k]) * inv);
  int steps = 0, subs = 0;
  eng.work = 0;
  eng.nops_budget = 1;
  const bool ok = eng.propagate(B, dtau[v], xr, ell, steps, subs);
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = eng.row(k);
    if (r < B.dim) y[int64_t(v) * B.dim + r] = xr[k];
  }
  if (threadIdx.x == 0) {
    log_scale[v] = ok ? ell : NAN;
    if (steps_out) steps_out[v] = steps;
  }
}

// ---------------------------------------------------------------------------
// kernel variants
// ---------------------------------------------------------------------------

struct Variant {
  const char* name;
  int fp64;   // 1: float64 vectors, 0: float32 (mixed)
  int nt, rpt, maxm;
  int mf;     // 1: matrix-free rows (needs no off-diagonal matrix on the device)
  const void* init_fn;   // k_path_init
  const void* op_fn;     // k_path_op
  const void* step_fn;   // k_path_prop
  const void* final_fn;  // k_path_final
  const void* prop_fn;   // k_propagate (parity hook)
  const void* chunk_fn;  // k_path_chunk
};

// MF: matrix-free rows; VL: Krylov basis in LDS; OCC: workgroups per CU the compiler
// must leave register room for
#define VARIANT(VT, NT, RPT, MAXM, MF, VL, OCC, NAME)                                             \
  {NAME, sizeof(VT) == 8, NT, RPT, MAXM, MF, reinterpret_cast<const void*>(&k_path_init<VT, NT>),   \
   reinterpret_cast<const void*>(&k_path_op<VT, NT, RPT>),                                        \
   reinterpret_cast<const void*>(&k_path_prop<VT, NT, RPT, MAXM, MF, VL, OCC>),                   \
   reinterpret_cast<const void*>(&k_path_final<VT, NT, RPT>),                                     \
   reinterpret_cast<const void*>(&k_propagate<VT, NT, RPT, MAXM, MF, VL, OCC>),                   \
   reinterpret_cast<const void*>(&k_path_chunk<VT, NT, RPT, MAXM, MF, VL, OCC>)}

static const Variant kVariants[] = {
    VARIANT(double, 64, 1, 12, false, false, 2, "f64_nt64_r1_m12"),
    VARIANT(double, 64, 2, 12, false, false, 2, "f64_nt64_r2_m12"),
    VARIANT(double, 64, 2, 16, false, false, 1, "f64_nt64_r2_m16"),
    VARIANT(double, 128, 1, 12, false, false, 1, "f64_nt128_r1_m12"),
    VARIANT(double, 128, 4, 12, false, false, 1, "f64_nt128_r4_m12"),
    VARIANT(double, 256, 2, 12, false, false, 1, "f64_nt256_r2_m12"),
    VARIANT(double, 256, 5, 12, false, false, 1, "f64_nt256_r5_m12"),
    VARIANT(float, 64, 2, 12, false, false, 1, "f32_nt64_r2_m12"),
    VARIANT(float, 256, 5, 12, false, false, 1, "f32_nt256_r5_m12"),
    VARIANT(float, 256, 5, 16, false, false, 1, "f32_nt256_r5_m16"),
    VARIANT(float, 512, 3, 12, false, false, 1, "f32_nt512_r3_m12"),
    VARIANT(double, 64, 2, 12, true, false, 2, "f64_nt64_r2_m12_mf"),
    VARIANT(double, 256, 5, 12, true, false, 1, "f64_nt256_r5_m12_mf"),
    VARIANT(float, 64, 2, 12, true, false, 1, "f32_nt64_r2_m12_mf"),
    VARIANT(float, 256, 5, 12, true, false, 1, "f32_nt256_r5_m12_mf"),
    VARIANT(float, 64, 20, 8, false, true, 1, "f32_nt64_r20_m8_vl"),
    VARIANT(float, 64, 20, 8, true, true, 1, "f32_nt64_r20_m8_vl_mf"),
    VARIANT(double, 64, 2, 12, false, true, 2, "f64_nt64_r2_m12_vl"),
};
static const int kNumVariants = int(sizeof(kVariants) / sizeof(kVariants[0]));

// A variant fits a model of its precision whose largest block it holds; models
// stored matrix-free take the matrix-free variants only (the others read the
// off-diagonal matrix, which such a model does not keep on the device).
static bool variant_fits(const Variant& v, const hyb_model* m) {
  const int want_fp64 = (m->p.precision == HYB_FP64) ? 1 : 0;
  if (m->p.storage == HYB_MATRIX_FREE && !v.mf) return false;
  if (v.mf && m->n_orb > 7) return false;
  return v.fp64 == want_fp64 && v.nt * v.rpt >= m->max_dim;
}

// Automatic choice: the smallest workgroup that holds the largest block, with the
// Lanczos register depth that covers krylov_max when possible.
static int auto_variant(const hyb_model* m) {
  int best = -1;
  long best_cost = 0;
  for (int i = 0; i < kNumVariants; ++i) {
    const Variant& v = kVariants[i];
    if (!variant_fits(v, m)) continue;
    // CSR models prefer the variants that read the matrix (matrix-free ones are picked
    // by the autotuner when faster)
    const long mf_cost = (v.mf && m->p.storage == HYB_CSR) ? 100000L : 0;
    const long cost = long(v.nt) * v.rpt * 4 + (v.maxm >= m->p.krylov_max ? 0 : 1000000L) + v.maxm + mf_cost;
    if (best < 0 || cost < best_cost) {
      best = i;
      best_cost = cost;
    }
  }
  return best;
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

template <typename T>
static int dev_upload(T*& dst, const T* src, size_t n, hipStream_t s) {
  // an empty array gets a one-element placeholder and no copy
  HIP_TRY(hipMalloc(reinterpret_cast<void**>(&dst), std::max<size_t>(n, 1) * sizeof(T)));
  if (src && n) HIP_TRY(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, s));
  return 0;
}

void free_device(hyb_model* m) {
  matrix_release(m);
  if (!m || !m->uploaded) return;
  DeviceModel& d = m->dev;
  void* ptrs[] = {d.states, d.rank, d.rank_half, d.blocks, d.rowptr, d.col, d.val64, d.val32, d.diag64,
                  d.ell_col, d.ell_val32, d.ell_perm, d.ell_len, d.tell_col, d.tell_val64, d.tell_val32, d.ret_block, d.ret_energy, d.ret_off, d.ret_vec64, d.ret_vec32, d.ws};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (void*& e : m->events)
    if (e) {
      (void)hipEventDestroy(reinterpret_cast<hipEvent_t>(e));
      e = nullptr;
    }
  for (void* e : m->step_events) (void)hipEventDestroy(reinterpret_cast<hipEvent_t>(e));
  m->step_events.clear();
  d = DeviceModel{};
  m->uploaded = false;
}

static int ensure_ws(hyb_model* m, size_t bytes) {
  if (m->dev.ws_bytes >= bytes) return 0;
  if (m->dev.ws) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(m->dev.ws));
    m->dev.ws = nullptr;
    m->dev.ws_bytes = 0;
  }
  const size_t want = std::max(bytes, size_t(1) << 20);
  if (hipMalloc(&m->dev.ws, want) != hipSuccess) return set_error(HYB_E_OOM, "device workspace of %zu bytes", want);
  m->dev.ws_bytes = want;
  return 0;
}

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

static TraceParams base_params(const hyb_model* m) {
  TraceParams P{};
  const DeviceModel& d = m->dev;
  P.states = d.states;
  P.rank = d.rank;
  P.blocks = d.blocks;
  P.rowptr = d.rowptr;
  P.col = d.col;
  P.val64 = d.val64;
  P.val32 = d.val32;
  P.diag64 = d.diag64;
  P.ecol = d.tell_col;
  P.eval64 = d.tell_val64;
  P.eval32 = d.tell_val32;
  P.ek = m->tell_k;
  P.rank_half = d.rank_half;
  P.jsf = m->p.J_sf;
  P.jph = m->p.J_ph;
  P.ret_block = d.ret_block;
  P.ret_energy = d.ret_energy;
  P.ret_off = d.ret_off;
  P.ret_vec64 = d.ret_vec64;
  P.ret_vec32 = d.ret_vec32;
  P.n_orb = m->n_orb;
  P.n_ret = int32_t(m->ret_block.size());
  P.E0 = m->E0;
  P.tol = m->p.krylov_tol;
  P.kmax = m->p.krylov_max;
  P.max_substeps = 32;
  P.work_budget = 200000;
  P.zero_tol2 = (m->p.precision == HYB_FP64) ? 1e-20 : 1e-10;
  return P;
}

static int error_from_bits(int bits) {
  if (bits & ERR_UNSORTED) return set_error(HYB_E_UNSORTED, "operator times not strictly increasing in [0, beta)");
  if (bits & ERR_FLAVOR) return set_error(HYB_E_FLAVOR, "flavor or dagger out of range");
  if (bits & ERR_NONFINITE) return set_error(HYB_E_NONFINITE, "non-finite value in the propagation");
  if (bits & ERR_NOCONV) return set_error(HYB_E_NOCONV, "Krylov propagation exceeded the substep limit");
  return 0;
}

// ---------------------------------------------------------------------------
// device-resident launch (no host round trip)
// ---------------------------------------------------------------------------

namespace {
struct ResidentLayout {
  size_t cnt, work, pbucket, psign, plog, psteps, psub, prs, prw, srs, srw, sblock, sstatus, ssteps, ssubs, sell, midblk, svec,
      total;
};
ResidentLayout resident_layout(const hyb_model* m, int nc, size_t vbytes) {
  const int64_t npairs = int64_t(nc) * int64_t(m->ret_block.size());
  const int vstride = (m->max_dim + 63) & ~63;
  ResidentLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.cnt = take(COUNTERS_LEN * sizeof(int32_t));
  L.work = take(npairs * sizeof(int32_t));
  L.pbucket = take(npairs * sizeof(int32_t));
  L.psign = take(npairs * sizeof(int8_t));
  L.plog = take(npairs * sizeof(double));
  L.psteps = take(npairs * sizeof(int32_t));
  L.psub = take(npairs * sizeof(int32_t));
  L.prs = take(npairs * sizeof(int64_t));
  L.prw = take(npairs * sizeof(int64_t));
  L.srs = take(npairs * sizeof(int64_t));
  L.srw = take(npairs * sizeof(int64_t));
  L.sblock = take(npairs * sizeof(int32_t));
  L.sstatus = take(npairs * sizeof(int32_t));
  L.ssteps = take(npairs * sizeof(int32_t));
  L.ssubs = take(npairs * sizeof(int32_t));
  L.sell = take(npairs * sizeof(double));
  L.midblk = take(npairs * sizeof(int32_t));
  L.svec = take(2 * size_t(npairs) * vstride * vbytes);
  L.total = off;
  return L;
}
}  // namespace

size_t trace_ws_bytes(const hyb_model* m, int n_configs) {
  return resident_layout(m, n_configs, sizeof(double)).total;
}

// Workspace pointers of a device-resident launch for nc configurations at ws.
static TraceParams resident_params(const hyb_model* m, int nc, void* ws, size_t vbytes) {
  const ResidentLayout L = resident_layout(m, nc, vbytes);
  char* w = static_cast<char*>(ws);
  TraceParams P = base_params(m);
  P.n_configs = nc;
  P.n_pairs = int32_t(int64_t(nc) * int64_t(m->ret_block.size()));
  P.counters = reinterpret_cast<int32_t*>(w + L.cnt);
  P.work = reinterpret_cast<int32_t*>(w + L.work);
  P.p_bucket = reinterpret_cast<int32_t*>(w + L.pbucket);
  P.p_sign = reinterpret_cast<int8_t*>(w + L.psign);
  P.p_log = reinterpret_cast<double*>(w + L.plog);
  P.p_steps = reinterpret_cast<int32_t*>(w + L.psteps);
  P.p_sub = reinterpret_cast<int32_t*>(w + L.psub);
  P.p_rowsteps = reinterpret_cast<int64_t*>(w + L.prs);
  P.p_rows = reinterpret_cast<int64_t*>(w + L.prw);
  P.st_rowsteps = reinterpret_cast<int64_t*>(w + L.srs);
  P.st_rows = reinterpret_cast<int64_t*>(w + L.srw);
  P.st_block = reinterpret_cast<int32_t*>(w + L.sblock);
  P.st_status = reinterpret_cast<int32_t*>(w + L.sstatus);
  P.st_steps = reinterpret_cast<int32_t*>(w + L.ssteps);
  P.st_subs = reinterpret_cast<int32_t*>(w + L.ssubs);
  P.st_ell = reinterpret_cast<double*>(w + L.sell);
  P.st_vec = w + L.svec;
  P.vstride = (m->max_dim + 63) & ~63;
  P.p_midblk = reinterpret_cast<int32_t*>(w + L.midblk);
  return P;
}

// Scan, path kernels with grids sized for every (configuration, retained state)
// pair (workgroups past the queued paths return at once), then the signed log-sum.
// No host synchronisation; the counters are cleared by a kernel, so the sequence
// may be captured.  Optional outputs may be NULL.
static int resident_launch(const Variant& V, TraceParams& P, int max_ops, double* out_log, int8_t* out_sign,
                           int32_t* out_steps, int32_t* out_sub, int32_t* out_feas, int64_t* out_rs, int64_t* out_rw,
                           hipStream_t s) {
  const int64_t npairs = P.n_pairs;
  k_init_counters<<<1, 256, 0, s>>>(P.counters, COUNTERS_LEN);
  const int scan_threads = 256;
  k_scan<<<unsigned((npairs + scan_threads - 1) / scan_threads), scan_threads, 0, s>>>(P);
  if (npairs > 0) {
    k_order_base<<<1, ORDER_NB, 0, s>>>(P.counters);
    k_order_place<<<unsigned((npairs + 255) / 256), 256, 0, s>>>(P);
    int k0 = 0, k1 = max_ops;
    void* a0[] = {&P};
    void* ak[] = {&P, &k0, &k1};
    HIP_TRY(hipLaunchKernel(V.init_fn, dim3(unsigned(npairs)), dim3(V.nt), a0, 0, s));
    HIP_TRY(hipLaunchKernel(V.chunk_fn, dim3(unsigned(npairs)), dim3(V.nt), ak, 0, s));
    HIP_TRY(hipLaunchKernel(V.final_fn, dim3(unsigned(npairs)), dim3(V.nt), a0, 0, s));
  }
  k_reduce<<<(P.n_configs + 255) / 256, 256, 0, s>>>(P, out_log, out_sign, out_steps, out_sub, out_feas, out_rs, out_rw);
  HIP_TRY(hipGetLastError());
  return 0;
}

int trace_resident(hyb_model* m, int nc, const int64_t* begin, const int64_t* ends, const double* tau,
                   const int16_t* flavor, const int8_t* dagger, int max_ops, double beta, void* ws,
                   double* out_log, int8_t* out_sign, int32_t* err_accum, hipStream_t s) {
  const int vi = m->variant >= 0 ? m->variant : auto_variant(m);
  const Variant& V = kVariants[vi];
  TraceParams P = resident_params(m, nc, ws, V.fp64 ? sizeof(double) : sizeof(float));
  P.beta = beta;
  P.tau_mid = 0.5 * beta;
  P.offsets = begin;
  P.ends = ends;
  P.tau = tau;
  P.flavor = flavor;
  P.dagger = dagger;
  const int rc = resident_launch(V, P, max_ops, out_log, out_sign, nullptr, nullptr, nullptr, nullptr, nullptr, s);
  if (rc) return rc;
  k_fold_errors<<<1, 64, 0, s>>>(P.counters, err_accum);
  HIP_TRY(hipGetLastError());
  return 0;
}

// ---------------------------------------------------------------------------
// allocation-free entry point: the workspace is a file-scope device array
// ---------------------------------------------------------------------------

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
// Workspace of hyb_trace_batch_noalloc.  Host code never uses this name as an
// address: each device's copy is reached through the pointer hipGetSymbolAddress
// returned for it (scratch_ptr).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void* scratch_ptr[kMaxDevices] = {};
static std::mutex scratch_mu;

// Looks up the current device's copy of `scratch` once per device (the model
// upload calls it with the model's device current).
static int scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(HYB_E_STATE, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_ptr[dev]) return 0;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return set_error(HYB_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
  scratch_ptr[dev] = p;
  return 0;
}

static void* scratch_of(int dev) {
  std::lock_guard<std::mutex> lock(scratch_mu);
  return (dev >= 0 && dev < kMaxDevices) ? scratch_ptr[dev] : nullptr;
}

int trace_resident_variant(const hyb_model* m) { return m->variant >= 0 ? m->variant : auto_variant(m); }

ResidentPairs trace_resident_pairs(const hyb_model* m, int nc, void* ws) {
  const int vi = m->variant >= 0 ? m->variant : auto_variant(m);
  const ResidentLayout L = resident_layout(m, nc, kVariants[vi].fp64 ? sizeof(double) : sizeof(float));
  char* w = static_cast<char*>(ws);
  return {reinterpret_cast<const int8_t*>(w + L.psign), reinterpret_cast<const double*>(w + L.plog),
          reinterpret_cast<const int32_t*>(w + L.midblk)};
}

}  // namespace hyb

using namespace hyb;

extern "C" {

int hyb_model_upload(hyb_model* m, void* stream) {
  if (!m) return set_error(HYB_E_ARG, "NULL model");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  free_device(m);
  ++m->dev_gen;
  DeviceModel& d = m->dev;
  HIP_TRY(hipGetDevice(&d.device));
  int rc = 0;
  std::vector<double> diag_shifted(m->n_states);
  for (int b = 0; b < m->n_blocks; ++b)
    for (int i = 0; i < m->blocks[b].dim; ++i) {
      const int64_t g = m->blocks[b].state_off + i;
      diag_shifted[g] = m->diag[g] - m->blocks[b].shift;
    }
  std::vector<float> val32(m->val.begin(), m->val.end());
  std::vector<float> rv32(m->ret_vec.begin(), m->ret_vec.end());
  // ELL copy of each block's off-diagonal rows for the block SpMM: the row pairs
  // (2q, 2q + 1), which share a 128-byte line of a 16-vector panel, are kept together
  // and sorted by their longer row, descending (stable), so that a wavefront's rows
  // need about the same number of slots and each line of Y is written whole by two
  // neighbouring lanes.  ELL row i is row perm[i] of the block, slot k of ELL row i at
  // off + k * dim + i; short rows are padded with their own index and 0
  m->ell_k.assign(m->n_blocks, 0);
  m->ell_off.assign(m->n_blocks, 0);
  int64_t ell_total = 0;
  for (int b = 0; b < m->n_blocks; ++b) {
    const BlockDev& B = m->blocks[b];
    int kmax = 0;
    for (int r = 0; r < B.dim; ++r)
      kmax = std::max(kmax, m->rowptr[B.state_off + r + 1] - m->rowptr[B.state_off + r]);
    m->ell_k[b] = kmax;
    m->ell_off[b] = ell_total;
    ell_total += int64_t(kmax) * B.dim;
  }
  std::vector<int16_t> ell_col(std::max<int64_t>(ell_total, 1));
  std::vector<float> ell_val(std::max<int64_t>(ell_total, 1));
  std::vector<int16_t> ell_perm(std::max<int64_t>(m->n_states, 1)), ell_len(std::max<int64_t>(m->n_states, 1));
  for (int b = 0; b < m->n_blocks; ++b) {
    const BlockDev& B = m->blocks[b];
    auto len = [&](int r) { return m->rowptr[B.state_off + r + 1] - m->rowptr[B.state_off + r]; };
    // whole pairs first (so every pair starts at an even ELL row), the odd last row
    // of an odd-dimensional block after them
    std::vector<int> pairs(B.dim / 2);
    for (int q = 0; q < int(pairs.size()); ++q) pairs[q] = q;
    std::stable_sort(pairs.begin(), pairs.end(), [&](int x, int y) {
      return std::max(len(2 * x), len(2 * x + 1)) > std::max(len(2 * y), len(2 * y + 1));
    });
    std::vector<int> order;
    order.reserve(B.dim);
    for (int q : pairs) {
      order.push_back(2 * q);
      order.push_back(2 * q + 1);
    }
    if (B.dim % 2) order.push_back(B.dim - 1);
    for (int i = 0; i < B.dim; ++i) {
      const int r = order[i];
      const int g = B.state_off + r;
      const int n = len(r);
      ell_perm[B.state_off + i] = int16_t(r);
      ell_len[B.state_off + i] = int16_t(n);
      for (int k = 0; k < m->ell_k[b]; ++k) {
        const int64_t at = m->ell_off[b] + int64_t(k) * B.dim + i;
        ell_col[at] = int16_t(k < n ? m->col[m->rowptr[g] + k] : r);
        ell_val[at] = k < n ? float(m->val[m->rowptr[g] + k]) : 0.0f;
      }
    }
  }
  // natural-order ELL for the trace kernels (padding: own index, value 0)
  int kt = 0;
  for (int g = 0; g < m->n_states; ++g) kt = std::max(kt, m->rowptr[g + 1] - m->rowptr[g]);
  m->tell_k = kt;
  const int64_t tell_total = std::max<int64_t>(int64_t(kt) * m->n_states, 1);
  std::vector<int16_t> tell_col(tell_total, 0);
  std::vector<double> tell_val(tell_total, 0.0);
  std::vector<float> tell_val32(tell_total, 0.0f);
  for (int b = 0; b < m->n_blocks; ++b) {
    const BlockDev& B = m->blocks[b];
    for (int r = 0; r < B.dim; ++r) {
      const int g = B.state_off + r, n = m->rowptr[g + 1] - m->rowptr[g];
      for (int k = 0; k < kt; ++k) {
        const int64_t at = int64_t(B.state_off) * kt + int64_t(k) * B.dim + r;
        tell_col[at] = int16_t(k < n ? m->col[m->rowptr[g] + k] : r);
        tell_val[at] = k < n ? m->val[m->rowptr[g] + k] : 0.0;
        tell_val32[at] = float(tell_val[at]);
      }
    }
  }
  m->uploaded = true;  // so that free_device releases partial uploads
  if ((rc = dev_upload(d.states, m->states.data(), m->states.size(), s))) return rc;
  if ((rc = dev_upload(d.rank, m->rank.data(), m->rank.size(), s))) return rc;
  if ((rc = dev_upload(d.rank_half, m->rank_half.data(), m->rank_half.size(), s))) return rc;
  // spectral width of every block (exact from the host spectrum, else a Gershgorin
  // bound): the scan's cost estimate for ordering the path queue
  for (int b = 0; b < m->n_blocks; ++b) {
    BlockDev& B = m->blocks[b];
    double w = 0.0;
    if (!m->evals.empty() && !m->evals[b].empty()) {
      w = m->evals[b].back() - m->evals[b].front();
    } else if (B.dim > 0) {
      double lo = INFINITY, hi = -INFINITY;
      for (int i = 0; i < B.dim; ++i) {
        const int64_t g = B.state_off + i;
        double r = 0.0;
        for (int j = m->rowptr[g]; j < m->rowptr[g + 1]; ++j) r += std::fabs(m->val[j]);
        lo = std::min(lo, m->diag[g] - r);
        hi = std::max(hi, m->diag[g] + r);
      }
      w = hi - lo;
    }
    B.width = float(w);
  }
  if ((rc = dev_upload(d.blocks, m->blocks.data(), m->blocks.size(), s))) return rc;
  // the off-diagonal matrix (CSR and both ELL copies) only for CSR storage; a
  // matrix-free model keeps one-element placeholders
  const bool keep = m->p.storage == HYB_CSR;
  auto up_matrix = [&](auto*& dst, const auto& v) {
    return dev_upload(dst, keep ? v.data() : nullptr, keep ? v.size() : size_t(0), s);
  };
  if ((rc = up_matrix(d.rowptr, m->rowptr))) return rc;
  if ((rc = up_matrix(d.col, m->col))) return rc;
  if ((rc = up_matrix(d.val64, m->val))) return rc;
  if ((rc = up_matrix(d.val32, val32))) return rc;
  if ((rc = dev_upload(d.diag64, diag_shifted.data(), diag_shifted.size(), s))) return rc;
  if ((rc = up_matrix(d.ell_col, ell_col))) return rc;
  if ((rc = up_matrix(d.ell_val32, ell_val))) return rc;
  if ((rc = up_matrix(d.ell_perm, ell_perm))) return rc;
  if ((rc = up_matrix(d.ell_len, ell_len))) return rc;
  if ((rc = up_matrix(d.tell_col, tell_col))) return rc;
  if ((rc = up_matrix(d.tell_val64, tell_val))) return rc;
  if ((rc = up_matrix(d.tell_val32, tell_val32))) return rc;
  if ((rc = dev_upload(d.ret_block, m->ret_block.data(), m->ret_block.size(), s))) return rc;
  if ((rc = dev_upload(d.ret_energy, m->ret_energy.data(), m->ret_energy.size(), s))) return rc;
  if ((rc = dev_upload(d.ret_off, m->ret_off.data(), m->ret_off.size(), s))) return rc;
  if ((rc = dev_upload(d.ret_vec64, m->ret_vec.data(), m->ret_vec.size(), s))) return rc;
  if ((rc = dev_upload(d.ret_vec32, rv32.data(), rv32.size(), s))) return rc;
  // host staging vectors above are pageable: make sure the copies finished
  HIP_TRY(hipStreamSynchronize(s));
  for (void*& e : m->events) HIP_TRY(hipEventCreate(reinterpret_cast<hipEvent_t*>(&e)));
  if ((rc = scratch_init(d.device))) return rc;
  if (m->variant < 0 && auto_variant(m) < 0)
    return set_error(HYB_E_ARG, "no trace kernel variant holds blocks of dimension %d", m->max_dim);
  return HYB_OK;
}

int hyb_build_hloc(const hyb_model_params* p, void* stream, hyb_model** out) {
  int rc = hyb_model_create(p, out);
  if (rc) return rc;
  rc = hyb_model_upload(*out, stream);
  if (rc) {
    hyb_model_destroy(*out);
    *out = nullptr;
  }
  return rc;
}

int hyb_trace_variant_count(int32_t* n) {
  if (!n) return set_error(HYB_E_ARG, "NULL argument");
  *n = kNumVariants;
  return HYB_OK;
}

int hyb_trace_variant_name(int32_t v, char* buf, size_t len) {
  if (v < 0 || v >= kNumVariants || !buf || len == 0) return set_error(HYB_E_ARG, "bad variant / buffer");
  std::snprintf(buf, len, "%s", kVariants[v].name);
  return HYB_OK;
}

int hyb_set_trace_variant(hyb_model* m, int32_t v) {
  if (!m) return set_error(HYB_E_ARG, "NULL model");
  if (v < 0) {
    m->variant = -1;
    return HYB_OK;
  }
  if (v >= kNumVariants) return set_error(HYB_E_ARG, "unknown variant %d", v);
  if (!variant_fits(kVariants[v], m))
    return set_error(HYB_E_ARG, "variant %s does not fit this model (precision / block size)", kVariants[v].name);
  m->variant = v;
  return HYB_OK;
}

int hyb_get_trace_variant(const hyb_model* m, int32_t* v) {
  if (!m || !v) return set_error(HYB_E_ARG, "NULL argument");
  *v = m->variant >= 0 ? m->variant : auto_variant(m);
  return HYB_OK;
}

int hyb_set_chunk(hyb_model* m, int32_t chunk) {
  if (!m) return set_error(HYB_E_ARG, "NULL model");
  if (chunk < 0) return set_error(HYB_E_ARG, "chunk must be >= 0");
  m->chunk = chunk == 0 ? (1 << 30) : chunk;
  return HYB_OK;
}

int hyb_get_chunk(const hyb_model* m, int32_t* chunk) {
  if (!m || !chunk) return set_error(HYB_E_ARG, "NULL argument");
  *chunk = m->chunk;
  return HYB_OK;
}

int hyb_set_timing(hyb_model* m, int32_t on) {
  if (!m) return set_error(HYB_E_ARG, "NULL model");
  m->timing = on != 0;
  return HYB_OK;
}

int hyb_last_timing(const hyb_model* m, float* ms) {
  if (!m || !ms) return set_error(HYB_E_ARG, "NULL argument");
  std::memcpy(ms, m->last_ms, sizeof m->last_ms);
  return HYB_OK;
}

int hyb_trace_batch(hyb_model* m, const hyb_config_batch* cfg, double beta, hyb_trace_out* out, void* stream) {
  if (!m || !cfg || !out) return set_error(HYB_E_ARG, "NULL argument");
  if (!m->uploaded) return set_error(HYB_E_STATE, "model not uploaded to a device");
  if (int rc0 = require_spectrum(m)) return rc0;
  if (!(beta > 0.0) || !std::isfinite(beta)) return set_error(HYB_E_ARG, "beta must be positive and finite");
  if (cfg->n_configs < 0) return set_error(HYB_E_ARG, "negative n_configs");
  if (cfg->n_configs == 0) return HYB_OK;
  if (!cfg->offsets || !out->log_abs || !out->sign) return set_error(HYB_E_ARG, "NULL array");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != m->dev.device) return set_error(HYB_E_STATE, "model lives on device %d, current is %d", m->dev.device, dev);
  const int vi = m->variant >= 0 ? m->variant : auto_variant(m);
  const Variant& V = kVariants[vi];
  const int nc = cfg->n_configs;
  const int n_ret = int(m->ret_block.size());
  const int64_t npairs = int64_t(nc) * n_ret;
  if (npairs > (int64_t(1) << 31) - 1) return set_error(HYB_E_ARG, "too many (config, state) pairs");

  // host configs: their size is needed for staging
  int64_t n_ops = 0;
  if (!cfg->on_device) {
    if (cfg->offsets[0] != 0) return set_error(HYB_E_ARG, "offsets must start at 0");
    for (int c = 0; c < nc; ++c)
      if (cfg->offsets[c + 1] < cfg->offsets[c]) return set_error(HYB_E_ARG, "offsets must not decrease");
    n_ops = cfg->offsets[nc];
  }
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t o_cnt = take(COUNTERS_LEN * sizeof(int32_t));
  const size_t o_work = take(npairs * sizeof(int32_t));
  const size_t o_pbucket = take(npairs * sizeof(int32_t));
  const size_t o_psign = take(npairs * sizeof(int8_t));
  const size_t o_plog = take(npairs * sizeof(double));
  const size_t o_psteps = take(npairs * sizeof(int32_t));
  const size_t o_psub = take(npairs * sizeof(int32_t));
  const size_t o_prs = take(npairs * sizeof(int64_t));
  const size_t o_prw = take(npairs * sizeof(int64_t));
  const size_t o_srs = take(npairs * sizeof(int64_t));
  const size_t o_srw = take(npairs * sizeof(int64_t));
  size_t o_offs = 0, o_tau = 0, o_fl = 0, o_dg = 0;
  if (!cfg->on_device) {
    o_offs = take((nc + 1) * sizeof(int64_t));
    o_tau = take(std::max<int64_t>(n_ops, 1) * sizeof(double));
    o_fl = take(std::max<int64_t>(n_ops, 1) * sizeof(int16_t));
    o_dg = take(std::max<int64_t>(n_ops, 1) * sizeof(int8_t));
  }
  const size_t vbytes = V.fp64 ? sizeof(double) : sizeof(float);
  const int vstride = (m->max_dim + 63) & ~63;
  const size_t o_sblock = take(npairs * sizeof(int32_t));
  const size_t o_sstatus = take(npairs * sizeof(int32_t));
  const size_t o_ssteps = take(npairs * sizeof(int32_t));
  const size_t o_ssubs = take(npairs * sizeof(int32_t));
  const size_t o_sell = take(npairs * sizeof(double));
  const size_t o_svec = take(2 * size_t(npairs) * vstride * vbytes);
  size_t o_olog = 0, o_osign = 0, o_osteps = 0, o_osub = 0, o_ofeas = 0, o_ors = 0, o_orw = 0;
  if (!out->on_device) {
    o_olog = take(nc * sizeof(double));
    o_osign = take(nc * sizeof(int8_t));
    o_osteps = take(nc * sizeof(int32_t));
    o_osub = take(nc * sizeof(int32_t));
    o_ofeas = take(nc * sizeof(int32_t));
    o_ors = take(nc * sizeof(int64_t));
    o_orw = take(nc * sizeof(int64_t));
  }
  int rc = ensure_ws(m, off);
  if (rc) return rc;
  char* ws = static_cast<char*>(m->dev.ws);

  TraceParams P = base_params(m);
  P.n_configs = nc;
  P.n_pairs = int32_t(npairs);
  P.beta = beta;
  P.counters = reinterpret_cast<int32_t*>(ws + o_cnt);
  P.work = reinterpret_cast<int32_t*>(ws + o_work);
  P.p_bucket = reinterpret_cast<int32_t*>(ws + o_pbucket);
  P.p_sign = reinterpret_cast<int8_t*>(ws + o_psign);
  P.p_log = reinterpret_cast<double*>(ws + o_plog);
  P.p_steps = reinterpret_cast<int32_t*>(ws + o_psteps);
  P.p_sub = reinterpret_cast<int32_t*>(ws + o_psub);
  P.st_block = reinterpret_cast<int32_t*>(ws + o_sblock);
  P.st_status = reinterpret_cast<int32_t*>(ws + o_sstatus);
  P.st_steps = reinterpret_cast<int32_t*>(ws + o_ssteps);
  P.st_subs = reinterpret_cast<int32_t*>(ws + o_ssubs);
  P.st_ell = reinterpret_cast<double*>(ws + o_sell);
  P.st_rowsteps = reinterpret_cast<int64_t*>(ws + o_srs);
  P.st_rows = reinterpret_cast<int64_t*>(ws + o_srw);
  P.p_rowsteps = reinterpret_cast<int64_t*>(ws + o_prs);
  P.p_rows = reinterpret_cast<int64_t*>(ws + o_prw);
  P.st_vec = ws + o_svec;
  P.vstride = vstride;
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
    HIP_TRY(hipMemcpyAsync(const_cast<int64_t*>(P.offsets), cfg->offsets, (nc + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    if (n_ops > 0) {
      if (!cfg->tau || !cfg->flavor || !cfg->dagger) return set_error(HYB_E_ARG, "NULL operator array");
      HIP_TRY(hipMemcpyAsync(const_cast<double*>(P.tau), cfg->tau, n_ops * sizeof(double), hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(const_cast<int16_t*>(P.flavor), cfg->flavor, n_ops * sizeof(int16_t),
                             hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(const_cast<int8_t*>(P.dagger), cfg->dagger, n_ops * sizeof(int8_t),
                             hipMemcpyHostToDevice, s));
    }
  }
  double* d_log = out->on_device ? out->log_abs : reinterpret_cast<double*>(ws + o_olog);
  int8_t* d_sign = out->on_device ? out->sign : reinterpret_cast<int8_t*>(ws + o_osign);
  int32_t* d_steps = out->on_device ? out->krylov_steps : reinterpret_cast<int32_t*>(ws + o_osteps);
  int32_t* d_sub = out->on_device ? out->substeps : reinterpret_cast<int32_t*>(ws + o_osub);
  int32_t* d_feas = out->on_device ? out->feasible_paths : reinterpret_cast<int32_t*>(ws + o_ofeas);
  int64_t* d_rs = out->on_device ? out->rowsteps : reinterpret_cast<int64_t*>(ws + o_ors);
  int64_t* d_rw = out->on_device ? out->rows : reinterpret_cast<int64_t*>(ws + o_orw);

  hipEvent_t ev[4];
  for (int i = 0; i < 4; ++i) ev[i] = reinterpret_cast<hipEvent_t>(m->events[i]);
  k_init_counters<<<1, 256, 0, s>>>(P.counters, COUNTERS_LEN);
  if (m->timing) HIP_TRY(hipEventRecord(ev[0], s));
  const int scan_threads = 256;
  k_scan<<<unsigned((npairs + scan_threads - 1) / scan_threads), scan_threads, 0, s>>>(P);
  if (npairs > 0) {
    k_order_base<<<1, ORDER_NB, 0, s>>>(P.counters);
    k_order_place<<<unsigned((npairs + 255) / 256), 256, 0, s>>>(P);
  }
  HIP_TRY(hipGetLastError());
  // queued paths, longest configuration and validation errors
  int32_t cnt[3] = {0, 0, 0};
  HIP_TRY(hipMemcpyAsync(cnt, P.counters, sizeof cnt, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (cnt[2]) return error_from_bits(cnt[2]);
  const int nwork = cnt[0], max_ops = cnt[1];
  if (nwork < 0 || nwork > npairs) return set_error(HYB_E_HIP, "corrupt path queue (%d)", nwork);
  if (m->timing) HIP_TRY(hipEventRecord(ev[1], s));
  if (nwork > 0) {
    void* a0[] = {&P};
    HIP_TRY(hipLaunchKernel(V.init_fn, dim3(unsigned(nwork)), dim3(V.nt), a0, 0, s));
    const size_t need_ev = m->timing ? size_t(4) * max_ops : 0;
    while (m->step_events.size() < need_ev) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      m->step_events.push_back(e);
    }
    auto ev_at = [&](size_t i) { return reinterpret_cast<hipEvent_t>(m->step_events[i]); };
    if (m->chunk <= 1) {
      for (int k = 0; k < max_ops; ++k) {
        void* ak[] = {&P, &k};
        if (k > 0) {
          if (m->timing) HIP_TRY(hipEventRecord(ev_at(4 * k), s));
          HIP_TRY(hipLaunchKernel(V.step_fn, dim3(unsigned(nwork)), dim3(V.nt), ak, 0, s));
          if (m->timing) HIP_TRY(hipEventRecord(ev_at(4 * k + 1), s));
        }
        if (m->timing) HIP_TRY(hipEventRecord(ev_at(4 * k + 2), s));
        HIP_TRY(hipLaunchKernel(V.op_fn, dim3(unsigned(nwork)), dim3(V.nt), ak, 0, s));
        if (m->timing) HIP_TRY(hipEventRecord(ev_at(4 * k + 3), s));
      }
    } else {
      // chunks of operators per launch; the events bracket whole chunks (reported
      // as propagation time: the chunk kernel spends nearly all of it there)
      int c = 0;
      for (int k0 = 0; k0 < max_ops; k0 += m->chunk, ++c) {
        int k1 = std::min(max_ops, k0 + m->chunk);
        void* ak[] = {&P, &k0, &k1};
        if (m->timing) HIP_TRY(hipEventRecord(ev_at(4 * c), s));
        HIP_TRY(hipLaunchKernel(V.chunk_fn, dim3(unsigned(nwork)), dim3(V.nt), ak, 0, s));
        if (m->timing) HIP_TRY(hipEventRecord(ev_at(4 * c + 1), s));
      }
    }
    HIP_TRY(hipLaunchKernel(V.final_fn, dim3(unsigned(nwork)), dim3(V.nt), a0, 0, s));
  }
  if (m->timing) HIP_TRY(hipEventRecord(ev[2], s));
  k_reduce<<<(nc + 255) / 256, 256, 0, s>>>(P, d_log, d_sign, d_steps, d_sub, d_feas, d_rs, d_rw);
  if (m->timing) HIP_TRY(hipEventRecord(ev[3], s));
  HIP_TRY(hipGetLastError());
  int32_t flags = 0;
  HIP_TRY(hipMemcpyAsync(&flags, P.counters + 2, sizeof flags, hipMemcpyDeviceToHost, s));
  if (!out->on_device) {
    HIP_TRY(hipMemcpyAsync(out->log_abs, d_log, nc * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(out->sign, d_sign, nc * sizeof(int8_t), hipMemcpyDeviceToHost, s));
    if (out->krylov_steps)
      HIP_TRY(hipMemcpyAsync(out->krylov_steps, d_steps, nc * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (out->substeps) HIP_TRY(hipMemcpyAsync(out->substeps, d_sub, nc * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (out->feasible_paths)
      HIP_TRY(hipMemcpyAsync(out->feasible_paths, d_feas, nc * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (out->rowsteps) HIP_TRY(hipMemcpyAsync(out->rowsteps, d_rs, nc * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (out->rows) HIP_TRY(hipMemcpyAsync(out->rows, d_rw, nc * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (m->timing) {
    HIP_TRY(hipEventElapsedTime(&m->last_ms[0], ev[0], ev[1]));
    HIP_TRY(hipEventElapsedTime(&m->last_ms[1], ev[1], ev[2]));
    HIP_TRY(hipEventElapsedTime(&m->last_ms[2], ev[2], ev[3]));
    float prop = 0.f, op = 0.f;
    int nprop = 0, nop = 0;
    if (nwork > 0 && m->chunk > 1) {
      for (int c = 0, k0 = 0; k0 < max_ops; k0 += m->chunk, ++c) {
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, reinterpret_cast<hipEvent_t>(m->step_events[4 * c]),
                                    reinterpret_cast<hipEvent_t>(m->step_events[4 * c + 1])));
        prop += t;
        ++nprop;
      }
    } else if (nwork > 0)
      for (int k = 0; k < max_ops; ++k) {
        float t = 0.f;
        if (k > 0) {
          HIP_TRY(hipEventElapsedTime(&t, reinterpret_cast<hipEvent_t>(m->step_events[4 * k]),
                                      reinterpret_cast<hipEvent_t>(m->step_events[4 * k + 1])));
          prop += t;
          ++nprop;
        }
        HIP_TRY(hipEventElapsedTime(&t, reinterpret_cast<hipEvent_t>(m->step_events[4 * k + 2]),
                                    reinterpret_cast<hipEvent_t>(m->step_events[4 * k + 3])));
        op += t;
        ++nop;
      }
    m->last_ms[3] = prop;
    m->last_ms[4] = float(nprop);
    m->last_ms[5] = op;
    m->last_ms[6] = float(nop);
  }
  return error_from_bits(flags);
}

int hyb_trace_batch_noalloc(hyb_model* m, const hyb_config_batch* cfg, double beta, hyb_trace_out* out,
                            void* stream) {
  if (!m || !cfg || !out) return set_error(HYB_E_ARG, "NULL argument");
  if (!m->uploaded) return set_error(HYB_E_STATE, "model not uploaded to a device");
  if (int rc0 = require_spectrum(m)) return rc0;
  if (!(beta > 0.0) || !std::isfinite(beta)) return set_error(HYB_E_ARG, "beta must be positive and finite");
  if (cfg->n_configs < 0) return set_error(HYB_E_ARG, "negative n_configs");
  if (cfg->n_configs == 0) return HYB_OK;
  if (!cfg->on_device || !out->on_device)
    return set_error(HYB_E_ARG, "hyb_trace_batch_noalloc takes device inputs and outputs only");
  if (!cfg->offsets || !cfg->tau || !cfg->flavor || !cfg->dagger || !out->log_abs || !out->sign)
    return set_error(HYB_E_ARG, "NULL array");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != m->dev.device) return set_error(HYB_E_STATE, "model lives on device %d, current is %d", m->dev.device, dev);
  void* ws = scratch_of(dev);
  if (!ws) return set_error(HYB_E_STATE, "scratch of device %d not initialised (upload the model first)", dev);
  const int vi = m->variant >= 0 ? m->variant : auto_variant(m);
  const Variant& V = kVariants[vi];
  const int nc = cfg->n_configs;
  const int64_t npairs = int64_t(nc) * int64_t(m->ret_block.size());
  if (npairs > (int64_t(1) << 31) - 1) return set_error(HYB_E_ARG, "too many (config, state) pairs");
  const size_t vbytes = V.fp64 ? sizeof(double) : sizeof(float);
  const size_t need = resident_layout(m, nc, vbytes).total;
  if (need > kScratchBytes) {
    const size_t per = resident_layout(m, 1, vbytes).total;
    return set_error(HYB_E_ARG, "%d configurations need %zu bytes of scratch; the maximum is %zu (about %zu "
                     "configurations of this model)", nc, need, kScratchBytes, kScratchBytes / std::max<size_t>(per, 1));
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  TraceParams P = resident_params(m, nc, ws, vbytes);
  P.beta = beta;
  P.tau_mid = 0.5 * beta;
  P.offsets = cfg->offsets;
  P.ends = nullptr;
  P.tau = cfg->tau;
  P.flavor = cfg->flavor;
  P.dagger = cfg->dagger;
  // every path stops at its own last operator
  const int rc = resident_launch(V, P, 1 << 30, out->log_abs, out->sign, out->krylov_steps, out->substeps,
                                 out->feasible_paths, out->rowsteps, out->rows, s);
  if (rc) return rc;
  int32_t flags = 0;
  HIP_TRY(hipMemcpyAsync(&flags, P.counters + 2, sizeof flags, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return error_from_bits(flags);
}

int hyb_apply_op_device(hyb_model* m, int32_t f, int32_t dagger, int32_t bin, int32_t n_vec, const double* x,
                        double* y, int32_t* bout, void* stream) {
  if (!m || !x || !y || !bout) return set_error(HYB_E_ARG, "NULL argument");
  if (!m->uploaded) return set_error(HYB_E_STATE, "model not uploaded");
  if (f < 0 || f >= m->F || (dagger != 0 && dagger != 1)) return set_error(HYB_E_FLAVOR, "bad operator");
  if (bin < 0 || bin >= m->n_blocks || n_vec < 0) return set_error(HYB_E_ARG, "bad block / count");
  const BlockDev& B = m->blocks[bin];
  int nu = B.n_up, nd = B.n_dn;
  if (f < m->n_orb) nu += dagger ? 1 : -1; else nd += dagger ? 1 : -1;
  if (nu < 0 || nu > m->n_orb || nd < 0 || nd > m->n_orb) {
    *bout = -1;
    return HYB_OK;
  }
  const int bt = nd * (m->n_orb + 1) + nu;
  *bout = bt;
  const int64_t total = int64_t(n_vec) * m->blocks[bt].dim;
  if (total == 0) return HYB_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const TraceParams P = base_params(m);
  k_apply_op<<<unsigned((total + 255) / 256), 256, 0, s>>>(P, B, m->blocks[bt], f, dagger, n_vec, x, y);
  HIP_TRY(hipGetLastError());
  return HYB_OK;
}

int hyb_propagate_device(hyb_model* m, int32_t block, int32_t n_vec, const void* x, const double* dtau, void* y,
                         double* log_scale, int32_t* steps, void* stream) {
  if (!m || !x || !dtau || !y || !log_scale) return set_error(HYB_E_ARG, "NULL argument");
  if (!m->uploaded) return set_error(HYB_E_STATE, "model not uploaded");
  if (int rc0 = require_spectrum(m)) return rc0;
  if (block < 0 || block >= m->n_blocks || n_vec < 0) return set_error(HYB_E_ARG, "bad block / count");
  if (m->blocks[block].dim == 0 || n_vec == 0) return HYB_OK;
  const int vi = m->variant >= 0 ? m->variant : auto_variant(m);
  const Variant& V = kVariants[vi];
  int rc = ensure_ws(m, 256);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  TraceParams P = base_params(m);
  P.counters = static_cast<int32_t*>(m->dev.ws);
  k_init_counters<<<1, 64, 0, s>>>(P.counters, 4);
  void* args[] = {&P, &block, (void*)&x, (void*)&dtau, &y, &log_scale, &steps};
  HIP_TRY(hipLaunchKernel(V.prop_fn, dim3(unsigned(n_vec)), dim3(V.nt), args, 0, s));
  int32_t flags = 0;
  HIP_TRY(hipMemcpyAsync(&flags, P.counters + 2, sizeof flags, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return error_from_bits(flags);
}

}  // extern "C"
