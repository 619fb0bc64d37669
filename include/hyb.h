/*
 * hyb.h -- C ABI of the MI355X (gfx950) Krylov hybridization-expansion trace library.
 *
 * Method: Laeuchli & Werner, "Krylov-implementation of the hybridization
 * expansion impurity solver and application to 5-orbital models"
 * (arXiv:0908.0681).  The library evaluates the truncated local trace of the
 * Monte Carlo weight, Eq.(2) (Sec. II),
 *
 *   Tr_R(c) = sum_{i in R} <E_i| e^{-(beta-tau_n) H} O_n e^{-(tau_n-tau_{n-1}) H} ... O_1 e^{-tau_1 H} |E_i>,
 *
 * in the occupation-number basis with sparse H_loc (Kanamori form, Eq.(4),
 * Sec. IV.A) and Krylov (Lanczos) time evolution (Sec. III, steps 3-8), summed
 * over the retained low-energy states R (truncation of type (i), Sec. II).
 *
 * General conventions
 *  - Every function returns an int status: HYB_OK (0) or a negative HYB_E_*
 *    code.  No C++ exception and no abort crosses this boundary.
 *    hyb_last_error() returns a thread-local human-readable message for the
 *    last failing call on the calling thread.
 *  - The caller owns every input and output buffer.  The library owns the
 *    opaque handles; each *_create / hyb_build_hloc has a matching destroy.
 *  - "stream" arguments are a hipStream_t passed as void* (NULL = the null
 *    stream).  Device work is enqueued on that stream.  Calls whose outputs are
 *    host memory synchronise that stream before returning.
 *  - Flavor f = a + n_orb * sigma (orbital a, sigma = 0 up / 1 down).  Bit f
 *    of a basis-state integer is the occupation of flavor f.  Fermion signs
 *    follow the Jordan-Wigner string in flavor order:
 *      c_f |s> = (-1)^{popcount(s & ((1<<f)-1))} |s ^ (1<<f)>  if bit f of s is set.
 *  - Blocks are the (n_up, n_dn) quantum-number sectors (Sec. II, quantum
 *    number ordering; Sec. IV.C orders them with n_up fastest):
 *      block = n_dn * (n_orb + 1) + n_up,
 *    and states inside a block are ordered by ascending state integer.
 */
#ifndef HYB_H
#define HYB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define HYB_OK            0
#define HYB_E_ARG        -1  /* invalid argument (NULL pointer, size or range) */
#define HYB_E_UNSORTED   -2  /* operator times not strictly increasing or outside [0, beta) */
#define HYB_E_FLAVOR     -3  /* flavor index outside [0, 2*n_orb) or dagger not 0/1 */
#define HYB_E_NOCONV     -4  /* Krylov propagation exceeded the substep limit */
#define HYB_E_NONFINITE  -5  /* NaN / Inf met in an input or intermediate */
#define HYB_E_HIP        -6  /* a HIP runtime call failed */
#define HYB_E_OOM        -7  /* host or device allocation failed */
#define HYB_E_STATE      -8  /* handle used in a state that does not allow the call */

/* ---- model --------------------------------------------------------------- */
#define HYB_CSR          0   /* H_loc blocks stored as CSR (and padded ELL copies) on the device */
#define HYB_MATRIX_FREE  1   /* no off-diagonal matrix on the device: the trace kernels generate the
                                spin-flip and pair-hopping entries of Eq.(4) of each row from its bit
                                pattern at every SpMV (hyb_block_spmm needs HYB_CSR) */
#define HYB_FP64         0   /* Krylov vectors, SpMV and recurrences in float64 */
#define HYB_MIXED        1   /* float32 Krylov vectors and off-diagonal SpMV with float32
                                accumulation; float64 diagonal, Lanczos alpha/beta,
                                re-orthogonalisation coefficients, tridiagonal exponential
                                and running log-norm */
#define HYB_SPECTRUM_HOST    0  /* hyb_model_create diagonalises every block on the host */
#define HYB_SPECTRUM_DEVICE  1  /* no host eigensolver: E0, the block shifts and the retained
                                   set come from hyb_init_lanczos on the device */

typedef struct {
  int32_t n_orb;          /* orbitals, 1..7 (F = 2*n_orb flavors <= 14) */
  const double* eps;      /* host [n_orb]: one-body energy of orbital a, -(mu + Delta_a) (Eq.(4)) */
  double U;               /* intra-orbital repulsion (Eq.(4)) */
  double Up;              /* inter-orbital opposite-spin repulsion U'; same spin gets Up - J */
  double J;               /* Hund coupling in the density-density part (Up - J) */
  double J_sf;            /* spin-flip amplitude (J in Eq.(4); 0 gives a density-density model) */
  double J_ph;            /* pair-hopping amplitude (J in Eq.(4)) */
  int32_t storage;        /* HYB_CSR or HYB_MATRIX_FREE */
  int32_t precision;      /* HYB_FP64 or HYB_MIXED */
  double retain_window;   /* retained set R = {E_i - E0 <= retain_window}; < 0: all states
                             (full trace).  Sec. III step 2, Sec. IV.C (energy window) */
  int32_t krylov_max;     /* Lanczos depth cap per (sub)interval, 2..20 (the tuned kernels
                             support 12, 16 and 20; the cap is rounded up to one of them
                             for register sizing but never exceeded) */
  double krylov_tol;      /* a-posteriori relative tolerance per (sub)interval:
                             beta_m |[exp(-dtau T_m)]_{m,1}| / ||exp(-dtau T_m) e_1|| <= tol.
                             Sec. III step 5 leaves the criterion open; this is the
                             Saad (1992) estimate.  Typical 1e-13 (FP64), 1e-7 (mixed). */
  int32_t spectrum;       /* HYB_SPECTRUM_HOST (0, the default of a zeroed struct) or
                             HYB_SPECTRUM_DEVICE.  Sec. III step 1: full diagonalisation,
                             or the lowest states by band Lanczos */
} hyb_model_params;

typedef struct hyb_model hyb_model;

typedef struct {
  int32_t n_orb, n_flavors, n_blocks, max_dim, n_retained, precision;
  int64_t n_states, nnz_offdiag;
  double E0;              /* lowest eigenvalue of H_loc */
} hyb_model_info_t;

/* Builds the bit-encoded basis, the (n_up, n_dn) blocks, H_loc per block (Eq.(4)
 * with spin-flip and pair-hopping summed once per ordered orbital pair a != b),
 * the spectrum of every block by dense FP64 Householder tridiagonalisation and
 * implicit QR with Wilkinson shifts (Sec. III step 1, full diagonalisation), E0 and the retained set
 * (step 2).  With spectrum = HYB_SPECTRUM_DEVICE the eigensolver is skipped: E0 is NaN
 * and the retained set empty until hyb_init_lanczos, and every call that needs them
 * (traces, propagation, Monte Carlo, matrix formulation) returns HYB_E_STATE before.
 * Host memory only; no GPU is touched.  *out receives a new handle. */
int hyb_model_create(const hyb_model_params* p, hyb_model** out);

/* Copies the model (basis tables, CSR blocks, retained vectors) to the current
 * HIP device on `stream`, with two padded ELL copies of the off-diagonal rows: one
 * in natural row order for the trace kernels, one with rows sorted by length for
 * the block SpMM.  Must precede any device call on the model; the device copies
 * live until hyb_model_destroy. */
int hyb_model_upload(hyb_model* m, void* stream);

/* Device initialisation, Sec. III steps 1-2 by band Lanczos (for blocks too large to
 * diagonalise fully): for every (n_up, n_dn) block, a block Krylov space of H_b from
 * block_size pseudo-random start vectors, fully reorthogonalised (two Gram-Schmidt
 * passes per vector; a vector with no new direction is replaced by a fresh one), its
 * projection T diagonalised on the host.  Phase 1 takes every block to a converged
 * lowest Ritz value, which fixes E0; phase 2 continues the blocks that reach within
 * retain_window of E0 until every Ritz value up to E0 + retain_window and the first one
 * above it have residual ||H x - theta x|| <= tol * ||H_b|| (||H_b|| bounded by the
 * largest absolute row sum), or the space spans the block.  The Ritz vectors up to
 * E0 + retain_window become the retained set (Sec. IV.C: an energy window, which near
 * a level crossing holds the multiplets on both sides), E0 the smallest Ritz value,
 * each block's shift its lowest one; the device copies are then rewritten as by
 * hyb_model_upload (device pointers captured earlier, and a matrix formulation built
 * earlier, become stale).  Works for HYB_SPECTRUM_HOST models too (it replaces their
 * host retained set).  FP64 throughout: a custom SpMM kernel and rocBLAS DGEMM/DGEMV.
 * Degeneracy: block Krylov holds at most block_size copies of a level, so a retained
 * level found block_size times (space not spanning its block) is an HYB_E_ARG error;
 * choose block_size above the largest in-block multiplicity of a retained level.
 * steps / resid (host [n_blocks], may be NULL): block steps taken and the largest
 * residual among a block's retained pairs (its lowest pair for other blocks).
 * Errors: HYB_E_STATE (not uploaded, other device), HYB_E_ARG (retain_window < 0,
 * block_size outside 2..64, tol outside [1e-15, 1e-4], multiplicity), HYB_E_NOCONV,
 * HYB_E_OOM, HYB_E_HIP. */
int hyb_init_lanczos(hyb_model* m, int32_t block_size, double tol, int32_t* steps, double* resid,
                     void* stream);

/* hyb_model_create + hyb_model_upload. */
int hyb_build_hloc(const hyb_model_params* p, void* stream, hyb_model** out);

void hyb_model_destroy(hyb_model* m);

int hyb_model_info(const hyb_model* m, hyb_model_info_t* out);

/* Per-block data (host). dim / nnz_offdiag / e_min may be NULL.  e_min is the block's
 * lowest eigenvalue (HYB_SPECTRUM_DEVICE: its lowest Ritz value, NaN before
 * hyb_init_lanczos). */
int hyb_block_info(const hyb_model* m, int32_t block, int32_t* dim, int32_t* nnz_offdiag, double* e_min);

/* Block spectrum (host): e[0..dim) ascending eigenvalues of block `block`.  HYB_E_STATE
 * for a HYB_SPECTRUM_DEVICE model (only its retained levels are known). */
int hyb_block_eigenvalues(const hyb_model* m, int32_t block, double* e);

/* Basis parity hooks (host): state integer <-> (block, index in block). */
int hyb_basis_state(const hyb_model* m, int32_t block, int32_t idx, uint32_t* bits);
int hyb_basis_index(const hyb_model* m, uint32_t bits, int32_t* block, int32_t* idx);

/* Dense copy of H_loc restricted to a block (host), row-major dim x dim. */
int hyb_block_dense(const hyb_model* m, int32_t block, double* h);

/* Retained set (host). block[n_retained], energy[n_retained]; vec (optional) receives
 * the eigenvectors concatenated in retained order, each of its block's dim. */
int hyb_retained(const hyb_model* m, int32_t* block, double* energy, double* vec);

/* Host reference application of c_f (dagger = 0) or c_f^dag (dagger = 1) to a
 * vector x of block block_in (Sec. III, operator application).  *block_out gets
 * the target block or -1 if the operator leaves the physical range (then y is
 * untouched).  y has the target block's dimension. */
int hyb_apply_op(const hyb_model* m, int32_t flavor, int32_t dagger, int32_t block_in,
                 const double* x, int32_t* block_out, double* y);

/* ---- device parity hooks --------------------------------------------------- */

/* Device operator application to n_vec vectors of block block_in, through the
 * same gather function (gather_tab: target states and source ranks from the
 * model's block and spin-pattern tables in LDS) that the whole-path trace kernel
 * applies at every operator of a path (Sec. III step 4).  x: device [n_vec][dim_in], y: device
 * [n_vec][dim_out].  Bit-exact: only sign flips and moves.  *block_out = -1 (and y
 * untouched) when the operator leaves the physical range. */
int hyb_apply_op_device(hyb_model* m, int32_t flavor, int32_t dagger, int32_t block_in,
                        int32_t n_vec, const double* x, double* y, int32_t* block_out, void* stream);

/* Device Krylov propagation (Sec. III step 5) of n_vec vectors of one block over
 * dtau[v] each:  y_v = exp(-dtau_v (H_b - E0)) x_v / s_v with log(s_v) in log_scale[v]
 * and the normalised result in y.  Lanczos steps used in steps[v] (may be NULL).
 * All pointers are device; x and y are [n_vec][dim] in the model's precision
 * (float64 for HYB_FP64, float32 for HYB_MIXED). */
int hyb_propagate_device(hyb_model* m, int32_t block, int32_t n_vec, const void* x,
                         const double* dtau, void* y, double* log_scale, int32_t* steps,
                         void* stream);

/* ---- the hot path: batched traces ----------------------------------------- */

typedef struct {
  int32_t n_configs;
  const int64_t* offsets; /* [n_configs + 1]; ops of config c are [offsets[c], offsets[c+1]) */
  const double* tau;      /* [n_ops] strictly increasing in [0, beta) inside a config */
  const int16_t* flavor;  /* [n_ops] */
  const int8_t* dagger;   /* [n_ops] 1 = creator c^dag, 0 = annihilator c */
  int32_t on_device;      /* 1: the five arrays are device pointers, 0: host */
} hyb_config_batch;

typedef struct {
  double* log_abs;        /* [n_configs] log|Tr_R| (includes -beta*E0); -inf when sign = 0 */
  int8_t* sign;           /* [n_configs] -1, 0, +1.  A zero trace is not an error. */
  int32_t* krylov_steps;  /* optional [n_configs]: Lanczos steps summed over the config's paths */
  int32_t* substeps;      /* optional [n_configs]: extra substeps forced by the depth cap */
  int32_t* feasible_paths;/* optional [n_configs]: retained states whose sector path stays physical */
  int64_t* rowsteps;      /* optional [n_configs]: sum over paths and intervals of (Lanczos steps x
                             block dimension), the vector traffic of the propagation */
  int64_t* rows;          /* optional [n_configs]: sum over paths and intervals of the block dimension */
  int32_t on_device;      /* 1: outputs are device pointers (no host sync), 0: host */
} hyb_trace_out;

/* Evaluates Tr_R for every configuration of the batch (Eq.(2) trace factor;
 * Sec. III steps 3-8): a scan finds the feasible (config, retained state)
 * paths, one workgroup per path then alternates Krylov propagation and operator
 * application with a running log-norm (all operators of a path in one launch by
 * default, see hyb_set_chunk), and a last kernel forms the signed log-sum over R
 * per config.  The returned value is the literal operator product in time order
 * (latest operator leftmost) without a time-ordering permutation sign.
 * Errors: HYB_E_UNSORTED / HYB_E_FLAVOR for bad configurations (checked on the
 * device; the call synchronises `stream` to read the check), HYB_E_NOCONV if a
 * propagation needs more than 32 substeps of the depth cap, HYB_E_NONFINITE for
 * NaN/Inf. */
int hyb_trace_batch(hyb_model* m, const hyb_config_batch* cfg, double beta,
                    hyb_trace_out* out, void* stream);

/* hyb_trace_batch for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * kernels and results as hyb_trace_batch (bitwise), launched with grids sized for
 * every (configuration, retained state) pair so that no host round trip sits
 * between the scan and the path kernels.  The workspace is a static device array
 * of 64 MiB per GPU (held from the model upload until the process ends); it holds
 * about 5,000 five-orbital FP64 or 800 seven-orbital mixed-precision
 * configurations.  No hipMalloc, hipFree or other allocation happens in the call.
 *  - cfg and out must be device pointers (on_device = 1 in both), else HYB_E_ARG.
 *  - A batch whose workspace exceeds the static array is refused with HYB_E_ARG
 *    (the message gives the bytes needed and the maximum).
 *  - Every call on one GPU uses that GPU's single array: calls that overlap on one
 *    GPU (several host threads or streams) race and must be serialised by the
 *    caller.  Counters are cleared by a kernel at the start of each call.
 *  - Returns after `stream` has drained (it reads the error flags); errors as
 *    hyb_trace_batch. */
int hyb_trace_batch_noalloc(hyb_model* m, const hyb_config_batch* cfg, double beta,
                            hyb_trace_out* out, void* stream);

/* Kernel tuning: which trace-kernel variant hyb_trace_batch launches.
 * variant < 0 restores the automatic choice. Returns HYB_E_ARG for an unknown id. */
int hyb_set_trace_variant(hyb_model* m, int32_t variant);
int hyb_get_trace_variant(const hyb_model* m, int32_t* variant);
/* Number of trace-kernel variants compiled in and a short name of each. */
int hyb_trace_variant_count(int32_t* n);
int hyb_trace_variant_name(int32_t variant, char* buf, size_t len);

/* Operators processed per launch of the path kernels: 1 launches one propagation
 * and one operator kernel per operator index; c > 1 launches one kernel that takes
 * every path through c operators (propagation + operator each); 0 = all operators
 * in one launch.  Results are identical; only the schedule changes. */
int hyb_set_chunk(hyb_model* m, int32_t chunk);
int hyb_get_chunk(const hyb_model* m, int32_t* chunk);

/* Device time of the last hyb_trace_batch (HIP events on the call's stream):
 * out[0] = scan, out[1] = all path-step launches, out[2] = reduce (ms),
 * out[3] = summed duration of the Krylov propagation launches (ms; with chunk > 1
 * the chunk launches, propagation and operators together),
 * out[4] = number of propagation launches, out[5] = summed duration of the
 * operator launches (ms), out[6] = number of operator launches.
 * Requires hyb_set_timing(m, 1) before the call. */
int hyb_set_timing(hyb_model* m, int32_t on);
int hyb_last_timing(const hyb_model* m, float* out7);

/* ---- the matrix formulation (the comparison path) ----------------------------- */

/* Builds the matrix formulation of Sec. II (Eq.(3)) on the model's device: every
 * block's full eigendecomposition (host, FP64, threads over blocks) and, for every
 * block b and operator c_f / c_f^dag with a physical target block t, the dense FP64
 * block U_t^T O U_b in the two eigenbases (one rocBLAS DGEMM per block on the
 * device).  Device memory: the sum of d_t d_b over those blocks, 8 bytes each
 * (2.3 GB at 7 orbitals); host time: the eigendecompositions.  Replaces an
 * earlier build; freed with the model.  Errors: HYB_E_STATE (model not uploaded),
 * HYB_E_OOM, HYB_E_HIP. */
int hyb_matrix_build(hyb_model* m, void* stream);

/* Device bytes of the operator blocks and the seconds the build took. */
int hyb_matrix_info(const hyb_model* m, int64_t* op_bytes, double* build_seconds);

/* Tr_R of every configuration by the matrix formulation: one workgroup per feasible
 * (configuration, retained state) path, each interval a diagonal scaling by
 * exp(-dtau (E_b - E0)) in the eigenbasis, each operator a dense product with its
 * eigenbasis block, renormalisation with a running log-norm, and the signed
 * log-sum over R.  Same arguments, outputs, zero rule (squared norm below 1e-20 of
 * a unit vector) and errors as hyb_trace_batch; krylov_steps and substeps are 0,
 * rowsteps counts the operator-block elements read and rows the target
 * dimensions.  FP64 whatever the model's precision.  HYB_E_STATE before
 * hyb_matrix_build or after a new hyb_model_upload. */
int hyb_trace_batch_matrix(hyb_model* m, const hyb_config_batch* cfg, double beta, hyb_trace_out* out,
                           void* stream);

/* ---- block SpMM over many vectors ------------------------------------------ */

/* Y = (H_b - c_b) X for n_vec float32 vectors of block b (c_b = lowest eigenvalue
 * of the block), the SpMV of the Krylov step applied to a panel of vectors.
 * Layout: X and Y are device float32 panels [n_vec / 16][dim][16]: 16 vectors are
 * interleaved per row and each panel is one contiguous dim*16 chunk, so a panel
 * streams from HBM in one pass.  n_vec must be a multiple of 16. */
int hyb_block_spmm(hyb_model* m, int32_t block, int64_t n_vec, const float* X, float* Y, void* stream);

/* ---- Monte Carlo sampling of the expansion (Sec. II) ------------------------ */

/* Weight of a configuration (Eq.(2) with a diagonal hybridization):
 *   w = s_perm * Tr_R(literal time-ordered product) * prod_f det A_f,
 *   A_f[i][j] = Delta(tau'_{f,i} - tau_{f,j}),
 * row i = i-th creator of flavor f, column j = its j-th annihilator (label order).
 * s_perm is the sign of the permutation taking the canonical string (flavor by
 * flavor, label by label: c_f(tau_{f,i}) c^dag_f(tau'_{f,i})) to descending time
 * order, i.e. the fermionic sign of the time-ordering operator.  Delta is given as a
 * table on a uniform grid of [0, beta], interpolated linearly and extended
 * antiperiodically (Delta(tau - beta) = -Delta(tau)).
 *
 * Moves (one per chain per step): flavor f = floor(u0 F); if u1 < 1/2 insert a
 * creator at ts = u2 beta and an annihilator at te = ts + u3 beta (mod beta) as label
 * k_f (acceptance factor beta^2 / (k_f+1)^2), else remove creator label floor(u2 k_f)
 * and annihilator label floor(u3 k_f), filling each hole with the last label
 * (factor k_f^2 / beta^2); accept when u4 < |w'/w| * factor.  u0..u5 come from
 * Philox4x32-10 (Salmon et al., SC'11) with counter (move low word, move high word,
 * chain, call 0..2) and key (seed low word, seed high word); a double is
 * ((a >> 5) 2^26 + (b >> 6)) / 2^53 from two output words.  Determinant ratios
 * and inverse updates are O(k^2) (Sec. II, fast updates); every move evaluates one
 * Krylov trace per chain through the batched trace path.
 *
 * G(tau) estimator (per flavor, after every meas_every-th move):
 *   G_f(tau) = -(1/beta) < sum_ij M_f[j][i] delta~(tau, tau_{f,j} - tau'_{f,i}) >,
 * M_f = A_f^{-1}; a negative difference is shifted by +beta and enters with a minus
 * sign; histogram of n_tau bins on [0, beta); samples weighted by sign(w). */
typedef struct {
  int32_t n_chains;
  double beta;
  int32_t n_delta;        /* intervals of the Delta table (table has n_delta + 1 values) */
  const double* delta;    /* host, [n_delta + 1]: Delta(k beta / n_delta); copied */
  int32_t kmax;           /* pair capacity per flavor, 1..63 */
  int32_t nmax_ops;       /* operator capacity per configuration, 2..4096 */
  uint64_t seed;          /* generator key */
  int32_t n_tau;          /* G(tau) bins */
  int32_t meas_every;     /* measure after every meas_every-th move */
  int32_t moves_per_sweep;
  int32_t rebuild_every;  /* > 0: M_f = A_f^{-1} is rebuilt from scratch (Gauss-Jordan with partial
                             pivoting, FP64) after every rebuild_every-th move, bounding the drift of
                             the O(k^2) updates; 0: never */
} hyb_mc_params;

typedef struct {
  int64_t insert_proposed, insert_accepted, remove_proposed, remove_accepted;
  int64_t impossible;     /* capacity reached or flavor empty */
  int64_t zero_weight;    /* proposals whose weight was zero (trace zero, time tie) */
  int64_t moves;          /* chain-moves counted */
  double order_sum;       /* sum over chain-moves of the total pair number */
  double sign_sum;        /* sum over chain-moves of sign(w) */
  double max_drift;       /* largest max|M_f - inv(A_f)| / max|inv(A_f)| found at a rebuild of M
                             (the accumulated error of the fast updates); 0 before any rebuild */
} hyb_mc_stats;

typedef struct hyb_mc hyb_mc;

/* Allocates n_chains chains on the model's device, all starting from the empty
 * configuration (weight Tr_R of no operators > 0).  The model must stay alive and
 * uploaded.  Errors: HYB_E_ARG (parameters), HYB_E_STATE, HYB_E_OOM, HYB_E_HIP. */
int hyb_mc_create(hyb_model* m, const hyb_mc_params* p, hyb_mc** out);
int hyb_mc_destroy(hyb_mc* mc);

/* Replaces every chain's configuration (host arrays): k [n_chains][F] pair numbers,
 * cre / ann [n_chains][F][kmax] creator / annihilator times in label order.  Builds
 * M_f = A_f^{-1} by LU on the host, traces the configurations, and resets the move
 * counter, statistics and accumulators.  HYB_E_ARG for a zero weight, a singular
 * A_f or a capacity overflow; HYB_E_UNSORTED for equal or out-of-range times. */
int hyb_mc_set_configs(hyb_mc* mc, const int32_t* k, const double* cre, const double* ann, void* stream);

/* n_sweeps * moves_per_sweep moves of every chain on `stream`; returns after the
 * stream drained.  HYB_E_NOCONV / HYB_E_NONFINITE if a trace inside failed. */
int hyb_mc_sweep(hyb_mc* mc, int32_t n_sweeps, void* stream);

/* Current state (host outputs, each may be NULL): k, cre, ann as in set_configs,
 * M [n_chains][F][kmax][kmax] (row = annihilator label, column = creator label),
 * logw = log|w| and sign = sign(w) per chain. */
int hyb_mc_get_state(const hyb_mc* mc, int32_t* k, double* cre, double* ann, double* M, double* logw,
                     int8_t* sign, void* stream);
int hyb_mc_get_stats(const hyb_mc* mc, hyb_mc_stats* out, void* stream);
/* Raw per-chain accumulators: gacc [n_chains][F][n_tau] = sum of sign * signed M
 * entries per bin, meas_sign [n_chains] = sum of signs, n_meas [n_chains]. */
int hyb_mc_get_accumulators(const hyb_mc* mc, double* gacc, double* meas_sign, int64_t* n_meas, void* stream);
/* G [F][n_tau] over all chains: -sum gacc / (beta * (beta / n_tau) * sum meas_sign);
 * *sign_avg = <sign>.  HYB_E_STATE before any measurement. */
int hyb_mc_measure(const hyb_mc* mc, double* G, double* sign_avg, void* stream);
int hyb_mc_reset_measurements(hyb_mc* mc, void* stream);
int hyb_mc_step_count(const hyb_mc* mc, int64_t* step);

/* Weights of the (n_up, n_dn) sectors at tau = beta/2 (Sec. IV.C, Fig. 4; Sec. III
 * measures at beta/2): for a configuration, P_s = sum_{r: path r in sector s at
 * beta/2} t_r / sum_r t_r over the retained-state paths of its trace (the blocks are
 * conserved between operators, so each path's sector at beta/2 follows from its
 * operators alone); accumulated with sign(w) at every measurement.
 * w (host [n_blocks], may be NULL): sum over chains of the accumulators / sum of
 * signs, indexed by block = n_dn (n_orb + 1) + n_up.  acc (host [n_chains][n_blocks],
 * may be NULL): the raw per-chain accumulators (for error analysis).  Reset by
 * hyb_mc_reset_measurements; part of the checkpoint. */
int hyb_mc_sector_weights(const hyb_mc* mc, double* w, double* acc, void* stream);

/* Checkpoint of every chain (the checkpoint/resume of a long run): pair lists, M,
 * the time-ordered operator lists and weight factors, the move counter (which
 * keys the Philox counters, so the random stream resumes where it stopped), the
 * statistics and the G(tau) accumulators.  hyb_mc_save with buf = NULL writes the
 * size needed to *len; otherwise *len is the buffer size on entry and the bytes
 * written on return (HYB_E_ARG if too small).  The blob is host memory owned by
 * the caller; its layout is a fixed header (magic "HYBMCCK2", sizes, beta, seed,
 * move counter, a hash of the Delta table) followed by the raw arrays.
 * hyb_mc_load restores a checkpoint into chains created with the same sizes, beta,
 * seed, Delta table and model precision (else HYB_E_ARG).  It then checks the
 * stored state: the trace of every stored operator list is evaluated again and
 * must equal the stored one (1e-8 relative in log for FP64), and A_f^{-1} is
 * recomputed from the stored times and must equal the stored M (1e-6 relative)
 * and log|det| (1e-8); a mismatch is HYB_E_ARG.  The stored M itself is kept, so
 * moves after a load repeat the uninterrupted run bit for bit.  After a load that
 * failed its checks the chain state is unspecified until a good checkpoint is
 * loaded or hyb_mc_set_configs is called.  The attached network and the graph
 * setting are not part of the checkpoint. */
int hyb_mc_save(const hyb_mc* mc, void* buf, size_t* len, void* stream);
int hyb_mc_load(hyb_mc* mc, const void* buf, size_t len, void* stream);
/* enable != 0: hyb_mc_sweep captures one sweep (moves_per_sweep moves of every chain,
 * with no host synchronisation inside) into a HIP graph on first use and replays it
 * n_sweeps times on `stream`.  The move counter lives on the device, so every replay
 * draws new random numbers, and the chains evolve bit for bit as with enable = 0.  The
 * sweep is captured again when anything it depends on has changed: the attached network
 * or its buffers, the mixture weight, the model's device copy or its kernel variant.
 * enable = 0 (the default) launches every move directly and frees the graph.  Capture
 * uses a private stream of the default priority; calls on one hyb_mc must not overlap. */
int hyb_mc_set_graphs(hyb_mc* mc, int32_t enable);

/* ---- DMFT self-consistency on the Bethe lattice (Sec. V) -------------------------- */

/* Replaces the Delta table of every chain (host [n_delta + 1], same grid) and rebuilds
 * each chain's M_f = A_f^{-1}, log|det A_f| and the weight's sign from its times
 * (Gauss-Jordan, FP64, on the device).  Measurements already accumulated are kept;
 * callers normally reset them.  HYB_E_ARG for a non-finite table or when a chain's
 * A_f becomes singular (the chain state is then unspecified until hyb_mc_set_configs). */
int hyb_mc_set_delta(hyb_mc* mc, const double* delta, void* stream);

/* The Bethe-lattice update for a semicircular density of states of half-bandwidth
 * 2t: Delta_new(tau) = (1 - mix) Delta(tau) + mix t^2 G(tau), with G the measured
 * G(tau) (hyb_mc_measure) averaged over the flavors (one Delta serves every flavor:
 * paramagnetic, orbitally degenerate bath), with symmetrize & 1 also made
 * particle-hole symmetric, G(tau) = G(beta - tau).  G is taken at the bin centres;
 * its values at 0+ and beta- are extrapolated linearly from the two nearest bins and
 * shifted together to satisfy G(0+) + G(beta-) = -1; the grid values of Delta come
 * from linear interpolation.  delta_out: host [n_delta + 1].  HYB_E_STATE before any
 * measurement. */
int hyb_mc_bethe_delta(const hyb_mc* mc, double t, double mix, int32_t symmetrize, double* delta_out,
                       void* stream);

typedef struct {
  double t;               /* Bethe-lattice hopping: Delta = t^2 G (bandwidth 4t) */
  double mix;             /* linear mixing of the new Delta, (0, 1] */
  int32_t n_iter;         /* self-consistency iterations */
  int32_t therm_sweeps;   /* sweeps after each Delta update before measuring */
  int32_t meas_sweeps;    /* measured sweeps per iteration */
  int32_t symmetrize;     /* bit 0: particle-hole symmetric G */
} hyb_dmft_params;

/* n_iter DMFT iterations on the Bethe lattice: thermalise, reset and measure G(tau),
 * record the flavor average of G at the two middle bins (g_half[it], host, may be
 * NULL) and the average sign (sign_avg[it]), then hyb_mc_bethe_delta and
 * hyb_mc_set_delta.  The final Delta is the chains' table (hyb_mc_get_delta). */
int hyb_dmft_bethe(hyb_mc* mc, const hyb_dmft_params* p, double* g_half, double* sign_avg, void* stream);

/* The chains' current Delta table (host out [n_delta + 1]). */
int hyb_mc_get_delta(const hyb_mc* mc, double* delta);

/* ---- learned insertion proposal ---------------------------------------------- */

/* A 3-layer perceptron 352 -> 128 -> 128 -> 128 (ReLU between layers) mapping the
 * features of (configuration without the pair, flavor f) to 64 logits for the bin
 * of the creator time tau_s and 64 logits for the bin of the pair length
 * l = (tau_e - tau_s) mod beta.  Features: one-hot f (F entries), k_g / 32 for every
 * flavor (F), and per flavor the count of creators minus annihilators before the
 * centre of each of 32 equal time bins (32 F); zero-padded to 352 (F <= 10).
 * BF16 weights and activations on the matrix cores with FP32 accumulation; FP32
 * master weights.  Insertion density
 *   q(tau_s, l) = (1 - eps) p_tau(bin tau_s) (64/beta) p_l(bin l) (64/beta) + eps / beta^2.
 * Training target: cross-entropy of the two bins of a pair removed uniformly from a
 * sampled configuration (maximum likelihood of the pairs the chains produce).
 * Weight layout (FP32, output-major): W1 [128][352], W2 [128][128], W3 [128][128]
 * concatenated; biases b1 [128], b2 [128], b3 [128] concatenated. */
typedef struct hyb_mlp hyb_mlp;
int hyb_mlp_create(uint64_t seed, hyb_mlp** out);   /* He-uniform weights from seed, zero biases */
int hyb_mlp_destroy(hyb_mlp* p);
int hyb_mlp_get_weights(const hyb_mlp* p, float* w, float* b);   /* host outputs */
int hyb_mlp_set_weights(hyb_mlp* p, const float* w, const float* b);   /* host inputs; resets Adam */
/* logits [n][128] (device) of features X [n][352] (device, bf16) */
int hyb_mlp_forward(hyb_mlp* p, int32_t n, const void* X, float* logits, void* stream);
/* Gradients of the mean loss over the batch (host outputs, may be NULL; same layouts
 * as the weights) and the mean loss; X device bf16 [n][352], targets device [n][2]. */
int hyb_mlp_gradients(hyb_mlp* p, int32_t n, const void* X, const int32_t* targets, float* w_grad, float* b_grad,
                      float* loss, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on a batch; *loss (host, may be
 * NULL) = mean loss before the step. */
int hyb_mlp_train_step(hyb_mlp* p, int32_t n, const void* X, const int32_t* targets, float lr, float* loss,
                       void* stream);
/* Use the network (NULL: back to uniform insertion) with mixture weight eps in (0, 1]
 * for every following insertion / removal of mc.  The network must outlive its use. */
int hyb_mc_attach_mlp(hyb_mc* mc, hyb_mlp* mlp, double eps);
/* One training sample per chain from the current states: X [n_chains][352] (device,
 * bf16) and targets [n_chains][2] (device; (-1, -1) for a chain without pairs).  The
 * flavor (uniform among those with pairs) and the pair come from Philox calls 8 and 9
 * at counter `index`. */
int hyb_mc_harvest(hyb_mc* mc, int64_t index, void* X, int32_t* targets, void* stream);

/* ---- misc ------------------------------------------------------------------ */
const char* hyb_last_error(void);
const char* hyb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HYB_H */
