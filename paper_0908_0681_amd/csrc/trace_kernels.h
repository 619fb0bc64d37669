// Device code of the Krylov trace (gfx950, wave64).
//
// One workgroup carries one feasible (configuration, retained state) path through
// all of its operators in one launch (k_path_chunk with the whole operator range;
// shorter chunks, down to one operator per launch, give the same arithmetic in
// another launch schedule).  Inside a launch a path's state (block, log-scale,
// unit vector) stays on chip (path_run); it passes through global memory only
// between launches.  The vector lives in registers, RPT rows per thread (row =
// tid + k*NT), the Lanczos basis V_0..V_m lives in registers too, and LDS holds the
// vector being gathered by the SpMV or the operator, the block's off-diagonal rows,
// the model's block and spin-pattern tables, the reduction partials and the small
// tridiagonal problem.
//
// Steps (Sec. III): the retained eigenstate enters with the scalar phase of the
// two edge intervals (step 3); each operator is a signed gather between blocks
// (step 4); each interval is a Lanczos/Krylov propagation with an a-posteriori
// stopping rule (step 5); the overlap with <E_i| closes the path (step 7); the
// signed log-sum over R is a separate kernel (step 8).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

#include "hyb_internal.h"

namespace hyb {

enum : int32_t { ERR_UNSORTED = 1, ERR_FLAVOR = 2, ERR_NOCONV = 4, ERR_NONFINITE = 8, ERR_SINGULAR = 16 };

// The path queue is ordered by an estimate of each path's cost, longest first, so
// that the launch does not end with long paths started late: the sum over the path's
// intervals of (dtau * width of the block)^(3/4), in ORDER_NB logarithmic buckets.
constexpr int ORDER_NB = 128;
constexpr int COUNTERS_LEN = 4 + 2 * ORDER_NB;

struct TraceParams {
  // model
  const uint32_t* states;
  const int32_t* rank;
  const BlockDev* blocks;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val64;
  const float* val32;
  const double* diag64;
  const int32_t* ret_block;
  const double* ret_energy;
  const int64_t* ret_off;
  const double* ret_vec64;
  const float* ret_vec32;
  int32_t n_orb, n_ret;
  double E0;
  // configurations
  int32_t n_configs;
  const int64_t* offsets;
  const int64_t* ends;  // nullptr: ops of config c are [offsets[c], offsets[c+1]); else [offsets[c], ends[c])
  const double* tau;
  const int16_t* flavor;
  const int8_t* dagger;
  double beta;
  // work queue and per-path results (path id = config * n_ret + r)
  int32_t* work;
  int32_t* counters;  // [0] queued paths, [1] longest configuration, [2] error bits;
                      // [4, 4 + ORDER_NB) paths per cost bucket, then each bucket's next slot
  int32_t* p_bucket;  // per pair: cost bucket of a feasible path, -1 otherwise (nullptr:
                      // the scan queues paths in the order it finds them)
  int8_t* p_sign;
  double* p_log;
  int32_t* p_steps;
  int32_t* p_sub;
  // Krylov settings
  double tol;
  int32_t kmax;
  int32_t max_substeps;
  int32_t n_pairs;     // n_configs * n_ret
  int32_t work_budget; // QR sweeps allowed per path before it is abandoned
  // step-synchronous path state, indexed by queue slot w < counters[0]
  int32_t* st_block;   // current block of the path
  int32_t* st_status;  // PATH_ACTIVE / PATH_EMPTY / PATH_ZERO / PATH_FAILED
  int32_t* st_steps;   // Lanczos steps so far
  int32_t* st_subs;    // extra substeps forced by the depth cap
  double* st_ell;      // running log-scale
  int64_t* st_rowsteps;  // sum of Lanczos steps x block dimension
  int64_t* st_rows;      // sum of block dimensions over intervals
  int64_t* p_rowsteps;   // per (config, retained state) pair
  int64_t* p_rows;
  void* st_vec;        // two ping-pong vector buffers [2][n_pairs][vstride] of VT
  int32_t vstride;     // elements per path vector (>= largest block)
  double zero_tol2;    // an operator leaving less than this squared norm ends the path
  // off-diagonal rows as padded ELL in natural order: slot k of row r of block b at
  // state_off_b * ek + k * dim_b + r (padding: column r, value 0)
  const int16_t* ecol;
  const double* eval64;
  const float* eval32;
  int32_t ek;          // slots per row
  // matrix-free rows (HYB_MATRIX_FREE and the *_mf variants): one spin's pattern ->
  // rank among patterns of its popcount, and the spin-flip / pair-hopping amplitudes
  const int16_t* rank_half;
  double jsf, jph;
  // optional: the block each (config, retained state) path occupies at time tau_mid
  // (the block after every operator earlier than tau_mid); nullptr to skip
  int32_t* p_midblk;
  double tau_mid;
};

__device__ __forceinline__ int64_t cfg_end(const TraceParams& P, int c) {
  return P.ends ? P.ends[c] : P.offsets[c + 1];
}


enum : int32_t { PATH_ACTIVE = 0, PATH_EMPTY = 1, PATH_ZERO = 2, PATH_FAILED = 3 };

// ---------------------------------------------------------------------------
// wavefront reductions (DPP inside rows of 16 lanes, then readlane)
// ---------------------------------------------------------------------------

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double shfl_xor_d(double v, int mask) {
  const int lo = __shfl_xor(__double2loint(v), mask), hi = __shfl_xor(__double2hiint(v), mask);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes; every lane receives the same (bitwise) result.
__device__ __forceinline__ double wave_sum(double x) {
  x += dpp_d<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_d<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_d<0x141>(x);  // row_half_mirror
  x += dpp_d<0x140>(x);  // row_mirror: every lane holds its 16-lane row sum
  return (readlane_d(x, 0) + readlane_d(x, 16)) + (readlane_d(x, 32) + readlane_d(x, 48));
}

// Wave totals of NV values per lane (NV = 4, 8 or 16): every lane receives all of
// them, bitwise identical across lanes.  A reduce-scatter inside each 16-lane row
// first: at each step a lane pairs with a partner (rotate by 8, mirror within 8,
// swap pairs, swap neighbours), keeps half of its values and adds the partner's copy
// of that half, so after log2(NV) steps each lane holds one value summed over
// NV lanes; the rest of its row and the four rows are then summed with two DPP and
// two cross-row exchanges, and each total is read from a lane that holds it.  About
// half the instructions of NV separate wave sums.
template <int NV>
__device__ __forceinline__ void wave_sums(double* v) {
  static_assert(NV == 4 || NV == 8 || NV == 16, "NV is 4, 8 or 16");
  const int lane = threadIdx.x & 63;
  double a[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) a[q] = v[q];
  // step s keeps the upper half on lanes with bit (8 >> s) set
  auto step = [&](auto ctrl_tag, int bit, int n) {
    constexpr int CTRL = decltype(ctrl_tag)::value;
    const bool upper = (lane & bit) != 0;
#pragma unroll
    for (int q = 0; q < NV / 2; ++q) {
      if (q < n) {
        const double send = upper ? a[q] : a[q + n];
        const double keep = upper ? a[q + n] : a[q];
        a[q] = keep + dpp_d<CTRL>(send);
      }
    }
  };
  step(std::integral_constant<int, 0x128>{}, 8, NV / 2);  // row_ror:8 (lane ^ 8)
  step(std::integral_constant<int, 0x141>{}, 4, NV / 4);  // row_half_mirror (bit 2 differs)
  if constexpr (NV >= 8) step(std::integral_constant<int, 0x4E>{}, 2, NV / 8);  // lane ^ 2
  if constexpr (NV >= 16) step(std::integral_constant<int, 0xB1>{}, 1, NV / 16);  // lane ^ 1
  double x = a[0];
  if constexpr (NV < 8) x += dpp_d<0x4E>(x);
  if constexpr (NV < 16) x += dpp_d<0xB1>(x);
  // the four rows
  x += shfl_xor_d(x, 16);
  x += shfl_xor_d(x, 32);
  // value c sits on the lane whose bits 3, 2, 1, 0 spell c from its top bit down
  constexpr int S = (NV == 4) ? 2 : (NV == 8) ? 3 : 4;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    int l = 0;
#pragma unroll
    for (int t = 0; t < S; ++t)
      if ((c >> (S - 1 - t)) & 1) l |= (8 >> t);
    v[c] = readlane_d(x, l);
  }
}

// 1/d to about one ulp: the hardware estimate refined by two Newton steps (d finite
// and nonzero, far from the exponent range's ends).
__device__ __forceinline__ double rcp_d(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// Root of y^2 - w y - s = 0 (s > 0) on the side right > 0 or right = false < 0,
// without cancellation.
__device__ __forceinline__ double pole_root(double w, double s, bool right) {
  const double sq = sqrt(w * w + 4.0 * s);
  if (right) return (w < 0.0) ? 2.0 * s * rcp_d(sq - w) : 0.5 * (w + sq);
  return (w > 0.0) ? -2.0 * s * rcp_d(w + sq) : 0.5 * (w - sq);
}

// True on every lane when p holds on at least one lane of the wavefront.
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

template <typename VT>
__device__ __forceinline__ double to_d(VT x) { return static_cast<double>(x); }

// ---------------------------------------------------------------------------
// the per-workgroup path evaluator
// ---------------------------------------------------------------------------

// VL: the Krylov basis V_0..V_m lives in LDS (row r of V_i at i * NT * RPT + r)
// instead of registers; the SpMV then gathers straight from V_j.  This is the shape
// for wide single-wave paths (many rows per lane), where a register basis would
// spill and where several paths share a CU.
template <typename VT, int NT, int RPT, int MAXM, bool MF = false, bool VL = false>
struct PathEngine {
  static constexpr int NW = NT / 64;
  static constexpr int NRED = (MAXM + 2 > 16) ? MAXM + 2 : 16;  // partial sums per reduction round
  static constexpr int QLD = MAXM + 1;   // padded row length of Q in LDS

  // Tridiagonal work space of one wavefront (uniform values; every wave of the
  // workgroup keeps its own copy so that no extra barrier is needed).
  struct Small {
    double alpha[MAXM], beta[MAXM];  // Lanczos T_m
    double a[2][MAXM], b[2][MAXM];   // QR snapshot / output buffers
    double q[2][MAXM * QLD];         // eigenvectors, row r = component r (buffer qc)
    double u[MAXM * QLD];            // eigenvectors of the arrowhead extension
    double tho[MAXM], xr[MAXM];      // root j = tho[j] + xr[j] (origin pole, offset)
    double zh[MAXM];                 // couplings recomputed from the roots
    double tz[2 * MAXM];             // pole i: theta_i at 2i, z_i^2 at 2i + 1
    double wk[MAXM];                 // exp(-tau (theta_i - theta_min)) Q[0][i]
    int rank[MAXM];                  // sorting permutation after a QR solve
    int cur;                         // buffer holding the eigenvalues (ascending)
    int qc;                          // buffer holding the eigenvectors
  };
  // Off-diagonal slots of each thread's rows held in LDS during a propagation, up to
  // KL per row within a per-variant budget (rows with more entries use the CSR in HBM)
  static constexpr int NR = NT * RPT;
  // LDS budget for staged rows: none for matrix-free rows and for wide single-wave
  // paths (RPT > 4: those read their rows from L2 at every SpMV so that several paths
  // share a CU)
  static constexpr int SLAB_BYTES = (MF || (NT == 64 && RPT > 4)) ? 0
                                    : (NT >= 512) ? 64 * 1024 : (NT >= 256) ? 96 * 1024 : 10 * 1024 * (NT / 64);
  static constexpr int KL0 = SLAB_BYTES / (NR * int(sizeof(VT) + sizeof(int16_t)));
  // Slots are staged in chunks of CH (16 bytes of values, 2 doubles or 4 floats):
  // chunk c of local row r holds the row's slots c*CH .. c*CH+CH-1, so that one
  // 16-byte LDS read brings CH values and one 4- or 8-byte read their columns.
  static constexpr int CH = 16 / int(sizeof(VT));
  static constexpr int KL = (KL0 > 16 ? 16 : KL0) / CH * CH;
  static constexpr int NCH = KL / CH;  // chunks per row
  using VV = std::conditional_t<sizeof(VT) == 8, double2, float4>;   // CH values
  using CV = std::conditional_t<sizeof(VT) == 8, uint32_t, uint2>;   // CH int16 columns
  struct Smem {
    VT vec[VL ? 1 : NT * RPT];
    VT vb[VL ? (MAXM + 1) * NT * RPT : 1];  // the Krylov basis when VL
    double red[2][NW][NRED];
    Small small[NW];
    VV sval[NCH > 0 ? NCH * NR : 1];     // chunk c of local row r at c * NR + r
    CV scol[NCH > 0 ? NCH * NR : 1];
    int16_t rh[MF ? 128 : 1];            // matrix-free: rank_half of the model (2^n_orb <= 128)
  };

  const TraceParams& P;
  Smem& S;
  const int tid, lane, wid;
  int rbuf = 0;

  __device__ PathEngine(const TraceParams& p, Smem& s)
      : P(p), S(s), tid(threadIdx.x), lane(threadIdx.x & 63), wid(threadIdx.x >> 6) {}

  uint32_t rstate[MF ? RPT : 1];  // matrix-free: the basis state of each of this thread's rows

  __device__ __forceinline__ const VT* ret_vec() const {
    if constexpr (sizeof(VT) == 8) return reinterpret_cast<const VT*>(P.ret_vec64);
    else return reinterpret_cast<const VT*>(P.ret_vec32);
  }
  __device__ __forceinline__ VT offval(int j) const {
    if constexpr (sizeof(VT) == 8) return static_cast<VT>(P.val64[j]);
    else return static_cast<VT>(P.val32[j]);
  }

  // Orders this wave's LDS traffic (all lanes of a wave run in lock step).
  __device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }

  // Workgroup sum of kact (<= K) per-thread partials; all threads get the totals
  // in a fixed summation order.
  template <int K>
  __device__ __forceinline__ void block_sum(double (&v)[K], int kact) {
    if (kact <= 2 || kact > 16 || K < 16) {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k < kact) v[k] = wave_sum(v[k]);
    } else if constexpr (K >= 16) {
      // several values at once, in place (entries from kact up are zero on entry)
      if (kact <= 4) wave_sums<4>(v);
      else if (kact <= 8) wave_sums<8>(v);
      else wave_sums<16>(v);
    }
    if constexpr (NW > 1) {
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (k < kact) S.red[rbuf][wid][k] = v[k];
      }
      __syncthreads();
      // lane k adds the waves' partials of value k (all loads in flight at once),
      // then every lane reads the totals from those lanes
      double s = 0.0;
      if (lane < kact) {
        double part[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) part[w] = S.red[rbuf][w][lane];
#pragma unroll
        for (int w = 0; w < NW; ++w) s += part[w];
      }
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k < kact) v[k] = readlane_d(s, k);
      rbuf ^= 1;
    }
  }

  __device__ __forceinline__ double block_sum1(double x) {
    double v[1] = {x};
    block_sum<1>(v, 1);
    return v[0];
  }

  __device__ __forceinline__ int row(int k) const { return tid + k * NT; }

  // Off-diagonal part of row t of H_b applied to the vector in S.vec, generated from
  // t's bits (Eq.(4), each ordered orbital pair a != c once): spin flip
  // -J_sf c+_{a dn} c+_{c up} c_{c dn} c_{a up} needs a singly occupied by up and c
  // by down; pair hopping -J_ph c+_{c up} c+_{c dn} c_{a up} c_{a dn} needs a doubly
  // occupied and c empty.  Both flip orbitals a and c in both spin strings; the sign
  // is the Jordan-Wigner parity of the four operators applied right to left.  The
  // target's index inside the block is rank_half[dn'] * up_states + rank_half[up'].
  __device__ __forceinline__ double row_free(const BlockDev& B, uint32_t t, const VT* xs) const {
    const int n = P.n_orb;
    const uint32_t lo = (1u << n) - 1u;
    const uint32_t up = t & lo, dn = t >> n;
    VT sf = VT(0), ph = VT(0);
    auto parity_step = [](uint32_t& cur, uint32_t bit) {
      const int par = __popc(cur & (bit - 1u)) & 1;
      cur ^= bit;
      return par;
    };
    auto take = [&](uint32_t t2) {
      return xs[int(S.rh[t2 >> n]) * B.up_states + int(S.rh[t2 & lo])];
    };
    if (P.jsf != 0.0) {
      for (uint32_t ma = up & ~dn; ma; ma &= ma - 1u) {
        const int a = __ffs(ma) - 1;
        for (uint32_t mc = dn & ~up; mc; mc &= mc - 1u) {
          const int c = __ffs(mc) - 1;
          uint32_t cur = t;
          int par = parity_step(cur, 1u << a);
          par ^= parity_step(cur, 1u << (c + n));
          par ^= parity_step(cur, 1u << c);
          par ^= parity_step(cur, 1u << (a + n));
          const VT v = take(cur);
          sf += par ? -v : v;
        }
      }
    }
    if (P.jph != 0.0) {
      for (uint32_t ma = up & dn; ma; ma &= ma - 1u) {
        const int a = __ffs(ma) - 1;
        for (uint32_t mc = lo & ~(up | dn); mc; mc &= mc - 1u) {
          const int c = __ffs(mc) - 1;
          uint32_t cur = t;
          int par = parity_step(cur, 1u << (a + n));
          par ^= parity_step(cur, 1u << a);
          par ^= parity_step(cur, 1u << (c + n));
          par ^= parity_step(cur, 1u << c);
          const VT v = take(cur);
          ph += par ? -v : v;
        }
      }
    }
    return -P.jsf * to_d(sf) - P.jph * to_d(ph);
  }

  // y = (H_b - c_b) x for the rows owned by this thread.  The whole vector is read
  // from LDS: from xsrc when it is there already (the basis of VL engines), else
  // after staging x into S.vec.  Each thread's rows come from its own LDS slots when
  // staged (stage_rows), from the ELL copy in L2 when the variant keeps no slots,
  // from the CSR in HBM otherwise, or are generated from the bits (MF).
  __device__ __forceinline__ void spmv(const BlockDev& B, const VT (&x)[RPT], VT (&y)[RPT],
                                       const double (&dg)[RPT], bool staged, const VT* xsrc = nullptr) {
    const VT* xs = xsrc;
    if (!xs) {
#pragma unroll
      for (int k = 0; k < RPT; ++k)
        if (row(k) < B.dim) S.vec[row(k)] = x[k];
      xs = S.vec;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = row(k);
      if (r < B.dim) {
        VT acc = VT(0);
        if constexpr (MF) {
          y[k] = static_cast<VT>(dg[k] * to_d(x[k]) + row_free(B, rstate[k], xs));
          continue;
        }
        if constexpr (NCH > 0) {
          if (staged) {
            // The columns and values of up to G chunks are requested together, then
            // all of their gathers, so a row costs two LDS round trips rather than
            // one per slot.  Chunks past the row's last are re-read (clamped) with
            // their values taken as 0; slots are summed in slot order.
            constexpr int G = NCH < 4 ? NCH : 4;
            const int nch = (P.ek + CH - 1) / CH;
            for (int c0 = 0; c0 < nch; c0 += G) {
              CV cw[G];
              VV vw[G];
#pragma unroll
              for (int g = 0; g < G; ++g) {
                const bool real = c0 + g < nch;
                const int c = real ? c0 + g : nch - 1;
                cw[g] = S.scol[c * NR + r];
                vw[g] = S.sval[c * NR + r];
                if (!real) vw[g] = VV{};
              }
              VT xg[G][CH];
#pragma unroll
              for (int g = 0; g < G; ++g) {
                if constexpr (CH == 2) {
                  xg[g][0] = xs[cw[g] & 0xffffu];
                  xg[g][1] = xs[cw[g] >> 16];
                } else {
                  xg[g][0] = xs[cw[g].x & 0xffffu];
                  xg[g][1] = xs[cw[g].x >> 16];
                  xg[g][2] = xs[cw[g].y & 0xffffu];
                  xg[g][3] = xs[cw[g].y >> 16];
                }
              }
#pragma unroll
              for (int g = 0; g < G; ++g) {
                if constexpr (CH == 2) {
                  acc += vw[g].x * xg[g][0];
                  acc += vw[g].y * xg[g][1];
                } else {
                  acc += vw[g].x * xg[g][0];
                  acc += vw[g].y * xg[g][1];
                  acc += vw[g].z * xg[g][2];
                  acc += vw[g].w * xg[g][3];
                }
              }
            }
            y[k] = static_cast<VT>(dg[k] * to_d(x[k]) + to_d(acc));
            continue;
          }
        }
        if constexpr (KL == 0) {
          // the block's natural-order ELL rows straight from global memory (L2): slot q
          // of row r at state_off * K + q * dim + r, so a wave's loads are contiguous
          const int K = P.ek;
          const int64_t base = int64_t(B.state_off) * K + r;
#pragma unroll 4
          for (int q = 0; q < K; ++q) {
            const int64_t at = base + int64_t(q) * B.dim;
            VT v;
            if constexpr (sizeof(VT) == 8) v = static_cast<VT>(P.eval64[at]);
            else v = static_cast<VT>(P.eval32[at]);
            acc += v * xs[P.ecol[at]];
          }
        } else {
          const int g = B.state_off + r;
          const int j0 = P.rowptr[g], j1 = P.rowptr[g + 1];
          for (int j = j0; j < j1; ++j) acc += offval(j) * xs[P.col[j]];
        }
        y[k] = static_cast<VT>(dg[k] * to_d(x[k]) + to_d(acc));
      } else {
        y[k] = VT(0);
      }
    }
    __syncthreads();  // the source is rewritten by the next staging / basis update
  }

  // Loads the diagonal of this thread's rows of block B into registers and, when
  // they fit, their off-diagonal ELL slots into this thread's LDS slots (read only
  // by this thread, so no barrier is needed).  Returns whether the slots are staged.
  __device__ __forceinline__ bool stage_rows(const BlockDev& B, double (&dg)[RPT]) {
    const int K = P.ek;
    const int nch = (K + CH - 1) / CH;
    const bool staged = nch <= NCH;
    const int64_t base = int64_t(B.state_off) * K;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = row(k);
      dg[k] = (r < B.dim) ? P.diag64[B.state_off + r] : 0.0;
    }
    if constexpr (MF) {
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int r = row(k);
        rstate[k] = (r < B.dim) ? P.states[B.state_off + r] : 0u;
      }
      // read after the barrier of the first SpMV's vector staging
      for (int i = tid; i < (1 << P.n_orb); i += NT) S.rh[i] = P.rank_half[i];
      return false;
    }
#pragma unroll 1
    for (int k = 0; k < RPT; ++k) {
      const int r = row(k);
      const bool in = r < B.dim;
      if constexpr (NCH > 0) {
        if (staged && in && K > 0) {
          // every slot of the row is requested before the first LDS store (slots past
          // K re-read slot K - 1 of the same row), so the loads are in flight
          // together; the last chunk is padded with value 0 at column 0
          VT vv[KL];
          int16_t cc[KL];
#pragma unroll
          for (int q = 0; q < KL; ++q) {
            const int64_t at = base + int64_t(q < K ? q : K - 1) * B.dim + r;
            if constexpr (sizeof(VT) == 8) vv[q] = static_cast<VT>(P.eval64[at]);
            else vv[q] = static_cast<VT>(P.eval32[at]);
            cc[q] = P.ecol[at];
          }
#pragma unroll
          for (int q = 0; q < KL; ++q)
            if (q >= K) {
              vv[q] = VT(0);
              cc[q] = 0;
            }
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            if (c < nch) {
              const int q = c * CH;
              VV v;
              CV w;
              if constexpr (CH == 2) {
                v = VV{vv[q], vv[q + 1]};
                w = uint32_t(uint16_t(cc[q])) | (uint32_t(uint16_t(cc[q + 1])) << 16);
              } else {
                v = VV{vv[q], vv[q + 1], vv[q + 2], vv[q + 3]};
                w = CV{uint32_t(uint16_t(cc[q])) | (uint32_t(uint16_t(cc[q + 1])) << 16),
                       uint32_t(uint16_t(cc[q + 2])) | (uint32_t(uint16_t(cc[q + 3])) << 16)};
              }
              S.sval[c * NR + r] = v;
              S.scol[c * NR + r] = w;
            }
          }
        }
      }
    }
    return staged;
  }

  // Eigendecomposition of the m x m symmetric tridiagonal T_m = (alpha, beta) of this
  // wave, called for m = 1, 2, 3, ... as the Lanczos recursion grows T.  On return
  // the eigenvalues are in ascending order in W.a[W.cur][0..m) and lane r (< m) has
  // row r of the eigenvector matrix in W.q.  From m = 3 on, the decomposition of
  // T_{m-1} is extended by one row and column (extend_eig); where that is not safe,
  // T_m is solved from scratch by QR and the result sorted.  Returns a work count.
  __device__ int small_eig(Small& W, int m) {
    if (m <= 2) {
      // closed forms: no sweep needed for the first two Lanczos steps
      double l0, l1, q00 = 1.0, q01 = 0.0, q10 = 0.0, q11 = 1.0;
      if (m == 1) {
        l0 = W.alpha[0];
        l1 = 0.0;
      } else {
        const double a = W.alpha[0], c = W.alpha[1], b = W.beta[0];
        const double t = 0.5 * (a + c), d = 0.5 * (a - c), r = hypot(d, b);
        l0 = t - r;
        l1 = t + r;
        if (b != 0.0) {
          // eigenvector of l0 from the row without cancellation
          double x0, x1;
          if (d >= 0.0) {
            x0 = b;
            x1 = -d - r;
          } else {
            x0 = r - d;
            x1 = -b;
          }
          const double nx = hypot(x0, x1);
          x0 /= nx;
          x1 /= nx;
          q00 = x0;
          q10 = x1;   // column 0 = eigenvector of l0
          q01 = -x1;
          q11 = x0;   // column 1 = eigenvector of l1
        } else if (a > c) {
          l0 = c;
          l1 = a;
          q00 = 0.0;
          q10 = 1.0;
          q01 = 1.0;
          q11 = 0.0;
        }
      }
      if (lane == 0) {
        W.a[0][0] = l0;
        W.a[0][1] = l1;
        W.q[0][0] = q00;
        W.q[0][1] = q01;
        W.q[0][QLD] = q10;
        W.q[0][QLD + 1] = q11;
        W.cur = 0;
        W.qc = 0;
      }
      wave_sync();
      return 0;
    }
    if (extend_eig(W, m)) return 1;
    const int sweeps = qr_eig(W, m);
    sort_eig(W, m);
    return sweeps + 1;
  }

  // Rank-one extension.  In the basis of T_{m-1}'s eigenvectors plus the new Lanczos
  // vector, T_m is an arrowhead matrix: the poles theta_0 < ... < theta_{n-1}
  // (n = m - 1) and alpha_{m-1} on the diagonal, the couplings z_i = beta_{m-2}
  // Q[m-2][i] in the last row and column.  Its eigenvalues are the roots of
  //   h(lam) = alpha_{m-1} - lam - sum_i z_i^2 / (theta_i - lam),
  // which decreases between poles: one root below theta_0, one between each pair of
  // neighbouring poles, one above theta_{n-1}.  A group of lanes finds root k as an
  // offset x from its nearer pole (so that roots close to a pole keep their relative
  // accuracy) by steps on a rational model of h, bracketed by bisection.  The
  // couplings are then recomputed from the computed roots with Loewner's formula,
  // which makes the roots exact for a nearby arrowhead and the eigenvectors
  // orthogonal to working precision (Gu and Eisenstat); eigenvector k is
  // (z_i / (lam_k - theta_i), 1) normalised, and Q_m = diag(Q_{m-1}, 1) U.
  // Returns false, before anything the QR path reads has changed, when a coupling or
  // a pole gap is negligible against ||T_m|| or an iteration does not settle.
  __device__ bool extend_eig(Small& W, int m) {
    constexpr int NP = MAXM - 1;  // most poles
    const int n = m - 1, cur = W.cur, qc = W.qc;
    const double* th = W.a[cur];
    const double* Q = W.q[qc];
    const double eps = 2.220446049250313e-16;
    const double bc = W.beta[m - 2], alpha = W.alpha[m - 1];
    const double tnorm = fmax(fabs(th[0]), fabs(th[n - 1])) + fabs(alpha) + bc;
    const double tiny = 64.0 * eps * tnorm;
    // lane i < n: pole i and its squared coupling into LDS; negligible couplings or
    // pole gaps end the attempt
    bool bad = !(tnorm < 1e300);
    if (lane < n) {
      const double ti = th[lane], zi = bc * Q[(m - 2) * QLD + lane];
      W.tz[2 * lane] = ti;
      W.tz[2 * lane + 1] = zi * zi;
      if (!(zi * zi > tiny * tiny)) bad = true;
      if (lane + 1 < n && !(th[lane + 1] - ti > tiny)) bad = true;
    }
    if (wave_any(bad)) return false;
    wave_sync();

    // Lanes in groups of G (8 when m <= 8, else 4): group g finds root g.  A lane
    // takes the poles i = sub, sub + G, ... of the pole sums, and the group adds its
    // lanes' parts with DPP, so every lane of the group holds the same sums (additions
    // are commutative, the butterfly order is the same on every lane) and the group's
    // iteration is uniform.
    const int G = (m <= 8) ? 8 : 4;
    const int k = lane / G, sub = lane - (lane / G) * G;
    const bool act = k < m;
    // this lane's poles (i = sub, sub + G, ...) and squared couplings in registers,
    // so that the iterations below read no LDS
    constexpr int NPL = (NP + 3) / 4;
    double pth[NPL], pzz[NPL];
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int i = sub + t * G;
      const int ic = i < n ? i : 0;
      pth[t] = W.tz[2 * ic];
      pzz[t] = W.tz[2 * ic + 1];
    }
    auto gsum = [&](double v) {
      v += dpp_d<0xB1>(v);                 // lane ^ 1
      v += dpp_d<0x4E>(v);                 // lane ^ 2
      if (G == 8) v += dpp_d<0x141>(v);    // the other quad of the half-row
      return v;
    };
    // h and the parts of -h' from poles left (dl_sum) and right (dr_sum) of root k,
    // at lam = tho + x; sabs = sum of |z_i^2 / (theta_i - lam)|
    auto eval = [&](double tho, double x, double& dl_sum, double& dr_sum, double& sabs) {
      double sum = 0.0, dl = 0.0, dr = 0.0, sa = 0.0;
#pragma unroll
      for (int t = 0; t < NPL; ++t) {
        const int i = sub + t * G;
        if (i < n) {
          const double r = rcp_d((pth[t] - tho) - x);
          const double ti = pzz[t] * r;
          sum += ti;
          if (i < k) dl += ti * r;
          else dr += ti * r;
          sa += fabs(ti);
        }
      }
      sum = gsum(sum);
      dl_sum = gsum(dl);
      dr_sum = gsum(dr);
      sabs = gsum(sa);
      return (alpha - tho) - x - sum;
    };

    double tho = 0.0, x = 0.0, lo = 0.0, hi = 0.0, h = 0.0, dls = 0.0, drs = 0.0, sabs = 0.0;
    double DL = 0.0, DR = 0.0;  // poles bracketing an interior root, relative to tho
    const bool interior = act && k > 0 && k < n;
    const double tl = (act && k > 0) ? th[k - 1] : 0.0, tr = (act && k < n) ? th[k] : 0.0;
    int o = 0;  // origin pole
    {
      // interior roots: the midpoint decides the nearer pole (evaluated by every group
      // so that the DPP sums stay uniform; outer groups discard it)
      const double g = tr - tl;
      const double hm = eval(tl, 0.5 * g, dls, drs, sabs);
      if (interior) {
        h = hm;
        if (h > 0.0) {  // root in the right half: origin at theta_k
          o = k;
          tho = tr;
          x = -0.5 * g;
          lo = x;
          hi = 0.0;
          DL = -g;
        } else {
          o = k - 1;
          tho = tl;
          x = 0.5 * g;
          lo = 0.0;
          hi = x;
          DR = g;
        }
      } else if (act) {
        o = (k == 0) ? 0 : n - 1;
        tho = (k == 0) ? tr : tl;
      }
    }
    // the outer roots' Weyl bounds and every group's start: the root of the model that
    // keeps the linear term and the origin pole and freezes the other poles at
    // lam = theta_o
    {
      double a = 0.0, zp = 0.0;
#pragma unroll
      for (int t = 0; t < NPL; ++t) {
        const int i = sub + t * G;
        if (i < n) {
          zp += pzz[t];
          if (i != o) a += pzz[t] * rcp_d(pth[t] - tho);
        }
      }
      a = gsum(a);
      const double zn = sqrt(gsum(zp));
      if (act && !interior) {
        const double A0 = alpha - tho;
        lo = (k == 0) ? 2.0 * (fmin(0.0, A0) - zn) : 0.0;
        hi = (k == 0) ? 0.0 : 2.0 * (fmax(0.0, A0) + zn);
      }
      const double xp = act ? pole_root((alpha - tho) - a, W.tz[2 * o + 1], k > o) : 0.0;
      bool take = false;
      if (act) {
        if (xp > lo && xp < hi) {
          x = xp;
          take = true;
        } else if (!interior) {
          x = 0.5 * (lo + hi);
          take = true;
        }
      }
      double d1, d2, d3;
      const double he = eval(tho, x, d1, d2, d3);
      if (take) {
        h = he;
        dls = d1;
        drs = d2;
        sabs = d3;
      }
    }
    bool done = !act, conv = !act;
    for (int it = 0; it < 60; ++it) {
      if (!done) {
        if (!(h == h)) {
          done = true;
        } else {
          if (h > 0.0) lo = x;
          else hi = x;
          const double A0 = alpha - tho, hp = 1.0 + dls + drs;
          const double errb = eps * (8.0 * sabs + 4.0 * fabs(A0) + 4.0 * fabs(x) + 2.0 * fabs(x) * hp);
          if (fabs(h) <= errb || hi - lo <= 4.0 * eps * fmax(fabs(lo), fabs(hi))) {
            done = conv = true;
          } else {
            // one-pole model: the exact linear term and the origin pole carrying all
            // of the poles' part of -h' (the whole step for an outer root)
            const double s1 = (dls + drs) * x * x;
            const double a1 = ((alpha - tho) - x - h) + (dls + drs) * x;
            double xn = pole_root(A0 - a1, s1, x > 0.0);
            if (interior) {
              // two-pole model: the linear term, and the bracketing poles carrying the
              // poles' part of -h' of their side; two Newton steps from the one-pole root
              const double dl = DL - x, dr = DR - x;
              const double sL = dls * dl * dl, sR = drs * dr * dr;
              const double c = h + x + dls * dl + drs * dr;
              double y = (xn > lo && xn < hi) ? xn : x;
              for (int q = 0; q < 2; ++q) {
                const double rl = rcp_d(DL - y), rr = rcp_d(DR - y);
                const double f = c - y - sL * rl - sR * rr;
                const double fp = -1.0 - sL * rl * rl - sR * rr * rr;
                const double y2 = y - f * rcp_d(fp);
                if (!(y2 > lo && y2 < hi)) break;
                y = y2;
              }
              xn = y;
            }
            const bool bis = !(xn > lo && xn < hi);
            if (bis) xn = 0.5 * (lo + hi);
            if (xn == x) {
              done = conv = true;
            } else if (!bis && fabs(xn - x) <= 0x1p-30 * fabs(xn)) {
              // a model step this small leaves an error far below rounding: take it
              x = xn;
              done = conv = true;
            } else {
              x = xn;
            }
          }
        }
      }
      if (!wave_any(!done)) break;
      double d1, d2, d3;
      const double he = eval(tho, x, d1, d2, d3);
      if (!done) {
        h = he;
        dls = d1;
        drs = d2;
        sabs = d3;
      }
    }
    if (act && sub == 0) {
      W.tho[k] = tho;
      W.xr[k] = x;
      W.a[cur ^ 1][k] = tho + x;
    }
    if (wave_any(!conv)) return false;
    wave_sync();

    // Loewner: zh_i^2 = -prod_j (lam_j - theta_i) / prod_{l != i} (theta_l - theta_i),
    // as a product of interlaced ratios (each of order one, so no overflow)
    bool okz = true;
    if (lane < n) {
      const int i = lane;
      const double ti = W.tz[2 * i];
      // every operand is requested before the first product (entries at and past m
      // are read but not used)
      double f[MAXM], dn[MAXM];
#pragma unroll
      for (int j = 0; j < MAXM; ++j) {
        // denominator pole of factor j: theta_j left of i, theta_{j-1} right of i+1
        const int pj = (j < i) ? j : (j > 0 ? j - 1 : 0);
        dn[j] = W.tz[2 * pj];
        f[j] = (W.tho[j] - ti) + W.xr[j];
      }
#pragma unroll
      for (int j = 0; j < MAXM; ++j) {
        if (j < m) {
          if (j < i || j > i + 1) f[j] *= rcp_d(dn[j] - ti);
        } else {
          f[j] = 1.0;
        }
      }
#pragma unroll
      for (int st = 1; st < MAXM; st *= 2)
#pragma unroll
        for (int j = 0; j + st < MAXM; j += 2 * st) f[j] *= f[j + st];
      const double pr = f[0];
      okz = (pr < 0.0) && (pr > -1e300);
      W.zh[i] = copysign(sqrt(fabs(pr)), Q[(m - 2) * QLD + i]);
    }
    if (wave_any(!okz)) return false;
    wave_sync();

    // eigenvector k of the arrowhead into column k of U
    bool oku = true;
    if (lane < m) {
      const double thl = W.tho[lane], xrl = W.xr[lane];
      double uv[NP], tv[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        uv[i] = W.zh[i];
        tv[i] = W.tz[2 * i];
      }
      double nrm = 1.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        if (i < n) {
          uv[i] *= rcp_d((thl - tv[i]) + xrl);
          nrm += uv[i] * uv[i];
        }
      }
      oku = (nrm < 1e300);
      const double inv = rcp_d(sqrt(nrm));
#pragma unroll
      for (int i = 0; i < NP; ++i)
        if (i < n) W.u[i * QLD + lane] = uv[i] * inv;
      W.u[n * QLD + lane] = inv;
    }
    if (wave_any(!oku)) return false;
    wave_sync();

    // Q_m = diag(Q_{m-1}, 1) U into the other buffer, entries (r, j) spread over lanes
    double* Qn = W.q[qc ^ 1];
    for (int p0 = 0; p0 < 16 * m; p0 += 64) {
      const int pair = p0 + lane, r = pair >> 4, j = pair & 15;
      if (r < m && j < m) {
        double acc;
        if (r < n) {
          double qv[NP], uv[NP];
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            qv[i] = Q[r * QLD + i];
            uv[i] = W.u[i * QLD + j];
          }
          acc = 0.0;
#pragma unroll
          for (int i = 0; i < NP; ++i)
            if (i < n) acc += qv[i] * uv[i];
        } else {
          acc = W.u[n * QLD + j];
        }
        Qn[r * QLD + j] = acc;
      }
    }
    wave_sync();
    if (lane == 0) {
      W.cur = cur ^ 1;
      W.qc = qc ^ 1;
    }
    wave_sync();
    return true;
  }

  // Sorts the eigenpairs of a QR solve into ascending order (ties by index).
  __device__ void sort_eig(Small& W, int m) {
    const int cur = W.cur;
    const double* th = W.a[cur];
    if (lane < m) {
      const double v = th[lane];
      int r = 0;
      for (int j = 0; j < m; ++j) r += (th[j] < v || (th[j] == v && j < lane)) ? 1 : 0;
      W.rank[lane] = r;
      W.a[cur ^ 1][r] = v;
    }
    wave_sync();
    if (lane < m) {
      double row[MAXM];
      double* Q = W.q[W.qc];
#pragma unroll
      for (int c = 0; c < MAXM; ++c) row[c] = (c < m) ? Q[lane * QLD + c] : 0.0;
#pragma unroll
      for (int c = 0; c < MAXM; ++c)
        if (c < m) Q[lane * QLD + W.rank[c]] = row[c];
    }
    wave_sync();
    if (lane == 0) W.cur = cur ^ 1;
    wave_sync();
  }

  // Implicit QR sweeps with the Wilkinson shift on T_m from scratch (the host
  // eigensolver's algorithm).  Every lane reads the same snapshot of T (buffer `in`)
  // and takes the same decisions; lane 0 writes the swept T into the other buffer,
  // which becomes the snapshot after a wave synchronisation, so no lane ever reads an
  // entry while another writes it.  Lane r (< m) keeps row r of the eigenvector
  // matrix in W.q.  Eigenvalues in W.a[W.cur][0..m), unsorted.  Returns the sweeps.
  __device__ int qr_eig(Small& W, int m) {
    if (lane < m) {
      W.a[0][lane] = W.alpha[lane];
      W.b[0][lane] = (lane + 1 < m) ? W.beta[lane] : 0.0;
      for (int c = 0; c < m; ++c) W.q[W.qc][lane * QLD + c] = (c == lane) ? 1.0 : 0.0;
    }
    int in = 0;
    wave_sync();
    const double eps = 2.220446049250313e-16;
    int q = m - 1;
    int sweeps = 0;
    for (; sweeps < 30 * MAXM; ++sweeps) {
      // decisions from the snapshot: trailing unreduced block [p, q]
      const double* A = W.a[in];
      const double* Bv = W.b[in];
      auto negligible = [&](int i) {
        return fabs(Bv[i]) <= eps * (fabs(A[i]) + fabs(A[i + 1]));
      };
      while (q > 0 && negligible(q - 1)) --q;
      if (q == 0) break;
      int p = q - 1;
      while (p > 0 && !negligible(p - 1)) --p;
      // copy the snapshot into the output buffer with negligible couplings zeroed
      const int out = in ^ 1;
      if (lane < m) {
        W.a[out][lane] = A[lane];
        W.b[out][lane] = (lane + 1 < m && !negligible(lane)) ? Bv[lane] : 0.0;
      }
      wave_sync();
      const double aq1 = A[q - 1], aq = A[q], bq = Bv[q - 1];
      const double dd = 0.5 * (aq1 - aq);
      const double den = dd + (dd >= 0.0 ? 1.0 : -1.0) * hypot(dd, bq);
      const double mu = aq - bq * bq / den;
      double x = A[p] - mu, z = Bv[p];
      double ak = A[p], bk = Bv[p];
      for (int k = p; k < q; ++k) {
        const double ak1 = A[k + 1];
        const double bk1 = (k + 1 < q) ? Bv[k + 1] : 0.0;
        const double r = hypot(x, z);
        double c = 1.0, s = 0.0;
        if (r != 0.0) {
          c = x / r;
          s = z / r;
        }
        const double na = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
        const double na1 = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
        const double nb = c * s * (ak1 - ak) + (c * c - s * s) * bk;
        const double bulge = s * bk1;
        const double nb1 = c * bk1;
        if (lane == 0) {
          if (k > p) W.b[out][k - 1] = r;
          W.a[out][k] = na;
          W.a[out][k + 1] = na1;
          W.b[out][k] = nb;
          if (k + 1 < q) W.b[out][k + 1] = nb1;
        }
        if (lane < m) {
          double* qr = &W.q[W.qc][lane * QLD];
          const double qk = qr[k], qk1 = qr[k + 1];
          qr[k] = c * qk + s * qk1;
          qr[k + 1] = -s * qk + c * qk1;
        }
        ak = na1;
        bk = nb1;
        x = nb;
        z = bulge;
      }
      wave_sync();  // the swept T becomes the next snapshot
      in = out;
    }
    W.cur = in;
    wave_sync();
    return sweeps;
  }

  int work = 0;         // QR sweeps spent on the current path
  int nops_budget = 1;  // operators of the current path (sizes the step budget)

  __device__ bool propagate(const BlockDev& B, double dtau, VT (&x)[RPT], double& ell, int& steps,
                            int& subs) {
    Small& W = S.small[wid];
    const int kmax = (P.kmax < MAXM) ? P.kmax : MAXM;
    const double shift = B.shift - P.E0;  // H - E0 = (H - c_b) + (c_b - E0)
    constexpr double EPSV = (sizeof(VT) == 8) ? 2.220446049250313e-16 : 5.9604644775390625e-08;
    double dg[RPT];
    const bool staged = stage_rows(B, dg);
    double remaining = dtau;
    VT V[VL ? 1 : MAXM + 1][RPT];
    // element (i, k) of the basis: V_i at this thread's k-th row
    auto VA = [&](int i, int k) -> VT& {
      if constexpr (VL) return S.vb[i * NR + row(k)];
      else return V[i][k];
    };
    for (int nsub = 0; remaining > 0.0; ++nsub) {
      if (nsub > P.max_substeps) {
        atomicOr(&P.counters[2], ERR_NOCONV);
        return false;
      }
#pragma unroll
      for (int k = 0; k < RPT; ++k) VA(0, k) = x[k];
      int m = 0;
      double tau_used = remaining, theta_min = 0.0, ynorm = 1.0, yv = 0.0, tscale = 0.0;
      for (int j = 0; j < kmax; ++j) {
        VT vj[RPT], w[RPT];
        if constexpr (VL) {
#pragma unroll
          for (int k = 0; k < RPT; ++k) vj[k] = VA(j, k);
          spmv(B, vj, w, dg, staged, S.vb + j * NR);
        } else {
#pragma unroll
          for (int k = 0; k < RPT; ++k) vj[k] = V[0][k];
#pragma unroll
          for (int i = 1; i < MAXM; ++i)
            if (i == j) {
#pragma unroll
              for (int k = 0; k < RPT; ++k) vj[k] = V[i][k];
            }
          spmv(B, vj, w, dg, staged);
        }
        // classical Gram-Schmidt twice against V_0..V_j; the second round also
        // reduces ||w||^2 so that beta_j needs no extra round.  A lane's products
        // and updates run in the vector precision VT (FP32 for mixed paths, whose
        // basis is stored in FP32 anyway), the sums across lanes and ||w||^2 in FP64.
        double hj;
        {
          double h[NRED];
#pragma unroll
          for (int i = 0; i < NRED; ++i) h[i] = 0.0;
#pragma unroll
          for (int i = 0; i < MAXM; ++i)
            if (i <= j) {
              VT hp = VT(0);
#pragma unroll
              for (int k = 0; k < RPT; ++k) hp += VA(i, k) * w[k];
              h[i] = to_d(hp);
            }
          block_sum<NRED>(h, j + 1);
#pragma unroll
          for (int k = 0; k < RPT; ++k) {
            VT t = w[k];
#pragma unroll
            for (int i = 0; i < MAXM; ++i)
              if (i <= j) t -= static_cast<VT>(h[i]) * VA(i, k);
            w[k] = t;
          }
          hj = h[0];
#pragma unroll
          for (int i = 1; i < MAXM; ++i)
            if (i == j) hj = h[i];
        }
        double bj;
        {
          double h[NRED];
#pragma unroll
          for (int i = 0; i < NRED; ++i) h[i] = 0.0;
          double wn = 0.0;
          VT hp[MAXM];
#pragma unroll
          for (int i = 0; i < MAXM; ++i) hp[i] = VT(0);
#pragma unroll
          for (int k = 0; k < RPT; ++k) {
            const double wd = to_d(w[k]);
#pragma unroll
            for (int i = 0; i < MAXM; ++i)
              if (i <= j) hp[i] += VA(i, k) * w[k];
            wn += wd * wd;
          }
#pragma unroll
          for (int i = 0; i < MAXM; ++i)
            if (i <= j) h[i] = to_d(hp[i]);
#pragma unroll
          for (int i = 1; i < NRED; ++i)
            if (i == j + 1) h[i] = wn;
          block_sum<NRED>(h, j + 2);
          double wn2 = 0.0, corr = 0.0;
#pragma unroll
          for (int i = 1; i < NRED; ++i)
            if (i == j + 1) wn2 = h[i];
#pragma unroll
          for (int i = 0; i < MAXM; ++i)
            if (i <= j) corr += h[i] * h[i];
#pragma unroll
          for (int k = 0; k < RPT; ++k) {
            VT t = w[k];
#pragma unroll
            for (int i = 0; i < MAXM; ++i)
              if (i <= j) t -= static_cast<VT>(h[i]) * VA(i, k);
            w[k] = t;
          }
          double h2j = h[0];
#pragma unroll
          for (int i = 1; i < MAXM; ++i)
            if (i == j) h2j = h[i];
          hj += h2j;
          const double b2 = wn2 - corr;
          bj = b2 > 0.0 ? sqrt(b2) : 0.0;
        }
        if (lane == 0) {
          W.alpha[j] = hj;
          W.beta[j] = bj;
        }
        wave_sync();
        tscale = fmax(tscale, fabs(hj) + bj);
        ++steps;
        // small problem: eigendecomposition of T_{j+1}, then
        // y = Q exp(-tau (Theta - theta_min)) Q^T e_1 and the a-posteriori estimate
        work += small_eig(W, j + 1);
        if (work > P.work_budget || steps > 40 * nops_budget + 400) {
          // far beyond any healthy propagation: report instead of grinding on
          atomicOr(&P.counters[2], ERR_NOCONV);
          return false;
        }
        // eigenvalues ascend, so theta_0 is the smallest; lane i (<= j) takes the
        // term of eigenpair i: w_i = exp(-tau (theta_i - theta_0)) Q[0][i], with
        // ||y||^2 = sum_i w_i^2 and y_j = sum_i Q[j][i] w_i
        const double* theta = W.a[W.cur];
        const double* Q = W.q[W.qc];
        theta_min = theta[0];
        const double dth = (lane <= j) ? theta[lane] - theta_min : 0.0;
        const double q0 = (lane <= j) ? Q[lane] : 0.0;
        const double qj = (lane <= j) ? Q[j * QLD + lane] : 0.0;
        const double breakdown = 4.0 * EPSV * (tscale + 1e-300);
        const bool last = (j + 1 >= kmax);
        double tau_try = remaining;
        bool ok = false;
        double wl = 0.0;
        for (int attempt = 0; attempt < 60; ++attempt) {
          wl = exp(-tau_try * dth) * q0;
          const double yn2 = wave_sum(wl * wl);
          const double ylast = wave_sum(qj * wl);
          ynorm = sqrt(yn2);
          const double est = bj * fabs(ylast) * rcp_d(ynorm);
          ok = (est <= P.tol) || (bj <= breakdown);
          if (ok || !last) break;
          tau_try *= 0.5;  // depth cap reached: shorten the substep
        }
        if (ok) {
          // y = Q w: lane r (<= j) gets component r
          if (lane <= j) W.wk[lane] = wl;
          wave_sync();
          const int rr = lane <= j ? lane : 0;
          double qv[MAXM], wv[MAXM];
#pragma unroll
          for (int i = 0; i < MAXM; ++i) {
            qv[i] = Q[rr * QLD + i];
            wv[i] = W.wk[i];
          }
          double yr = 0.0;
#pragma unroll
          for (int i = 0; i < MAXM; ++i)
            if (i <= j) yr += qv[i] * wv[i];
          m = j + 1;
          tau_used = tau_try;
          yv = (lane <= j) ? yr : 0.0;
          break;
        }
        if (last) {
          atomicOr(&P.counters[2], ERR_NOCONV);
          return false;
        }
        const double inv = rcp_d(bj);
#pragma unroll
        for (int i = 1; i <= MAXM; ++i)
          if (i == j + 1) {
#pragma unroll
            for (int k = 0; k < RPT; ++k) VA(i, k) = static_cast<VT>(to_d(w[k]) * inv);
          }
      }
      // recombination x = V_m y / ||y||
      const double inv = rcp_d(ynorm);
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < MAXM; ++i)
          if (i < m) t += readlane_d(yv, i) * to_d(VA(i, k));
        x[k] = static_cast<VT>(t * inv);
      }
      ell += -tau_used * (shift + theta_min) + log(ynorm);
      remaining -= tau_used;
      if (remaining > 0.0) ++subs;
    }
    return true;
  }

};

__device__ inline void scan_pair(const TraceParams& P, int64_t id, const float* width) {
  const int c = int(id / P.n_ret), r = int(id - int64_t(c) * P.n_ret);
  const int64_t o0 = P.offsets[c], o1 = cfg_end(P, c);
  int err = 0;
  const BlockDev B0 = P.blocks[P.ret_block[r]];
  int nu = B0.n_up, nd = B0.n_dn;
  int mid = P.ret_block[r];
  bool feas = true;
  double prev = -1.0, cost = 0.0;
  if (o1 < o0) err |= ERR_UNSORTED;
  for (int64_t k = o0; k < o1; ++k) {
    const double t = P.tau[k];
    if (!(t >= 0.0) || !(t < P.beta) || !(t > prev)) err |= ERR_UNSORTED;
    // the interval before operator k, spent in the block the path is in
    if (k > o0 && feas) {
      const double sq = sqrt(fmax(t - prev, 0.0) * double(width[nd * (P.n_orb + 1) + nu]));
      cost += sq * sqrt(sq);
    }
    prev = t;
    const int f = P.flavor[k];
    const int dg = P.dagger[k];
    if (f < 0 || f >= 2 * P.n_orb || (dg != 0 && dg != 1)) {
      err |= ERR_FLAVOR;
      continue;
    }
    const int step = dg ? 1 : -1;
    if (f < P.n_orb) nu += step; else nd += step;
    if (nu < 0 || nu > P.n_orb || nd < 0 || nd > P.n_orb) feas = false;
    if (feas && t < P.tau_mid) mid = nd * (P.n_orb + 1) + nu;
  }
  if (P.p_midblk) P.p_midblk[id] = feas ? mid : -1;
  if (nu != B0.n_up || nd != B0.n_dn) feas = false;
  if (err) feas = false;
  P.p_sign[id] = 0;
  P.p_log[id] = -INFINITY;
  P.p_steps[id] = 0;
  P.p_sub[id] = feas ? 0 : -1;
  P.p_rowsteps[id] = 0;
  P.p_rows[id] = 0;
  if (err && r == 0) atomicOr(&P.counters[2], err);
  if (r == 0 && o1 > o0) atomicMax(&P.counters[1], int(o1 - o0));
  if (P.p_bucket) {
    int b = -1;
    if (feas) {
      b = min(ORDER_NB - 1, int(8.0 * log2(1.0 + cost)));
      atomicAdd(&P.counters[0], 1);
      atomicAdd(&P.counters[4 + b], 1);
    }
    P.p_bucket[id] = b;
  } else if (feas) {
    const int slot = atomicAdd(&P.counters[0], 1);
    P.work[slot] = int32_t(id);
  }
}

// Signed log-sum over the retained states of every configuration (step 8),
// in a fixed order so that repeated runs are bitwise identical.
__device__ inline void reduce_config(const TraceParams& P, int c, double* out_log, int8_t* out_sign,
                                     int32_t* out_steps, int32_t* out_sub, int32_t* out_feas,
                                     int64_t* out_rowsteps, int64_t* out_rows) {
  const int64_t base = int64_t(c) * P.n_ret;
  double mx = -INFINITY;
  int steps = 0, subs = 0, feas = 0;
  int64_t rs = 0, rw = 0;
  for (int r = 0; r < P.n_ret; ++r) {
    if (P.p_sign[base + r] != 0) mx = fmax(mx, P.p_log[base + r]);
    steps += P.p_steps[base + r];
    rs += P.p_rowsteps[base + r];
    rw += P.p_rows[base + r];
    if (P.p_sub[base + r] >= 0) {
      ++feas;
      subs += P.p_sub[base + r];
    }
  }
  int8_t sg = 0;
  double lg = -INFINITY;
  if (mx > -INFINITY) {
    double s = 0.0;
    for (int r = 0; r < P.n_ret; ++r) {
      const int8_t q = P.p_sign[base + r];
      if (q != 0) s += q * exp(P.p_log[base + r] - mx);
    }
    if (s != 0.0) {
      sg = s > 0.0 ? 1 : -1;
      lg = mx + log(fabs(s));
    }
  }
  out_log[c] = lg;
  out_sign[c] = sg;
  if (out_steps) out_steps[c] = steps;
  if (out_sub) out_sub[c] = subs;
  if (out_feas) out_feas[c] = feas;
  if (out_rowsteps) out_rowsteps[c] = rs;
  if (out_rows) out_rows[c] = rw;
}

// ---- step-synchronous path kernels (one workgroup per queued path) ----------

template <typename VT>
__device__ __forceinline__ VT* path_vec(const TraceParams& P, int parity, int w) {
  return static_cast<VT*>(P.st_vec) + (int64_t(parity) * P.n_pairs + w) * P.vstride;
}

// Step 3: the retained eigenstate enters with the phase of the two edge intervals.
template <typename VT, int NT>
__device__ inline void path_init(const TraceParams& P, int w) {
  const int id = P.work[w];
  const int c = id / P.n_ret, r = id - c * P.n_ret;
  const int64_t o0 = P.offsets[c], o1 = cfg_end(P, c);
  const int b = P.ret_block[r];
  const int dim = P.blocks[b].dim;
  const VT* src = (sizeof(VT) == 8) ? reinterpret_cast<const VT*>(P.ret_vec64 + P.ret_off[r])
                                    : reinterpret_cast<const VT*>(P.ret_vec32 + P.ret_off[r]);
  VT* dst = path_vec<VT>(P, 0, w);
  for (int i = threadIdx.x; i < dim; i += NT) dst[i] = src[i];
  if (threadIdx.x == 0) {
    const double Ei = P.ret_energy[r];
    P.st_block[w] = b;
    P.st_status[w] = (o1 > o0) ? PATH_ACTIVE : PATH_EMPTY;
    P.st_steps[w] = 0;
    P.st_subs[w] = 0;
    P.st_rowsteps[w] = 0;
    P.st_rows[w] = 0;
    P.st_ell[w] = (o1 > o0) ? -(P.beta - P.tau[o1 - 1] + P.tau[o0]) * (Ei - P.E0) : 0.0;
  }
}

// Component r of O x in the target block Bt, for O = c_f (dg = 0) or c_f^dag
// (dg = 1) and x a vector of the source block (indexed by in-block rank): the
// source state s with O|s> ~ |t> is t with bit f flipped (a creator needs bit f set
// in t, an annihilator needs it clear), and the Jordan-Wigner sign is the parity
// of the occupied flavors below f.  Only moves and sign flips: bit-exact.
template <typename VT>
__device__ __forceinline__ VT gather_op(const uint32_t* states, const int32_t* rank, const BlockDev& Bt, int r,
                                        int f, int dg, const VT* x) {
  const uint32_t bit = 1u << f;
  const uint32_t t = states[Bt.state_off + r];
  const bool has = dg ? ((t & bit) != 0u) : ((t & bit) == 0u);
  if (!has) return VT(0);
  const uint32_t s = t ^ bit;
  const VT v = x[rank[s]];
  return (__popc(s & (bit - 1u)) & 1) ? -v : v;
}

// Step 4: operator k of the path's configuration, a signed gather from block b to
// the target block, then renormalisation with the log of the norm kept in ell.
template <typename VT, int NT, int RPT>
__device__ inline void path_op(const TraceParams& P, int w, int k, double* red) {
  if (P.st_status[w] != PATH_ACTIVE) return;
  const int id = P.work[w];
  const int c = id / P.n_ret;
  const int64_t o0 = P.offsets[c], o1 = cfg_end(P, c);
  if (k >= o1 - o0) return;
  const int f = P.flavor[o0 + k];
  const int dg = P.dagger[o0 + k] ? 1 : 0;
  const BlockDev B = P.blocks[P.st_block[w]];
  int nu = B.n_up, nd = B.n_dn;
  if (f < P.n_orb) nu += dg ? 1 : -1; else nd += dg ? 1 : -1;
  if (nu < 0 || nu > P.n_orb || nd < 0 || nd > P.n_orb) {  // excluded by the scan
    if (threadIdx.x == 0) P.st_status[w] = PATH_FAILED;
    return;
  }
  const int bt = nd * (P.n_orb + 1) + nu;
  const BlockDev Bt = P.blocks[bt];
  const VT* src = path_vec<VT>(P, k & 1, w);
  VT* dst = path_vec<VT>(P, (k + 1) & 1, w);
  VT val[RPT];
  double part = 0.0;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = threadIdx.x + q * NT;
    const VT v = (r < Bt.dim) ? gather_op<VT>(P.states, P.rank, Bt, r, f, dg, src) : VT(0);
    val[q] = v;
    part += to_d(v) * to_d(v);
  }
  part = wave_sum(part);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  double n2 = 0.0;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) n2 += red[q];
  // The input is a unit vector: a result this small is a zero imposed by symmetry
  // in exact arithmetic and rounding noise in floating point.
  if (!(n2 > P.zero_tol2) || !isfinite(n2)) {
    if (threadIdx.x == 0) {
      const bool zero = (n2 >= 0.0) && (n2 <= P.zero_tol2);
      P.st_status[w] = zero ? PATH_ZERO : PATH_FAILED;
      if (!zero) atomicOr(&P.counters[2], ERR_NONFINITE);
    }
    return;
  }
  const double inv = rcp_d(sqrt(n2));
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = threadIdx.x + q * NT;
    if (r < Bt.dim) dst[r] = static_cast<VT>(to_d(val[q]) * inv);
  }
  if (threadIdx.x == 0) {
    P.st_block[w] = bt;
    P.st_ell[w] += 0.5 * log(n2);
  }
}

// Step 5: Krylov propagation of the path's vector over tau_k - tau_{k-1}, in place.
template <typename VT, int NT, int RPT, int MAXM, bool MF, bool VL>
__device__ inline void path_prop(const TraceParams& P, int w, int k,
                                 typename PathEngine<VT, NT, RPT, MAXM, MF, VL>::Smem& S) {
  using E = PathEngine<VT, NT, RPT, MAXM, MF, VL>;
  if (P.st_status[w] != PATH_ACTIVE) return;
  const int id = P.work[w];
  const int c = id / P.n_ret;
  const int64_t o0 = P.offsets[c], o1 = cfg_end(P, c);
  if (k >= o1 - o0) return;
  E eng(P, S);
  const BlockDev B = P.blocks[P.st_block[w]];
  VT* vec = path_vec<VT>(P, k & 1, w);
  VT x[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = eng.row(q);
    x[q] = (r < B.dim) ? vec[r] : VT(0);
  }
  double ell = 0.0;
  int steps = 0, subs = 0;
  eng.work = 0;
  eng.nops_budget = 1;
  const bool ok = eng.propagate(B, P.tau[o0 + k] - P.tau[o0 + k - 1], x, ell, steps, subs);
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = eng.row(q);
    if (r < B.dim) vec[r] = x[q];
  }
  if (threadIdx.x == 0) {
    P.st_ell[w] += ell;
    P.st_steps[w] += steps;
    P.st_subs[w] += subs;
    P.st_rowsteps[w] += int64_t(steps) * B.dim;
    P.st_rows[w] += B.dim;
    if (!ok) P.st_status[w] = PATH_FAILED;
  }
}

// Running totals of one path between its first and last operator (kept in LDS by
// thread 0, so that they hold no registers during the propagations).
struct PathCarry {
  double ell;
  int64_t rowsteps, rows;
  int32_t steps, subs;
};

// The model's block table and the one-spin pattern tables (n_orb <= 7), copied into
// LDS once per launch, so that an operator's target block, the target states and the
// source ranks come from LDS and integer arithmetic instead of dependent global
// loads.  Pattern i (ascending) with c bits set is pat[off[c] + i]; rank_half inverts
// it; the state of row r of block (n_up, n_dn) is pat[off[n_up] + r % up_states] |
// pat[off[n_dn] + r / up_states] << n_orb.
struct PathTables {
  BlockDev blk[64];
  int16_t rh[128];
  uint8_t pat[128];
  int16_t off[8];
};

template <int NT>
__device__ inline void path_tables_load(const TraceParams& P, PathTables& T) {
  const int n = P.n_orb, nb = (n + 1) * (n + 1), ns = 1 << n;
  for (int i = threadIdx.x; i < nb; i += NT) T.blk[i] = P.blocks[i];
  for (int i = threadIdx.x; i < ns; i += NT) T.rh[i] = P.rank_half[i];
  if (int(threadIdx.x) <= n) {
    // patterns with fewer than c bits: sum of C(n, c') over c' < c
    const int c = threadIdx.x;
    int off = 0, b = 1;
    for (int q = 0; q < c; ++q) {
      off += b;
      b = b * (n - q) / (q + 1);
    }
    T.off[c] = int16_t(off);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ns; i += NT) T.pat[T.off[__popc(i)] + T.rh[i]] = uint8_t(i);
  __syncthreads();
}

// gather_op with the states and ranks from the LDS tables: component r of O x in the
// target block Bt for x in the source block B (the same moves and sign flips).
template <typename VT>
__device__ __forceinline__ VT gather_tab(const PathTables& T, int n, const BlockDev& B, const BlockDev& Bt, int r,
                                         int f, int dg, const VT* x) {
  const uint32_t bit = 1u << f, lo = (1u << n) - 1u;
  const int dr = r / Bt.up_states, ur = r - dr * Bt.up_states;
  const uint32_t t = uint32_t(T.pat[T.off[Bt.n_up] + ur]) | (uint32_t(T.pat[T.off[Bt.n_dn] + dr]) << n);
  const bool has = dg ? ((t & bit) != 0u) : ((t & bit) == 0u);
  if (!has) return VT(0);
  const uint32_t s = t ^ bit;
  const VT v = x[int(T.rh[s >> n]) * B.up_states + int(T.rh[s & lo])];
  return (__popc(s & (bit - 1u)) & 1) ? -v : v;
}

// Steps 4-5 for operators [k0, k1) of one path, fused: the same arithmetic as
// path_prop / path_op in the same order, with the vector in registers, the totals
// in LDS and the operator's gather reading the vector and the model tables from LDS,
// so that only the first and the last operator touch the path's global state.  k1
// must not exceed the configuration's operator count.
template <typename VT, int NT, int RPT, int MAXM, bool MF, bool VL>
__device__ inline void path_run(const TraceParams& P, int w, int k0, int k1,
                                typename PathEngine<VT, NT, RPT, MAXM, MF, VL>::Smem& S, double* red,
                                PathCarry& pc, const PathTables& T) {
  using E = PathEngine<VT, NT, RPT, MAXM, MF, VL>;
  if (k0 >= k1 || P.st_status[w] != PATH_ACTIVE) return;
  const int id = P.work[w];
  const int c = id / P.n_ret;
  const int64_t o0 = P.offsets[c];
  const int n = P.n_orb;
  E eng(P, S);
  int status = PATH_ACTIVE;
  int blk = P.st_block[w];
  if (threadIdx.x == 0) {
    pc.ell = P.st_ell[w];
    pc.steps = P.st_steps[w];
    pc.subs = P.st_subs[w];
    pc.rowsteps = P.st_rowsteps[w];
    pc.rows = P.st_rows[w];
  }
  VT x[RPT];
  {
    const int dim = T.blk[blk].dim;
    const VT* vec = path_vec<VT>(P, k0 & 1, w);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = eng.row(q);
      x[q] = (r < dim) ? vec[r] : VT(0);
    }
  }
  // the vector in LDS for the operator's gather (VL engines keep no separate copy)
  VT* xs = VL ? S.vb : S.vec;
  int k = k0;
  for (; k < k1; ++k) {
    const BlockDev B = T.blk[blk];
    if (k > 0) {
      double ell = 0.0;
      int steps = 0, subs = 0;
      eng.work = 0;
      eng.nops_budget = 1;
      const bool ok = eng.propagate(B, P.tau[o0 + k] - P.tau[o0 + k - 1], x, ell, steps, subs);
      if (threadIdx.x == 0) {
        pc.ell += ell;
        pc.steps += steps;
        pc.subs += subs;
        pc.rowsteps += int64_t(steps) * B.dim;
        pc.rows += B.dim;
      }
      if (!ok) {
        status = PATH_FAILED;
        break;
      }
    }
    // operator k: signed gather from the source block into the target block
    const int f = P.flavor[o0 + k];
    const int dg = P.dagger[o0 + k] ? 1 : 0;
    int nu = B.n_up, nd = B.n_dn;
    if (f < n) nu += dg ? 1 : -1; else nd += dg ? 1 : -1;
    if (nu < 0 || nu > n || nd < 0 || nd > n) {  // excluded by the scan
      status = PATH_FAILED;
      break;
    }
    const int bt = nd * (n + 1) + nu;
    const BlockDev Bt = T.blk[bt];
    __syncthreads();  // the propagation's last LDS reads are done
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = eng.row(q);
      if (r < B.dim) xs[r] = x[q];
    }
    __syncthreads();
    VT val[RPT];
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = eng.row(q);
      const VT v = (r < Bt.dim) ? gather_tab<VT>(T, n, B, Bt, r, f, dg, xs) : VT(0);
      val[q] = v;
      part += to_d(v) * to_d(v);
    }
    part = wave_sum(part);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    double n2 = 0.0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) n2 += red[q];
    __syncthreads();  // red and xs are rewritten by the next operator / propagation
    // a unit vector mapped to (almost) nothing: a zero imposed by symmetry
    if (!(n2 > P.zero_tol2) || !isfinite(n2)) {
      const bool zero = (n2 >= 0.0) && (n2 <= P.zero_tol2);
      status = zero ? PATH_ZERO : PATH_FAILED;
      if (!zero && threadIdx.x == 0) atomicOr(&P.counters[2], ERR_NONFINITE);
      break;
    }
    const double inv = rcp_d(sqrt(n2));
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = eng.row(q);
      x[q] = (r < Bt.dim) ? static_cast<VT>(to_d(val[q]) * inv) : VT(0);
    }
    blk = bt;
    if (threadIdx.x == 0) pc.ell += 0.5 * log(n2);
  }
  if (status == PATH_ACTIVE) {
    // operators [k0, k1) applied: the vector goes where operator k1 - 1 leaves it
    const int dim = T.blk[blk].dim;
    VT* vec = path_vec<VT>(P, k1 & 1, w);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = eng.row(q);
      if (r < dim) vec[r] = x[q];
    }
  }
  if (threadIdx.x == 0) {
    P.st_status[w] = status;
    P.st_block[w] = blk;
    P.st_ell[w] = pc.ell;
    P.st_steps[w] = pc.steps;
    P.st_subs[w] = pc.subs;
    P.st_rowsteps[w] = pc.rowsteps;
    P.st_rows[w] = pc.rows;
  }
}

// Step 7: overlap with <E_i| closes the path; writes the per-path sign / log.
template <typename VT, int NT, int RPT>
__device__ inline void path_final(const TraceParams& P, int w, double* red) {
  const int id = P.work[w];
  const int c = id / P.n_ret, r = id - c * P.n_ret;
  const int status = P.st_status[w];
  const double Ei = P.ret_energy[r];
  if (status == PATH_EMPTY) {
    if (threadIdx.x == 0) {
      P.p_sign[id] = 1;
      P.p_log[id] = -P.beta * Ei;
      P.p_steps[id] = 0;
      P.p_sub[id] = 0;
      P.p_rowsteps[id] = 0;
      P.p_rows[id] = 0;
    }
    return;
  }
  const int64_t nops = cfg_end(P, c) - P.offsets[c];
  const int b = P.ret_block[r];
  const int dim = P.blocks[b].dim;
  const VT* v = path_vec<VT>(P, int(nops & 1), w);
  const VT* e = (sizeof(VT) == 8) ? reinterpret_cast<const VT*>(P.ret_vec64 + P.ret_off[r])
                                  : reinterpret_cast<const VT*>(P.ret_vec32 + P.ret_off[r]);
  double part = 0.0;
  if (status == PATH_ACTIVE && P.st_block[w] == b) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int i = threadIdx.x + q * NT;
      if (i < dim) part += to_d(e[i]) * to_d(v[i]);
    }
  }
  part = wave_sum(part);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double ov = 0.0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) ov += red[q];
    // unit vectors: an overlap below the zero threshold is a symmetry zero
    if (status != PATH_ACTIVE || !(fabs(ov) * fabs(ov) > P.zero_tol2)) {
      P.p_sign[id] = 0;
      P.p_log[id] = -INFINITY;
    } else {
      P.p_sign[id] = ov > 0.0 ? 1 : -1;
      P.p_log[id] = P.st_ell[w] + log(fabs(ov)) - P.beta * P.E0;
    }
    P.p_steps[id] = P.st_steps[w];
    P.p_sub[id] = P.st_subs[w];
    P.p_rowsteps[id] = P.st_rowsteps[w];
    P.p_rows[id] = P.st_rows[w];
    if (status == PATH_FAILED) atomicOr(&P.counters[2], ERR_NOCONV);
  }
}

}  // namespace hyb
