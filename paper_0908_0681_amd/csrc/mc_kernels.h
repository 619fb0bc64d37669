// Device side of the Monte Carlo layer (included by mc.hip and by CPU builds of
// the same code): move records, the counter-based generator, the bath
// interpolation, and the bodies of the proposal and acceptance kernels.  One
// wavefront (64 lanes) per chain.
#pragma once

#include "trace_kernels.h"
#include "mlp_kernels.h"

// Operator times, table positions and acceptance ratios are computed with one
// rounding per operation (no fused multiply-add), so that they are the same
// doubles on every platform that follows IEEE 754.  The pragma covers this
// file; the library builds the including translation unit with
// -ffp-contract=off so that inlined helpers from other headers are covered too.
#ifdef __clang__
#pragma clang fp contract(off)
#endif

namespace hyb {

struct MoveRec {
  int32_t kind;   // 0 impossible, 1 insert, 2 remove
  int32_t valid;  // 0: the proposed configuration has zero weight (time tie)
  int32_t f, k, i, j;
  int32_t pad;
  double ts, te;  // insert: creator / annihilator times
  double ratio;   // det A_f' / det A_f (with the relabelling of a removal)
  double logq;    // learned proposal: log q(tau_s, l) of the inserted / removed pair
};

enum : int { ST_INS_PROP = 0, ST_INS_ACC, ST_REM_PROP, ST_REM_ACC, ST_IMPOSSIBLE, ST_ZERO, ST_ORDER, ST_MOVES, ST_N };

struct MCParams {
  int32_t n_chains, F, kmax, nmax, n_delta, n_tau;
  double beta;
  uint32_t key0, key1;
  const double* delta;
  int32_t* kf;   // [C][F]
  double* cre;   // [C][F][kmax]
  double* ann;   // [C][F][kmax]
  double* M;     // [C][F][kmax][kmax], row = annihilator label, column = creator label
  int32_t* cur_n;
  double* cur_tau;  // [C][nmax]
  int16_t* cur_fl;
  int8_t* cur_dg;
  const int64_t* p_begin;  // [C] = c * nmax
  int64_t* p_end;
  double* p_tau;
  int16_t* p_fl;
  int8_t* p_dg;
  MoveRec* mv;
  double* uvec;  // [C][kmax]: M b of an insertion
  double* vvec;  // [C][kmax]: c^T M of an insertion
  double* cur_logtr;
  int32_t* cur_signtr;
  double* cur_logdet;
  int32_t* cur_signdet;
  int32_t* cur_sign;
  const double* t_log;
  const int8_t* t_sign;
  int64_t* stats;     // [C][ST_N]
  double* sign_sum;   // [C]
  double* gacc;       // [C][F][n_tau]
  double* meas_sign;  // [C]
  int64_t* n_meas;    // [C]
  int64_t* step_dev;  // [1] move counter; move `off` of a launch sequence is *step_dev + off
  // learned proposal (learned != 0): features [C][MLP_IN] and logits [C][MLP_OUT]
  int32_t learned;
  double eps_mix;
  __bf16* X;
  const float* logits;
  // (n_up, n_dn) sector weights at beta/2: the trace workspace's per-path results of
  // the proposals (sign, log, block at beta/2; pair id = chain * n_ret + r), the
  // proposal's distribution over the n_blocks sectors, the current one, and the
  // sign-weighted accumulators, each [C][n_blocks]
  int32_t n_blocks, n_ret;
  const int8_t* pr_sign;
  const double* pr_log;
  const int32_t* pr_mid;
  double* psec_prop;
  double* cur_psec;
  double* sec_acc;
};

// The proposal's sector distribution at beta/2 (lane 0 of the chain's wavefront, in
// retained-state order so that repeated runs are bitwise equal):
// P_s = sum_{r: block_r(beta/2) = s} t_r / sum_r t_r over the retained-state paths.
__device__ inline void mc_sectors(const MCParams& Q, int c) {
  if (threadIdx.x != 0) return;
  const int64_t base = int64_t(c) * Q.n_ret;
  double mx = -INFINITY;
  for (int r = 0; r < Q.n_ret; ++r)
    if (Q.pr_sign[base + r] != 0) mx = fmax(mx, Q.pr_log[base + r]);
  double* out = Q.psec_prop + int64_t(c) * Q.n_blocks;
  for (int b = 0; b < Q.n_blocks; ++b) out[b] = 0.0;
  if (!(mx > -INFINITY)) return;
  double tot = 0.0;
  for (int r = 0; r < Q.n_ret; ++r) {
    const int8_t sg = Q.pr_sign[base + r];
    const int b = Q.pr_mid[base + r];
    if (sg == 0 || b < 0) continue;
    const double t = sg * exp(Q.pr_log[base + r] - mx);
    out[b] += t;
    tot += t;
  }
  if (tot != 0.0)
    for (int b = 0; b < Q.n_blocks; ++b) out[b] /= tot;
}

// ---- generator -------------------------------------------------------------

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = uint64_t(0xD2511F53u) * c[0];
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c[2];
    const uint32_t n0 = uint32_t(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = uint32_t(p0 >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = uint32_t(p1);
    c[2] = n2;
    c[3] = uint32_t(p0);
  }
}

// 53 random bits from two words; exact in double, identical on every platform.
__device__ __forceinline__ double u01(uint32_t a, uint32_t b) {
  return (double(a >> 5) * 67108864.0 + double(b >> 6)) * (1.0 / 9007199254740992.0);
}

__device__ inline void move_uniforms(const MCParams& Q, int chain, int64_t step, double (&u)[6]) {
#pragma unroll
  for (int call = 0; call < 3; ++call) {
    uint32_t c[4] = {uint32_t(uint64_t(step)), uint32_t(uint64_t(step) >> 32), uint32_t(chain), uint32_t(call)};
    philox4x32_10(c, Q.key0, Q.key1);
    u[2 * call] = u01(c[0], c[1]);
    u[2 * call + 1] = u01(c[2], c[3]);
  }
}

// u6..u9 of a move (calls 3 and 4), drawn only by the learned proposal.
__device__ inline void move_uniforms_extra(const MCParams& Q, int chain, int64_t step, double (&u)[4]) {
#pragma unroll
  for (int call = 3; call < 5; ++call) {
    uint32_t c[4] = {uint32_t(uint64_t(step)), uint32_t(uint64_t(step) >> 32), uint32_t(chain), uint32_t(call)};
    philox4x32_10(c, Q.key0, Q.key1);
    u[2 * (call - 3)] = u01(c[0], c[1]);
    u[2 * (call - 3) + 1] = u01(c[2], c[3]);
  }
}

// ---- learned proposal ---------------------------------------------------------

// Softmax probability of bin b among the 64 logits z[0..64) (uniform over lanes).
__device__ inline void softmax64(const float* z, float& mx, float& sum) {
  mx = z[0];
  for (int q = 1; q < MLP_BINS; ++q) mx = fmaxf(mx, z[q]);
  sum = 0.0f;
  for (int q = 0; q < MLP_BINS; ++q) sum += expf(z[q] - mx);
}

// log q(ts, l) = log[(1 - eps) p_tau(bin ts) (64/beta) p_l(bin l) (64/beta) + eps / beta^2]
__device__ inline double mlp_logq(const MCParams& Q, const float* z, double ts, double l) {
  float m0, s0, m1, s1;
  softmax64(z, m0, s0);
  softmax64(z + MLP_BINS, m1, s1);
  int bs = int(ts / Q.beta * MLP_BINS), bl = int(l / Q.beta * MLP_BINS);
  bs = bs > MLP_BINS - 1 ? MLP_BINS - 1 : bs;
  bl = bl > MLP_BINS - 1 ? MLP_BINS - 1 : bl;
  const double pt = double(expf(z[bs] - m0) / s0), pl = double(expf(z[MLP_BINS + bl] - m1) / s1);
  const double d = MLP_BINS / Q.beta;
  return log((1.0 - Q.eps_mix) * pt * d * pl * d + Q.eps_mix / (Q.beta * Q.beta));
}

// Inverse-CDF draw of a bin from 64 logits with uniform u.
__device__ inline int mlp_draw_bin(const float* z, double u) {
  float mx, sum;
  softmax64(z, mx, sum);
  const double target = u * double(sum);
  double acc = 0.0;
  for (int q = 0; q < MLP_BINS - 1; ++q) {
    acc += double(expf(z[q] - mx));
    if (target < acc) return q;
  }
  return MLP_BINS - 1;
}

// Phase A of a learned move: the move type, flavor and (for a removal) the pair,
// and the features of the configuration the pair is inserted into / removed from.
__device__ inline void mc_choose(const MCParams& Q, int c, int64_t step) {
  double u[6];
  move_uniforms(Q, c, step, u);
  const int F = Q.F, KM = Q.kmax;
  int f = int(__dmul_rn(u[0], double(F)));
  if (f > F - 1) f = F - 1;
  const bool ins = u[1] < 0.5;
  const int k = Q.kf[c * F + f];
  int i = -1, j = -1;
  if (!ins && k > 0) {
    i = int(__dmul_rn(u[2], double(k)));
    j = int(__dmul_rn(u[3], double(k)));
    if (i > k - 1) i = k - 1;
    if (j > k - 1) j = k - 1;
  }
  mlp_features(F, KM, Q.beta, Q.kf + c * F, Q.cre + int64_t(c) * F * KM, Q.ann + int64_t(c) * F * KM, f,
               (i >= 0) ? f : -1, i, j, Q.X + int64_t(c) * MLP_IN);
}

// ---- bath --------------------------------------------------------------------

// Linear interpolation of the tabulated Delta on [0, beta], antiperiodic outside.
__device__ __forceinline__ double delta_at(const MCParams& Q, double tau) {
  double sgn = 1.0;
  if (tau < 0.0) {
    tau = __dadd_rn(tau, Q.beta);
    sgn = -1.0;
  }
  const double x = __dmul_rn(__ddiv_rn(tau, Q.beta), double(Q.n_delta));
  int k = int(x);
  if (k > Q.n_delta - 1) k = Q.n_delta - 1;
  const double fr = __dadd_rn(x, -double(k));
  const double a = Q.delta[k], b = Q.delta[k + 1];
  return sgn * __dadd_rn(a, __dmul_rn(fr, __dadd_rn(b, -a)));
}

__device__ __forceinline__ double wave_sum64(double x) { return wave_sum(x); }

// ---- proposal ---------------------------------------------------------------------

// One workgroup (one wavefront) per chain: draws the move, computes the
// determinant ratio (and, for an insertion, M b and c^T M for the update) and
// writes the proposed time-ordered operator list into the chain's trace slot.
__device__ inline void mc_propose(const MCParams& Q, int c, int64_t step, double* sb, double* sc) {
  const int lane = threadIdx.x;
  double u[6];
  move_uniforms(Q, c, step, u);
  const int F = Q.F, KM = Q.kmax, NM = Q.nmax;
  int f = int(__dmul_rn(u[0], double(F)));
  if (f > F - 1) f = F - 1;
  const bool ins = u[1] < 0.5;
  const int k = Q.kf[c * F + f];
  const int n = Q.cur_n[c];
  const double* cre_f = Q.cre + (int64_t(c) * F + f) * KM;
  const double* ann_f = Q.ann + (int64_t(c) * F + f) * KM;
  const double* Mf = Q.M + (int64_t(c) * F + f) * KM * KM;
  const double* otau = Q.cur_tau + int64_t(c) * NM;
  const int16_t* ofl = Q.cur_fl + int64_t(c) * NM;
  const int8_t* odg = Q.cur_dg + int64_t(c) * NM;
  double* ntau = Q.p_tau + int64_t(c) * NM;
  int16_t* nfl = Q.p_fl + int64_t(c) * NM;
  int8_t* ndg = Q.p_dg + int64_t(c) * NM;
  MoveRec rec{};
  rec.f = f;
  rec.k = k;
  int n_new = 0;
  if (ins) {
    rec.kind = 1;
    if (k >= KM || n + 2 > NM) {
      rec.kind = 0;
    } else {
      double ts = __dmul_rn(u[2], Q.beta);
      double te = __dadd_rn(ts, __dmul_rn(u[3], Q.beta));
      if (Q.learned) {
        // mixture: eps uniform on [0, beta)^2, else bins from the network and a
        // uniform position inside each bin
        const float* z = Q.logits + int64_t(c) * MLP_OUT;
        double ux[4];
        move_uniforms_extra(Q, c, step, ux);
        double len = __dmul_rn(u[3], Q.beta);
        if (!(ux[2] < Q.eps_mix)) {
          const int bs = mlp_draw_bin(z, u[2]), bl = mlp_draw_bin(z + MLP_BINS, u[3]);
          ts = (bs + ux[0]) * (Q.beta / MLP_BINS);
          len = (bl + ux[1]) * (Q.beta / MLP_BINS);
          if (ts >= Q.beta) ts = nextafter(Q.beta, 0.0);   // a position that rounded up to beta
          if (len >= Q.beta) len = nextafter(Q.beta, 0.0);
        }
        te = ts + len;
        rec.logq = mlp_logq(Q, z, ts, len);
      }
      if (te >= Q.beta) te = __dadd_rn(te, -Q.beta);
      rec.ts = ts;
      rec.te = te;
      double cs = 0.0, ce = 0.0, tie = (ts == te) ? 1.0 : 0.0;
      for (int p = lane; p < n; p += 64) {
        const double t = otau[p];
        cs += (t < ts) ? 1.0 : 0.0;
        ce += (t < te) ? 1.0 : 0.0;
        if (t == ts || t == te) tie = 1.0;
      }
      cs = wave_sum64(cs);
      ce = wave_sum64(ce);
      tie = wave_sum64(tie);
      rec.valid = tie == 0.0;
      if (rec.valid) {
        for (int p = lane; p < n; p += 64) {
          const double t = otau[p];
          const int np = p + (ts < t ? 1 : 0) + (te < t ? 1 : 0);
          ntau[np] = t;
          nfl[np] = ofl[p];
          ndg[np] = odg[p];
        }
        if (lane == 0) {
          const int ps = int(cs) + (te < ts ? 1 : 0);
          const int pe = int(ce) + (ts < te ? 1 : 0);
          ntau[ps] = ts;
          nfl[ps] = int16_t(f);
          ndg[ps] = 1;
          ntau[pe] = te;
          nfl[pe] = int16_t(f);
          ndg[pe] = 0;
        }
        n_new = n + 2;
        // A' = [[A, b], [c^T, d]]: b_r = Delta(tau'_r - te), c_r = Delta(ts - tau_r)
        if (lane < k) {
          sb[lane] = delta_at(Q, __dadd_rn(cre_f[lane], -te));
          sc[lane] = delta_at(Q, __dadd_rn(ts, -ann_f[lane]));
        }
        __syncthreads();
        double dot = 0.0;
        if (lane < k) {
          double ur = 0.0, vr = 0.0;
          for (int q = 0; q < k; ++q) {
            ur += Mf[lane * KM + q] * sb[q];   // (M b)_lane
            vr += sc[q] * Mf[q * KM + lane];   // (c^T M)_lane
          }
          Q.uvec[int64_t(c) * KM + lane] = ur;
          Q.vvec[int64_t(c) * KM + lane] = vr;
          dot = sc[lane] * ur;
        }
        dot = wave_sum64(dot);
        rec.ratio = delta_at(Q, __dadd_rn(ts, -te)) - dot;
      }
    }
  } else {
    rec.kind = 2;
    if (k == 0) {
      rec.kind = 0;
    } else {
      int i = int(__dmul_rn(u[2], double(k)));
      int j = int(__dmul_rn(u[3], double(k)));
      if (i > k - 1) i = k - 1;
      if (j > k - 1) j = k - 1;
      rec.i = i;
      rec.j = j;
      rec.valid = 1;
      // det of A without row i and column j, after moving the last labels into the holes
      const double s_i = (i != k - 1) ? -1.0 : 1.0, s_j = (j != k - 1) ? -1.0 : 1.0;
      rec.ratio = s_i * s_j * Mf[j * KM + i];
      const double tc = cre_f[i], ta = ann_f[j];
      if (Q.learned) {
        double len = ta - tc;
        if (len < 0.0) len += Q.beta;
        rec.logq = mlp_logq(Q, Q.logits + int64_t(c) * MLP_OUT, tc, len);
      }
      double pc = 0.0, pa = 0.0;
      for (int p = lane; p < n; p += 64) {
        if (otau[p] == tc && ofl[p] == f && odg[p] == 1) pc = double(p);
        if (otau[p] == ta && ofl[p] == f && odg[p] == 0) pa = double(p);
      }
      const int pos_c = int(wave_sum64(pc)), pos_a = int(wave_sum64(pa));
      for (int p = lane; p < n; p += 64) {
        if (p == pos_c || p == pos_a) continue;
        const int np = p - (p > pos_c ? 1 : 0) - (p > pos_a ? 1 : 0);
        ntau[np] = otau[p];
        nfl[np] = ofl[p];
        ndg[np] = odg[p];
      }
      n_new = n - 2;
    }
  }
  if (lane == 0) {
    Q.mv[c] = rec;
    Q.p_end[c] = Q.p_begin[c] + ((rec.kind != 0 && rec.valid) ? n_new : 0);
  }
}

// ---- acceptance, update, measurement ------------------------------------------

// Sign of the permutation from the canonical string to descending time order,
// counted over the chain's current per-flavor lists (all 64 lanes take part).
__device__ int perm_sign(const MCParams& Q, int c, double* canon) {
  const int F = Q.F, KM = Q.kmax;
  int n = 0;
  for (int g = 0; g < F; ++g) {
    const int kg = Q.kf[c * F + g];
    const double* cg = Q.cre + (int64_t(c) * F + g) * KM;
    const double* ag = Q.ann + (int64_t(c) * F + g) * KM;
    for (int i = threadIdx.x; i < kg; i += 64) {
      canon[n + 2 * i] = ag[i];
      canon[n + 2 * i + 1] = cg[i];
    }
    n += 2 * kg;
  }
  __syncthreads();
  double inv = 0.0;
  for (int p = threadIdx.x; p < n; p += 64) {
    const double tp = canon[p];
    int cnt = 0;
    for (int q = p + 1; q < n; ++q) cnt += (tp < canon[q]) ? 1 : 0;
    inv += double(cnt);
  }
  inv = wave_sum64(inv);
  __syncthreads();
  return (int64_t(inv) & 1) ? -1 : 1;
}

// canon: LDS scratch of max(nmax, 64) doubles (its head doubles as a row buffer)
__device__ inline void mc_accept(const MCParams& Q, int c, int64_t step, int measure, double* canon) {
  const int lane = threadIdx.x;
  const int F = Q.F, KM = Q.kmax, NM = Q.nmax;
  double u[6];
  move_uniforms(Q, c, step, u);
  const MoveRec rec = Q.mv[c];
  const int f = rec.f, k = rec.k;
  int64_t* st = Q.stats + int64_t(c) * ST_N;
  bool accept = false;
  if (rec.kind != 0 && rec.valid && Q.t_sign[c] != 0 && rec.ratio != 0.0) {
    // Metropolis-Hastings factor q_reverse / q_forward: removal picks one of k^2
    // pairs; insertion has density 1 / beta^2 (uniform) or q(tau_s, l) (learned)
    double log_factor;
    if (Q.learned)
      log_factor = (rec.kind == 1) ? -2.0 * log(double(k + 1)) - rec.logq : 2.0 * log(double(k)) + rec.logq;
    else
      log_factor = (rec.kind == 1) ? 2.0 * (log(Q.beta) - log(double(k + 1))) : 2.0 * (log(double(k)) - log(Q.beta));
    const double log_ratio = (Q.t_log[c] - Q.cur_logtr[c]) + log(fabs(rec.ratio)) + log_factor;
    accept = u[4] < exp(log_ratio);
  }
  if (lane == 0) {
    if (rec.kind == 0) st[ST_IMPOSSIBLE] += 1;
    if (rec.kind == 1) st[ST_INS_PROP] += 1;
    if (rec.kind == 2) st[ST_REM_PROP] += 1;
    if (rec.kind != 0 && (!rec.valid || Q.t_sign[c] == 0 || rec.ratio == 0.0)) st[ST_ZERO] += 1;
    if (accept) st[rec.kind == 1 ? ST_INS_ACC : ST_REM_ACC] += 1;
  }
  if (accept) {
    double* Mf = Q.M + (int64_t(c) * F + f) * KM * KM;
    double* cre_f = Q.cre + (int64_t(c) * F + f) * KM;
    double* ann_f = Q.ann + (int64_t(c) * F + f) * KM;
    const double r = rec.ratio;
    if (rec.kind == 1) {
      // M' = [[M + u v^T / r, -u / r], [-v^T / r, 1 / r]]
      const double* uv = Q.uvec + int64_t(c) * KM;
      const double* vv = Q.vvec + int64_t(c) * KM;
      if (lane < k) {
        const double ur = uv[lane];
        for (int q = 0; q < k; ++q) Mf[lane * KM + q] += ur * vv[q] / r;
        Mf[lane * KM + k] = -ur / r;
      } else if (lane == k) {
        for (int q = 0; q < k; ++q) Mf[k * KM + q] = -vv[q] / r;
        Mf[k * KM + k] = 1.0 / r;
      }
      if (lane == 0) {
        cre_f[k] = rec.ts;
        ann_f[k] = rec.te;
        Q.kf[c * F + f] = k + 1;
      }
    } else {
      // swap row j <-> k-1 and column i <-> k-1 of M, then drop the last row and
      // column: M'[r][s] = M''[r][s] - M''[r][k-1] M''[k-1][s] / M''[k-1][k-1]
      const int i = rec.i, j = rec.j;
      double* rowj = canon;  // old row j of M
      for (int q = lane; q < k; q += 64) rowj[q] = Mf[j * KM + q];
      __syncthreads();
      const double mji = rowj[i];
      if (lane < k - 1) {
        const int src = (lane == j) ? k - 1 : lane;
        const double m_ri = Mf[src * KM + i];
        for (int q = 0; q < k - 1; ++q) {
          const int qs = (q == i) ? k - 1 : q;
          Mf[lane * KM + q] = Mf[src * KM + qs] - m_ri * rowj[qs] / mji;
        }
      }
      __syncthreads();
      if (lane == 0) {
        cre_f[i] = cre_f[k - 1];
        ann_f[j] = ann_f[k - 1];
        Q.kf[c * F + f] = k - 1;
      }
    }
    // the proposed operator list becomes the current one
    const int n_new = int(Q.p_end[c] - Q.p_begin[c]);
    for (int p = lane; p < n_new; p += 64) {
      Q.cur_tau[int64_t(c) * NM + p] = Q.p_tau[int64_t(c) * NM + p];
      Q.cur_fl[int64_t(c) * NM + p] = Q.p_fl[int64_t(c) * NM + p];
      Q.cur_dg[int64_t(c) * NM + p] = Q.p_dg[int64_t(c) * NM + p];
    }
    __syncthreads();
    const int sp = perm_sign(Q, c, canon);
    for (int b = lane; b < Q.n_blocks; b += 64)
      Q.cur_psec[int64_t(c) * Q.n_blocks + b] = Q.psec_prop[int64_t(c) * Q.n_blocks + b];
    if (lane == 0) {
      Q.cur_n[c] = n_new;
      Q.cur_logtr[c] = Q.t_log[c];
      Q.cur_signtr[c] = Q.t_sign[c];
      Q.cur_logdet[c] += log(fabs(r));
      Q.cur_signdet[c] *= (r > 0.0) ? 1 : -1;
      Q.cur_sign[c] = sp * Q.cur_signtr[c] * Q.cur_signdet[c];
    }
  }
  __syncthreads();
  const double sgn = double(Q.cur_sign[c]);
  if (lane == 0) {
    int64_t order = 0;
    for (int g = 0; g < F; ++g) order += Q.kf[c * F + g];
    st[ST_ORDER] += order;
    st[ST_MOVES] += 1;
    Q.sign_sum[c] += sgn;
  }
  if (measure) {
    // G_f(tau) += sign * sum_ij M[j][i] delta~(tau, tau_j - tau'_i), binned
    for (int g = 0; g < F; ++g) {
      const int kg = Q.kf[c * F + g];
      const double* cg = Q.cre + (int64_t(c) * F + g) * KM;
      const double* ag = Q.ann + (int64_t(c) * F + g) * KM;
      const double* Mg = Q.M + (int64_t(c) * F + g) * KM * KM;
      double* acc = Q.gacc + (int64_t(c) * F + g) * Q.n_tau;
      for (int e = lane; e < kg * kg; e += 64) {
        const int i = e / kg, j = e - i * kg;
        double d = __dadd_rn(ag[j], -cg[i]);
        double s = 1.0;
        if (d < 0.0) {
          d = __dadd_rn(d, Q.beta);
          s = -1.0;
        }
        int b = int(__dmul_rn(__ddiv_rn(d, Q.beta), double(Q.n_tau)));
        if (b > Q.n_tau - 1) b = Q.n_tau - 1;
        atomicAdd(&acc[b], sgn * s * Mg[j * KM + i]);
      }
    }
    for (int b = lane; b < Q.n_blocks; b += 64)
      Q.sec_acc[int64_t(c) * Q.n_blocks + b] += sgn * Q.cur_psec[int64_t(c) * Q.n_blocks + b];
    if (lane == 0) {
      Q.meas_sign[c] += sgn;
      Q.n_meas[c] += 1;
    }
  }
}

// ---- rebuild of M from scratch ---------------------------------------------------

constexpr int RB_LD = 65;  // LDS row stride of the rebuild (64 columns + 1 against bank conflicts)

// One wavefront per (chain c, flavor f): A_f from the chain's current times, its
// inverse by Gauss-Jordan elimination with partial pivoting (lane r owns row r),
// log|det A_f| and its sign.  The relative drift max|M_f - inv(A_f)| / max|inv(A_f)|
// of the incrementally updated M_f goes to drift_f[c][f], the log-determinant and
// sign to ld_f / sd_f.  apply != 0 replaces M_f by the fresh inverse.  A singular
// A_f (no nonzero pivot) sets ERR_SINGULAR and leaves M_f alone.
// a: LDS scratch of 64 * RB_LD doubles; piv: LDS scratch of 64 ints.
__device__ inline void mc_rebuild(const MCParams& Q, int c, int f, int apply, double* a, int* piv, double* ld_f,
                                  int32_t* sd_f, double* drift_f, int32_t* err) {
  const int lane = threadIdx.x;
  const int F = Q.F, KM = Q.kmax;
  const int k = Q.kf[c * F + f];
  const double* cre = Q.cre + (int64_t(c) * F + f) * KM;
  const double* ann = Q.ann + (int64_t(c) * F + f) * KM;
  double* Mf = Q.M + (int64_t(c) * F + f) * KM * KM;
  if (lane < k)
    for (int j = 0; j < k; ++j) a[lane * RB_LD + j] = delta_at(Q, __dadd_rn(cre[lane], -ann[j]));
  __syncthreads();
  double logdet = 0.0;
  int sg = 1;
  bool singular = false;
  for (int col = 0; col < k; ++col) {
    // every lane scans the same column, so the pivot choice is uniform
    int p = col;
    double best = fabs(a[col * RB_LD + col]);
    for (int r = col + 1; r < k; ++r) {
      const double v = fabs(a[r * RB_LD + col]);
      if (v > best) {
        best = v;
        p = r;
      }
    }
    if (!(best > 0.0)) {
      singular = true;
      break;
    }
    __syncthreads();
    if (p != col && lane < k) {
      const double t = a[col * RB_LD + lane];
      a[col * RB_LD + lane] = a[p * RB_LD + lane];
      a[p * RB_LD + lane] = t;
    }
    if (lane == 0) piv[col] = p;
    __syncthreads();
    const double d = a[col * RB_LD + col];
    logdet += log(fabs(d));
    if (d < 0.0) sg = -sg;
    if (p != col) sg = -sg;
    __syncthreads();
    // pivot row: a[col][j] / d, with the pivot position becoming 1 / d
    if (lane < k) a[col * RB_LD + lane] = ((lane == col) ? 1.0 : a[col * RB_LD + lane]) / d;
    __syncthreads();
    // other rows: a[r][j] -= a[r][col] * a[col][j], the pivot column becoming -a[r][col] / d
    if (lane < k && lane != col) {
      const double fct = a[lane * RB_LD + col];
      a[lane * RB_LD + col] = 0.0;
      for (int j = 0; j < k; ++j) a[lane * RB_LD + j] = __dadd_rn(a[lane * RB_LD + j], -__dmul_rn(fct, a[col * RB_LD + j]));
    }
    __syncthreads();
  }
  if (singular) {
    if (lane == 0) {
      atomicOr(err, ERR_SINGULAR);
      ld_f[c * F + f] = 0.0;
      sd_f[c * F + f] = 0;
      drift_f[c * F + f] = 0.0;
    }
    return;
  }
  // the row swaps of the elimination become column swaps of the inverse, undone in
  // reverse order
  for (int col = k - 1; col >= 0; --col) {
    const int p = piv[col];
    if (p != col && lane < k) {
      const double t = a[lane * RB_LD + col];
      a[lane * RB_LD + col] = a[lane * RB_LD + p];
      a[lane * RB_LD + p] = t;
    }
  }
  __syncthreads();
  double dmax = 0.0, amax = 0.0;
  if (lane < k)
    for (int j = 0; j < k; ++j) {
      const double v = a[lane * RB_LD + j];
      amax = fmax(amax, fabs(v));
      dmax = fmax(dmax, fabs(v - Mf[lane * KM + j]));
    }
  for (int o = 32; o >= 1; o >>= 1) {
    amax = fmax(amax, shfl_xor_d(amax, o));
    dmax = fmax(dmax, shfl_xor_d(dmax, o));
  }
  if (apply && lane < k)
    for (int j = 0; j < k; ++j) Mf[lane * KM + j] = a[lane * RB_LD + j];
  if (lane == 0) {
    ld_f[c * F + f] = logdet;
    sd_f[c * F + f] = sg;
    drift_f[c * F + f] = (amax > 0.0) ? dmax / amax : 0.0;
  }
}

// Per chain, after mc_rebuild of all its flavors: log|det| summed over the flavors
// in flavor order, the largest flavor drift folded into drift[c], and with
// apply != 0 the chain's determinant state replaced (the weight's sign follows a
// changed determinant sign).
__device__ inline void mc_rebuild_finish(const MCParams& Q, int c, int apply, const double* ld_f, const int32_t* sd_f,
                                         const double* drift_f, double* drift, double* ld_out, int32_t* sd_out) {
  double ld = 0.0, dr = 0.0;
  int sd = 1;
  for (int g = 0; g < Q.F; ++g) {
    ld += ld_f[c * Q.F + g];
    sd *= sd_f[c * Q.F + g];
    dr = fmax(dr, drift_f[c * Q.F + g]);
  }
  drift[c] = fmax(drift[c], dr);
  if (ld_out) ld_out[c] = ld;
  if (sd_out) sd_out[c] = sd;
  if (apply && sd != 0) {
    Q.cur_sign[c] = Q.cur_sign[c] * Q.cur_signdet[c] * sd;
    Q.cur_signdet[c] = sd;
    Q.cur_logdet[c] = ld;
  }
}

// One training sample per chain: a flavor with pairs (uniform among them), one of
// its k^2 (creator, annihilator) pairs (uniform), the features of the configuration
// without that pair, and the targets (bin of tau_s, bin of l) on 64 bins.  Chains
// without pairs give targets (-1, -1).  Uniforms: Philox calls 8 and 9 at counter
// `index`.
__device__ inline void mc_harvest(const MCParams& Q, int c, int64_t index, __bf16* X, int32_t* T) {
  double u[4];
#pragma unroll
  for (int call = 8; call < 10; ++call) {
    uint32_t w[4] = {uint32_t(uint64_t(index)), uint32_t(uint64_t(index) >> 32), uint32_t(c), uint32_t(call)};
    philox4x32_10(w, Q.key0, Q.key1);
    u[2 * (call - 8)] = u01(w[0], w[1]);
    u[2 * (call - 8) + 1] = u01(w[2], w[3]);
  }
  const int F = Q.F, KM = Q.kmax;
  const int32_t* kf = Q.kf + c * F;
  int nonempty = 0;
  for (int g = 0; g < F; ++g) nonempty += kf[g] > 0;
  if (nonempty == 0) {
    if (threadIdx.x == 0) {
      T[2 * c] = -1;
      T[2 * c + 1] = -1;
    }
    return;
  }
  int pick = int(u[0] * nonempty);
  if (pick > nonempty - 1) pick = nonempty - 1;
  int f = 0;
  for (int g = 0, seen = 0; g < F; ++g)
    if (kf[g] > 0) {
      if (seen == pick) f = g;
      ++seen;
    }
  const int k = kf[f];
  int i = int(u[1] * k), j = int(u[2] * k);
  if (i > k - 1) i = k - 1;
  if (j > k - 1) j = k - 1;
  const double* cre = Q.cre + int64_t(c) * F * KM;
  const double* ann = Q.ann + int64_t(c) * F * KM;
  mlp_features(F, KM, Q.beta, kf, cre, ann, f, f, i, j, X + int64_t(c) * MLP_IN);
  if (threadIdx.x == 0) {
    const double ts = cre[f * KM + i];
    double len = ann[f * KM + j] - ts;
    if (len < 0.0) len += Q.beta;
    int bs = int(ts / Q.beta * MLP_BINS), bl = int(len / Q.beta * MLP_BINS);
    T[2 * c] = bs > MLP_BINS - 1 ? MLP_BINS - 1 : bs;
    T[2 * c + 1] = bl > MLP_BINS - 1 ? MLP_BINS - 1 : bl;
  }
}

}  // namespace hyb
