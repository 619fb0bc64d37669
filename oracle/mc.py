"""Monte Carlo weight, moves and measurement of the hybridization expansion (FP64, CPU).

Test infrastructure only: the product path never imports this module.

Weight of a configuration (Eq.(2), Sec. II, diagonal hybridization):

    w = s_perm * Tr_R[ literal time-ordered product ] * prod_f det A_f,
    A_f[i][j] = Delta(tau'_{f,i} - tau_{f,j})

Row i of A_f belongs to the i-th creator (tau') of flavor f and column j to the
j-th annihilator (tau).  Tr_R is the truncated trace of `oracle.trace`.

s_perm is the sign of the permutation taking the canonical string to descending
time order.  The canonical string is built flavor by flavor and, within a
flavor, in label order i: ... c_f(tau_{f,i}) c^dag_f(tau'_{f,i}) ...  This is
the pairing of the operators in Eq.(2) with the time-ordering operator made
explicit.

Delta is the hybridization function of the bath, an input given as a table on
a uniform grid of [0, beta].  Values between grid points are interpolated
linearly, and negative arguments use the antiperiodic extension
Delta(tau - beta) = -Delta(tau).

Moves (random pair insertion and removal of Sec. II, one flavor at a time):
- Insert: a creator at tau_s = u2 * beta and an annihilator at
  tau_e = tau_s + u3 * beta (mod beta), appended as label k.  The proposal
  density is 1/beta^2, so the acceptance factor is beta^2 / (k+1)^2.
- Remove: creator label i = floor(u2 k) and annihilator label j = floor(u3 k),
  picked uniformly.  In each list the last label fills the hole ("swap-remove").
  The acceptance factor is k^2 / beta^2.
- The flavor is floor(u0 F), and the move inserts when u1 < 1/2.
- Accept when u4 < |w'/w| * factor.

The uniforms come from the counter-based generator Philox4x32-10 (Salmon et
al., SC'11), here written from its published definition.  The counter is
(step low word, step high word, chain, call), the key is (seed low word,
seed high word), and a double is formed from two output words as
((a >> 5) * 2^26 + (b >> 6)) / 2^53.  Each weight is computed from scratch, by
a dense log-determinant and the oracle trace: no fast updates.

G(tau) estimator (measured in the flavor's own configuration):

    G_f(tau) = -(1/beta) < sum_{ij} M_f[j][i] delta~(tau, tau_{f,j} - tau'_{f,i}) >

where M_f = A_f^{-1} and delta~ carries a minus sign when the difference is
negative (the difference is then shifted by +beta).  Histogram bins of width
beta/n_tau; the sign of w weights every sample.
"""
from __future__ import annotations

import numpy as np

from .trace import TraceOracle

M32 = 0xFFFFFFFF


# ---------------------------------------------------------------------------
# Philox4x32-10
# ---------------------------------------------------------------------------

def philox4x32_10(ctr, key):
    """Ten rounds of Philox4x32 on a 4-word counter with a 2-word key."""
    c0, c1, c2, c3 = (int(x) & M32 for x in ctr)
    k0, k1 = (int(x) & M32 for x in key)
    for r in range(10):
        if r > 0:
            k0 = (k0 + 0x9E3779B9) & M32
            k1 = (k1 + 0xBB67AE85) & M32
        p0 = 0xD2511F53 * c0
        p1 = 0xCD9E8D57 * c2
        hi0, lo0 = p0 >> 32, p0 & M32
        hi1, lo1 = p1 >> 32, p1 & M32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & M32, lo1, (hi0 ^ c3 ^ k1) & M32, lo0
    return c0, c1, c2, c3


def u01(a: int, b: int) -> float:
    """Double in [0, 1) from two 32-bit words (53 random bits)."""
    return ((a >> 5) * 67108864 + (b >> 6)) / 9007199254740992.0


def move_uniforms(seed: int, chain: int, step: int, calls=(0, 1, 2)):
    """u0..u5 of one move: three Philox calls (call index 0, 1, 2); the learned
    proposal also draws calls 3 and 4 (u6..u9)."""
    key = (seed & M32, (seed >> 32) & M32)
    out = []
    for call in calls:
        w = philox4x32_10((step & M32, (step >> 32) & M32, chain, call), key)
        out += [u01(w[0], w[1]), u01(w[2], w[3])]
    return out


# ---------------------------------------------------------------------------
# bath, determinants and the permutation sign
# ---------------------------------------------------------------------------

def delta_at(table: np.ndarray, beta: float, tau: float) -> float:
    """Linear interpolation of the tabulated Delta, extended antiperiodically."""
    sgn = 1.0
    if tau < 0.0:
        tau += beta
        sgn = -1.0
    n = len(table) - 1
    x = tau / beta * n
    k = min(int(x), n - 1)
    fr = x - k
    return sgn * (table[k] + fr * (table[k + 1] - table[k]))


def hyb_matrix(table, beta, cre, ann) -> np.ndarray:
    k = len(cre)
    A = np.empty((k, k))
    for i in range(k):
        for j in range(k):
            A[i, j] = delta_at(table, beta, cre[i] - ann[j])
    return A


def perm_sign(cre, ann) -> int:
    """Sign of the permutation from the canonical string to descending time order
    (brute-force inversion count)."""
    times = []
    for f in range(len(cre)):
        for i in range(len(cre[f])):
            times += [ann[f][i], cre[f][i]]
    inv = 0
    n = len(times)
    for p in range(n):
        for q in range(p + 1, n):
            if times[p] < times[q]:
                inv += 1
    return -1 if inv & 1 else 1


def merged(cre, ann):
    taus, fls, dgs = [], [], []
    for f in range(len(cre)):
        for t in cre[f]:
            taus.append(t); fls.append(f); dgs.append(1)
        for t in ann[f]:
            taus.append(t); fls.append(f); dgs.append(0)
    o = np.argsort(np.asarray(taus, dtype=np.float64), kind="stable")
    return (np.asarray(taus, np.float64)[o], np.asarray(fls, np.int16)[o], np.asarray(dgs, np.int8)[o])


def weight(tr: TraceOracle, table, beta, cre, ann):
    """(sign, log|w|) of a configuration from scratch; sign 0 for a zero weight."""
    from paper_0908_0681_amd.inputs import from_lists
    tau, fl, dg = merged(cre, ann)
    if len(tau) > 1 and np.any(np.diff(tau) <= 0.0):
        return 0, -np.inf
    r = tr.trace_batch(from_lists([(tau, fl, dg)], beta))
    s = int(r.sign[0])
    if s == 0:
        return 0, -np.inf
    logw = float(r.log_abs[0])
    for f in range(len(cre)):
        if len(cre[f]) == 0:
            continue
        sd, ld = np.linalg.slogdet(hyb_matrix(table, beta, cre[f], ann[f]))
        if sd == 0:
            return 0, -np.inf
        s *= int(sd)
        logw += float(ld)
    return s * perm_sign(cre, ann), logw


# ---------------------------------------------------------------------------
# one chain
# ---------------------------------------------------------------------------

class Chain:
    """State: cre[f], ann[f] (label order), the weight's sign and log|w|."""

    def __init__(self, tr: TraceOracle, table, beta, cre, ann, kmax: int, net=None, eps: float = 0.1):
        self.tr, self.table, self.beta, self.kmax = tr, table, float(beta), kmax
        self.net, self.eps = net, eps     # learned insertion density (oracle.mlp.Network) or None
        self.cre = [list(map(float, c)) for c in cre]
        self.ann = [list(map(float, a)) for a in ann]
        self.sign, self.logw = weight(tr, table, beta, self.cre, self.ann)
        self.last_margin = np.inf
        if self.sign == 0:
            raise ValueError("initial configuration has zero weight")

    def propose(self, u):
        """The move drawn by uniforms u[0..4]: (kind, cre', ann', sign', log|w'|, log_ratio)
        with log_ratio = log(|w'/w| * proposal factor); kind 1 insert, 2 remove,
        0 impossible (flavor at capacity, empty flavor); sign' = 0 for a zero weight."""
        F = len(self.cre)
        f = min(int(u[0] * F), F - 1)
        k = len(self.cre[f])
        cre = [list(c) for c in self.cre]
        ann = [list(a) for a in self.ann]
        if u[1] < 0.5:
            if k >= self.kmax:
                return 0, None, None, 0, -np.inf, -np.inf
            ts = u[2] * self.beta
            te = ts + u[3] * self.beta
            if self.net is None:
                log_factor = 2.0 * (np.log(self.beta) - np.log(k + 1))
            else:
                from . import mlp as NN
                ux = u[6:10]
                z = self.net.forward(NN.features(self.cre, self.ann, f, self.beta)[None])["Z3"][0]
                length = u[3] * self.beta
                if not ux[2] < self.eps:
                    bs, bl = _draw_bin(z[:NN.BINS], u[2]), _draw_bin(z[NN.BINS:], u[3])
                    ts = (bs + ux[0]) * (self.beta / NN.BINS)
                    length = (bl + ux[1]) * (self.beta / NN.BINS)
                te = ts + length
                log_factor = -2.0 * np.log(k + 1) - NN.logq(z, ts, length, self.beta, self.eps)
            if te >= self.beta:
                te -= self.beta
            cre[f].append(ts)
            ann[f].append(te)
            kind = 1
        else:
            if k == 0:
                return 0, None, None, 0, -np.inf, -np.inf
            i = min(int(u[2] * k), k - 1)
            j = min(int(u[3] * k), k - 1)
            if self.net is not None:
                from . import mlp as NN
                z = self.net.forward(NN.features(self.cre, self.ann, f, self.beta, exclude=(f, i, j))[None])["Z3"][0]
                length = self.ann[f][j] - self.cre[f][i]
                if length < 0.0:
                    length += self.beta
                lq = NN.logq(z, self.cre[f][i], length, self.beta, self.eps)
            cre[f][i] = cre[f][k - 1]
            cre[f].pop()
            ann[f][j] = ann[f][k - 1]
            ann[f].pop()
            log_factor = 2.0 * (np.log(k) - np.log(self.beta)) if self.net is None else 2.0 * np.log(k) + lq
            kind = 2
        s, lw = weight(self.tr, self.table, self.beta, cre, ann)
        if s == 0:
            return kind, cre, ann, 0, -np.inf, -np.inf
        return kind, cre, ann, s, lw, lw - self.logw + log_factor

    def step(self, u):
        """One move with uniforms u[0..5]; returns (kind, accepted): accept when
        u4 < |w'/w| * factor (Metropolis-Hastings with the proposal densities above)."""
        kind, cre, ann, s, lw, log_ratio = self.propose(u)
        if kind == 0 or s == 0:
            return kind, False
        # distance of the decision from its threshold (a replay in another
        # floating-point order can only differ when this is at rounding level)
        self.last_margin = abs(np.log(u[4]) - log_ratio) if u[4] > 0.0 else np.inf
        if u[4] < np.exp(log_ratio):
            self.cre, self.ann, self.sign, self.logw = cre, ann, s, lw
            return kind, True
        return kind, False

    def measure_sectors(self, acc: np.ndarray):
        """Adds sign(w) * P_s(beta/2) of the current configuration into acc[s]
        (TraceOracle.sector_weights)."""
        tau, fl, dg = merged(self.cre, self.ann)
        for b, p in self.tr.sector_weights(tau, fl, dg, self.beta, 0.5 * self.beta).items():
            acc[b] += self.sign * p

    def measure(self, acc: np.ndarray):
        """Adds sign(w) * sum_ij M[j][i] (signed, binned) into acc[f][bin]."""
        F, n_tau = acc.shape
        for f in range(F):
            k = len(self.cre[f])
            if k == 0:
                continue
            M = np.linalg.inv(hyb_matrix(self.table, self.beta, self.cre[f], self.ann[f]))
            for i in range(k):
                for j in range(k):
                    d = self.ann[f][j] - self.cre[f][i]
                    s = 1.0
                    if d < 0.0:
                        d += self.beta
                        s = -1.0
                    b = min(int(d / self.beta * n_tau), n_tau - 1)
                    acc[f, b] += self.sign * s * M[j, i]


def _draw_bin(z, u: float) -> int:
    """Inverse-CDF draw of a bin from logits z with uniform u."""
    e = np.exp(np.asarray(z, dtype=np.float64) - np.max(z))
    c = np.cumsum(e)
    b = int(np.searchsorted(c, u * c[-1], side="right"))
    return min(b, len(z) - 1)


def g_tau(acc_sum: np.ndarray, sign_sum: float, beta: float) -> np.ndarray:
    """G_f(tau_bin) from accumulated measurements (sum over samples of sign*X and of sign)."""
    n_tau = acc_sum.shape[1]
    h = beta / n_tau
    return -acc_sum / (beta * h * sign_sum)
