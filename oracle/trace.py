"""Truncated local trace Tr_R(c) by dense eigendecomposition (FP64).

Definition followed (trace factor of Eq.(2), Sec. II; truncation of type (i),
Sec. II; evaluation steps 3-8 of Sec. III):

    Tr_R(c) = sum_{i in R} <E_i| e^{-(beta - tau_n) H} O_n e^{-(tau_n - tau_{n-1}) H}
                                ... O_1 e^{-tau_1 H} |E_i>

with O_k = c^dag_{f_k} if dagger_k else c_{f_k}, 0 <= tau_1 < ... < tau_n < beta.
The value is the literal operator product in time order (latest operator
leftmost); no time-ordering permutation sign is attached.

Each imaginary-time evolution inside block b is the matrix exponential
exp(-dtau (H_b - e_b)) (e_b the block's lowest eigenvalue) applied to the
vector.  For blocks of up to EXPM_MAX_DIM states it is evaluated by scipy's
scaling-and-squaring Pade expm; for larger blocks by the block's eigen-
decomposition V_b diag(exp(-dtau (E_b - e_b))) V_b^T.  The two agree to
rounding, but the eigenvector route mixes symmetry sectors inside (near-)
degenerate eigenvalue clusters at the level eps*|H|/gap, and long intervals
then amplify that mixing into components that are zero by symmetry; the
polynomial route keeps the vector in its own symmetry sector (it is a power
series in H).  Because |E_i> is an eigenstate, the two edge intervals reduce
to the scalar exp(-(beta - tau_n + tau_1) (E_i - E0)) (step 3).

An operator that leaves less than zero_tol of the (unit) vector's norm ends
the path, and so does a closing overlap <E_i|v> below zero_tol: in exact arithmetic such results are zeros imposed by symmetry
(for instance c_f acting on a vector with no weight on occupied f inside the
sector reached), and numerically they are rounding noise.  Energies are
shifted by the ground energy E0 (and, inside a propagation, by the block's
own lowest eigenvalue), and the vector is renormalised after every step with
its log-norm kept aside; these are exact rescalings that keep the float64
numbers in range, and -beta*E0 is added back at the end.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np
import scipy.linalg as sla

from .fock import FockOperators, block_key
from .hamiltonian import BlockSpectrum, Retained


@dataclass
class TraceResult:
    sign: np.ndarray          # int8 [n_configs]: -1, 0, +1
    log_abs: np.ndarray       # float64: log|Tr_R|, -inf where sign = 0
    contrib_sign: np.ndarray  # int8 [n_configs, n_retained]
    contrib_log: np.ndarray   # float64 [n_configs, n_retained]: log|t_i| incl. -beta*E0
    feasible: np.ndarray      # bool [n_configs, n_retained]: sector path stays physical

    def rows(self, idx):
        """The results of the configurations idx (a list), in that order."""
        idx = list(idx)
        return TraceResult(self.sign[idx], self.log_abs[idx], self.contrib_sign[idx],
                           self.contrib_log[idx], self.feasible[idx])

    def kappa(self):
        """Conditioning sum_i |t_i| / |sum_i t_i| per config (inf for zero traces)."""
        out = np.full(len(self.sign), np.inf)
        for c in range(len(self.sign)):
            if self.sign[c] == 0:
                continue
            lg = self.contrib_log[c]
            m = np.max(lg)
            s_abs = np.sum(np.exp(lg - m))
            out[c] = s_abs * np.exp(m - self.log_abs[c])
        return out


EXPM_MAX_DIM = 400


class TraceOracle:
    """Holds a block spectrum, a retained set and cached operator blocks."""

    def __init__(self, spec: BlockSpectrum, retained: Retained, ops: FockOperators | None = None,
                 zero_tol: float = 1e-10, method: str = "auto"):
        self.spec = spec
        self.R = retained
        self.n = spec.n_orb
        self.ops = ops or FockOperators(self.n)
        self._opblk = {}
        self.zero_tol = zero_tol
        self.method = method   # "auto" | "expm" | "eigh"

    # -- sector bookkeeping -------------------------------------------------
    def _nud(self, b):
        return b % (self.n + 1), b // (self.n + 1)

    def target_block(self, b: int, f: int, dagger: int) -> int:
        """Block reached by O from block b, or -1 if it leaves the physical range."""
        nu, nd = self._nud(b)
        d = 1 if dagger else -1
        if f < self.n:
            nu += d
        else:
            nd += d
        if not (0 <= nu <= self.n and 0 <= nd <= self.n):
            return -1
        return block_key(self.n, nu, nd)

    def op_block(self, f: int, dagger: int, b: int):
        """Dense matrix of O restricted to block b -> target block."""
        key = (f, dagger, b)
        if key not in self._opblk:
            bt = self.target_block(b, f, dagger)
            M = self.ops.op(f, dagger)
            src, dst = self.spec.states[b], self.spec.states[bt]
            self._opblk[key] = (bt, M[dst][:, src].toarray())
        return self._opblk[key]

    def propagate(self, b: int, v: np.ndarray, dtau: float) -> np.ndarray:
        """exp(-dtau (H_b - E0)) v by the eigendecomposition of block b."""
        Vb, Eb = self.spec.V[b], self.spec.E[b]
        return Vb @ (np.exp(-dtau * (Eb - self.spec.E0)) * (Vb.T @ v))

    def propagate_log(self, b: int, v: np.ndarray, dtau: float):
        """exp(-dtau (H_b - E0)) v as (unit vector, log of its norm).

        The block's lowest eigenvalue is factored out before exponentiating so
        that long intervals in high-lying blocks do not underflow."""
        Vb, Eb, Hb = self.spec.V[b], self.spec.E[b], self.spec.H[b]
        emin = float(Eb.min())
        use_expm = self.method == "expm" or (self.method == "auto" and len(Eb) <= EXPM_MAX_DIM)
        if use_expm:
            y = sla.expm(-dtau * (Hb - emin * np.eye(len(Eb)))) @ v
        else:
            y = Vb @ (np.exp(-dtau * (Eb - emin)) * (Vb.T @ v))
        s = np.linalg.norm(y)
        return y / s, np.log(s) - dtau * (emin - self.spec.E0)

    # -- one term of the outer sum ------------------------------------------
    def path(self, tau, flavor, dagger, beta: float, r: int):
        """(feasible, sign, log|t_r|) for retained state r (log includes -beta*E0)."""
        b0 = int(self.R.block[r])
        Ei = float(self.R.energy[r])
        E0 = self.spec.E0
        nops = len(tau)
        # sector path first (block-level structural zeros, no arithmetic)
        b = b0
        for k in range(nops):
            b = self.target_block(b, int(flavor[k]), int(dagger[k]))
            if b < 0:
                return False, 0, -np.inf
        if b != b0:
            return False, 0, -np.inf
        ei = self.spec.V[b0][:, int(self.R.index[r])]
        if nops == 0:
            return True, 1, -beta * (Ei - E0) - beta * E0
        ell = -(beta - tau[-1] + tau[0]) * (Ei - E0)
        v = ei.copy()
        b = b0
        for k in range(nops):
            if k > 0:
                v, ls = self.propagate_log(b, v, float(tau[k] - tau[k - 1]))
                ell += ls
            b, M = self.op_block(int(flavor[k]), int(dagger[k]), b)
            v = M @ v
            s = np.linalg.norm(v)
            if s <= self.zero_tol:
                return True, 0, -np.inf
            ell += np.log(s)
            v = v / s
        ov = float(ei @ v)
        if abs(ov) <= self.zero_tol:      # unit vectors: a symmetry zero in exact arithmetic
            return True, 0, -np.inf
        return True, (1 if ov > 0 else -1), ell + np.log(abs(ov)) - beta * E0

    # -- sector weights at a time inside the interval ---------------------------
    def sector_weights(self, tau, flavor, dagger, beta: float, tau_m: float):
        """Weights of the (n_up, n_dn) sectors at time tau_m (Sec. IV.C, Fig. 4):
        P_s = sum_{i: path i in block s at tau_m} t_i / sum_i t_i, with t_i the
        retained-state contributions of path(); the block of path i at tau_m is the
        block reached after the operators earlier than tau_m (H conserves the blocks
        in between).  Returns a dict block -> weight (empty for a zero trace)."""
        out, tot, ts = {}, 0.0, []
        for r in range(len(self.R.block)):
            feas, sg, lg = self.path(tau, flavor, dagger, beta, r)
            if not feas or sg == 0:
                continue
            b = int(self.R.block[r])
            for k in range(len(tau)):
                if tau[k] < tau_m:
                    b = self.target_block(b, int(flavor[k]), int(dagger[k]))
            ts.append((b, sg, lg))
        if not ts:
            return out
        m = max(lg for _, _, lg in ts)
        for b, sg, lg in ts:
            t = sg * np.exp(lg - m)
            out[b] = out.get(b, 0.0) + t
            tot += t
        return {b: v / tot for b, v in out.items()}

    # -- conditioning ----------------------------------------------------------
    def path_condition(self, tau, flavor, dagger, r: int):
        """Cut-point condition numbers kappa_k = 1 / |<L_k|R_k>| of one path.

        Cut the operator product of Eq.(2) just before operator k:
        t_r = <E_i| A_k B_k |E_i>, with R_k = B_k|E_i> / |B_k|E_i>| the
        propagated vector the forward pass holds there and
        L_k = A_k^T|E_i> / |A_k^T|E_i>| the closing state carried backwards to
        the same point.  Replacing R_k by R_k + delta (|delta| <= eps) changes
        t_r by the relative amount <L_k|delta> / <L_k|R_k>, at most
        eps * kappa_k; a method whose propagations are accurate to eps in
        norm is therefore accurate to about eps * sum_k kappa_k on this path
        (first order).  Returns the array over k = 0..n-1, or None for a path
        that is zero (sector-infeasible or a symmetry zero)."""
        feas, sg, _ = self.path(tau, flavor, dagger, 0.0, r)
        nops = len(tau)
        if not feas or sg == 0:
            return None
        if nops == 0:
            return np.zeros(0)
        b0 = int(self.R.block[r])
        ei = self.spec.V[b0][:, int(self.R.index[r])]
        R, blocks, mats = [], [], []
        v, b = ei.copy(), b0
        for k in range(nops):
            if k > 0:
                v, _ = self.propagate_log(b, v, float(tau[k] - tau[k - 1]))
            R.append(v.copy())
            blocks.append(b)
            b, M = self.op_block(int(flavor[k]), int(dagger[k]), b)
            mats.append(M)
            v = M @ v
            v = v / np.linalg.norm(v)
        kap = np.empty(nops)
        u = ei.copy()
        for k in range(nops - 1, -1, -1):
            u = mats[k].T @ u
            u = u / np.linalg.norm(u)
            ov = abs(float(u @ R[k]))
            kap[k] = np.inf if ov == 0.0 else 1.0 / ov
            if k > 0:
                # exp(-dtau H_b) is symmetric: the backward step is the same propagation
                u, _ = self.propagate_log(blocks[k], u, float(tau[k] - tau[k - 1]))
        return kap

    def condition(self, batch, result: TraceResult, configs=None) -> np.ndarray:
        """Per configuration: sum_i |t_i| K_i / |sum_i t_i| with K_i = sum_k kappa_k
        of path i, the first-order amplification of per-propagation relative
        errors into the relative error of Tr_R (1 for an empty configuration,
        0 for an exact zero, inf for a cancelling sum)."""
        idx = list(range(batch.n_configs) if configs is None else configs)
        out = np.zeros(len(idx))
        for j, c in enumerate(idx):
            if result.sign[j] == 0:
                continue
            tau, fl, dg = batch.config(c)
            lg = result.contrib_log[j]
            m = np.max(lg[result.contrib_sign[j] != 0])
            acc = 0.0
            for r in range(len(lg)):
                if result.contrib_sign[j, r] == 0:
                    continue
                kap = self.path_condition(tau, fl, dg, r)
                K = max(1.0, float(np.sum(kap))) if kap is not None else 1.0
                acc += np.exp(lg[r] - m) * K
            out[j] = acc * np.exp(m - result.log_abs[j])
        return out

    # -- the batch -----------------------------------------------------------
    def trace_batch(self, batch, configs=None) -> TraceResult:
        idx = range(batch.n_configs) if configs is None else list(configs)
        idx = list(idx)
        nR = len(self.R.block)
        sg = np.zeros(len(idx), np.int8)
        la = np.full(len(idx), -np.inf)
        csg = np.zeros((len(idx), nR), np.int8)
        clg = np.full((len(idx), nR), -np.inf)
        feas = np.zeros((len(idx), nR), bool)
        for j, c in enumerate(idx):
            tau, fl, dg = batch.config(c)
            for r in range(nR):
                feas[j, r], csg[j, r], clg[j, r] = self.path(tau, fl, dg, batch.beta, r)
            sg[j], la[j] = signed_logsum(csg[j], clg[j])
        return TraceResult(sg, la, csg, clg, feas)


def signed_logsum(signs, logs):
    """(sign, log|sum_i sign_i exp(log_i)|) in a fixed order; sign 0 for an exact zero."""
    nz = signs != 0
    if not np.any(nz):
        return 0, -np.inf
    m = np.max(logs[nz])
    s = float(np.sum(signs[nz] * np.exp(logs[nz] - m)))
    if s == 0.0:
        return 0, -np.inf
    return (1 if s > 0 else -1), m + np.log(abs(s))


def build(params, window: float, ops: FockOperators | None = None, hc_literal: bool = False,
          zero_tol: float = 1e-10, method: str = "auto"):
    """Convenience: spectrum + retained set + oracle for a parameter set."""
    from .hamiltonian import block_spectrum, retained_set
    ops = ops or FockOperators(params.n_orb)
    spec = block_spectrum(params, hc_literal=hc_literal, ops=ops)
    R = retained_set(spec, window)
    return TraceOracle(spec, R, ops, zero_tol=zero_tol, method=method)
