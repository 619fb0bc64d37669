"""Kanamori local Hamiltonian of Eq.(4) and its block spectrum.

H_loc is assembled literally from products of the operator matrices of
oracle.fock (no bit arithmetic on matrix elements), then cut into the
(n_up, n_dn) blocks, and each block is diagonalised densely with
numpy.linalg.eigh (initialisation step 1 of Sec. III, "full diagonalization").

Reading of Eq.(4) (Sec. IV.A): the spin-flip and pair-hopping sum runs over
ordered pairs a != b, each term once.  The printed "+ h.c." is not added on
top: the hermitian conjugate of the (a, b) term is the (b, a) term, so adding
it would double J.  The tests show that this reading reproduces the ground
state degeneracies printed in Sec. IV.A, IV.C and V.C, and that the literal
reading (hc_literal=True here) does not.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np
import scipy.sparse as sp

from .fock import FockOperators, blocks


def kanamori_full(params, ops: FockOperators | None = None, hc_literal: bool = False):
    """Sparse H_loc on the full 2^F Fock space, Eq.(4).

    params: object with n_orb, eps[n_orb], U, Up, J, J_sf, J_ph.
      one-body  sum_{a,s} eps_a n_{a s}          (eps_a = -(mu + Delta_a))
      intra     U sum_a n_{a up} n_{a dn}
      inter     sum_{a>b,s} [Up n_{a s} n_{b -s} + (Up - J) n_{a s} n_{b s}]
      exchange  -J_sf sum_{a!=b} c+_{a dn} c+_{b up} c_{b dn} c_{a up}
      pair hop  -J_ph sum_{a!=b} c+_{b up} c+_{b dn} c_{a up} c_{a dn}
    """
    n = params.n_orb
    ops = ops or FockOperators(n)
    c, cd, nn = ops.c, ops.cdag, ops.n
    f = ops.flavor
    H = sp.csr_matrix((ops.dim, ops.dim))
    for a in range(n):
        for s in (0, 1):
            H = H + params.eps[a] * nn[f(a, s)]
        H = H + params.U * (nn[f(a, 0)] @ nn[f(a, 1)])
    for a in range(n):
        for b in range(a):
            for s in (0, 1):
                H = H + params.Up * (nn[f(a, s)] @ nn[f(b, 1 - s)])
                H = H + (params.Up - params.J) * (nn[f(a, s)] @ nn[f(b, s)])
    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            sf = cd[f(a, 1)] @ cd[f(b, 0)] @ c[f(b, 1)] @ c[f(a, 0)]
            ph = cd[f(b, 0)] @ cd[f(b, 1)] @ c[f(a, 0)] @ c[f(a, 1)]
            term = params.J_sf * sf + params.J_ph * ph
            if hc_literal:
                term = term + term.T
            H = H - term
    return H.tocsr()


@dataclass
class BlockSpectrum:
    n_orb: int
    states: list            # per block: ascending state integers
    H: list                 # per block: dense H_b
    E: list                 # per block: ascending eigenvalues
    V: list                 # per block: eigenvectors as columns
    E0: float

    @property
    def n_blocks(self):
        return len(self.states)

    def all_energies(self):
        return np.sort(np.concatenate([e for e in self.E if len(e)]))


def block_spectrum(params, hc_literal: bool = False, ops: FockOperators | None = None) -> BlockSpectrum:
    """Dense eigendecomposition of every (n_up, n_dn) block (Sec. III step 1)."""
    H = kanamori_full(params, ops=ops, hc_literal=hc_literal)
    st = blocks(params.n_orb)
    Hb, Eb, Vb = [], [], []
    for states in st:
        sub = H[states][:, states].toarray()
        # H conserves (n_up, n_dn): nothing may leak out of the block
        e, v = np.linalg.eigh(sub)
        Hb.append(sub)
        Eb.append(e)
        Vb.append(v)
    E0 = min(e.min() for e in Eb if len(e))
    return BlockSpectrum(params.n_orb, st, Hb, Eb, Vb, float(E0))


def leakage(params) -> float:
    """Largest |H| element coupling two different blocks (must be 0)."""
    H = kanamori_full(params).tocoo()
    n = params.n_orb
    mask = (1 << n) - 1
    pc = np.vectorize(lambda x: bin(int(x)).count("1"))
    ru, rd = pc(H.row & mask), pc(H.row >> n)
    cu, cd = pc(H.col & mask), pc(H.col >> n)
    bad = (ru != cu) | (rd != cd)
    return float(np.abs(H.data[bad]).max()) if bad.any() else 0.0


@dataclass
class Retained:
    block: np.ndarray       # block key of each retained state
    index: np.ndarray       # index of the eigenvector inside its block
    energy: np.ndarray


def retained_set(spec: BlockSpectrum, window: float) -> Retained:
    """States kept in the outer trace (Sec. III step 2; Sec. IV.C window).

    R = {i : E_i - E0 <= window}; window < 0 keeps every state (full trace).
    Ordered by block key, then by energy inside the block."""
    bl, ix, en = [], [], []
    for b, e in enumerate(spec.E):
        for i, ei in enumerate(e):
            if window < 0 or ei - spec.E0 <= window:
                bl.append(b)
                ix.append(i)
                en.append(ei)
    return Retained(np.array(bl, np.int64), np.array(ix, np.int64), np.array(en))


def sector_ground_degeneracy(params, n_electrons: int, tol: float = 1e-9, spec=None):
    """Degeneracy of the lowest level inside the n-electron sector."""
    spec = spec or block_spectrum(params)
    n = params.n_orb
    es = []
    for nd in range(n + 1):
        nu = n_electrons - nd
        if 0 <= nu <= n:
            es.append(spec.E[nd * (n + 1) + nu])
    e = np.concatenate(es)
    return int(np.sum(e - e.min() <= tol)), float(e.min())
