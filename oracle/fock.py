"""Occupation-number (Fock) basis and fermion operators.

The Krylov method works in the occupation-number basis, where the
hybridization operators are sparse and trivial to apply (Sec. III, item 1 of
the strategy).  The basis is split into blocks with fixed (n_up, n_dn)
(Sec. II, quantum-number ordering; Sec. IV.C orders the sectors with n_up
running fastest).

Conventions (readings of points the paper leaves open):

* bit f of a state integer is the occupation of flavor f = a + n_orb*sigma
  (spin up in the low bits);
* Jordan-Wigner order = flavor order: c_f |s> = (-1)^{#occupied flavors g<f}
  |s - f> for an occupied f, else 0;
* block key = n_dn * (n_orb + 1) + n_up; inside a block states are ordered by
  ascending state integer.
"""
from __future__ import annotations

import itertools
import numpy as np
import scipy.sparse as sp


def n_flavors(n_orb: int) -> int:
    return 2 * n_orb


def occupations(n_orb: int, s: int):
    """Tuple of 0/1 occupations of the 2*n_orb flavors of state s."""
    return tuple((s >> f) & 1 for f in range(2 * n_orb))


def block_key(n_orb: int, n_up: int, n_dn: int) -> int:
    return n_dn * (n_orb + 1) + n_up


def spin_counts(n_orb: int, s: int):
    occ = occupations(n_orb, s)
    return sum(occ[:n_orb]), sum(occ[n_orb:])


def blocks(n_orb: int):
    """List over block keys of the ascending state integers in each block.

    Built by enumerating every occupation tuple with itertools (not by bit
    tricks), then sorting."""
    F = 2 * n_orb
    out = [[] for _ in range((n_orb + 1) ** 2)]
    for occ in itertools.product((0, 1), repeat=F):
        s = sum(bit << f for f, bit in enumerate(occ))
        nu, nd = sum(occ[:n_orb]), sum(occ[n_orb:])
        out[block_key(n_orb, nu, nd)].append(s)
    return [np.array(sorted(b), dtype=np.int64) for b in out]


def index_maps(n_orb: int):
    """(block_of[s], index_in_block[s]) for every state s."""
    bl = blocks(n_orb)
    dim = 1 << (2 * n_orb)
    block_of = np.full(dim, -1, dtype=np.int64)
    idx = np.full(dim, -1, dtype=np.int64)
    for b, states in enumerate(bl):
        for i, s in enumerate(states):
            block_of[s] = b
            idx[s] = i
    return block_of, idx


def annihilator(n_orb: int, f: int) -> sp.csr_matrix:
    """Matrix of c_f on the full 2^F Fock space (Jordan-Wigner, flavor order).

    Element <s - f| c_f |s> = (-1)^{sum_{g<f} n_g(s)} for n_f(s) = 1."""
    F = 2 * n_orb
    dim = 1 << F
    rows, cols, vals = [], [], []
    for s in range(dim):
        occ = occupations(n_orb, s)
        if occ[f] == 1:
            sign = -1.0 if (sum(occ[:f]) % 2) else 1.0
            rows.append(s - (1 << f))
            cols.append(s)
            vals.append(sign)
    return sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim), dtype=np.float64)


class FockOperators:
    """Cache of c_f, c_f^dag and n_f on the full Fock space of n_orb orbitals."""

    def __init__(self, n_orb: int, flavor_order=None):
        """flavor_order optionally permutes the Jordan-Wigner ordering: the JW
        string of flavor f then counts the flavors placed before it in
        flavor_order.  The default is the flavor order itself."""
        self.n_orb = n_orb
        self.F = 2 * n_orb
        self.dim = 1 << self.F
        if flavor_order is None:
            self.c = [annihilator(n_orb, f) for f in range(self.F)]
        else:
            self.c = [self._annihilator_order(f, list(flavor_order)) for f in range(self.F)]
        self.cdag = [m.T.tocsr() for m in self.c]
        self.n = [(self.cdag[f] @ self.c[f]).tocsr() for f in range(self.F)]

    def _annihilator_order(self, f, order):
        pos = {g: i for i, g in enumerate(order)}
        before = [g for g in range(self.F) if pos[g] < pos[f]]
        rows, cols, vals = [], [], []
        for s in range(self.dim):
            occ = occupations(self.n_orb, s)
            if occ[f] == 1:
                sign = -1.0 if (sum(occ[g] for g in before) % 2) else 1.0
                rows.append(s - (1 << f))
                cols.append(s)
                vals.append(sign)
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.dim, self.dim))

    def op(self, f: int, dagger: int) -> sp.csr_matrix:
        return self.cdag[f] if dagger else self.c[f]

    def flavor(self, a: int, sigma: int) -> int:
        return a + self.n_orb * sigma
