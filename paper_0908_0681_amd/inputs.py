"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds only input recipes: model parameters of the Kanamori
impurity of Eq.(4) (Sec. IV.A), and random hybridization-event configurations
(the configurations c~ of Eq.(2), Sec. II).  It contains none of the trace
arithmetic, so that both sides of a parity test read identical bytes without
sharing any of the method's code.

Conventions fixed here (they are input conventions, not arithmetic):

* flavor index f = a + n_orb * sigma, sigma = 0 for spin up, 1 for spin down;
* a configuration is a time-ordered list of operators (tau, flavor, dagger)
  with 0 <= tau_1 < ... < tau_n < beta; dagger = 1 is a creator;
* a batch of configurations is CSR: ops of config c are
  [offsets[c], offsets[c+1]).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


# --------------------------------------------------------------------------
# model parameters
# --------------------------------------------------------------------------

def mu_half(n_orb: int, U: float, J: float) -> float:
    """Half-filling chemical potential of the rotationally invariant model
    (Sec. IV.B): (n - 1/2) U - (n - 1) (5/2) J."""
    return (n_orb - 0.5) * U - (n_orb - 1) * 2.5 * J


@dataclass
class ModelParams:
    """Parameters of the Kanamori H_loc of Eq.(4).

    eps[a] is the spin-independent one-body energy -(mu + Delta_a);
    U intra-orbital, Up inter-orbital opposite spin, Up - J same spin,
    J_sf / J_ph the spin-flip / pair-hopping amplitudes (both J in Eq.(4)).
    """
    n_orb: int
    eps: np.ndarray
    U: float
    Up: float
    J: float
    J_sf: float
    J_ph: float

    @property
    def n_flavors(self) -> int:
        return 2 * self.n_orb


def kanamori(n_orb: int, U: float, J: float, mu: float,
             delta=None, density_density: bool = False) -> ModelParams:
    """Rotationally invariant Kanamori parameters, U' = U - 2J (Sec. IV.A)."""
    delta = np.zeros(n_orb) if delta is None else np.asarray(delta, dtype=np.float64)
    eps = -(mu + delta)
    jx = 0.0 if density_density else J
    return ModelParams(n_orb=n_orb, eps=np.ascontiguousarray(eps, dtype=np.float64),
                       U=float(U), Up=float(U - 2.0 * J), J=float(J),
                       J_sf=float(jx), J_ph=float(jx))


def crystal_field(n_orb: int, amp: float, seed: int) -> np.ndarray:
    """Crystal-field shifts Delta_a ~ U(-amp, amp), spin independent."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=n_orb)


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------

@dataclass
class ConfigBatch:
    offsets: np.ndarray      # int64 [n_configs + 1]
    tau: np.ndarray          # float64 [n_ops]
    flavor: np.ndarray       # int16 [n_ops]
    dagger: np.ndarray       # int8 [n_ops]
    beta: float
    meta: dict = field(default_factory=dict)

    @property
    def n_configs(self) -> int:
        return len(self.offsets) - 1

    def config(self, c: int):
        s, e = int(self.offsets[c]), int(self.offsets[c + 1])
        return self.tau[s:e], self.flavor[s:e], self.dagger[s:e]

    def subset(self, idx) -> "ConfigBatch":
        return from_lists([self.config(int(c)) for c in idx], self.beta)


def from_lists(cfgs, beta: float) -> ConfigBatch:
    """Build a batch from a list of (tau, flavor, dagger) triples."""
    offs = [0]
    taus, fls, dgs = [], [], []
    for tau, fl, dg in cfgs:
        taus.append(np.asarray(tau, dtype=np.float64))
        fls.append(np.asarray(fl, dtype=np.int16))
        dgs.append(np.asarray(dg, dtype=np.int8))
        offs.append(offs[-1] + len(taus[-1]))
    cat = lambda xs, dt: (np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt))
    return ConfigBatch(offsets=np.asarray(offs, dtype=np.int64),
                       tau=np.ascontiguousarray(cat(taus, np.float64)),
                       flavor=np.ascontiguousarray(cat(fls, np.int16)),
                       dagger=np.ascontiguousarray(cat(dgs, np.int8)),
                       beta=float(beta))


def random_config(rng: np.random.Generator, n_orb: int, beta: float, lam: float,
                  start: str = "reference"):
    """One configuration: per-flavor order k_f ~ Poisson(lam), 2 k_f operator
    times uniform in [0, beta), per-flavor alternation of c / c^dag in time.

    start = "reference": a reference Fock state with every orbital singly
    occupied and a random spin per orbital is drawn; a flavor occupied in it
    starts with an annihilator, otherwise with a creator (this keeps the
    sector path inside the physical range, so the truncated trace is rarely a
    structural zero).  start = "random": the first type of every flavor is a
    fair coin (most truncated traces are then structural zeros).
    """
    F = 2 * n_orb
    spins = rng.integers(0, 2, size=n_orb)
    occ = np.zeros(F, dtype=bool)
    for a in range(n_orb):
        occ[a + n_orb * spins[a]] = True
    k = rng.poisson(lam, size=F)
    taus, fls = [], []
    for f in range(F):
        taus.append(rng.uniform(0.0, beta, size=2 * k[f]))
        fls.append(np.full(2 * k[f], f, dtype=np.int16))
    tau = np.concatenate(taus) if taus else np.zeros(0)
    fl = np.concatenate(fls) if fls else np.zeros(0, np.int16)
    order = np.argsort(tau, kind="stable")
    tau, fl = tau[order], fl[order]
    if len(tau) > 1 and np.any(np.diff(tau) <= 0.0):   # measure-zero tie: redraw
        return random_config(rng, n_orb, beta, lam, start)
    dg = np.zeros(len(tau), dtype=np.int8)
    for f in range(F):
        pos = np.nonzero(fl == f)[0]
        if start == "reference":
            first_creator = not occ[f]
        else:
            first_creator = bool(rng.integers(0, 2))
        # alternate in time order
        dg[pos] = np.where((np.arange(len(pos)) % 2 == 0) == first_creator, 1, 0)
    return tau, fl, dg


def random_batch(seed: int, n_orb: int, n_configs: int, beta: float, lam: float,
                 start: str = "reference") -> ConfigBatch:
    rng = np.random.default_rng(seed)
    cfgs = [random_config(rng, n_orb, beta, lam, start) for _ in range(n_configs)]
    b = from_lists(cfgs, beta)
    b.meta = dict(seed=seed, n_orb=n_orb, lam=lam, start=start)
    return b


# --------------------------------------------------------------------------
# the workloads of the benchmark table
# --------------------------------------------------------------------------

MODEL_SEED = 1


@dataclass
class Workload:
    name: str
    params: ModelParams
    beta: float
    n_configs: int
    lam: float
    config_seed: int
    precision: str            # "fp64" | "mixed"
    retain_window: float      # < 0: every state (full trace)
    krylov_max: int = 20
    krylov_tol: float = 1e-12

    def batch(self, n_configs: int | None = None, start: str = "reference") -> ConfigBatch:
        n = self.n_configs if n_configs is None else n_configs
        return random_batch(self.config_seed, self.params.n_orb, n, self.beta, self.lam, start)


def workload(k: int) -> Workload:
    """Workload k of the benchmark table (k = 0, 1, 2)."""
    if k == 0:
        # 2 orbitals, eps = -mu, mu = (3U - 5J)/2, U = 4, J = 1, beta = 10
        p = kanamori(2, U=4.0, J=1.0, mu=(3 * 4.0 - 5 * 1.0) / 2)
        return Workload("kanamori-2orb-b10", p, 10.0, 64, 2.0, 1000, "fp64", -1.0)
    if k == 1:
        U, J = 4.0, 1.0
        p = kanamori(5, U=U, J=J, mu=mu_half(5, U, J),
                     delta=crystal_field(5, 0.1, MODEL_SEED))
        return Workload("kanamori-5orb-b50", p, 50.0, 4096, 5.0, 1001, "fp64", 1e-5)
    if k == 2:
        U, J = 6.0, 0.7
        p = kanamori(7, U=U, J=J, mu=mu_half(7, U, J),
                     delta=crystal_field(7, 0.05, MODEL_SEED))
        return Workload("kanamori-7orb-b40", p, 40.0, 1024, 6.0, 1002, "mixed", 1e-5,
                        krylov_max=20, krylov_tol=1e-7)
    raise ValueError(k)


def comparator_workload(n_orb: int, n_configs: int = 512) -> Workload:
    """The Krylov-against-matrix comparison of Sec. IV.B: n_orb = 2..7 orbitals at
    U = 6, J = U/6, half filling (mu_half), beta = 50, a crystal field of +-0.05,
    per-flavor orders ~ Poisson(5), the ground multiplet retained; FP64."""
    U, J = 6.0, 1.0
    p = kanamori(n_orb, U=U, J=J, mu=mu_half(n_orb, U, J), delta=crystal_field(n_orb, 0.05, MODEL_SEED))
    return Workload(f"kanamori-{n_orb}orb-U6-b50", p, 50.0, n_configs, 5.0, 1100 + n_orb, "fp64", 1e-5,
                    krylov_max=20, krylov_tol=1e-13)


# --------------------------------------------------------------------------
# bath and Monte Carlo inputs
# --------------------------------------------------------------------------

def parity_sample(n_configs: int, n: int, seed: int) -> np.ndarray:
    """Sorted indices of n of the n_configs configurations of a batch, drawn without
    replacement (the seeded sample a parity check evaluates)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_configs, n, replace=False))


def semicircle_delta(beta: float, n_tau: int, D: float = 2.0, t: float = 1.0,
                     n_quad: int = 6000) -> np.ndarray:
    """Hybridization function of a semicircular bath, tabulated on a uniform grid.

    Delta(tau) = t^2 G_sc(tau) with G_sc(tau) = -int rho(e) e^{-tau e} / (1 + e^{-beta e}) de,
    rho(e) = 2 / (pi D^2) sqrt(D^2 - e^2) (the bandwidth-4 semicircle of Sec. IV.A for
    D = 2), at tau_k = k beta / n_tau, k = 0..n_tau (k = 0 is 0^+, k = n_tau is beta^-).
    This is an *input* of the impurity solver (in a DMFT loop it would come from the
    self-consistency); the solver interpolates the table linearly and extends it
    antiperiodically.  Gauss-Chebyshev quadrature of the second kind with n_quad nodes.
    """
    i = np.arange(1, n_quad + 1)
    x = np.cos(i * np.pi / (n_quad + 1))
    w = np.pi / (n_quad + 1) * np.sin(i * np.pi / (n_quad + 1)) ** 2
    e = D * x
    taus = np.arange(n_tau + 1) * (beta / n_tau)
    out = np.empty(n_tau + 1)
    pos = e > 0
    for k, tau in enumerate(taus):
        # overflow-free Fermi-weighted exponential on both sides of the band centre
        g = np.empty_like(e)
        g[pos] = np.exp(-tau * e[pos]) / (1.0 + np.exp(-beta * e[pos]))
        g[~pos] = np.exp((beta - tau) * e[~pos]) / (np.exp(beta * e[~pos]) + 1.0)
        out[k] = -(2.0 / np.pi) * np.sum(w * g) * t * t
    return out


@dataclass
class McSetup:
    name: str
    workload: Workload
    n_chains: int
    n_tau_delta: int
    delta: np.ndarray          # [n_tau_delta + 1]
    init_seed: int
    max_init_pairs: int        # chains start at total pair numbers uniform in 0..max
    kmax_flavor: int           # capacity per flavor (pairs)
    seed: int                  # counter-based generator key of the chains


def mc_setup(k: int = 3, n_chains: int | None = None) -> McSetup:
    """Monte Carlo workloads.  k = 3: the 5-orbital model of workload 1 coupled to a
    semicircular bath (D = 2, t = 1), 256 chains whose initial total pair numbers are
    uniform in 0..200 (a scheduling stress).  k = 5: one orbital, U = 0, eps = 0, beta = 10
    (the non-interacting check: G(tau) must equal G_sc(tau)).  k = 6: the 2-orbital model
    of workload 0 with the bath, small chains for trajectory parity."""
    if k == 3:
        w = workload(1)
        n = 256 if n_chains is None else n_chains
        return McSetup("kanamori-5orb-b50-mc", w, n, 4096, semicircle_delta(w.beta, 4096), 3003, 200, 48, 7)
    if k == 5:
        p = kanamori(1, U=0.0, J=0.0, mu=0.0)
        w = Workload("free-1orb-b10", p, 10.0, 0, 0.0, 0, "fp64", -1.0)
        n = 64 if n_chains is None else n_chains
        return McSetup("free-1orb-b10-mc", w, n, 1000, semicircle_delta(10.0, 1000), 3005, 0, 48, 11)
    if k == 6:
        w = workload(0)
        n = 8 if n_chains is None else n_chains
        return McSetup("kanamori-2orb-b10-mc", w, n, 1000, semicircle_delta(w.beta, 1000), 3006, 12, 32, 13)
    raise ValueError(k)


def dmft_setup(n_orb: int, U: float, beta: float, n_chains: int = 128, n_delta: int = 1000) -> McSetup:
    """The Bethe-lattice DMFT models of Sec. V: n_orb degenerate orbitals, J = U/6,
    half filling (mu_half), every local state kept (full trace), chains starting
    empty, the initial bath the non-interacting semicircle (D = 2, t = 1)."""
    J = U / 6.0
    p = kanamori(n_orb, U=U, J=J, mu=mu_half(n_orb, U, J))
    w = Workload(f"kanamori-{n_orb}orb-U{U:g}-b{beta:g}", p, beta, 0, 0.0, 0, "fp64", -1.0)
    return McSetup(f"{w.name}-dmft", w, n_chains, n_delta, semicircle_delta(beta, n_delta), 3100 + n_orb, 0, 48,
                   17 + n_orb)


def mc_initial_configs(setup: McSetup, min_pairs: int = 0, refs=None):
    """Per chain: (cre, ann) with cre[f] / ann[f] the creator / annihilator times of
    flavor f in label order (the i-th creator in time is paired with the i-th
    annihilator).  Total pair number uniform in min_pairs..max_init_pairs, spread over
    the flavors uniformly; per flavor the operators alternate in time, starting with c
    if the flavor is occupied in a reference Fock state: single occupancy with random
    spins, or one of refs (bit f set = flavor f occupied) drawn at random per chain."""
    n_orb = setup.workload.params.n_orb
    F, beta = 2 * n_orb, setup.workload.beta
    rng = np.random.default_rng(setup.init_seed)
    chains = []
    for _ in range(setup.n_chains):
        K = int(rng.integers(min_pairs, setup.max_init_pairs + 1))
        kf = np.bincount(rng.integers(0, F, size=K), minlength=F)
        kf = np.minimum(kf, setup.kmax_flavor)
        occ = np.zeros(F, dtype=bool)
        if refs is None:
            spins = rng.integers(0, 2, size=n_orb)
            for a in range(n_orb):
                occ[a + n_orb * spins[a]] = True
        else:
            s = int(refs[int(rng.integers(0, len(refs)))])
            for f in range(F):
                occ[f] = bool((s >> f) & 1)
        cre, ann = [], []
        for f in range(F):
            ts = np.sort(rng.uniform(0.0, beta, size=2 * kf[f]))
            if occ[f]:       # c first: annihilators at even positions
                ann.append(ts[0::2].copy()); cre.append(ts[1::2].copy())
            else:
                cre.append(ts[0::2].copy()); ann.append(ts[1::2].copy())
        chains.append((cre, ann))
    return chains


def mc_merged(cre, ann):
    """Time-ordered operator list (tau, flavor, dagger) of a per-flavor pair state."""
    taus, fls, dgs = [], [], []
    for f in range(len(cre)):
        taus += [np.asarray(cre[f]), np.asarray(ann[f])]
        fls += [np.full(len(cre[f]), f, np.int16), np.full(len(ann[f]), f, np.int16)]
        dgs += [np.ones(len(cre[f]), np.int8), np.zeros(len(ann[f]), np.int8)]
    tau = np.concatenate(taus) if taus else np.zeros(0)
    fl = np.concatenate(fls) if fls else np.zeros(0, np.int16)
    dg = np.concatenate(dgs) if dgs else np.zeros(0, np.int8)
    o = np.argsort(tau, kind="stable")
    return tau[o], fl[o], dg[o]
