"""Host-side helpers of bench.py: the sign-weighted observable of the ESS measurement,
the depth histogram, and the oracle's feasible-path count (against a brute-force
walk of the 2-orbital sectors)."""
import numpy as np
import pytest

import bench
from paper_0908_0681_amd import inputs as I


def test_sign_weighted_observable_is_a_plain_average():
    rng = np.random.default_rng(1)
    g = rng.normal(size=(3, 4, 20))
    nm = np.array([1, 2, 5])
    beta, n_tau = 10.0, 20
    got = bench._sg_half(g, nm, beta, n_tau)
    want = [-(g[c, :, 9:11].mean()) / (beta * (beta / n_tau) * nm[c]) for c in range(3)]
    assert np.allclose(got, want, rtol=1e-14)
    # with one measurement per chain the sums come back unscaled
    assert np.allclose(bench._sg_half(g, 1, beta, n_tau), got * nm, rtol=1e-14)


def test_depth_histogram_counts_configurations():
    import torch
    offsets = np.array([0, 3, 7, 7, 10])          # 3, 4, 0 and 3 operators
    batch = type("B", (), {"offsets": offsets})()
    out = {"feasible_paths": torch.tensor([1, 2, 0, 1]), "krylov_steps": torch.tensor([5, 12, 0, 20])}
    h = bench.depth_histogram(batch, out)
    # mean depths 5/2 = 2.5, 12/6 = 2.0, (none), 20/2 = 10.0
    assert sum(h["configs"]) == 3
    assert h["configs"][2] == 2 and h["configs"][10] == 1


def test_oracle_feasible_paths_matches_the_full_oracle():
    """bench.oracle_feasible_paths walks sectors only; the full oracle path (which also
    does the arithmetic) reports the same feasibility (2-orbital batch)."""
    from oracle import trace as T
    w = I.workload(0)
    o = T.build(w.params, w.retain_window)
    b = w.batch()
    want = 0
    for c in range(b.n_configs):
        tau, fl, dg = b.config(c)
        for r in range(len(o.R.block)):
            want += int(o.path(tau, fl, dg, b.beta, r)[0])
    got = bench.oracle_feasible_paths(0)
    assert got == want and got > 0


def test_robust_variance_ignores_outlying_chains():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(4000) * 2.0
    v, n = bench._robust_var(x)
    assert v == pytest.approx(4.0, rel=0.1) and n == 0
    y = np.concatenate([x, [1e3, -5e2, 80.0]])
    v2, n2 = bench._robust_var(y)
    assert v2 == pytest.approx(v, rel=0.01) and n2 == 3
    assert np.var(y) > 50 * v2


def test_ratio_jackknife_matches_leave_one_out():
    rng = np.random.default_rng(5)
    C = 40
    s = rng.integers(50, 100, C).astype(float)
    sg = rng.normal(size=C) * 3.0 + 0.5 * s
    R, se = bench._ratio_jackknife(sg, s)
    assert R == pytest.approx(sg.sum() / s.sum(), rel=1e-14)
    loo = np.array([(sg.sum() - sg[c]) / (s.sum() - s[c]) for c in range(C)])
    want = np.sqrt((C - 1) / C * np.sum((loo - loo.mean()) ** 2))
    assert se == pytest.approx(want, rel=1e-12)
    # equal weights: the jackknife error of a mean is the plain standard error
    x = rng.normal(size=C)
    _, se2 = bench._ratio_jackknife(x, np.ones(C))
    assert se2 == pytest.approx(np.std(x, ddof=1) / np.sqrt(C), rel=1e-12)
    # per-bin curves at once
    sgk = np.stack([sg, 2 * sg], axis=1)
    Rk, sek = bench._ratio_jackknife(sgk, s)
    assert np.allclose(Rk, [R, 2 * R]) and np.allclose(sek, [se, 2 * se])


def test_drift_and_two_sample_statistics():
    rng = np.random.default_rng(6)
    a = rng.normal(size=400)
    assert abs(bench._drift_t(a, a + rng.normal(size=400) * 0.1)) < 4.0
    assert bench._drift_t(a, a + 1.0 + rng.normal(size=400) * 0.1) > 50.0
    chi2, zmax = bench._two_sample([1.0, 2.0], [0.1, 0.1], [1.0, 2.0], [0.1, 0.1])
    assert chi2 == 0.0 and zmax == 0.0
    chi2, zmax = bench._two_sample([1.0], [0.3], [0.0], [0.4])
    assert zmax == pytest.approx(2.0) and chi2 == pytest.approx(4.0)


def test_heldout_gain_of_flat_and_sharp_networks():
    N = 1000
    rng = np.random.default_rng(7)
    t = np.stack([rng.integers(0, 64, N), rng.integers(0, 64, N)], axis=1)
    mix, net = bench._heldout_gain(np.zeros((N, 128)), t, 50.0, 0.1)
    assert mix == pytest.approx(0.0, abs=1e-12) and net == pytest.approx(0.0, abs=1e-12)
    # a network certain of the right bins: network gain 2 log 64, mixture log(0.9*64^2 + 0.1)
    z = np.full((N, 128), -1e3)
    z[np.arange(N), t[:, 0]] = 0.0
    z[np.arange(N), 64 + t[:, 1]] = 0.0
    mix, net = bench._heldout_gain(z, t, 50.0, 0.1)
    assert net == pytest.approx(2 * np.log(64))
    assert mix == pytest.approx(np.log(0.9 * 64 ** 2 + 0.1))
