"""Pins of the oracle's Monte Carlo parts (weight of Eq.(2), moves, G(tau) estimator)
against facts that do not come from the oracle itself: published generator test
vectors, a hand-derived single-pair weight, the absence of negative weights for
density-density interactions, relabelling invariance, and the non-interacting
limit where the measured Green's function must equal the bath's own.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from paper_0908_0681_amd import inputs as I
from oracle import mc as MC
from oracle import trace as T


def test_philox_known_answers():
    """Philox4x32-10 known-answer vectors published with the generator (Salmon et al.,
    SC'11, Random123 distribution): zero counter/key, all-ones, and the pi digits."""
    assert MC.philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    ones = (0xFFFFFFFF,) * 4
    assert MC.philox4x32_10(ones, ones[:2]) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert MC.philox4x32_10((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0)) == \
        (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_uniforms_range():
    assert MC.u01(0, 0) == 0.0
    assert MC.u01(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    u = np.array([MC.move_uniforms(5, c, s) for c in range(4) for s in range(250)]).ravel()
    assert 0.0 <= u.min() and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.02


def test_semicircle_bath_table():
    """The bath input: sum rule Delta(0+) + Delta(beta-) = -t^2, particle-hole
    symmetry Delta(tau) = Delta(beta - tau), and adaptive quadrature at interior points."""
    beta, n = 10.0, 1000
    d = I.semicircle_delta(beta, n)
    assert d[0] + d[-1] == pytest.approx(-1.0, abs=1e-12)
    assert np.max(np.abs(d - d[::-1])) < 1e-13
    for k in (1, 137, 500, 999):
        tau = k * beta / n
        f = lambda e: (2 / (np.pi * 4)) * np.sqrt(4 - e * e) * np.exp(-tau * e) / (1 + np.exp(-beta * e))
        v, _ = quad(f, -2, 2, limit=400, epsabs=1e-15, epsrel=1e-13)
        assert d[k] == pytest.approx(-v, rel=1e-9)


def test_delta_interpolation_and_antiperiodicity():
    beta = 10.0
    d = I.semicircle_delta(beta, 1000)
    for k in (0, 3, 500, 999):
        assert MC.delta_at(d, beta, k * beta / 1000) == d[k]
    assert MC.delta_at(d, beta, 2.505) == pytest.approx(0.5 * (d[250] + d[251]), rel=1e-12)
    assert MC.delta_at(d, beta, 3.0 - beta) == pytest.approx(-MC.delta_at(d, beta, 3.0), rel=1e-15)


def _free_one_orbital():
    s = I.mc_setup(5)
    return s, T.build(s.workload.params, s.workload.retain_window)


def test_single_pair_weight_by_hand():
    """One orbital, U = 0, eps = 0 (H_loc = 0, all four states kept).  A segment
    c^dag_up(2) ... c_up(5): the literal product is already time ordered
    (s_perm = +1), the trace counts the two states without an up electron, and
    det A = Delta(2 - 5) = -Delta(beta - 3) > 0, so w = 2 |Delta(7)|.  The
    anti-segment (c at 2, c^dag at 5) has the same weight: the T-ordering sign
    -1 meets Delta(3) < 0."""
    s, o = _free_one_orbital()
    beta, d = s.workload.beta, s.delta
    want = math.log(2.0 * abs(MC.delta_at(d, beta, 7.0)))
    sg, lw = MC.weight(o, d, beta, [[2.0], []], [[5.0], []])
    assert sg == 1 and lw == pytest.approx(want, rel=1e-13)
    sg, lw = MC.weight(o, d, beta, [[5.0], []], [[2.0], []])
    want_anti = math.log(2.0 * abs(MC.delta_at(d, beta, 3.0)))
    assert sg == 1 and lw == pytest.approx(want_anti, rel=1e-13)
    assert MC.perm_sign([[5.0], []], [[2.0], []]) == -1


def _random_pairs(rng, F, beta, kmax):
    cre, ann = [], []
    for f in range(F):
        k = int(rng.integers(0, kmax + 1))
        ts = np.sort(rng.uniform(0, beta, 2 * k))
        if rng.integers(0, 2):
            cre.append(list(ts[0::2])); ann.append(list(ts[1::2]))
        else:
            ann.append(list(ts[0::2])); cre.append(list(ts[1::2]))
    return cre, ann


@pytest.mark.parametrize("window", [-1.0, 1e-6])
def test_density_density_weights_are_never_negative(window):
    """With density-density interactions (J_sf = J_ph = 0) the expansion has no sign
    problem (Sec. IV.A); a wrong permutation sign or determinant convention breaks this."""
    s = I.mc_setup(6)
    p = I.kanamori(2, 4.0, 1.0, 3.5, density_density=True)
    o = T.build(p, window)
    rng = np.random.default_rng(11)
    nonzero = 0
    for _ in range(150):
        cre, ann = _random_pairs(rng, 4, 10.0, 3)
        sg, _ = MC.weight(o, s.delta, 10.0, cre, ann)
        assert sg >= 0
        nonzero += sg > 0
    assert nonzero >= 40


def test_weight_is_independent_of_pair_labels():
    """Relabelling creators (or annihilators) of a flavor permutes rows (columns) of
    A_f and the canonical string together: the weight must not change."""
    s = I.mc_setup(6)
    w = s.workload
    o = T.build(w.params, w.retain_window)
    rng = np.random.default_rng(3)
    checked = 0
    for _ in range(40):
        cre, ann = _random_pairs(rng, 4, w.beta, 3)
        sg, lw = MC.weight(o, s.delta, w.beta, cre, ann)
        if sg == 0:
            continue
        cre2 = [list(np.asarray(c)[rng.permutation(len(c))]) for c in cre]
        ann2 = [list(np.asarray(a)[rng.permutation(len(a))]) for a in ann]
        sg2, lw2 = MC.weight(o, s.delta, w.beta, cre2, ann2)
        assert sg2 == sg and lw2 == pytest.approx(lw, rel=1e-12, abs=1e-12)
        checked += 1
    assert checked >= 10


def test_insert_then_remove_is_detailed_balance():
    """Insert a pair, then propose removing exactly that pair: the two
    Metropolis-Hastings ratios are |w'/w| q_rem / q_ins and its inverse, so their
    logs cancel (a mismatched pair of proposal factors fails this)."""
    s = I.mc_setup(6)
    w = s.workload
    o = T.build(w.params, w.retain_window)
    rng = np.random.default_rng(8)
    checked = 0
    while checked < 12:
        cre, ann = _random_pairs(rng, 4, w.beta, 2)
        if MC.weight(o, s.delta, w.beta, cre, ann)[0] == 0:
            continue
        ch = MC.Chain(o, s.delta, w.beta, cre, ann, 32)
        f = int(rng.integers(0, 4))
        k = len(ch.cre[f])
        u_ins = [(f + 0.5) / 4, 0.25, rng.uniform(), rng.uniform(), 0.0]
        kind, cre2, ann2, s2, lw2, lr_ins = ch.propose(u_ins)
        if s2 == 0:
            continue
        back = MC.Chain(o, s.delta, w.beta, cre2, ann2, 32)
        last = (k + 0.5) / (k + 1)     # labels i = j = k: the pair just inserted
        kind_r, cre3, ann3, s3, lw3, lr_rem = back.propose([(f + 0.5) / 4, 0.75, last, last, 0.0])
        assert kind == 1 and kind_r == 2
        assert cre3 == ch.cre and ann3 == ch.ann and s3 == ch.sign
        assert lr_ins + lr_rem == pytest.approx(0.0, abs=1e-11)
        checked += 1


def test_free_orbital_green_function_equals_bath():
    """U = 0, eps = 0 with Delta = t^2 G_sc (t = 1): the impurity Green's function is
    G_sc itself (the semicircle's self-consistency), so the sampled G(tau), binned,
    must match the bin averages of the Delta table within the statistical error."""
    s, o = _free_one_orbital()
    beta, n_tau = s.workload.beta, 20
    ch = MC.Chain(o, s.delta, beta, [[], []], [[], []], 48)
    blocks, step = [], 0
    for b in range(7):
        acc = np.zeros((2, n_tau))
        ssum = 0.0
        for it in range(3000):
            ch.step(MC.move_uniforms(s.seed, 0, step))
            step += 1
            if it % 4 == 0:
                ch.measure(acc)
                ssum += ch.sign
        if b > 0:                      # block 0 is thermalisation
            blocks.append(MC.g_tau(acc, ssum, beta))
    G = np.array(blocks)
    mean = G.mean(axis=0)
    err = G.std(axis=0, ddof=1) / np.sqrt(len(G))
    ref = np.array([np.mean([MC.delta_at(s.delta, beta, x) for x in
                             np.linspace(b * beta / n_tau, (b + 1) * beta / n_tau, 41)[1:-1]])
                    for b in range(n_tau)])
    z = (mean - ref) / err
    assert np.abs(z).max() < 4.5 and np.mean(z ** 2) < 2.5, (np.abs(z).max(), np.mean(z ** 2))
