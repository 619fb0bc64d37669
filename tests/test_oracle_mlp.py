"""Pins of the oracle's learned-proposal parts: BF16 rounding, the feature map by hand,
the backward pass against central differences of the FP64 network, normalisation of
the insertion density, and detailed balance of the Metropolis-Hastings factors with
the learned density."""
import math

import numpy as np
import pytest

from paper_0908_0681_amd import inputs as I
from oracle import mc as MC
from oracle import mlp as NN
from oracle import trace as T


def test_bf16_rounding():
    assert NN.bf16(1.0) == 1.0
    assert NN.bf16(1.0 + 2.0 ** -8) == 1.0                     # tie -> even
    assert NN.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6     # tie -> even (upwards)
    assert NN.bf16(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7
    assert NN.bf16(3.14159) == 3.140625
    assert NN.bf16(-0.1) == -0.10009765625


def test_features_by_hand():
    beta = 10.0
    cre, ann = [[2.0], []], [[5.0], []]
    x = NN.features(cre, ann, 1, beta)
    assert x[0] == 0.0 and x[1] == 1.0          # one-hot of the proposing flavor
    assert x[2] == 1.0 / 32 and x[3] == 0.0     # k / 32
    steps = x[4:4 + 32]
    centres = (np.arange(32) + 0.5) * beta / 32
    assert np.array_equal(steps, ((centres > 2.0) & (centres < 5.0)).astype(float))
    assert np.all(x[4 + 32:] == 0.0)
    y = NN.features(cre, ann, 0, beta, exclude=(0, 0, 0))
    assert y[0] == 1.0 and y[2] == 0.0 and np.all(y[4:] == 0.0)


def _random_net(seed, quantize, scale=0.05):
    rng = np.random.default_rng(seed)
    Ws = [rng.standard_normal((NN.H, NN.IN)) * scale, rng.standard_normal((NN.H, NN.H)) * scale,
          rng.standard_normal((NN.OUT, NN.H)) * scale]
    bs = [rng.standard_normal(NN.H) * 0.1, rng.standard_normal(NN.H) * 0.1, rng.standard_normal(NN.OUT) * 0.1]
    return NN.Network(Ws, bs, quantize=quantize), Ws, bs


def test_backward_matches_central_differences():
    net, Ws, bs = _random_net(1, quantize=False, scale=0.2)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((5, NN.IN))
    Tg = rng.integers(0, NN.BINS, size=(5, 2))
    dWs, dbs, loss = net.gradients(X, Tg)
    assert loss == pytest.approx(net.loss(X, Tg), rel=1e-12)
    h = 1e-6
    for L in range(3):
        for _ in range(6):
            i, j = rng.integers(0, net.W[L].shape[0]), rng.integers(0, net.W[L].shape[1])
            old = net.W[L][i, j]
            net.W[L][i, j] = old + h
            lp = net.loss(X, Tg)
            net.W[L][i, j] = old - h
            lm = net.loss(X, Tg)
            net.W[L][i, j] = old
            assert dWs[L][i, j] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-8), (L, i, j)
        i = rng.integers(0, len(net.b[L]))
        old = net.b[L][i]
        net.b[L][i] = old + h
        lp = net.loss(X, Tg)
        net.b[L][i] = old - h
        lm = net.loss(X, Tg)
        net.b[L][i] = old
        assert dbs[L][i] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-8), (L, i)


def test_insertion_density_is_normalised():
    net, _, _ = _random_net(3, quantize=True)
    z = net.forward(np.random.default_rng(4).standard_normal((1, NN.IN)))["Z3"][0]
    beta, eps = 7.0, 0.1
    w = beta / NN.BINS
    tot = sum(math.exp(NN.logq(z, (a + 0.5) * w, (b + 0.5) * w, beta, eps)) * w * w
              for a in range(NN.BINS) for b in range(NN.BINS))
    assert tot == pytest.approx(1.0, rel=1e-12)


@pytest.mark.parametrize("mix", [0.9, 0.05])   # network branch, uniform branch of the mixture
def test_learned_insert_then_remove_is_detailed_balance(mix):
    s = I.mc_setup(6)
    w = s.workload
    o = T.build(w.params, w.retain_window)
    net, _, _ = _random_net(5, quantize=True, scale=0.1)
    rng = np.random.default_rng(9)
    checked = 0
    while checked < 6:
        cre = [sorted(rng.uniform(0, w.beta, rng.integers(0, 3)).tolist()) for _ in range(4)]
        ann = [sorted(rng.uniform(0, w.beta, len(c)).tolist()) for c in cre]
        if MC.weight(o, s.delta, w.beta, cre, ann)[0] == 0:
            continue
        ch = MC.Chain(o, s.delta, w.beta, cre, ann, 32, net=net, eps=0.1)
        f = int(rng.integers(0, 4))
        k = len(ch.cre[f])
        u = [(f + 0.5) / 4, 0.25, rng.uniform(), rng.uniform(), 0.0, 0.0, rng.uniform(), rng.uniform(), mix, 0.0]
        kind, cre2, ann2, s2, lw2, lr_ins = ch.propose(u)
        if s2 == 0:
            continue
        back = MC.Chain(o, s.delta, w.beta, cre2, ann2, 32, net=net, eps=0.1)
        last = (k + 0.5) / (k + 1)
        kind_r, cre3, ann3, s3, _, lr_rem = back.propose([(f + 0.5) / 4, 0.75, last, last, 0.0, 0.0, 0, 0, 0, 0])
        assert kind == 1 and kind_r == 2 and cre3 == ch.cre and ann3 == ch.ann and s3 == ch.sign
        assert lr_ins + lr_rem == pytest.approx(0.0, abs=1e-10)
        checked += 1
