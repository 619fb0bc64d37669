"""GPU learned proposal (hyb_mlp_*, hyb_mc_attach_mlp, hyb_mc_harvest) through the C ABI.

Forward and backward are compared with the oracle's FP64 network, which rounds to
BF16 at the same points as the device.  The remaining differences come from FP32
accumulation and the rare BF16 rounding decisions it flips.  Every element is
checked, against the largest magnitude of its tensor:
- logits: max |z - z_ref| <= 5e-3 max |z_ref|;
- gradients: max |g - g_ref| <= 1e-2 max |g_ref| per tensor (the stated BF16/FP32
  tolerance against FP64).
Harvested training samples are exact (integer features, bins).  Learned moves replay
the oracle's chain move by move (configurations exact, divergence allowed only where a
BF16-level change of the logits can flip a bin draw or an acceptance, which then resyncs
the oracle).  A sampler using the learned density must sample the same distribution as
the uniform one:
- G(tau) = G_sc(tau) for a free orbital;
- learned and uniform G(tau) agree on the 2-orbital model (two-sample test).
"""
import math
import sys

import numpy as np
import pytest

from paper_0908_0681_amd import inputs as I
from paper_0908_0681_amd import hyb
from oracle import mc as MC
from oracle import mlp as NN
from oracle import trace as T

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def announce(request):
    print(f"\n[gpu-test] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _random_weights(seed, scale=0.1):
    rng = np.random.default_rng(seed)
    Ws = [(rng.standard_normal(s) * scale).astype(np.float32) for s in hyb.MLP_W_SHAPES]
    bs = [(rng.standard_normal(s) * 0.1).astype(np.float32) for s in hyb.MLP_B_SHAPES]
    return Ws, bs


def _features_batch(n, seed):
    """Features of random 5-orbital configurations (one flavor each) and pair bins."""
    rng = np.random.default_rng(seed)
    X, T = [], []
    for _ in range(n):
        k = rng.integers(0, 6, size=10)
        cre = [sorted(rng.uniform(0, 50.0, kk).tolist()) for kk in k]
        ann = [sorted(rng.uniform(0, 50.0, kk).tolist()) for kk in k]
        X.append(NN.features(cre, ann, int(rng.integers(0, 10)), 50.0))
        T.append(rng.integers(0, NN.BINS, size=2))
    return np.array(X), np.array(T, dtype=np.int32)


def _rel(a, b):
    """Largest element error against the largest element of the reference."""
    return float(np.max(np.abs(np.asarray(a, np.float64) - b)) / np.max(np.abs(b)))


def test_mlp_forward_matches_oracle():
    _require_gpu()
    Ws, bs = _random_weights(1)
    net = hyb.MLP(seed=3)
    net.set_weights(Ws, bs)
    X, _ = _features_batch(200, 2)
    Xd = torch.tensor(X, device="cuda").to(torch.bfloat16)
    assert torch.equal(Xd.double().cpu(), torch.tensor(X))           # features are exact in BF16
    Z = torch.empty(200, NN.OUT, device="cuda")
    net.forward(Xd, Z)
    torch.cuda.synchronize()
    ref = NN.Network(Ws, bs, quantize=True).forward(X)["Z3"]
    err = _rel(Z.cpu().numpy(), ref)
    print(f"logits: relative error {err:.2e} (vs unrounded FP64: "
          f"{_rel(Z.cpu().numpy(), NN.Network(Ws, bs, quantize=False).forward(X)['Z3']):.2e})")
    assert err <= 5e-3
    net.close()


def test_mlp_gradients_match_oracle():
    _require_gpu()
    Ws, bs = _random_weights(4)
    net = hyb.MLP(seed=3)
    net.set_weights(Ws, bs)
    X, Tg = _features_batch(256, 5)
    Xd = torch.tensor(X, device="cuda").to(torch.bfloat16)
    Td = torch.tensor(Tg, device="cuda")
    gW, gb, loss = net.gradients(Xd, Td)
    rW, rb, rloss = NN.Network(Ws, bs, quantize=True).gradients(X, Tg)
    assert loss == pytest.approx(rloss, rel=1e-3)
    for L in range(3):
        ew, eb = _rel(gW[L], rW[L]), _rel(gb[L], rb[L])
        print(f"layer {L + 1}: dW {ew:.2e}, db {eb:.2e}")
        assert ew <= 1e-2 and eb <= 1e-2
    net.close()


def test_mlp_training_reduces_loss():
    """Targets that depend on the features (bins from the first occupied time bin of
    the proposing flavor): Adam steps on the device lower the loss."""
    _require_gpu()
    rng = np.random.default_rng(7)
    X, _ = _features_batch(1024, 8)
    f = np.argmax(X[:, :10], axis=1)
    T = np.stack([(f * 6 + 3) % NN.BINS, (X[:, 10:20].sum(axis=1) * 32 * 2).astype(int) % NN.BINS], axis=1)
    Xd = torch.tensor(X, device="cuda").to(torch.bfloat16)
    Td = torch.tensor(T.astype(np.int32), device="cuda")
    net = hyb.MLP(seed=11)
    first = net.train_step(Xd[:256], Td[:256], 1e-3, want_loss=True)
    for it in range(400):
        idx = torch.tensor(rng.integers(0, 1024, 256), device="cuda")
        net.train_step(Xd[idx].contiguous(), Td[idx].contiguous(), 1e-3)
    _, _, last = net.gradients(Xd, Td)
    print(f"loss {first:.3f} -> {last:.3f}")
    assert last < 0.5 * first
    net.close()


def test_mc_harvest_matches_oracle():
    _require_gpu()
    setup = I.mc_setup(6, 8)
    w = setup.workload
    m = hyb.model_for_workload(w)
    mc = hyb.MC(m, setup.n_chains, w.beta, setup.delta, kmax=32, nmax_ops=512, seed=setup.seed, n_tau=10)
    mc.sweep(60)
    st = mc.state()
    X = torch.zeros(setup.n_chains, NN.IN, device="cuda", dtype=torch.bfloat16)
    T = torch.zeros(setup.n_chains, 2, device="cuda", dtype=torch.int32)
    mc.harvest(17, X, T)
    torch.cuda.synchronize()
    Xh, Th = X.double().cpu().numpy(), T.cpu().numpy()
    F = 4
    for c in range(setup.n_chains):
        cre = [list(st["cre"][c, f, :st["k"][c, f]]) for f in range(F)]
        ann = [list(st["ann"][c, f, :st["k"][c, f]]) for f in range(F)]
        u = MC.move_uniforms(setup.seed, c, 17, calls=(8, 9))
        nonempty = [g for g in range(F) if len(cre[g])]
        if not nonempty:
            assert list(Th[c]) == [-1, -1]
            continue
        f = nonempty[min(int(u[0] * len(nonempty)), len(nonempty) - 1)]
        k = len(cre[f])
        i, j = min(int(u[1] * k), k - 1), min(int(u[2] * k), k - 1)
        assert np.array_equal(Xh[c], NN.features(cre, ann, f, w.beta, exclude=(f, i, j))), c
        ln = ann[f][j] - cre[f][i]
        ln += w.beta if ln < 0 else 0.0
        assert list(Th[c]) == [min(int(cre[f][i] / w.beta * 64), 63), min(int(ln / w.beta * 64), 63)], c
    mc.close()


def _g_per_chain(mc, beta, n_tau):
    g, ms, nm = mc.accumulators()
    return -g / (beta * (beta / n_tau) * ms[:, None, None])


def test_mc_learned_free_orbital_green_function():
    """Any valid insertion density samples the same distribution: with a (random)
    network attached, G(tau) = G_sc(tau) still holds."""
    _require_gpu()
    setup = I.mc_setup(5, 128)
    w = setup.workload
    m = hyb.model_for_workload(w)
    n_tau = 20
    mc = hyb.MC(m, setup.n_chains, w.beta, setup.delta, kmax=48, nmax_ops=256, seed=setup.seed + 1,
                n_tau=n_tau, meas_every=2)
    net = hyb.MLP(seed=5)
    mc.attach_mlp(net, eps=0.2)
    mc.sweep(500)
    mc.reset_measurements()
    mc.sweep(3000)
    per = _g_per_chain(mc, w.beta, n_tau)
    mean, err = per.mean(axis=0), per.std(axis=0, ddof=1) / math.sqrt(setup.n_chains)
    h = w.beta / n_tau
    ref = np.array([np.mean([MC.delta_at(setup.delta, w.beta, x) for x in np.linspace(b * h, (b + 1) * h, 41)[1:-1]])
                    for b in range(n_tau)])
    z = (mean - ref[None, :]) / err
    st = mc.stats()
    print(f"learned, free orbital: max |z| {np.abs(z).max():.2f}, chi2/dof {np.mean(z ** 2):.2f}, acceptance "
          f"{(st['insert_accepted'] + st['remove_accepted']) / st['moves']:.3f}")
    assert np.abs(z).max() < 5.0 and np.mean(z ** 2) < 2.5
    mc.close()
    net.close()


def test_mc_learned_matches_uniform_two_orbital():
    """2-orbital Kanamori model with the bath: G(tau) from the learned proposal (a
    network trained briefly on harvested pairs) agrees with the uniform proposal's,
    and the trained network raises the acceptance of the moves over the uniform
    proposal (what it gains; the effective sample size of G(beta/2) from the spread
    of the chain means is printed beside it)."""
    _require_gpu()
    setup = I.mc_setup(6, 256)
    w = setup.workload
    m = hyb.model_for_workload(w)
    n_tau = 16
    runs, accept = {}, {}
    net = hyb.MLP(seed=9)
    for mode in ("uniform", "learned"):
        mc = hyb.MC(m, setup.n_chains, w.beta, setup.delta, kmax=32, nmax_ops=512,
                    seed=setup.seed + (0 if mode == "uniform" else 100), n_tau=n_tau, meas_every=2)
        if mode == "learned":
            # harvest pairs from the uniform chains' distribution and train briefly
            mc.sweep(400)
            Xs, Ts = [], []
            for hv in range(24):
                X = torch.zeros(setup.n_chains, NN.IN, device="cuda", dtype=torch.bfloat16)
                T = torch.zeros(setup.n_chains, 2, device="cuda", dtype=torch.int32)
                mc.harvest(hv, X, T)
                mc.sweep(5)
                Xs.append(X)
                Ts.append(T)
            X, T = torch.cat(Xs), torch.cat(Ts)
            keep = T[:, 0] >= 0
            X, T = X[keep].contiguous(), T[keep].contiguous()
            gen = torch.Generator(device="cuda").manual_seed(1)
            for it in range(300):
                idx = torch.randint(0, X.shape[0], (256,), device="cuda", generator=gen)
                net.train_step(X[idx].contiguous(), T[idx].contiguous(), 2e-3)
            mc.attach_mlp(net, eps=0.1)
        mc.sweep(1000)
        mc.reset_measurements()
        mc.sweep(4000)
        runs[mode] = _g_per_chain(mc, w.beta, n_tau)
        st = mc.stats()
        accept[mode] = (st['insert_accepted'] + st['remove_accepted']) / st['moves']
        print(f"{mode}: acceptance {accept[mode]:.3f}, "
              f"<order> {st['order_sum'] / st['moves']:.2f}, <sign> {st['sign_sum'] / st['moves']:.3f}")
        mc.close()
    a, b = runs["uniform"], runs["learned"]
    z = (a.mean(0) - b.mean(0)) / np.sqrt(a.var(0, ddof=1) / len(a) + b.var(0, ddof=1) / len(b))
    # 64 z values (4 flavors x 16 bins) that are strongly correlated (neighbouring bins,
    # spin-equivalent flavors): two independent uniform runs of this size give
    # chi2/dof up to ~1.5, so the bar is 3
    print(f"learned vs uniform: max |z| {np.abs(z).max():.2f}, chi2/dof {np.mean(z ** 2):.2f}")
    assert np.abs(z).max() < 5.0 and np.mean(z ** 2) < 3.0
    # G(beta/2) per chain (flavor average of the two middle bins); equal run lengths,
    # so the ratio of the spreads of the chain means is the ratio of effective samples
    mid = lambda g: g[:, :, n_tau // 2 - 1:n_tau // 2 + 1].mean(axis=(1, 2))
    ess_ratio = np.var(mid(a), ddof=1) / np.var(mid(b), ddof=1)
    print(f"acceptance learned / uniform {accept['learned'] / accept['uniform']:.3f}; "
          f"ESS of G(beta/2) learned / uniform {ess_ratio:.2f}")
    # the margin is many standard errors of an acceptance over 10^6 moves per sampler
    assert accept["learned"] > 1.08 * accept["uniform"]
    net.close()


def _edge_distance(z, u):
    """Distance of u * total from the nearest bin edge of the inverse-CDF draw, as a
    fraction of the total (a draw this close to an edge can flip between bins when
    the logits change at BF16 level)."""
    e = np.exp(np.asarray(z, dtype=np.float64) - np.max(z))
    c = np.cumsum(e)
    return float(np.min(np.abs(c[:-1] - u * c[-1])) / c[-1])


@pytest.mark.parametrize("which,n_chains,n_moves", [(6, 8, 120), (3, 16, 30)])
def test_mc_learned_trajectory_matches_oracle(which, n_chains, n_moves):
    """Learned moves replayed move by move: the oracle chain with the same network
    (FP64 with BF16 rounding points) and the same counter-based uniforms against the
    device chain (BF16 matrix cores, FP32 accumulation).  The logits differ at the
    1e-3 level, so a move may go another way, but only where that is explained: a bin
    draw within 1% of a bin edge, or an acceptance within 0.05 of its threshold.  The
    oracle chain is then restarted from the device state.  Every other move must leave
    both chains in the same configuration (times and labels exact), and at the end
    signs, log|w| and M agree as in the uniform replay."""
    _require_gpu()
    setup = I.mc_setup(which, n_chains)
    w = setup.workload
    F = 2 * w.params.n_orb
    kmax = setup.kmax_flavor
    o = T.build(w.params, w.retain_window)
    m = hyb.model_for_workload(w)
    net = hyb.MLP(seed=17)
    Ws, bs = _random_weights(21, scale=0.15)
    net.set_weights(Ws, bs)
    onet = NN.Network(Ws, bs, quantize=True)
    eps = 0.2
    mc = hyb.MC(m, setup.n_chains, w.beta, setup.delta, kmax=kmax, nmax_ops=512, seed=setup.seed, n_tau=10)
    chains = []
    for cre, ann in I.mc_initial_configs(setup):
        try:
            ch = MC.Chain(o, setup.delta, w.beta, cre, ann, kmax, net=onet, eps=eps)
        except ValueError:
            ch = MC.Chain(o, setup.delta, w.beta, [[]] * F, [[]] * F, kmax, net=onet, eps=eps)
        chains.append(ch)
    mc.set_configs([(ch.cre, ch.ann) for ch in chains])
    mc.attach_mlp(net, eps=eps)
    same = diverged = accepted = 0
    for step in range(n_moves):
        mc.sweep(1)
        st = mc.state()
        for c, ch in enumerate(chains):
            u = MC.move_uniforms(setup.seed, c, step, calls=(0, 1, 2, 3, 4))
            f = min(int(u[0] * F), F - 1)
            near_edge = False
            if u[1] < 0.5 and len(ch.cre[f]) < kmax and not u[8] < eps:
                z = onet.forward(NN.features(ch.cre, ch.ann, f, w.beta)[None])["Z3"][0]
                near_edge = min(_edge_distance(z[:NN.BINS], u[2]), _edge_distance(z[NN.BINS:], u[3])) < 0.01
            ch.last_margin = np.inf
            kind, a = ch.step(u)
            accepted += a
            dev = ([list(st["cre"][c, g, :st["k"][c, g]]) for g in range(F)],
                   [list(st["ann"][c, g, :st["k"][c, g]]) for g in range(F)])
            if dev == (ch.cre, ch.ann):
                same += 1
                continue
            assert near_edge or ch.last_margin < 0.05, (which, step, c, kind, ch.last_margin)
            diverged += 1
            chains[c] = MC.Chain(o, setup.delta, w.beta, dev[0], dev[1], kmax, net=onet, eps=eps)
    print(f"learned replay: {same} moves identical, {diverged} explained divergences, {accepted} accepted")
    assert diverged <= max(2, 0.05 * (same + diverged))
    st = mc.state(with_M=True)
    worst_M = worst_w = 0.0
    for c, ch in enumerate(chains):
        for g in range(F):
            k = len(ch.cre[g])
            assert st["k"][c, g] == k
            if k:
                Mi = np.linalg.inv(MC.hyb_matrix(setup.delta, w.beta, ch.cre[g], ch.ann[g]))
                worst_M = max(worst_M, np.max(np.abs(st["M"][c, g, :k, :k] - Mi)) / np.max(np.abs(Mi)))
        assert st["sign"][c] == ch.sign, c
        worst_w = max(worst_w, abs(st["logw"][c] - ch.logw))
    assert worst_M <= 1e-10 and worst_w <= 1e-10, (worst_M, worst_w)
    mc.close()
    net.close()
