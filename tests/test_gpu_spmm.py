"""GPU parity of the block SpMM Y = (H_b - c_b) X on interleaved 16-vector panels
(the SpMV of the Krylov step, applied to many vectors) against the oracle's own
Eq.(4) block and its lowest eigenvalue, in FP64.  FP32 inputs and outputs with a
short FP32 sum per row (<= ~10 terms): relative error bar 2e-6 in the Frobenius
norm of each panel set."""
import sys

import numpy as np
import pytest

from paper_0908_0681_amd import inputs as I
from paper_0908_0681_amd import hyb
from oracle import fock as Fk
from oracle import hamiltonian as Hm

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def announce(request):
    print(f"\n[gpu-test] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def _oracle_block(params, n_up, n_dn):
    H = Hm.kanamori_full(params)
    states = Fk.blocks(params.n_orb)[Fk.block_key(params.n_orb, n_up, n_dn)]
    Hb = H[states][:, states].toarray()
    return Hb - np.linalg.eigvalsh(Hb).min() * np.eye(len(states))


def _panels(X):          # [n_vec][dim] -> [n_vec/16][dim][16]
    n, d = X.shape
    return np.ascontiguousarray(X.reshape(n // 16, 16, d).transpose(0, 2, 1))


@pytest.mark.parametrize("k,n_up,n_dn,n_vec", [(1, 2, 3, 48), (1, 0, 1, 16), (2, 3, 4, 64), (2, 1, 0, 32)])
def test_block_spmm_matches_oracle(k, n_up, n_dn, n_vec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = I.workload(k)
    m = hyb.model_for_workload(w)
    b = Fk.block_key(w.params.n_orb, n_up, n_dn)
    A = _oracle_block(w.params, n_up, n_dn)
    d = A.shape[0]
    rng = np.random.default_rng(21 + b)
    X = rng.standard_normal((n_vec, d)).astype(np.float32)
    Xd = torch.tensor(_panels(X), device="cuda")
    Yd = torch.full_like(Xd, float("nan"))
    m.block_spmm(b, Xd, Yd, n_vec)
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy().transpose(0, 2, 1).reshape(n_vec, d)
    ref = X.astype(np.float64) @ A.T
    err = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
    print(f"block ({n_up},{n_dn}) dim {d}: relative error {err:.2e}")
    assert err <= 2e-6


def test_block_spmm_full_size_sampled():
    """The benchmark's pass: the 7-orbital (3,4) block on N_v = 262144 vectors.  Three
    panels (first, a seeded middle one, last) are checked against the oracle's block,
    and every panel through linearity: the sum of all output panels against the block
    applied to the sum of all input panels (both sums in FP64)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = I.workload(2)
    m = hyb.model_for_workload(w)
    b = Fk.block_key(w.params.n_orb, 3, 4)
    A = _oracle_block(w.params, 3, 4)
    d, n_vec = A.shape[0], 262144
    gen = torch.Generator(device="cuda").manual_seed(2024)
    Xd = torch.randn(n_vec // 16, d, 16, device="cuda", dtype=torch.float32, generator=gen)
    Yd = torch.full_like(Xd, float("nan"))
    m.block_spmm(b, Xd, Yd, n_vec)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(Yd).all())
    mid = int(np.random.default_rng(5).integers(1, n_vec // 16 - 1))
    for p in (0, mid, n_vec // 16 - 1):
        X = Xd[p].double().cpu().numpy()
        Y = Yd[p].cpu().numpy()
        ref = A @ X
        err = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
        print(f"panel {p}: relative error {err:.2e}")
        assert err <= 2e-6, p
    xs = Xd.sum(dim=0, dtype=torch.float64).cpu().numpy()
    ys = Yd.sum(dim=0, dtype=torch.float64).cpu().numpy()
    ref = A @ xs
    err = np.linalg.norm(ys - ref) / np.linalg.norm(ref)
    print(f"sum of all {n_vec // 16} panels: relative error {err:.2e}")
    assert err <= 2e-6


def test_block_spmm_rejects_bad_sizes():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = I.workload(1)
    m = hyb.model_for_workload(w)
    X = torch.zeros(16 * 100, device="cuda")
    with pytest.raises(hyb.HybError):
        m.block_spmm(14, X, X, 15)
    with pytest.raises(hyb.HybError):
        m.block_spmm(99, X, X, 16)
