"""GPU parity of the block SpMM Y = (H_b - c_b) X on interleaved 16-vector panels
(the SpMV of the Krylov step, applied to many vectors) against the oracle's own
Eq.(4) block and its lowest eigenvalue, in FP64.  FP32 inputs and outputs with a
short FP32 sum per row (at most 13 terms, FP32 matrix values): every element must
satisfy |y - y_ref| <= 16 u32 (|A| |x|) (u32 = 2^-24; the rounding bound of such a
sum, with the rounding of A's values to FP32 included), and the largest element
error must stay below 2e-6 of the largest |y_ref|."""
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


U32 = 2.0 ** -24


def _check(Y, ref, bound, what):
    """Element-wise check of Y against ref (all float64 arrays of one shape)."""
    over = np.abs(Y - ref) - 16 * U32 * bound
    rel = float(np.max(np.abs(Y - ref)) / np.max(np.abs(ref)))
    print(f"{what}: max element error {rel:.2e} of max |y|, worst against the bound {float(np.max(over)):.2e}")
    assert np.all(over <= 1e-30), what
    assert rel <= 2e-6, what


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
    _check(Y.astype(np.float64), ref, np.abs(X.astype(np.float64)) @ np.abs(A).T, f"block ({n_up},{n_dn}) dim {d}")


def test_block_spmm_full_size_every_element():
    """The benchmark's pass: the 7-orbital (3,4) block on N_v = 262144 vectors.  Every
    output element is checked against the oracle's block applied in FP64 (a plain
    FP64 matrix product on the device, 1024 panels at a time)."""
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
    Ad = torch.tensor(A, device="cuda", dtype=torch.float64)
    Aa = Ad.abs()
    worst_rel, worst_over, ymax = 0.0, -1.0, 0.0
    step = 1024
    for p0 in range(0, n_vec // 16, step):
        # panels [p][d][16] -> columns [d][p * 16]
        X = Xd[p0:p0 + step].double().permute(1, 0, 2).reshape(d, -1).contiguous()
        Y = Yd[p0:p0 + step].double().permute(1, 0, 2).reshape(d, -1)
        ref = Ad @ X
        bound = Aa @ X.abs()
        diff = (Y - ref).abs()
        worst_over = max(worst_over, float((diff - 16 * U32 * bound).max()))
        worst_rel = max(worst_rel, float(diff.max()))
        ymax = max(ymax, float(ref.abs().max()))
    print(f"all {n_vec} vectors: max element error {worst_rel / ymax:.2e} of max |y|, "
          f"worst against the bound {worst_over:.2e}")
    assert worst_over <= 1e-30
    assert worst_rel <= 2e-6 * ymax


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
