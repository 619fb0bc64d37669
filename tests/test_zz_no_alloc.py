"""hyb_trace_batch_noalloc (the entry point for callers that cannot allocate)
against hyb_trace_batch, through the C ABI.

Both run the same kernels on the same configurations, so the results must agree
bitwise: signs, logs, Lanczos step counts, substeps and feasible-path counts.
Two calls in a row share the library's static workspace, the second with a
smaller batch; the second result must not carry anything over from the first.
The 5-orbital results are also held to the oracle's bar on a sample.  A batch
beyond the static workspace and host buffers are refused with HYB_E_ARG.
"""
import math
import sys

import numpy as np
import pytest

from paper_0908_0681_amd import inputs as I
from paper_0908_0681_amd import hyb
from oracle import trace as T

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def announce(request):
    print(f"\n[gpu-test] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def _device_batch(batch):
    return {"offsets": torch.tensor(batch.offsets, device="cuda"), "tau": torch.tensor(batch.tau, device="cuda"),
            "flavor": torch.tensor(batch.flavor, device="cuda"), "dagger": torch.tensor(batch.dagger, device="cuda")}


def _device_out(n, fill):
    return {"log_abs": torch.full((n,), fill, dtype=torch.float64, device="cuda"),
            "sign": torch.full((n,), 7, dtype=torch.int8, device="cuda"),
            "krylov_steps": torch.full((n,), -7, dtype=torch.int32, device="cuda"),
            "substeps": torch.full((n,), -7, dtype=torch.int32, device="cuda"),
            "feasible_paths": torch.full((n,), -7, dtype=torch.int32, device="cuda"),
            "rowsteps": torch.full((n,), -7, dtype=torch.int64, device="cuda"),
            "rows": torch.full((n,), -7, dtype=torch.int64, device="cuda")}


def _host(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("k,sizes", [(1, (512, 96)), (2, (48, 20))])
def test_noalloc_matches_trace_batch(k, sizes):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = I.workload(k)
    m = hyb.model_for_workload(w)
    full = w.batch()
    for call, n in enumerate(sizes):
        # the second call takes other configurations than the first, so a stale
        # result left in the shared workspace cannot match by accident
        b = full.subset(np.arange(n) + call * 7)
        db = _device_batch(b)
        ref, got = _device_out(n, -1.0), _device_out(n, 123.0)
        m.trace_batch_device(db, b.beta, ref)
        m.trace_batch_noalloc(db, b.beta, got)
        torch.cuda.synchronize()
        r, g = _host(ref), _host(got)
        for key in r:
            assert np.array_equal(r[key], g[key]), (call, key)
        assert np.all(np.isin(g["sign"], (-1, 0, 1))) and np.all(g["feasible_paths"] >= 0)
        print(f"workload {k}, call {call}: {n} configurations, bitwise equal to hyb_trace_batch")
        if k == 1:
            o = T.build(w.params, w.retain_window)
            idx = np.arange(0, n, max(1, n // 16))
            ref_o = o.trace_batch(b, configs=idx)
            for j, c in enumerate(idx):
                assert int(g["sign"][c]) == int(ref_o.sign[j])
                if ref_o.sign[j] != 0:
                    assert abs(math.expm1(float(g["log_abs"][c]) - float(ref_o.log_abs[j]))) <= 1e-10


def test_noalloc_refuses_what_it_cannot_hold():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = I.workload(2)
    m = hyb.model_for_workload(w)
    b = w.batch()          # 1024 seven-orbital configurations: beyond the static workspace
    db = _device_batch(b)
    out = _device_out(b.n_configs, 0.0)
    with pytest.raises(hyb.HybError) as e:
        m.trace_batch_noalloc(db, b.beta, out)
    assert e.value.code == -1 and "scratch" in str(e.value)
    # host buffers are refused as well
    small = b.subset(np.arange(4))
    cfg = hyb.ConfigBatchC(n_configs=4, offsets=small.offsets.ctypes.data, tau=small.tau.ctypes.data,
                           flavor=small.flavor.ctypes.data, dagger=small.dagger.ctypes.data, on_device=0)
    res = _device_out(4, 0.0)
    o = hyb.TraceOutC(log_abs=res["log_abs"].data_ptr(), sign=res["sign"].data_ptr(), on_device=1)
    import ctypes
    rc = hyb.lib().hyb_trace_batch_noalloc(m.h, ctypes.byref(cfg), b.beta, ctypes.byref(o), None)
    assert rc == -1
    # the entry point still works after the refusals
    sb = _device_batch(small)
    r1, r2 = _device_out(4, 0.0), _device_out(4, 1.0)
    m.trace_batch_device(sb, b.beta, r1)
    m.trace_batch_noalloc(sb, b.beta, r2)
    torch.cuda.synchronize()
    assert torch.equal(r1["log_abs"], r2["log_abs"]) and torch.equal(r1["sign"], r2["sign"])
