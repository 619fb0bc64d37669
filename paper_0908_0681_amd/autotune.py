"""Kernel-variant autotuner for the trace path.

For a workload, times every compiled trace-kernel variant that fits the model
(precision, largest block, Lanczos register depth) on the real batch and
records the fastest in a JSON cache keyed by (gpu arch, n_orb, precision).
hyb.model_for_workload applies the cached choice; without a cache the
library's own heuristic is used.

Usage (on a GPU): python -m paper_0908_0681_amd.autotune [--workloads 1 2] [--comparator 2 3 4 6 7] [--reps 3]
(--comparator tunes the FP64 models of the Krylov-against-matrix comparison at the
given orbital counts.)
"""
from __future__ import annotations

import argparse
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "autotune_cache.json")


def cache_key(arch: str, n_orb: int, precision: str) -> str:
    return f"{arch}/n{n_orb}/{precision}"


def load_cache() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def gpu_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def tune(w, reps: int = 3, n_configs: int | None = None) -> dict:
    """Times every fitting variant with the whole path in one launch, then the launch
    schedules of the fastest, on workload w (an inputs.Workload)."""
    import torch
    from . import hyb
    model = hyb.model_for_workload(w, use_cache=False)
    batch = w.batch(n_configs)
    dev = {key: torch.tensor(getattr(batch, key), device="cuda") for key in ("offsets", "tau", "flavor", "dagger")}
    out = {"log_abs": torch.empty(batch.n_configs, dtype=torch.float64, device="cuda"),
           "sign": torch.empty(batch.n_configs, dtype=torch.int8, device="cuda")}
    results = {}
    model.set_chunk(0)  # variants are ranked under the schedule they will run with
    for v, name in enumerate(hyb.variant_names()):
        try:
            model.set_variant(v)
        except hyb.HybError:
            continue
        model.trace_batch_device(dev, batch.beta, out)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            model.trace_batch_device(dev, batch.beta, out)
        torch.cuda.synchronize()
        results[name] = (time.perf_counter() - t0) / reps * 1e3
    best = min(results, key=results.get)
    # launch schedule of the best variant: operators per path-kernel launch
    model.set_variant(hyb.variant_names().index(best))
    chunks = {}
    for chunk in (1, 8, 32, 0):
        model.set_chunk(chunk)
        model.trace_batch_device(dev, batch.beta, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            model.trace_batch_device(dev, batch.beta, out)
        torch.cuda.synchronize()
        chunks[chunk] = (time.perf_counter() - t0) / reps * 1e3
    best_chunk = min(chunks, key=chunks.get)
    return {"workload": w.name, "best": best, "ms": results, "chunk": best_chunk, "chunk_ms": chunks}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", type=int, nargs="*", default=[1, 2])
    ap.add_argument("--comparator", type=int, nargs="*", default=[])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=CACHE)
    a = ap.parse_args()
    from . import inputs as I
    cache = load_cache()
    arch = gpu_arch()
    for w in [I.workload(k) for k in a.workloads] + [I.comparator_workload(n) for n in a.comparator]:
        r = tune(w, a.reps)
        cache[cache_key(arch, w.params.n_orb, w.precision)] = {
            "variant": r["best"], "ms": r["ms"], "chunk": r["chunk"], "chunk_ms": r["chunk_ms"]}
        print(json.dumps(r), flush=True)
    with open(a.out, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
