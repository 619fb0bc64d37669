"""The oracle over a pool of worker processes (test infrastructure only).

Each worker is a fresh interpreter (spawn) with one BLAS thread; it builds its
own copy of the oracle once and then evaluates the share of the work it is
handed.  The arithmetic is exactly that of `oracle.trace` and `oracle.mc`: the
pool only splits independent configurations (or independent Markov chains)
over processes and puts the results back in input order.

Worker count: min(16, os.cpu_count()) unless given.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import numpy as np

_BLAS_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS",
              "NUMEXPR_NUM_THREADS")

_W = {}   # per-worker state: the oracle and its inputs


def default_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _spawn_pool(workers, initializer, initargs):
    saved = {k: os.environ.get(k) for k in _BLAS_VARS}
    for k in _BLAS_VARS:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")
        return ctx.Pool(workers, initializer=initializer, initargs=initargs)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


# ---------------------------------------------------------------------------
# traces
# ---------------------------------------------------------------------------

def _trace_init(params, window, zero_tol, batch, method):
    from . import trace as T
    _W["oracle"] = T.build(params, window, zero_tol=zero_tol, method=method)
    _W["batch"] = batch


def _trace_chunk(idx):
    t0 = time.perf_counter()
    r = _W["oracle"].trace_batch(_W["batch"], configs=idx)
    return idx, r, time.perf_counter() - t0


def trace_batch(params, window, batch, configs=None, zero_tol=1e-10, workers=None, chunk=1, method="auto"):
    """oracle.trace.build(params, window, zero_tol, method).trace_batch(batch, configs),
    evaluated by a process pool.  Returns (TraceResult, info) where info holds the
    worker count and the seconds spent in trace evaluation (model setup excluded)."""
    from .trace import TraceResult
    idx = list(range(batch.n_configs) if configs is None else configs)
    workers = workers or default_workers()
    workers = max(1, min(workers, len(idx)))
    chunks = [idx[i:i + chunk] for i in range(0, len(idx), chunk)]
    with _spawn_pool(workers, _trace_init, (params, window, zero_tol, batch, method)) as pool:
        # the first round of tasks is timed from the moment every worker holds its oracle
        pool.map(_noop, range(workers), chunksize=1)
        t0 = time.perf_counter()
        parts = pool.map(_trace_chunk, chunks, chunksize=1)
        wall = time.perf_counter() - t0
    pos = {c: j for j, c in enumerate(idx)}
    nR = parts[0][1].contrib_sign.shape[1] if parts else 0
    out = TraceResult(np.zeros(len(idx), np.int8), np.full(len(idx), -np.inf), np.zeros((len(idx), nR), np.int8),
                      np.full((len(idx), nR), -np.inf), np.zeros((len(idx), nR), bool))
    busy = 0.0
    for cidx, r, sec in parts:
        busy += sec
        for j, c in enumerate(cidx):
            k = pos[c]
            out.sign[k], out.log_abs[k] = r.sign[j], r.log_abs[j]
            out.contrib_sign[k], out.contrib_log[k], out.feasible[k] = r.contrib_sign[j], r.contrib_log[j], r.feasible[j]
    return out, {"workers": workers, "wall_s": wall, "busy_s": busy}


def _noop(_):
    return None


# ---------------------------------------------------------------------------
# Markov chains
# ---------------------------------------------------------------------------

def _chain_init(params, window, table, beta, kmax):
    from . import trace as T
    _W["oracle"] = T.build(params, window)
    _W["table"], _W["beta"], _W["kmax"] = table, beta, kmax


def _chain_run(task):
    """Replays one chain: (chain id, initial cre, ann, seed, moves, n_tau, meas_every)."""
    from . import mc as MC
    c, cre, ann, seed, n_moves, n_tau, meas_every = task
    F = len(cre)
    try:
        ch = MC.Chain(_W["oracle"], _W["table"], _W["beta"], cre, ann, _W["kmax"])
    except ValueError:
        ch = MC.Chain(_W["oracle"], _W["table"], _W["beta"], [[]] * F, [[]] * F, _W["kmax"])
    start = ([list(x) for x in ch.cre], [list(x) for x in ch.ann], ch.sign, ch.logw)
    acc = np.zeros((F, n_tau))
    sec = np.zeros(len(_W["oracle"].spec.states))
    accepted, margins = 0, []
    for step in range(n_moves):
        kind, a = ch.step(MC.move_uniforms(seed, c, step))
        accepted += int(a)
        if kind:
            margins.append(ch.last_margin)
        if (step + 1) % meas_every == 0:
            ch.measure(acc)
            ch.measure_sectors(sec)
    return dict(chain=c, start=start, cre=ch.cre, ann=ch.ann, sign=ch.sign, logw=ch.logw, acc=acc, sec=sec,
                accepted=accepted, min_margin=min(margins) if margins else np.inf)


def replay_chains(params, window, table, beta, kmax, starts, seed, n_moves, n_tau, meas_every, workers=None,
                  chain_ids=None):
    """oracle.mc.Chain replays of len(starts) chains (chain c starts from starts[c] =
    (cre, ann), or empty when that configuration has zero weight) for n_moves moves
    with the uniforms of chain c, measuring after every meas_every-th move.  With
    chain_ids, starts[j] is the start of chain chain_ids[j] (a sample of the chains)."""
    workers = max(1, min(workers or default_workers(), len(starts)))
    ids = list(range(len(starts))) if chain_ids is None else [int(c) for c in chain_ids]
    tasks = [(c, cre, ann, seed, n_moves, n_tau, meas_every) for c, (cre, ann) in zip(ids, starts)]
    with _spawn_pool(workers, _chain_init, (params, window, table, beta, kmax)) as pool:
        return pool.map(_chain_run, tasks, chunksize=1)
