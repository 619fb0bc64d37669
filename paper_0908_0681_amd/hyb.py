"""Thin ctypes binding of libhyb (argument marshalling only).

Every step of the trace runs in the library's HIP kernels; this module only
converts numpy arrays / torch device tensors into pointers and sizes.  It
refuses to run when libhyb.so is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhyb.so")

HYB_OK = 0
ERRORS = {-1: "HYB_E_ARG", -2: "HYB_E_UNSORTED", -3: "HYB_E_FLAVOR", -4: "HYB_E_NOCONV",
          -5: "HYB_E_NONFINITE", -6: "HYB_E_HIP", -7: "HYB_E_OOM", -8: "HYB_E_STATE"}
HYB_CSR, HYB_MATRIX_FREE = 0, 1
HYB_FP64, HYB_MIXED = 0, 1
HYB_SPECTRUM_HOST, HYB_SPECTRUM_DEVICE = 0, 1


class HybError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class ModelParamsC(C.Structure):
    _fields_ = [("n_orb", C.c_int32), ("eps", C.POINTER(C.c_double)), ("U", C.c_double),
                ("Up", C.c_double), ("J", C.c_double), ("J_sf", C.c_double), ("J_ph", C.c_double),
                ("storage", C.c_int32), ("precision", C.c_int32), ("retain_window", C.c_double),
                ("krylov_max", C.c_int32), ("krylov_tol", C.c_double), ("spectrum", C.c_int32)]


class ModelInfoC(C.Structure):
    _fields_ = [("n_orb", C.c_int32), ("n_flavors", C.c_int32), ("n_blocks", C.c_int32),
                ("max_dim", C.c_int32), ("n_retained", C.c_int32), ("precision", C.c_int32),
                ("n_states", C.c_int64), ("nnz_offdiag", C.c_int64), ("E0", C.c_double)]


class ConfigBatchC(C.Structure):
    _fields_ = [("n_configs", C.c_int32), ("offsets", C.c_void_p), ("tau", C.c_void_p),
                ("flavor", C.c_void_p), ("dagger", C.c_void_p), ("on_device", C.c_int32)]


class TraceOutC(C.Structure):
    _fields_ = [("log_abs", C.c_void_p), ("sign", C.c_void_p), ("krylov_steps", C.c_void_p),
                ("substeps", C.c_void_p), ("feasible_paths", C.c_void_p), ("rowsteps", C.c_void_p),
                ("rows", C.c_void_p), ("on_device", C.c_int32)]


class McParamsC(C.Structure):
    _fields_ = [("n_chains", C.c_int32), ("beta", C.c_double), ("n_delta", C.c_int32),
                ("delta", C.POINTER(C.c_double)), ("kmax", C.c_int32), ("nmax_ops", C.c_int32),
                ("seed", C.c_uint64), ("n_tau", C.c_int32), ("meas_every", C.c_int32),
                ("moves_per_sweep", C.c_int32), ("rebuild_every", C.c_int32)]


class McStatsC(C.Structure):
    _fields_ = [("insert_proposed", C.c_int64), ("insert_accepted", C.c_int64),
                ("remove_proposed", C.c_int64), ("remove_accepted", C.c_int64),
                ("impossible", C.c_int64), ("zero_weight", C.c_int64), ("moves", C.c_int64),
                ("order_sum", C.c_double), ("sign_sum", C.c_double), ("max_drift", C.c_double)]


class DmftParamsC(C.Structure):
    _fields_ = [("t", C.c_double), ("mix", C.c_double), ("n_iter", C.c_int32), ("therm_sweeps", C.c_int32),
                ("meas_sweeps", C.c_int32), ("symmetrize", C.c_int32)]


# name -> (restype, argtypes)
_P = C.c_void_p
_SIGS = {
    "hyb_model_create": (C.c_int, [C.POINTER(ModelParamsC), C.POINTER(_P)]),
    "hyb_model_upload": (C.c_int, [_P, _P]),
    "hyb_build_hloc": (C.c_int, [C.POINTER(ModelParamsC), _P, C.POINTER(_P)]),
    "hyb_init_lanczos": (C.c_int, [_P, C.c_int32, C.c_double, _P, _P, _P]),
    "hyb_model_destroy": (None, [_P]),
    "hyb_model_info": (C.c_int, [_P, C.POINTER(ModelInfoC)]),
    "hyb_block_info": (C.c_int, [_P, C.c_int32, _P, _P, _P]),
    "hyb_block_eigenvalues": (C.c_int, [_P, C.c_int32, _P]),
    "hyb_basis_state": (C.c_int, [_P, C.c_int32, C.c_int32, _P]),
    "hyb_basis_index": (C.c_int, [_P, C.c_uint32, _P, _P]),
    "hyb_block_dense": (C.c_int, [_P, C.c_int32, _P]),
    "hyb_retained": (C.c_int, [_P, _P, _P, _P]),
    "hyb_apply_op": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, _P, _P, _P]),
    "hyb_apply_op_device": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, _P, _P, _P]),
    "hyb_propagate_device": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P, _P, _P, _P, _P]),
    "hyb_trace_batch": (C.c_int, [_P, C.POINTER(ConfigBatchC), C.c_double, C.POINTER(TraceOutC), _P]),
    "hyb_trace_batch_noalloc": (C.c_int, [_P, C.POINTER(ConfigBatchC), C.c_double, C.POINTER(TraceOutC), _P]),
    "hyb_set_trace_variant": (C.c_int, [_P, C.c_int32]),
    "hyb_get_trace_variant": (C.c_int, [_P, _P]),
    "hyb_trace_variant_count": (C.c_int, [_P]),
    "hyb_trace_variant_name": (C.c_int, [C.c_int32, C.c_char_p, C.c_size_t]),
    "hyb_set_chunk": (C.c_int, [_P, C.c_int32]),
    "hyb_get_chunk": (C.c_int, [_P, _P]),
    "hyb_set_timing": (C.c_int, [_P, C.c_int32]),
    "hyb_last_timing": (C.c_int, [_P, _P]),
    "hyb_block_spmm": (C.c_int, [_P, C.c_int32, C.c_int64, _P, _P, _P]),
    "hyb_matrix_build": (C.c_int, [_P, _P]),
    "hyb_matrix_info": (C.c_int, [_P, _P, _P]),
    "hyb_trace_batch_matrix": (C.c_int, [_P, C.POINTER(ConfigBatchC), C.c_double, C.POINTER(TraceOutC), _P]),
    "hyb_mc_create": (C.c_int, [_P, C.POINTER(McParamsC), C.POINTER(_P)]),
    "hyb_mc_destroy": (C.c_int, [_P]),
    "hyb_mc_set_configs": (C.c_int, [_P, _P, _P, _P, _P]),
    "hyb_mc_sweep": (C.c_int, [_P, C.c_int32, _P]),
    "hyb_mc_get_state": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "hyb_mc_get_stats": (C.c_int, [_P, C.POINTER(McStatsC), _P]),
    "hyb_mc_get_accumulators": (C.c_int, [_P, _P, _P, _P, _P]),
    "hyb_mc_measure": (C.c_int, [_P, _P, _P, _P]),
    "hyb_mc_reset_measurements": (C.c_int, [_P, _P]),
    "hyb_mc_step_count": (C.c_int, [_P, _P]),
    "hyb_mc_set_graphs": (C.c_int, [_P, C.c_int32]),
    "hyb_mc_save": (C.c_int, [_P, _P, C.POINTER(C.c_size_t), _P]),
    "hyb_mc_set_delta": (C.c_int, [_P, _P, _P]),
    "hyb_mc_sector_weights": (C.c_int, [_P, _P, _P, _P]),
    "hyb_mc_get_delta": (C.c_int, [_P, _P]),
    "hyb_mc_bethe_delta": (C.c_int, [_P, C.c_double, C.c_double, C.c_int32, _P, _P]),
    "hyb_dmft_bethe": (C.c_int, [_P, C.POINTER(DmftParamsC), _P, _P, _P]),
    "hyb_mc_load": (C.c_int, [_P, _P, C.c_size_t, _P]),
    "hyb_mc_attach_mlp": (C.c_int, [_P, _P, C.c_double]),
    "hyb_mc_harvest": (C.c_int, [_P, C.c_int64, _P, _P, _P]),
    "hyb_mlp_create": (C.c_int, [C.c_uint64, C.POINTER(_P)]),
    "hyb_mlp_destroy": (C.c_int, [_P]),
    "hyb_mlp_get_weights": (C.c_int, [_P, _P, _P]),
    "hyb_mlp_set_weights": (C.c_int, [_P, _P, _P]),
    "hyb_mlp_forward": (C.c_int, [_P, C.c_int32, _P, _P, _P]),
    "hyb_mlp_gradients": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P, _P]),
    "hyb_mlp_train_step": (C.c_int, [_P, C.c_int32, _P, _P, C.c_float, _P, _P]),
    "hyb_last_error": (C.c_char_p, []),
    "hyb_version": (C.c_char_p, []),
}

_lib = None
_VERBOSE = os.environ.get("HYB_VERBOSE", "") not in ("", "0")


def _log(msg):
    if _VERBOSE:
        print(f"[hyb] {msg}", flush=True)


def lib():
    """Loads libhyb.so (raises if it was not built).

    torch, when importable, is loaded first: its HIP runtime and rocBLAS carry the same
    sonames as the ones libhyb links, so libhyb then binds to torch's copies and the two
    share one HIP runtime (device pointers and streams pass between them, and the
    device is seen the same way by both)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_0908_0681_amd.build first")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc):
    if rc != HYB_OK:
        raise HybError(rc, lib().hyb_last_error().decode())


def _ptr(a):
    """Pointer of a numpy array or a torch tensor (host or device)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    return a.data_ptr()   # torch tensor


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:
            pass
        return None
    return stream if isinstance(stream, int) else stream.cuda_stream


@dataclass
class TraceResult:
    sign: np.ndarray
    log_abs: np.ndarray
    krylov_steps: np.ndarray
    substeps: np.ndarray
    feasible_paths: np.ndarray
    rowsteps: np.ndarray = None
    rows: np.ndarray = None


class Model:
    """Owns a hyb_model handle."""

    def __init__(self, params, precision="fp64", retain_window=1e-5, krylov_max=12,
                 krylov_tol=None, upload=True, stream=None, storage="csr", spectrum="host",
                 lanczos_block=8, lanczos_tol=1e-12):
        """spectrum="device": no host eigensolver; after the upload hyb_init_lanczos
        (block size lanczos_block, residual tolerance lanczos_tol) supplies E0 and the
        retained set (its per-block steps and residuals in self.lanczos)."""
        prec = {"fp64": HYB_FP64, "mixed": HYB_MIXED}[precision]
        store = {"csr": HYB_CSR, "matrix_free": HYB_MATRIX_FREE}[storage]
        spec = {"host": HYB_SPECTRUM_HOST, "device": HYB_SPECTRUM_DEVICE}[spectrum]
        if krylov_tol is None:
            krylov_tol = 1e-13 if prec == HYB_FP64 else 1e-7
        self._eps = np.ascontiguousarray(params.eps, dtype=np.float64)
        p = ModelParamsC(n_orb=params.n_orb, eps=self._eps.ctypes.data_as(C.POINTER(C.c_double)),
                         U=params.U, Up=params.Up, J=params.J, J_sf=params.J_sf, J_ph=params.J_ph,
                         storage=store, precision=prec, retain_window=retain_window,
                         krylov_max=krylov_max, krylov_tol=krylov_tol, spectrum=spec)
        h = C.c_void_p()
        _check(lib().hyb_model_create(C.byref(p), C.byref(h)))
        self.h = h
        self.precision = precision
        self.lanczos = None
        if upload:
            self.upload(stream)
            if spec == HYB_SPECTRUM_DEVICE:
                self.init_lanczos(lanczos_block, lanczos_tol, stream)

    def init_lanczos(self, block_size=8, tol=1e-12, stream=None):
        """hyb_init_lanczos: E0, block shifts and the retained set by band Lanczos on the
        device.  Returns (and keeps in self.lanczos) the block steps and the largest
        retained-pair residual of every block."""
        nb = self.info()["n_blocks"]
        steps = np.zeros(nb, np.int32)
        resid = np.zeros(nb)
        _check(lib().hyb_init_lanczos(self.h, block_size, tol, _ptr(steps), _ptr(resid), _stream(stream)))
        self.lanczos = {"steps": steps, "resid": resid}
        return self.lanczos

    def upload(self, stream=None):
        _check(lib().hyb_model_upload(self.h, _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            lib().hyb_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- host information / parity hooks ------------------------------------
    def info(self):
        i = ModelInfoC()
        _check(lib().hyb_model_info(self.h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in ModelInfoC._fields_}

    def block_info(self, b):
        d, n, e = C.c_int32(), C.c_int32(), C.c_double()
        _check(lib().hyb_block_info(self.h, b, C.byref(d), C.byref(n), C.byref(e)))
        return d.value, n.value, e.value

    def block_eigenvalues(self, b):
        d = self.block_info(b)[0]
        e = np.zeros(d)
        _check(lib().hyb_block_eigenvalues(self.h, b, _ptr(e)))
        return e

    def basis_state(self, b, i):
        s = C.c_uint32()
        _check(lib().hyb_basis_state(self.h, b, i, C.byref(s)))
        return s.value

    def basis_index(self, s):
        b, i = C.c_int32(), C.c_int32()
        _check(lib().hyb_basis_index(self.h, s, C.byref(b), C.byref(i)))
        return b.value, i.value

    def block_dense(self, b):
        d = self.block_info(b)[0]
        h = np.zeros((d, d))
        _check(lib().hyb_block_dense(self.h, b, _ptr(h)))
        return h

    def retained(self):
        n = self.info()["n_retained"]
        blk = np.zeros(n, np.int32)
        en = np.zeros(n)
        _check(lib().hyb_retained(self.h, _ptr(blk), _ptr(en), None))
        tot = sum(self.block_info(int(b))[0] for b in blk)
        vec = np.zeros(max(tot, 1))
        _check(lib().hyb_retained(self.h, None, None, _ptr(vec)))
        return blk, en, vec[:tot]

    def apply_op(self, f, dagger, b, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        bo = C.c_int32()
        y = np.zeros(max(self.info()["max_dim"], 1))
        _check(lib().hyb_apply_op(self.h, f, dagger, b, _ptr(x), C.byref(bo), _ptr(y)))
        if bo.value < 0:
            return -1, None
        return bo.value, y[: self.block_info(bo.value)[0]].copy()

    # ---- device calls ---------------------------------------------------------
    def apply_op_device(self, f, dagger, b, x, y, stream=None):
        """x, y: device tensors [n_vec, dim] float64."""
        bo = C.c_int32()
        _check(lib().hyb_apply_op_device(self.h, f, dagger, b, x.shape[0], _ptr(x), _ptr(y),
                                         C.byref(bo), _stream(stream)))
        return bo.value

    def propagate_device(self, b, x, dtau, y, log_scale, steps=None, stream=None):
        _log(f"propagate_device block={b} n_vec={x.shape[0]}")
        _check(lib().hyb_propagate_device(self.h, b, x.shape[0], _ptr(x), _ptr(dtau), _ptr(y),
                                          _ptr(log_scale), _ptr(steps), _stream(stream)))

    def set_variant(self, v):
        _check(lib().hyb_set_trace_variant(self.h, v))

    def variant(self):
        v = C.c_int32()
        _check(lib().hyb_get_trace_variant(self.h, C.byref(v)))
        return v.value

    def set_chunk(self, chunk):
        _check(lib().hyb_set_chunk(self.h, chunk))

    def chunk(self):
        c = C.c_int32()
        _check(lib().hyb_get_chunk(self.h, C.byref(c)))
        return c.value

    def set_timing(self, on=True):
        _check(lib().hyb_set_timing(self.h, 1 if on else 0))

    def last_timing(self):
        ms = np.zeros(7, np.float32)
        _check(lib().hyb_last_timing(self.h, _ptr(ms)))
        return ms

    def trace_batch(self, batch, beta=None, stream=None):
        """Host batch (inputs.ConfigBatch) -> TraceResult (host)."""
        beta = batch.beta if beta is None else beta
        n = batch.n_configs
        cfg = ConfigBatchC(n_configs=n, offsets=_ptr(batch.offsets), tau=_ptr(batch.tau),
                           flavor=_ptr(batch.flavor), dagger=_ptr(batch.dagger), on_device=0)
        res = TraceResult(np.zeros(n, np.int8), np.zeros(n), np.zeros(n, np.int32),
                          np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(n, np.int64),
                          np.zeros(n, np.int64))
        out = TraceOutC(log_abs=_ptr(res.log_abs), sign=_ptr(res.sign),
                        krylov_steps=_ptr(res.krylov_steps), substeps=_ptr(res.substeps),
                        feasible_paths=_ptr(res.feasible_paths), rowsteps=_ptr(res.rowsteps),
                        rows=_ptr(res.rows), on_device=0)
        _log(f"trace_batch n_configs={n} n_ops={len(batch.tau)} beta={beta} variant={self.variant()}")
        _check(lib().hyb_trace_batch(self.h, C.byref(cfg), beta, C.byref(out), _stream(stream)))
        _log("trace_batch done")
        return res

    @staticmethod
    def _device_args(dev_batch, out):
        cfg = ConfigBatchC(n_configs=dev_batch["offsets"].numel() - 1, offsets=_ptr(dev_batch["offsets"]),
                           tau=_ptr(dev_batch["tau"]), flavor=_ptr(dev_batch["flavor"]),
                           dagger=_ptr(dev_batch["dagger"]), on_device=1)
        o = TraceOutC(log_abs=_ptr(out["log_abs"]), sign=_ptr(out["sign"]),
                      krylov_steps=_ptr(out.get("krylov_steps")), substeps=_ptr(out.get("substeps")),
                      feasible_paths=_ptr(out.get("feasible_paths")), rowsteps=_ptr(out.get("rowsteps")),
                      rows=_ptr(out.get("rows")), on_device=1)
        return cfg, o

    def trace_batch_device(self, dev_batch, beta, out, stream=None):
        """dev_batch / out: dicts of torch device tensors (see bench.py)."""
        cfg, o = self._device_args(dev_batch, out)
        _check(lib().hyb_trace_batch(self.h, C.byref(cfg), beta, C.byref(o), _stream(stream)))

    def trace_batch_noalloc(self, dev_batch, beta, out, stream=None):
        """hyb_trace_batch_noalloc: as trace_batch_device, with the library's static
        device workspace instead of an allocated one."""
        cfg, o = self._device_args(dev_batch, out)
        _check(lib().hyb_trace_batch_noalloc(self.h, C.byref(cfg), beta, C.byref(o), _stream(stream)))

    def matrix_build(self, stream=None):
        """hyb_matrix_build: the eigenbasis operator blocks of the matrix formulation."""
        _check(lib().hyb_matrix_build(self.h, _stream(stream)))

    def matrix_info(self):
        nb, sec = C.c_int64(), C.c_double()
        _check(lib().hyb_matrix_info(self.h, C.byref(nb), C.byref(sec)))
        return {"op_bytes": nb.value, "build_seconds": sec.value}

    def trace_batch_matrix(self, batch, beta=None, stream=None):
        """Host batch -> TraceResult by the matrix formulation (hyb_trace_batch_matrix)."""
        beta = batch.beta if beta is None else beta
        n = batch.n_configs
        cfg = ConfigBatchC(n_configs=n, offsets=_ptr(batch.offsets), tau=_ptr(batch.tau),
                           flavor=_ptr(batch.flavor), dagger=_ptr(batch.dagger), on_device=0)
        res = TraceResult(np.zeros(n, np.int8), np.zeros(n), np.zeros(n, np.int32), np.zeros(n, np.int32),
                          np.zeros(n, np.int32), np.zeros(n, np.int64), np.zeros(n, np.int64))
        out = TraceOutC(log_abs=_ptr(res.log_abs), sign=_ptr(res.sign), krylov_steps=_ptr(res.krylov_steps),
                        substeps=_ptr(res.substeps), feasible_paths=_ptr(res.feasible_paths),
                        rowsteps=_ptr(res.rowsteps), rows=_ptr(res.rows), on_device=0)
        _check(lib().hyb_trace_batch_matrix(self.h, C.byref(cfg), beta, C.byref(out), _stream(stream)))
        return res

    def trace_batch_matrix_device(self, dev_batch, beta, out, stream=None):
        cfg, o = self._device_args(dev_batch, out)
        _check(lib().hyb_trace_batch_matrix(self.h, C.byref(cfg), beta, C.byref(o), _stream(stream)))

    def block_spmm(self, b, X, Y, n_vec, stream=None):
        _check(lib().hyb_block_spmm(self.h, b, n_vec, _ptr(X), _ptr(Y), _stream(stream)))


def variant_names():
    n = C.c_int32()
    _check(lib().hyb_trace_variant_count(C.byref(n)))
    out = []
    for i in range(n.value):
        buf = C.create_string_buffer(64)
        _check(lib().hyb_trace_variant_name(i, buf, 64))
        out.append(buf.value.decode())
    return out


def model_for_workload(w, upload=True, use_cache=True, **kw):
    """Model of a benchmark workload; applies the autotuned kernel variant if cached."""
    args = dict(precision=w.precision, retain_window=w.retain_window,
                krylov_max=min(w.krylov_max, 12),
                krylov_tol=(1e-13 if w.precision == "fp64" else 1e-7))
    args.update(kw)
    m = Model(w.params, upload=upload, **args)
    if upload and use_cache:
        try:
            import torch
            from . import autotune
            key = autotune.cache_key(autotune.gpu_arch(), w.params.n_orb, m.precision)
            entry = autotune.load_cache().get(key, {})
            name = entry.get("variant")
            if name in variant_names():
                m.set_variant(variant_names().index(name))
                _log(f"autotuned variant {name} for {key}")
            if "chunk" in entry:
                m.set_chunk(int(entry["chunk"]))
        except HybError:
            pass
    return m


class MC:
    """Monte Carlo chains on the model's device (hyb_mc_*)."""

    def __init__(self, model: Model, n_chains, beta, delta, kmax=48, nmax_ops=1024, seed=7, n_tau=200,
                 meas_every=1, moves_per_sweep=1, rebuild_every=1000):
        self.model = model
        self.delta = np.ascontiguousarray(delta, dtype=np.float64)
        self.n_chains, self.beta, self.kmax, self.n_tau = int(n_chains), float(beta), int(kmax), int(n_tau)
        self.F = model.info()["n_flavors"]
        p = McParamsC(self.n_chains, self.beta, len(self.delta) - 1,
                      self.delta.ctypes.data_as(C.POINTER(C.c_double)), self.kmax, int(nmax_ops),
                      int(seed), self.n_tau, int(meas_every), int(moves_per_sweep), int(rebuild_every))
        h = _P()
        _check(lib().hyb_mc_create(model.h, C.byref(p), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().hyb_mc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_configs(self, chains, stream=None):
        """chains: list of (cre, ann) with cre[f], ann[f] sequences of times (label order)."""
        k = np.zeros((self.n_chains, self.F), np.int32)
        cre = np.zeros((self.n_chains, self.F, self.kmax))
        ann = np.zeros((self.n_chains, self.F, self.kmax))
        for c, (cr, an) in enumerate(chains):
            for f in range(self.F):
                n = len(cr[f])
                if n != len(an[f]) or n > self.kmax:
                    raise ValueError(f"chain {c} flavor {f}: {n} creators, {len(an[f])} annihilators")
                k[c, f] = n
                cre[c, f, :n] = cr[f]
                ann[c, f, :n] = an[f]
        _check(lib().hyb_mc_set_configs(self.h, _ptr(k), _ptr(cre), _ptr(ann), _stream(stream)))

    def sweep(self, n_sweeps=1, stream=None):
        _check(lib().hyb_mc_sweep(self.h, int(n_sweeps), _stream(stream)))

    def state(self, with_M=False, stream=None):
        k = np.zeros((self.n_chains, self.F), np.int32)
        cre = np.zeros((self.n_chains, self.F, self.kmax))
        ann = np.zeros((self.n_chains, self.F, self.kmax))
        M = np.zeros((self.n_chains, self.F, self.kmax, self.kmax)) if with_M else None
        logw = np.zeros(self.n_chains)
        sign = np.zeros(self.n_chains, np.int8)
        _check(lib().hyb_mc_get_state(self.h, _ptr(k), _ptr(cre), _ptr(ann), _ptr(M) if with_M else None,
                                      _ptr(logw), _ptr(sign), _stream(stream)))
        return dict(k=k, cre=cre, ann=ann, M=M, logw=logw, sign=sign)

    def stats(self, stream=None):
        st = McStatsC()
        _check(lib().hyb_mc_get_stats(self.h, C.byref(st), _stream(stream)))
        return {name: getattr(st, name) for name, _ in McStatsC._fields_}

    def accumulators(self, stream=None):
        g = np.zeros((self.n_chains, self.F, self.n_tau))
        ms = np.zeros(self.n_chains)
        nm = np.zeros(self.n_chains, np.int64)
        _check(lib().hyb_mc_get_accumulators(self.h, _ptr(g), _ptr(ms), _ptr(nm), _stream(stream)))
        return g, ms, nm

    def measure(self, stream=None):
        G = np.zeros((self.F, self.n_tau))
        sa = C.c_double()
        _check(lib().hyb_mc_measure(self.h, _ptr(G), C.byref(sa), _stream(stream)))
        return G, sa.value

    def reset_measurements(self, stream=None):
        _check(lib().hyb_mc_reset_measurements(self.h, _stream(stream)))

    def step_count(self):
        s = C.c_int64()
        _check(lib().hyb_mc_step_count(self.h, C.byref(s)))
        return s.value

    def save(self, stream=None) -> bytes:
        """Checkpoint of every chain (hyb_mc_save) as bytes."""
        n = C.c_size_t()
        _check(lib().hyb_mc_save(self.h, None, C.byref(n), _stream(stream)))
        buf = C.create_string_buffer(n.value)
        _check(lib().hyb_mc_save(self.h, buf, C.byref(n), _stream(stream)))
        return buf.raw[: n.value]

    def load(self, blob: bytes, stream=None):
        """Restores a checkpoint written by save() (hyb_mc_load)."""
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().hyb_mc_load(self.h, buf, len(blob), _stream(stream)))

    def sector_weights(self, stream=None):
        """(weights [n_blocks], per-chain accumulators [n_chains][n_blocks]) of the
        (n_up, n_dn) sectors at beta/2."""
        nb = self.model.info()["n_blocks"]
        w = np.zeros(nb)
        acc = np.zeros((self.n_chains, nb))
        _check(lib().hyb_mc_sector_weights(self.h, _ptr(w), _ptr(acc), _stream(stream)))
        return w, acc

    def set_delta(self, delta, stream=None):
        """Replaces the Delta table (same grid); M, log|det| and signs rebuilt per chain."""
        d = np.ascontiguousarray(delta, dtype=np.float64)
        if d.shape != self.delta.shape:
            raise ValueError(f"Delta table of {d.shape}, the chains use {self.delta.shape}")
        _check(lib().hyb_mc_set_delta(self.h, _ptr(d), _stream(stream)))
        self.delta = d

    def get_delta(self):
        d = np.zeros_like(self.delta)
        _check(lib().hyb_mc_get_delta(self.h, _ptr(d)))
        return d

    def bethe_delta(self, t=1.0, mix=1.0, symmetrize=True, stream=None):
        """Delta_new = (1 - mix) Delta + mix t^2 G from the current measurements."""
        d = np.zeros_like(self.delta)
        _check(lib().hyb_mc_bethe_delta(self.h, float(t), float(mix), 1 if symmetrize else 0, _ptr(d),
                                        _stream(stream)))
        return d

    def dmft_bethe(self, n_iter, therm_sweeps, meas_sweeps, t=1.0, mix=1.0, symmetrize=True, stream=None):
        """hyb_dmft_bethe: returns (G(beta/2) per iteration, <sign> per iteration)."""
        p = DmftParamsC(float(t), float(mix), int(n_iter), int(therm_sweeps), int(meas_sweeps),
                        1 if symmetrize else 0)
        gh, sa = np.zeros(n_iter), np.zeros(n_iter)
        _check(lib().hyb_dmft_bethe(self.h, C.byref(p), _ptr(gh), _ptr(sa), _stream(stream)))
        self.delta = self.get_delta()
        return gh, sa

    def set_graphs(self, enable=True):
        """Replay each sweep from a captured HIP graph (same chains bit for bit)."""
        _check(lib().hyb_mc_set_graphs(self.h, 1 if enable else 0))

    def attach_mlp(self, mlp, eps=0.1):
        """Learned insertion proposal (mlp: MLP or None for uniform)."""
        self._mlp = mlp
        _check(lib().hyb_mc_attach_mlp(self.h, mlp.h if mlp is not None else None, float(eps)))

    def harvest(self, index, X, T, stream=None):
        """One training sample per chain into device tensors X [n_chains][352] (bf16)
        and T [n_chains][2] (int32)."""
        _check(lib().hyb_mc_harvest(self.h, int(index), _ptr(X), _ptr(T), _stream(stream)))


MLP_IN, MLP_H, MLP_OUT, MLP_BINS = 352, 128, 128, 64
MLP_W_SHAPES = [(MLP_H, MLP_IN), (MLP_H, MLP_H), (MLP_OUT, MLP_H)]
MLP_B_SHAPES = [(MLP_H,), (MLP_H,), (MLP_OUT,)]


class MLP:
    """The learned proposal network (hyb_mlp_*); weights as lists of numpy arrays."""

    def __init__(self, seed=1):
        h = _P()
        _check(lib().hyb_mlp_create(int(seed), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().hyb_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _split(flat, shapes):
        out, o = [], 0
        for sh in shapes:
            n = int(np.prod(sh))
            out.append(flat[o:o + n].reshape(sh).copy())
            o += n
        return out

    def weights(self):
        w = np.zeros(sum(int(np.prod(s)) for s in MLP_W_SHAPES), np.float32)
        b = np.zeros(sum(int(np.prod(s)) for s in MLP_B_SHAPES), np.float32)
        _check(lib().hyb_mlp_get_weights(self.h, _ptr(w), _ptr(b)))
        return self._split(w, MLP_W_SHAPES), self._split(b, MLP_B_SHAPES)

    def set_weights(self, Ws, bs):
        w = np.ascontiguousarray(np.concatenate([np.asarray(x, np.float32).ravel() for x in Ws]))
        b = np.ascontiguousarray(np.concatenate([np.asarray(x, np.float32).ravel() for x in bs]))
        _check(lib().hyb_mlp_set_weights(self.h, _ptr(w), _ptr(b)))

    def forward(self, X, logits, stream=None):
        _check(lib().hyb_mlp_forward(self.h, int(X.shape[0]), _ptr(X), _ptr(logits), _stream(stream)))

    def gradients(self, X, T, stream=None):
        w = np.zeros(sum(int(np.prod(s)) for s in MLP_W_SHAPES), np.float32)
        b = np.zeros(sum(int(np.prod(s)) for s in MLP_B_SHAPES), np.float32)
        loss = C.c_float()
        _check(lib().hyb_mlp_gradients(self.h, int(X.shape[0]), _ptr(X), _ptr(T), _ptr(w), _ptr(b),
                                       C.byref(loss), _stream(stream)))
        return self._split(w, MLP_W_SHAPES), self._split(b, MLP_B_SHAPES), loss.value

    def train_step(self, X, T, lr, want_loss=False, stream=None):
        loss = C.c_float()
        _check(lib().hyb_mlp_train_step(self.h, int(X.shape[0]), _ptr(X), _ptr(T), float(lr),
                                        C.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None

