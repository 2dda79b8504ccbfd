"""Python binding of librl0 (include/rl0.h): argument marshalling only.

Every step of the decoder runs in the HIP library.  Tensors are torch CUDA (HIP)
tensors; torch supplies device memory and the current stream and nothing else.  If the
library is not built the import fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RL0_LIBRARY names another build of the same library (e.g. one with host sanitizers)
LIB_PATH = os.environ.get("RL0_LIBRARY") or os.path.join(_HERE, "librl0.so")

RL0_TABLE_N = 4096
RL0_MAX_D = 16
RL0_TABLES_FLOATS = 2 * (RL0_TABLE_N + 1) + 2
LAWS = {"gaussian": 0, "laplace": 1}          # RL0_LAW_GAUSSIAN, RL0_LAW_LAPLACE

ERRORS = {
    -1: "RL0_EINVAL",
    -2: "RL0_EINDEX",
    -3: "RL0_ENOMEM",
    -4: "RL0_EHIP",
    -5: "RL0_ENOWEIGHTS",
    -6: "RL0_ERANGE",
    -7: "RL0_EIO",
}


class Params(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("sigma", ctypes.c_float),
        ("sigma_signal", ctypes.c_float),
        ("alpha", ctypes.c_float),
        ("c", ctypes.c_float),
        ("series_terms", ctypes.c_int32),
        ("max_iters", ctypes.c_int32),
        ("l1_test", ctypes.c_int32),
        ("posterior", ctypes.c_int32),
        ("mlp", ctypes.c_void_p),
        ("validate", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("adaptive_k", ctypes.c_int32),
        ("signal_law", ctypes.c_int32),
        ("noise_law", ctypes.c_int32),
        ("log", ctypes.c_int32),
        ("tables", ctypes.c_void_p),
        ("wg_order", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("accepted", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("updates_total", ctypes.c_int32),
        ("l1_final_fx", ctypes.c_int64),
        ("l1_final", ctypes.c_double),
        ("l1_tol", ctypes.c_double),
        ("t_final", ctypes.c_float),
        ("error_flags", ctypes.c_int32),
        ("ms_total", ctypes.c_float),
        ("fx_inexact_y", ctypes.c_int32),
        ("fx_inexact_x", ctypes.c_int32),
        ("k_post", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


# stats fields that depend only on the inputs (ms_total is a timing), and of those the
# ones a batched decode reports too (it does not count fixed-point roundings)
DETERMINISTIC_STATS = tuple(f for f, _ in Stats._fields_ if f != "ms_total")


def stats_subset(st: dict, fields=DETERMINISTIC_STATS) -> dict:
    return {f: st[f] for f in fields}


class Constants(ctypes.Structure):
    _fields_ = [
        ("n_iters", ctypes.c_int32),
        ("exact", ctypes.c_int32),
        ("c", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("range_z", ctypes.c_double),
        ("range_e", ctypes.c_double),
        ("inv_h_z", ctypes.c_float),
        ("inv_h_e", ctypes.c_float),
        ("table_z", ctypes.c_float * (RL0_TABLE_N + 1)),
        ("table_e", ctypes.c_float * (RL0_TABLE_N + 1)),
    ]


RL0_SIZE_CLASSES = 12
RL0_BATCH_MAX_M = 524288


class Problem(ctypes.Structure):
    _fields_ = [
        ("A_cols", ctypes.c_void_p),
        ("n", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("d", ctypes.c_int32),
        ("y", ctypes.c_void_p),
        ("params", Params),
        ("x_out", ctypes.c_void_p),
    ]


class BatchSchedule(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int32),
        ("per_cu", ctypes.c_int32),
        ("cols", ctypes.c_int32 * RL0_SIZE_CLASSES),
        ("group", ctypes.c_int32 * RL0_SIZE_CLASSES),
    ]

    def as_dict(self) -> dict:
        return {"block": self.block, "per_cu": self.per_cu, "cols": list(self.cols), "group": list(self.group)}

    @classmethod
    def from_dict(cls, d: dict) -> "BatchSchedule":
        s = cls()
        s.block = d["block"]
        s.per_cu = d["per_cu"]
        for i, c in enumerate(d["cols"]):
            s.cols[i] = c
        for i, g in enumerate(d.get("group", [1] * RL0_SIZE_CLASSES)):
            s.group[i] = g
        return s


class TrainCfg(ctypes.Structure):
    _fields_ = [
        ("lr", ctypes.c_float),
        ("beta1", ctypes.c_float),
        ("beta2", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("lam", ctypes.c_float),
        ("batch", ctypes.c_int32),
        ("steps", ctypes.c_int32),
        ("t0", ctypes.c_int32),
    ]


class MlpCkpt(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("P", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("step", ctypes.c_int64),
        ("cfg", TrainCfg),
    ]


class Rl0Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded librl0.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1704_09012_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, V = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        L.rl0_params_default.argtypes = [ctypes.POINTER(Params), I32, I32, I32, I32, ctypes.c_float]
        L.rl0_compute_constants.argtypes = [ctypes.POINTER(Params), I32, I32, I32, ctypes.POINTER(Constants), P, P]
        L.rl0_sketch.argtypes = [P, I32, I32, I32, P, P, V]
        L.rl0_sketch_static.argtypes = [P, I32, I32, I32, P, P, V]
        L.rl0_validate.argtypes = [P, I32, I32, I32, V]
        L.rl0_decode.argtypes = [P, I32, I32, I32, P, ctypes.POINTER(Params), P, ctypes.POINTER(Stats), V]
        L.rl0_step.argtypes = [P, I32, I32, I32, P, ctypes.POINTER(Params), I32, P, P,
                               ctypes.POINTER(I64), ctypes.POINTER(I32), P, P, P, P, V]
        L.rl0_profile_enable.argtypes = [I32]
        L.rl0_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)]
        L.rl0_profile_read_kernels.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)]
        L.rl0_profile_read_learned.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)]
        L.rl0_last_log.argtypes = [P, I32, ctypes.POINTER(I32), V]
        L.rl0_decode_batched.argtypes = [ctypes.POINTER(Problem), I32, ctypes.POINTER(Stats), V]
        L.rl0_batch_schedule_get.argtypes = [ctypes.POINTER(BatchSchedule)]
        L.rl0_batch_timeline.argtypes = [I32, P, P, P, V]
        L.rl0_batch_schedule_set.argtypes = [ctypes.POINTER(BatchSchedule)]
        L.rl0_autotune_batched.argtypes = [ctypes.POINTER(Problem), I32, I32, ctypes.POINTER(BatchSchedule),
                                           ctypes.POINTER(ctypes.c_double), V]
        L.rl0_mlp_num_params.argtypes = [I32]
        L.rl0_mlp_num_params.restype = I32
        L.rl0_mlp_pack_bf16.argtypes = [P, I32, P]
        L.rl0_validate_host.argtypes = [P, I32, I32, I32]
        L.rl0_workspace_bytes.argtypes = [I32, I32, I32, I32]
        L.rl0_workspace_bytes.restype = ctypes.c_size_t
        L.rl0_mlp_init.argtypes = [P, I32, ctypes.c_uint64, V]
        L.rl0_mlp_features.argtypes = [P, I32, I32, I32, P, ctypes.c_float, P, V]
        L.rl0_mlp_labels.argtypes = [P, P, I32, I32, ctypes.c_float, P, V]
        L.rl0_mlp_grad.argtypes = [P, P, I32, I32, P, ctypes.c_float, P, ctypes.POINTER(ctypes.c_float), V]
        L.rl0_mlp_train.argtypes = [P, P, I64, I32, P, P, P, ctypes.POINTER(TrainCfg),
                                    ctypes.POINTER(ctypes.c_float), V]
        L.rl0_mlp_forward.argtypes = [P, I32, I32, P, P, I32, V]
        L.rl0_mlp_adam.argtypes = [P, P, P, P, I32, I32, ctypes.POINTER(TrainCfg), V]
        L.rl0_mlp_save.argtypes = [ctypes.c_char_p, ctypes.POINTER(MlpCkpt), P, P, P, V]
        L.rl0_mlp_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(MlpCkpt), P, P, P, V]
        L.rl0_device_check.argtypes = [ctypes.POINTER(I32), V]
        L.rl0_last_error.restype = ctypes.c_char_p
        L.rl0_release.argtypes = []
        for name in ("rl0_params_default", "rl0_compute_constants", "rl0_sketch", "rl0_sketch_static", "rl0_validate",
                     "rl0_decode", "rl0_step", "rl0_decode_batched", "rl0_batch_schedule_get", "rl0_profile_read_learned",
                     "rl0_last_log",
                     "rl0_batch_schedule_set", "rl0_autotune_batched", "rl0_batch_timeline", "rl0_mlp_init", "rl0_mlp_features",
                     "rl0_mlp_labels", "rl0_mlp_grad", "rl0_mlp_train", "rl0_mlp_forward", "rl0_mlp_adam",
                     "rl0_mlp_save", "rl0_mlp_load", "rl0_device_check"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != 0:
        raise Rl0Error(rc, lib().rl0_last_error().decode())


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype, shape=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def pack_tables(Tz, Te, inv_h_z, inv_h_e) -> np.ndarray:
    """Score tables in the layout of rl0_params.tables (RL0_TABLES_FLOATS float32)."""
    out = np.empty(RL0_TABLES_FLOATS, np.float32)
    out[:RL0_TABLE_N + 1] = np.asarray(Tz, np.float32)
    out[RL0_TABLE_N + 1:2 * (RL0_TABLE_N + 1)] = np.asarray(Te, np.float32)
    out[-2:] = (np.float32(inv_h_z), np.float32(inv_h_e))
    return out


def _set_param(p: Params, key: str, val) -> None:
    if not hasattr(p, key):
        raise KeyError(key)
    if key == "mlp" and hasattr(val, "data_ptr"):
        # a parameter tensor: the learned decision
        val = val.data_ptr()
        p.posterior = 1
    elif key in ("signal_law", "noise_law") and isinstance(val, str):
        val = LAWS[val]
    elif key == "tables" and val is not None and not isinstance(val, int):
        arr = np.ascontiguousarray(val, dtype=np.float32)
        if arr.shape != (RL0_TABLES_FLOATS,):
            raise ValueError(f"tables must hold {RL0_TABLES_FLOATS} floats (pack_tables)")
        p._tables_keep = arr            # the library reads it during each call
        val = arr.ctypes.data
    setattr(p, key, val)


def params_default(n: int, m: int, d: int, k: int, sigma: float, **overrides) -> Params:
    p = Params()
    _check(lib().rl0_params_default(ctypes.byref(p), n, m, d, k, ctypes.c_float(sigma)))
    for key, val in overrides.items():
        _set_param(p, key, val)
    return p


@dataclass
class HostConstants:
    n_iters: int
    exact: bool
    c: float
    tol: float
    range_z: float
    range_e: float
    inv_h_z: np.float32
    inv_h_e: np.float32
    table_z: np.ndarray
    table_e: np.ndarray
    t: np.ndarray
    tau: np.ndarray


def compute_constants(p: Params, n: int, m: int, d: int) -> HostConstants:
    out = Constants()
    cap = max(200, p.max_iters + 1)
    t = np.zeros(cap, np.float32)
    tau = np.zeros(cap, np.float32)
    _check(lib().rl0_compute_constants(ctypes.byref(p), n, m, d, ctypes.byref(out),
                                       t.ctypes.data_as(ctypes.c_void_p), tau.ctypes.data_as(ctypes.c_void_p)))
    k = out.n_iters
    return HostConstants(n_iters=k, exact=bool(out.exact), c=out.c, tol=out.tol, range_z=out.range_z,
                         range_e=out.range_e, inv_h_z=np.float32(out.inv_h_z), inv_h_e=np.float32(out.inv_h_e),
                         table_z=np.ctypeslib.as_array(out.table_z).copy(),
                         table_e=np.ctypeslib.as_array(out.table_e).copy(), t=t[:k].copy(), tau=tau[:k].copy())


def validate(A_cols, m: int) -> None:
    torch = _torch()
    n, d = A_cols.shape
    _check(lib().rl0_validate(_dev_ptr(A_cols, torch.int32, name="A_cols"), n, m, d, _stream()))


def sketch(A_cols, x, m: int, out=None):
    """y = A x on the device (rl0_sketch)."""
    torch = _torch()
    n, d = A_cols.shape
    y = out if out is not None else torch.empty(m, dtype=torch.float32, device=x.device)
    _check(lib().rl0_sketch(_dev_ptr(A_cols, torch.int32, (n, d), "A_cols"), n, m, d,
                            _dev_ptr(x, torch.float32, (n,), "x"), _dev_ptr(y, torch.float32, (m,), "y"),
                            _stream()))
    return y


RL0_SKETCH_STATIC_MAX_M = 2097152


def sketch_static(A_cols, x, m: int, out=None):
    """y = A x through rl0_sketch_static (no allocation; m <= RL0_SKETCH_STATIC_MAX_M)."""
    torch = _torch()
    n, d = A_cols.shape
    y = out if out is not None else torch.empty(m, dtype=torch.float32, device=x.device)
    _check(lib().rl0_sketch_static(_dev_ptr(A_cols, torch.int32, (n, d), "A_cols"), n, m, d,
                                   _dev_ptr(x, torch.float32, (n,), "x"), _dev_ptr(y, torch.float32, (m,), "y"),
                                   _stream()))
    return y


def decode(A_cols, y, sigma: float | None = None, d: int | None = None, params: Params | None = None,
           k: int | None = None, out=None, **overrides):
    """Robust-l0 (rl0_decode).  Returns (x_hat tensor, stats dict)."""
    torch = _torch()
    n, dd = A_cols.shape
    if d is not None and d != dd:
        raise ValueError("d does not match A_cols")
    m = y.shape[0]
    if params is None:
        if sigma is None or k is None:
            raise ValueError("give params, or sigma and k")
        params = params_default(n, m, dd, k, sigma, **overrides)
    else:
        for key, val in overrides.items():
            _set_param(params, key, val)
    x = out if out is not None else torch.empty(n, dtype=torch.float32, device=y.device)
    st = Stats()
    _check(lib().rl0_decode(_dev_ptr(A_cols, torch.int32, (n, dd), "A_cols"), n, m, dd,
                            _dev_ptr(y, torch.float32, (m,), "y"), ctypes.byref(params),
                            _dev_ptr(x, torch.float32, (n,), "x_out"), ctypes.byref(st), _stream()))
    return x, st.as_dict()


def step(A_cols, y, params: Params, it: int, x_hat, r_hat, L_hat: int, debug: bool = True):
    """One loop iteration (rl0_step) in place on x_hat, r_hat.  Returns a dict."""
    torch = _torch()
    n, d = A_cols.shape
    m = y.shape[0]
    L = ctypes.c_int64(L_hat)
    acc = ctypes.c_int32(0)
    dbg = {}
    if debug:
        dbg = {
            "updated": torch.zeros(n, dtype=torch.int32, device=y.device),
            "omega": torch.zeros(n, dtype=torch.float32, device=y.device),
            "x_trial": torch.zeros(n, dtype=torch.float32, device=y.device),
            "r_trial": torch.zeros(m, dtype=torch.float32, device=y.device),
        }
    ptr = lambda key: ctypes.c_void_p(dbg[key].data_ptr()) if debug else None  # noqa: E731
    _check(lib().rl0_step(_dev_ptr(A_cols, torch.int32, (n, d), "A_cols"), n, m, d,
                          _dev_ptr(y, torch.float32, (m,), "y"), ctypes.byref(params), it,
                          _dev_ptr(x_hat, torch.float32, (n,), "x_hat"),
                          _dev_ptr(r_hat, torch.float32, (m,), "r_hat"), ctypes.byref(L), ctypes.byref(acc),
                          ptr("updated"), ptr("omega"), ptr("x_trial"), ptr("r_trial"), _stream()))
    out = {"L_hat": int(L.value), "accepted": bool(acc.value)}
    out.update(dbg)
    return out


def device_check() -> int:
    """rl0_device_check: the kernels' source line of the first failed index check since the
    last call (0: none), or -1 when the loaded library is the normal one."""
    line = ctypes.c_int32(0)
    _check(lib().rl0_device_check(ctypes.byref(line), None))   # the default stream
    return line.value


def profile_enable(enable: bool = True) -> None:
    """Time every sweep launch of rl0_decode with HIP events (resets the total)."""
    _check(lib().rl0_profile_enable(1 if enable else 0))


def profile_read() -> tuple[float, int]:
    """(total sweep milliseconds, sweep launches) since the last profile_enable."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().rl0_profile_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def profile_read_kernels() -> dict:
    """Total milliseconds per kernel since profile_enable: over every launched iteration
    ("all") and over the iterations that ran before the stopping condition ("executed")."""
    arr = (ctypes.c_double * 4)()
    cnt = (ctypes.c_int64 * 2)()
    _check(lib().rl0_profile_read_kernels(arr, cnt))
    names = ("sweep", "hk_rows")
    return {"all": {k: arr[i] for i, k in enumerate(names)}, "all_launches": cnt[0],
            "executed": {k: arr[2 + i] for i, k in enumerate(names)}, "executed_launches": cnt[1]}


ITER_LOG = np.dtype([("l1_trial_fx", np.int64), ("l1_hat_fx", np.int64), ("accepted", np.int32),
                     ("updates", np.int32), ("t", np.float32), ("it", np.int32), ("rows_start", np.uint64),
                     ("rows_end", np.uint64)])


def last_log(cap: int = 4096) -> np.ndarray:
    """rl0_last_log: the per-iteration records of the last decode on the current stream (a
    numpy structured array of dtype ITER_LOG)."""
    out = np.zeros(cap, ITER_LOG)
    count = ctypes.c_int32(0)
    _check(lib().rl0_last_log(out.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(count), _stream()))
    return out[:min(count.value, cap)]


def profile_read_learned() -> tuple[float, int]:
    """(total ms, launches) of the learned column decision timed in rl0_step since the last
    profile_enable."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(lib().rl0_profile_read_learned(ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, int(cnt.value)


def validate_host(A_cols, m: int) -> None:
    """rl0_validate_host on a host int32 [n][d] array; raises Rl0Error if malformed."""
    import numpy as np
    a = np.ascontiguousarray(A_cols, dtype=np.int32)
    n, d = a.shape
    _check(lib().rl0_validate_host(a.ctypes.data, n, m, d))


def workspace_bytes(n: int, m: int, d: int, k: int) -> int:
    """rl0_workspace_bytes: device bytes a decode of this size allocates (0: invalid)."""
    return int(lib().rl0_workspace_bytes(n, m, d, k))


def mlp_pack_bf16(w, d: int):
    """rl0_mlp_pack_bf16: the fp32 parameters (host) as bf16 bit patterns (uint16)."""
    import numpy as np
    wf = np.ascontiguousarray(w, dtype=np.float32)
    P = mlp_num_params(d)
    if wf.shape != (P,):
        raise ValueError(f"w must hold {P} values")
    out = np.empty(P, dtype=np.uint16)
    _check(lib().rl0_mlp_pack_bf16(wf.ctypes.data, d, out.ctypes.data))
    return out


def release() -> None:
    lib().rl0_release()


# ---------------------------------------------------------------- batched decoding

def _problems(problems):
    """Marshal a list of dicts {A, y, out, params} (or {A, y, out, sigma, k, **overrides})
    into an rl0_problem array; returns (array, kept tensors)."""
    torch = _torch()
    arr = (Problem * len(problems))()
    keep = []
    for i, pr in enumerate(problems):
        A, y = pr["A"], pr["y"]
        n, d = A.shape
        m = y.shape[0]
        out = pr.get("out")
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=y.device)
            pr["out"] = out
        params = pr.get("params")
        if params is None:
            extra = {k: v for k, v in pr.items() if k not in ("A", "y", "out", "params", "sigma", "k")}
            params = params_default(n, m, d, pr["k"], pr["sigma"], **extra)
        arr[i].A_cols = _dev_ptr(A, torch.int32, (n, d), f"problems[{i}].A").value
        arr[i].n, arr[i].m, arr[i].d = n, m, d
        arr[i].y = _dev_ptr(y, torch.float32, (m,), f"problems[{i}].y").value
        arr[i].params = params
        arr[i].x_out = _dev_ptr(out, torch.float32, (n,), f"problems[{i}].out").value
        keep.append((A, y, out))
    return arr, keep


class PreparedBatch:
    """A list of problem dicts marshalled once into the rl0_problem array, for repeated
    batched decodes of the same tensors (their contents may change between calls)."""

    def __init__(self, problems):
        self.problems = problems
        self.arr, self._keep = _problems(problems)
        self.stats = (Stats * max(len(problems), 1))()

    def __len__(self):
        return len(self.problems)


def decode_batched(problems, stats: bool = True):
    """rl0_decode_batched over a list of problem dicts (or a PreparedBatch of them); each
    dict's "out" (created if absent) receives x_hat.  Returns the per-instance stats
    dicts, or None with stats=False (a PreparedBatch keeps them in .stats)."""
    if isinstance(problems, PreparedBatch):
        arr, st, count = problems.arr, problems.stats, len(problems)
    else:
        arr, _keep = _problems(problems)
        count = len(problems)
        st = (Stats * max(count, 1))()
    _check(lib().rl0_decode_batched(arr, count, st, _stream()))
    return [st[i].as_dict() for i in range(count)] if stats else None


def batch_timeline(count: int):
    """(start_ms, end_ms, group) arrays of the last batched call's first `count` instances."""
    import numpy as np
    a = np.zeros(count, np.float64)
    b = np.zeros(count, np.float64)
    g = np.zeros(count, np.int32)
    _check(lib().rl0_batch_timeline(count, a.ctypes.data_as(ctypes.c_void_p), b.ctypes.data_as(ctypes.c_void_p),
                                    g.ctypes.data_as(ctypes.c_void_p), _stream()))
    return a, b, g


def batch_schedule_get() -> dict:
    s = BatchSchedule()
    _check(lib().rl0_batch_schedule_get(ctypes.byref(s)))
    return s.as_dict()


def batch_schedule_set(sched: dict) -> None:
    s = BatchSchedule.from_dict(sched)
    _check(lib().rl0_batch_schedule_set(ctypes.byref(s)))


def autotune_batched(problems, reps: int = 3) -> tuple[dict, float]:
    """rl0_autotune_batched: installs and returns (best schedule, its median ms)."""
    arr, _keep = _problems(problems)
    best = BatchSchedule()
    ms = ctypes.c_double(0.0)
    _check(lib().rl0_autotune_batched(arr, len(problems), reps, ctypes.byref(best), ctypes.byref(ms), _stream()))
    return best.as_dict(), ms.value


# ---------------------------------------------------------------- learned decision

def mlp_num_params(d: int) -> int:
    n = lib().rl0_mlp_num_params(d)
    if n < 0:
        raise ValueError("d must be in [1, 16]")
    return n


def mlp_init(d: int, seed: int, device="cuda"):
    """A new parameter vector (rl0_mlp_init)."""
    torch = _torch()
    w = torch.empty(mlp_num_params(d), dtype=torch.float32, device=device)
    _check(lib().rl0_mlp_init(_dev_ptr(w, torch.float32, None, "w"), d, seed, _stream()))
    return w


def mlp_features(A_cols, r, sigma: float, out=None):
    torch = _torch()
    n, d = A_cols.shape
    m = r.shape[0]
    f = out if out is not None else torch.empty((n, d + 1), dtype=torch.float32, device=r.device)
    _check(lib().rl0_mlp_features(_dev_ptr(A_cols, torch.int32, (n, d), "A_cols"), n, m, d,
                                  _dev_ptr(r, torch.float32, (m,), "r"), ctypes.c_float(sigma),
                                  _dev_ptr(f, torch.float32, (n, d + 1), "feats"), _stream()))
    return f


def mlp_labels(x_true, x_hat, d: int, sigma: float, out=None):
    torch = _torch()
    n = x_true.shape[0]
    lab = out if out is not None else torch.empty((n, 2), dtype=torch.float32, device=x_true.device)
    _check(lib().rl0_mlp_labels(_dev_ptr(x_true, torch.float32, (n,), "x_true"),
                                _dev_ptr(x_hat, torch.float32, (n,), "x_hat"), n, d, ctypes.c_float(sigma),
                                _dev_ptr(lab, torch.float32, (n, 2), "labels"), _stream()))
    return lab


def mlp_grad(feats, labels, w, lam: float = 1.0):
    """(gradient tensor, loss) of the mean loss at w."""
    torch = _torch()
    N, F = feats.shape
    g = torch.empty_like(w)
    loss = ctypes.c_float(0.0)
    _check(lib().rl0_mlp_grad(_dev_ptr(feats, torch.float32, (N, F), "feats"),
                              _dev_ptr(labels, torch.float32, (N, 2), "labels"), N, F - 1,
                              _dev_ptr(w, torch.float32, None, "w"), ctypes.c_float(lam),
                              _dev_ptr(g, torch.float32, None, "grad"), ctypes.byref(loss), _stream()))
    return g, loss.value


def mlp_train(feats, labels, w, m, v, steps: int, t0: int = 0, lr: float = 1e-3, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8, lam: float = 1.0, batch: int = 4096) -> float:
    """rl0_mlp_train in place on (w, m, v); returns the mean loss of the last steps."""
    torch = _torch()
    N, F = feats.shape
    cfg = TrainCfg(lr, beta1, beta2, eps, lam, batch, steps, t0)
    loss = ctypes.c_float(0.0)
    _check(lib().rl0_mlp_train(_dev_ptr(feats, torch.float32, (N, F), "feats"),
                               _dev_ptr(labels, torch.float32, (N, 2), "labels"), N, F - 1,
                               _dev_ptr(w, torch.float32, None, "w"), _dev_ptr(m, torch.float32, None, "m"),
                               _dev_ptr(v, torch.float32, None, "v"), ctypes.byref(cfg), ctypes.byref(loss),
                               _stream()))
    return loss.value


def mlp_adam(w, grad, m, v, d: int, t: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8) -> None:
    """rl0_mlp_adam: one Adam update of (w, m, v) in place with the gradient grad at step t."""
    torch = _torch()
    P = mlp_num_params(d)
    cfg = TrainCfg(lr, beta1, beta2, eps, 1.0, 1, 1, 0)
    _check(lib().rl0_mlp_adam(_dev_ptr(w, torch.float32, (P,), "w"), _dev_ptr(grad, torch.float32, (P,), "grad"),
                              _dev_ptr(m, torch.float32, (P,), "m"), _dev_ptr(v, torch.float32, (P,), "v"), d, t,
                              ctypes.byref(cfg), _stream()))


def _ckpt_dict(c: MlpCkpt) -> dict:
    cfg = {f: getattr(c.cfg, f) for f, _ in TrainCfg._fields_}
    return {"d": c.d, "dtype": c.dtype, "P": c.P, "seed": c.seed, "step": c.step, "cfg": cfg}


def mlp_save(path: str, w, m, v, d: int, step: int, seed: int = 0, lr: float = 1e-3, beta1: float = 0.9,
             beta2: float = 0.999, eps: float = 1e-8, lam: float = 1.0, batch: int = 4096) -> None:
    """rl0_mlp_save: the weights w and Adam's moments m, v (device tensors of
    mlp_num_params(d) floats) after `step` Adam steps with these hyper-parameters."""
    torch = _torch()
    P = mlp_num_params(d)
    info = MlpCkpt(d, 0, P, seed, step, TrainCfg(lr, beta1, beta2, eps, lam, batch, 0, 0))
    _check(lib().rl0_mlp_save(os.fsencode(path), ctypes.byref(info), _dev_ptr(w, torch.float32, (P,), "w"),
                              _dev_ptr(m, torch.float32, (P,), "m"), _dev_ptr(v, torch.float32, (P,), "v"),
                              _stream()))


def mlp_checkpoint_info(path: str) -> dict:
    """The header of a checkpoint after rl0_mlp_load has checked the whole file (no GPU)."""
    info = MlpCkpt()
    _check(lib().rl0_mlp_load(os.fsencode(path), ctypes.byref(info), None, None, None, None))
    return _ckpt_dict(info)


def mlp_load(path: str, device="cuda", moments: bool = True):
    """(header dict, w, m, v) of a checkpoint; m and v are None when moments is False."""
    torch = _torch()
    info = mlp_checkpoint_info(path)
    P = info["P"]
    w = torch.empty(P, dtype=torch.float32, device=device)
    m = torch.empty_like(w) if moments else None
    v = torch.empty_like(w) if moments else None
    ptr = lambda t, name: _dev_ptr(t, torch.float32, (P,), name) if t is not None else None
    again = MlpCkpt()
    _check(lib().rl0_mlp_load(os.fsencode(path), ctypes.byref(again), ptr(w, "w"), ptr(m, "m"), ptr(v, "v"),
                              _stream()))
    return _ckpt_dict(again), w, m, v


def mlp_forward(feats, w, bf16: bool = True):
    torch = _torch()
    N, F = feats.shape
    out = torch.empty((N, 2), dtype=torch.float32, device=feats.device)
    _check(lib().rl0_mlp_forward(_dev_ptr(feats, torch.float32, (N, F), "feats"), N, F - 1,
                                 _dev_ptr(w, torch.float32, None, "w"),
                                 _dev_ptr(out, torch.float32, (N, 2), "out"), 1 if bf16 else 0, _stream()))
    return out
