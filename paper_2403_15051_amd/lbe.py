"""Thin Python binding of liblbe (include/lbe.h): argument marshalling only.

Every step of the solver runs in the HIP kernels of ``csrc/``; PyTorch provides the device
workspace (a uint8 tensor) and the stream.  There is no CPU fallback: if the shared library
is missing, importing or constructing a solver raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBE_LIB selects another build of the library (the host-sanitized one of build.py --sanitize)
LIB_PATH = os.environ.get("LBE_LIB") or os.path.join(_HERE, "liblbe.so")

LBE_OK, LBE_EINVAL, LBE_ENOMEM, LBE_EDEVICE, LBE_ENOTCONV, LBE_ENAN, LBE_ESTATE = 0, -1, -2, -3, -4, -5, -6
CYL, SPH, PLANAR = 0, 1, 2
FIELDS = ("n", "u_r", "u_t1", "u_t2", "T", "q_r", "P_rt1", "nbar", "chi")
MF_FIELDS = ("Phi", "F")  # mean-field potential and radial force (lbe_moments with 11 fields)
WARM_FIELDS = ("n", "u_t1", "T", "q_r", "P_rt1")
GEMM_BF16, GEMM_FP32 = 0, 1
FP64, FP32_STORE = 0, 1
INFO_KEYS = ("nr", "nv", "n0", "n1", "n2", "chi0", "C", "L", "sigma", "rcl", "rcr", "dr", "dt", "steps", "N0", "N1",
             "N2", "fp32_now", "promoted_at")


class LbeError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        super().__init__(f"liblbe status {status}: {msg}")


class Params(ctypes.Structure):
    """Mirror of ``lbe_params`` (include/lbe.h)."""

    _fields_ = [
        ("geometry", ctypes.c_int32),
        ("r_inner", ctypes.c_double),
        ("r_outer", ctypes.c_double),
        ("u_wall_inner", ctypes.c_double),
        ("t_wall_inner", ctypes.c_double),
        ("t_wall_outer", ctypes.c_double),
        ("eta0", ctypes.c_double),
        ("kn", ctypes.c_double),
        ("nr", ctypes.c_int32),
        ("q_radial", ctypes.c_int32),
        ("q_t1", ctypes.c_int32),
        ("q_t2", ctypes.c_int32),
        ("n_expand", ctypes.c_int32 * 3),
        ("cfl", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("reduced", ctypes.c_int32),
        ("phi_a", ctypes.c_double),
    ]


PARAM_KEYS = ("geometry", "r_inner", "r_outer", "u_wall_inner", "t_wall_inner", "t_wall_outer", "eta0", "kn", "nr",
              "q_radial", "q_t1", "q_t2", "cfl")


def make_params(d: dict) -> Params:
    p = Params()
    for k in PARAM_KEYS:
        setattr(p, k, d[k])
    p.precision = int(d.get("precision", FP64))
    p.reduced = int(d.get("reduced", 0))
    p.phi_a = float(d.get("phi_a", 0.0))
    ne = d.get("n_expand", (0, 0, 0))
    for a in range(3):
        p.n_expand[a] = int(ne[a])
    return p


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    P = ctypes.POINTER(Params)
    lib.lbe_query.argtypes = [P, i32, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.lbe_init.argtypes = [P, i32, vp, sz, vp, ctypes.POINTER(vp)]
    lib.lbe_init_static.argtypes = [P, i32, vp, ctypes.POINTER(vp)]
    lib.lbe_step.argtypes = [vp, i64]
    lib.lbe_sync.argtypes = [vp]
    lib.lbe_moments.argtypes = [vp, i32, _D, i64]
    lib.lbe_run_to_steady.argtypes = [vp, ctypes.c_double, i64, i32, _I64, _D]
    lib.lbe_get_state.argtypes = [vp, i32, _D, i64]
    lib.lbe_set_state.argtypes = [vp, i32, _D, i64]
    lib.lbe_rhs.argtypes = [vp, i32, _D, i64]
    lib.lbe_checkpoint_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.lbe_checkpoint_save.argtypes = [vp, vp, sz]
    lib.lbe_checkpoint_load.argtypes = [vp, vp, sz]
    lib.lbe_info.argtypes = [vp, i32, _D, i64]
    lib.lbe_tables.argtypes = [P, i32, _D, _D, i64, _I64]
    lib.lbe_timing.argtypes = [vp, i32, _D, i64]
    lib.lbe_autotune.argtypes = [vp, i32, _D, i64, ctypes.POINTER(i32)]
    F = ctypes.POINTER(ctypes.c_float)
    u64 = ctypes.c_uint64
    lib.lbe_features.argtypes = [vp, vp, i64, _I64]
    lib.lbe_targets.argtypes = [vp, vp, i64]
    lib.lbe_set_init_moments.argtypes = [vp, i32, _D, i64]
    lib.lbe_warm_start.argtypes = [vp, vp, i32, ctypes.POINTER(i32), _D]
    lib.lbe_mlp_query.argtypes = [i32, ctypes.POINTER(sz), _I64]
    lib.lbe_mlp_init.argtypes = [i32, i32, vp, sz, vp, ctypes.POINTER(vp)]
    lib.lbe_mlp_init_params.argtypes = [vp, u64]
    lib.lbe_mlp_set_params.argtypes = [vp, F, i64]
    lib.lbe_mlp_get_params.argtypes = [vp, F, i64]
    lib.lbe_mlp_set_scaling.argtypes = [vp, _D, _D]
    lib.lbe_mlp_get_scaling.argtypes = [vp, _D, _D]
    lib.lbe_mlp_forward.argtypes = [vp, vp, i32, vp]
    lib.lbe_mlp_loss_grad.argtypes = [vp, vp, vp, i32, _D, F, i64]
    lib.lbe_mlp_set_grads.argtypes = [vp, F, i64]
    lib.lbe_mlp_adam_step.argtypes = [vp, ctypes.c_float]
    lib.lbe_mlp_train.argtypes = [vp, vp, vp, i64, i32, i32, ctypes.c_float, u64, _D]
    lib.lbe_mlp_last_error.argtypes = [vp]
    lib.lbe_mlp_last_error.restype = ctypes.c_char_p
    lib.lbe_mlp_free.argtypes = [vp]
    lib.lbe_mlp_free.restype = None
    lib.lbe_last_error.argtypes = [vp]
    lib.lbe_last_error.restype = ctypes.c_char_p
    lib.lbe_status_string.argtypes = [ctypes.c_int]
    lib.lbe_status_string.restype = ctypes.c_char_p
    lib.lbe_free.argtypes = [vp]
    lib.lbe_free.restype = None
    for name in ("lbe_query", "lbe_init", "lbe_init_static", "lbe_step", "lbe_sync", "lbe_moments", "lbe_run_to_steady", "lbe_get_state",
                 "lbe_set_state", "lbe_rhs", "lbe_checkpoint_size", "lbe_checkpoint_save", "lbe_checkpoint_load",
                 "lbe_info", "lbe_tables", "lbe_timing", "lbe_autotune",
                 "lbe_features", "lbe_targets", "lbe_set_init_moments", "lbe_warm_start", "lbe_mlp_query",
                 "lbe_mlp_init", "lbe_mlp_init_params", "lbe_mlp_set_params", "lbe_mlp_get_params",
                 "lbe_mlp_set_scaling", "lbe_mlp_get_scaling", "lbe_mlp_forward", "lbe_mlp_loss_grad",
                 "lbe_mlp_set_grads", "lbe_mlp_adam_step", "lbe_mlp_train", "lbe_status_string"):
        if name != "lbe_status_string":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


EXPORTS = ("lbe_query", "lbe_init", "lbe_init_static", "lbe_step", "lbe_sync", "lbe_moments", "lbe_run_to_steady", "lbe_get_state",
           "lbe_set_state", "lbe_rhs", "lbe_checkpoint_size", "lbe_checkpoint_save", "lbe_checkpoint_load",
           "lbe_info", "lbe_tables", "lbe_timing", "lbe_autotune", "lbe_last_error",
           "lbe_status_string", "lbe_free", "lbe_features", "lbe_targets", "lbe_set_init_moments", "lbe_warm_start",
           "lbe_mlp_query", "lbe_mlp_init", "lbe_mlp_init_params", "lbe_mlp_set_params", "lbe_mlp_get_params",
           "lbe_mlp_set_scaling", "lbe_mlp_get_scaling", "lbe_mlp_forward", "lbe_mlp_loss_grad", "lbe_mlp_set_grads",
           "lbe_mlp_adam_step", "lbe_mlp_train", "lbe_mlp_last_error", "lbe_mlp_free")


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def query(params: Sequence[dict]) -> tuple[int, int]:
    lib = load()
    arr = (Params * len(params))(*[make_params(p) for p in params])
    dev = ctypes.c_size_t(0)
    host = ctypes.c_size_t(0)
    st = lib.lbe_query(arr, len(params), ctypes.byref(dev), ctypes.byref(host))
    if st != LBE_OK:
        raise LbeError(st, "lbe_query rejected the parameters")
    return dev.value, host.value


def tables(params: dict, which: int, extra: Iterable[float] | None = None) -> np.ndarray:
    """Host-only tables of one instance (see lbe_tables in include/lbe.h)."""
    lib = load()
    p = make_params(params)
    ex = np.ascontiguousarray(np.array(list(extra) if extra is not None else [0.0, 1.0, 0.0], dtype=np.float64))
    n = ctypes.c_int64(0)
    lib.lbe_tables(ctypes.byref(p), which, _ptr(ex), None, 0, ctypes.byref(n))
    if n.value <= 0:
        raise LbeError(LBE_EINVAL, f"lbe_tables({which}) rejected the parameters")
    out = np.zeros(n.value)
    st = lib.lbe_tables(ctypes.byref(p), which, _ptr(ex), _ptr(out), n.value, ctypes.byref(n))
    if st != LBE_OK:
        raise LbeError(st, f"lbe_tables({which})")
    return out


class Solver:
    """A batch of FDLB instances on one GPU (the current torch device and stream)."""

    def __init__(self, params: dict | Sequence[dict], static_ws: bool = False):
        """static_ws: take the library's own device workspace (lbe_init_static) instead of a
        torch tensor; at most one such solver per GPU at a time, up to 64 MiB."""
        import torch

        if isinstance(params, dict):
            params = [params]
        self.params = [dict(p) for p in params]
        lib = load()
        self._lib = lib
        arr = (Params * len(self.params))(*[make_params(p) for p in self.params])
        stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p(0)
        if static_ws:
            self._ws = None
            st = lib.lbe_init_static(arr, len(self.params), ctypes.c_void_p(stream), ctypes.byref(h))
            if st != LBE_OK:
                raise LbeError(st, "lbe_init_static failed")
        else:
            dev_bytes, _ = query(self.params)
            self._ws = torch.empty(dev_bytes + 256, dtype=torch.uint8, device="cuda")
            base = self._ws.data_ptr()
            aligned = (base + 255) & ~255
            st = lib.lbe_init(arr, len(self.params), ctypes.c_void_p(aligned), dev_bytes, ctypes.c_void_p(stream),
                              ctypes.byref(h))
            if st != LBE_OK:
                raise LbeError(st, "lbe_init failed")
        self._h = h
        self.n_inst = len(self.params)
        self._infos = [self.info(k) for k in range(self.n_inst)]

    def close(self) -> None:
        """Free the context now (waits for its stream); the workspace tensor goes with the object."""
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                self._lib.lbe_sync(h)
            finally:
                self._lib.lbe_free(h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, st: int, what: str) -> int:
        if st not in (LBE_OK, LBE_ENOTCONV):
            msg = self._lib.lbe_last_error(self._h).decode()
            raise LbeError(st, f"{what}: {msg}")
        return st

    def info(self, inst: int = 0) -> dict:
        out = np.zeros(19)
        self._check(self._lib.lbe_info(self._h, inst, _ptr(out), 19), "lbe_info")
        return dict(zip(INFO_KEYS, out.tolist()))

    def step(self, n: int = 1) -> None:
        self._check(self._lib.lbe_step(self._h, n), "lbe_step")

    def sync(self) -> None:
        self._check(self._lib.lbe_sync(self._h), "lbe_sync")

    def moments(self, inst: int = 0, mean_field: bool = False) -> dict:
        nr = int(self._infos[inst]["nr"])
        keys = FIELDS + (MF_FIELDS if mean_field else ())
        out = np.zeros(len(keys) * nr)
        self._check(self._lib.lbe_moments(self._h, inst, _ptr(out), out.size), "lbe_moments")
        out = out.reshape(len(keys), nr)
        return {k: out[i].copy() for i, k in enumerate(keys)}

    def run_to_steady(self, tol: float, max_steps: int, check_every: int):
        steps = np.zeros(self.n_inst, dtype=np.int64)
        res = np.zeros(self.n_inst)
        st = self._lib.lbe_run_to_steady(self._h, tol, max_steps, check_every, steps.ctypes.data_as(_I64), _ptr(res))
        self._check(st, "lbe_run_to_steady")
        return st, steps, res

    def get_state(self, inst: int = 0) -> np.ndarray:
        nr, nv = int(self._infos[inst]["nr"]), int(self._infos[inst]["nv"])
        out = np.zeros(nr * nv)
        self._check(self._lib.lbe_get_state(self._h, inst, _ptr(out), out.size), "lbe_get_state")
        return out.reshape(nr, nv)

    def set_state(self, inst: int, f: np.ndarray) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        self._check(self._lib.lbe_set_state(self._h, inst, _ptr(f), f.size), "lbe_set_state")

    def timing_start(self) -> None:
        self._check(self._lib.lbe_timing(self._h, 1, None, 0), "lbe_timing")

    def timing_stop(self) -> dict:
        out = np.zeros(4)
        self._check(self._lib.lbe_timing(self._h, 0, _ptr(out), 4), "lbe_timing")
        return {"stage_ms": out[0], "stage_launches": int(out[1]), "node_ms": out[2], "node_launches": int(out[3])}

    def autotune(self, reps: int = 3) -> list[dict]:
        ng = ctypes.c_int32(0)
        out = np.zeros(4 * self.n_inst)  # at most one launch group per instance
        self._check(self._lib.lbe_autotune(self._h, reps, _ptr(out), out.size, ctypes.byref(ng)), "lbe_autotune")
        return [{"nv": int(out[4 * q]), "tile_nodes": int(out[4 * q + 1]), "ms": out[4 * q + 2],
                 "ms_before": out[4 * q + 3]} for q in range(ng.value)]

    def rows(self) -> int:
        return int(sum(int(i["nr"]) for i in self._infos))

    def features(self):
        """Network inputs of every node (torch float32 tensor [rows][6] on the device)."""
        import torch

        x = torch.empty((self.rows(), 6), dtype=torch.float32, device="cuda")
        self._check(self._lib.lbe_features(self._h, ctypes.c_void_p(x.data_ptr()), x.shape[0], None), "lbe_features")
        return x

    def targets(self):
        """Profiles (n, u_t1, T, q_r, P_rt1) of every node (torch float32 tensor [rows][5])."""
        import torch

        t = torch.empty((self.rows(), 5), dtype=torch.float32, device="cuda")
        self._check(self._lib.lbe_targets(self._h, ctypes.c_void_p(t.data_ptr()), t.shape[0]), "lbe_targets")
        return t

    def set_init_moments(self, inst: int, prof: dict) -> None:
        a = np.ascontiguousarray(np.stack([np.asarray(prof[k], dtype=np.float64) for k in WARM_FIELDS]).reshape(-1))
        self._check(self._lib.lbe_set_init_moments(self._h, inst, _ptr(a), a.size), "lbe_set_init_moments")

    def warm_start(self, net: "Mlp", judge: bool = True):
        kept = np.zeros(self.n_inst, dtype=np.int32)
        rho = np.zeros(2 * self.n_inst)
        self._check(self._lib.lbe_warm_start(self._h, net._h, int(judge),
                                             kept.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(rho)),
                    "lbe_warm_start")
        return kept, rho.reshape(self.n_inst, 2)

    def checkpoint(self) -> bytes:
        """Exact device state of the whole context (lbe_checkpoint_save)."""
        n = ctypes.c_size_t(0)
        self._check(self._lib.lbe_checkpoint_size(self._h, ctypes.byref(n)), "lbe_checkpoint_size")
        buf = ctypes.create_string_buffer(n.value)
        self._check(self._lib.lbe_checkpoint_save(self._h, buf, n.value), "lbe_checkpoint_save")
        return buf.raw

    def restore(self, blob: bytes) -> None:
        """Continue from a checkpoint of a context with the same problem statements."""
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self._lib.lbe_checkpoint_load(self._h, buf, len(blob)), "lbe_checkpoint_load")

    def rhs(self, inst: int = 0) -> np.ndarray:
        nr, nv = int(self._infos[inst]["nr"]), int(self._infos[inst]["nv"])
        out = np.zeros(nr * nv)
        self._check(self._lib.lbe_rhs(self._h, inst, _ptr(out), out.size), "lbe_rhs")
        return out.reshape(nr, nv)


class Mlp:
    """Network of the learned warm start on the current torch device and stream."""

    def __init__(self, max_rows: int = 4096, gemm: int = GEMM_BF16, seed: int | None = None):
        import torch

        lib = load()
        self._lib = lib
        nbytes = ctypes.c_size_t(0)
        npar = ctypes.c_int64(0)
        st = lib.lbe_mlp_query(max_rows, ctypes.byref(nbytes), ctypes.byref(npar))
        if st != LBE_OK:
            raise LbeError(st, "lbe_mlp_query")
        self.n_params = npar.value
        self.max_rows = max_rows
        self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        aligned = (self._ws.data_ptr() + 255) & ~255
        h = ctypes.c_void_p(0)
        st = lib.lbe_mlp_init(max_rows, gemm, ctypes.c_void_p(aligned), nbytes.value,
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(h))
        if st != LBE_OK:
            raise LbeError(st, "lbe_mlp_init")
        self._h = h
        if seed is not None:
            self._check(lib.lbe_mlp_init_params(h, seed), "lbe_mlp_init_params")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.lbe_mlp_free(h)
            self._h = None

    def _check(self, st: int, what: str) -> None:
        if st != LBE_OK:
            raise LbeError(st, f"{what}: {self._lib.lbe_mlp_last_error(self._h).decode()}")

    def set_params(self, p: np.ndarray) -> None:
        a = np.ascontiguousarray(p, dtype=np.float32)
        self._check(self._lib.lbe_mlp_set_params(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size),
                    "lbe_mlp_set_params")

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.n_params, dtype=np.float32)
        self._check(self._lib.lbe_mlp_get_params(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size),
                    "lbe_mlp_get_params")
        return a

    def set_scaling(self, mean, scale) -> None:
        m = np.ascontiguousarray(mean, dtype=np.float64)
        s = np.ascontiguousarray(scale, dtype=np.float64)
        self._check(self._lib.lbe_mlp_set_scaling(self._h, _ptr(m), _ptr(s)), "lbe_mlp_set_scaling")

    def get_scaling(self):
        m = np.zeros(5)
        s = np.zeros(5)
        self._check(self._lib.lbe_mlp_get_scaling(self._h, _ptr(m), _ptr(s)), "lbe_mlp_get_scaling")
        return m, s

    def forward(self, x):
        import torch

        y = torch.empty((x.shape[0], 5), dtype=torch.float32, device="cuda")
        self._check(self._lib.lbe_mlp_forward(self._h, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                              ctypes.c_void_p(y.data_ptr())), "lbe_mlp_forward")
        return y

    def loss_grad(self, x, t):
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = np.zeros(1)
        self._check(self._lib.lbe_mlp_loss_grad(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                                x.shape[0], _ptr(loss), g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                g.size), "lbe_mlp_loss_grad")
        return float(loss[0]), g

    def set_grads(self, g: np.ndarray) -> None:
        a = np.ascontiguousarray(g, dtype=np.float32)
        self._check(self._lib.lbe_mlp_set_grads(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size),
                    "lbe_mlp_set_grads")

    def adam_step(self, lr: float) -> None:
        self._check(self._lib.lbe_mlp_adam_step(self._h, lr), "lbe_mlp_adam_step")

    def train(self, x, t, epochs: int, batch: int, lr: float, seed: int) -> np.ndarray:
        hist = np.zeros(epochs)
        self._check(self._lib.lbe_mlp_train(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                            x.shape[0], epochs, batch, lr, seed, _ptr(hist)), "lbe_mlp_train")
        return hist
