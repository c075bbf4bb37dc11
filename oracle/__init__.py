"""Python access to the plain FP64 CPU oracle (``oracle/lbe_oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle is the slow reference that the GPU solver is checked
against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package; the product package never does, and the two share no code.

The oracle follows arXiv:2403.15051 (Busuioc, FDLB for the simplified Enskog equation in
vielbein coordinates); see the header of ``lbe_oracle.c`` for the section map.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbe_oracle.c")
_LIB = os.environ.get("LBE_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
SAN_LIB = os.path.join(_HERE, "liboracle_san.so")

_lib = None


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP over radial nodes).  sanitize: the
    AddressSanitizer + UndefinedBehaviorSanitizer build SAN_LIB (load it with LBE_ORACLE_LIB and
    gcc's libasan / libubsan preloaded)."""
    lib = SAN_LIB if sanitize else _LIB
    if force or not os.path.exists(lib):
        tmp = lib + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", "-o", tmp, _SRC, "-lquadmath", "-lm"]
        if sanitize:
            cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined",
                        "-g"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    return lib


class Params(ctypes.Structure):
    """Problem statement of one solve (mirrors ``orc_params`` in lbe_oracle.c)."""

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
        ("reduced", ctypes.c_int32),
        ("phi_a", ctypes.c_double),
    ]


_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    _lib = _setup(ctypes.CDLL(_LIB))
    return _lib


def load_variant(substitutions, workdir: str):
    """Compile a copy of the oracle with textual substitutions [(old, new), ...] applied (each
    ``old`` must occur exactly once) into ``workdir`` and load it.  Used only by the tests that
    plant a deliberate mistake in the oracle to show that a pin catches it."""
    src = open(_SRC).read()
    for old, new in substitutions:
        if src.count(old) != 1:
            raise ValueError(f"substitution target must occur exactly once: {old!r}")
        src = src.replace(old, new)
    tag = str(abs(hash(tuple(substitutions))))
    c = os.path.join(workdir, f"oracle_variant_{tag}.c")
    so = os.path.join(workdir, f"oracle_variant_{tag}.so")
    with open(c, "w") as fh:
        fh.write(src)
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", "-o", so, c, "-lquadmath", "-lm"],
                   check=True)
    return _setup(ctypes.CDLL(so))


def _setup(lib):
    vp = ctypes.c_void_p
    lib.orc_quad_half.argtypes = [ctypes.c_int, _D, _D]
    lib.orc_quad_full.argtypes = [ctypes.c_int, _D, _D]
    lib.orc_half_poly.argtypes = [ctypes.c_int, _D, _D, _D]
    lib.orc_kmat_full.argtypes = [ctypes.c_int, ctypes.c_int, _D]
    lib.orc_kmat_half.argtypes = [ctypes.c_int, ctypes.c_int, _D]
    lib.orc_geq.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D]
    for name in ("orc_chi",):
        getattr(lib, name).argtypes = [ctypes.c_double]
        getattr(lib, name).restype = ctypes.c_double
    lib.orc_prandtl.argtypes = [ctypes.c_double]
    lib.orc_prandtl.restype = ctypes.c_double
    lib.orc_confinement.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.orc_confinement.restype = ctypes.c_double
    lib.orc_knudsen.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.orc_knudsen.restype = ctypes.c_double
    lib.orc_tau.argtypes = [ctypes.c_double] * 7
    lib.orc_tau.restype = ctypes.c_double
    lib.orc_vol_sph.argtypes = [ctypes.c_double] * 3
    lib.orc_vol_sph.restype = ctypes.c_double
    lib.orc_vol_slab.argtypes = [ctypes.c_double] * 3
    lib.orc_vol_slab.restype = ctypes.c_double
    lib.orc_vol_cyl.argtypes = [ctypes.c_double] * 3
    lib.orc_vol_cyl.restype = ctypes.c_double
    lib.orc_mf_potential.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4
    lib.orc_mf_potential.restype = ctypes.c_double
    lib.orc_fd4.argtypes = [_D, ctypes.c_int, ctypes.c_int, ctypes.c_double]
    lib.orc_fd4.restype = ctypes.c_double
    lib.orc_weno5.argtypes = [ctypes.c_double] * 5
    lib.orc_weno5.restype = ctypes.c_double
    lib.orc_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_int)]
    lib.orc_create.restype = vp
    lib.orc_free.argtypes = [vp]
    lib.orc_step.argtypes = [vp, ctypes.c_int64]
    lib.orc_run_to_steady.argtypes = [vp, ctypes.c_double, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int64), _D]
    for name in ("orc_moments", "orc_node_coeffs", "orc_node_grads", "orc_rhs", "orc_get_f", "orc_set_f",
                 "orc_get_W", "orc_get_attraction", "orc_info"):
        getattr(lib, name).argtypes = [vp, _D]
    lib.orc_grid.argtypes = [vp, _D, _D, _D, _D]
    lib.orc_rhs_terms.argtypes = [vp, _D, _D, _D, _D]
    lib.orc_mean_field.argtypes = [vp, _D, _D]
    lib.orc_mass.argtypes = [vp]
    lib.orc_mass.restype = ctypes.c_double
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_get_threads.restype = ctypes.c_int
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


# ---------------------------------------------------------------- table-level entry points
def quad_half(Q: int):
    lib = _load()
    x = np.zeros(2 * Q)
    w = np.zeros(2 * Q)
    assert lib.orc_quad_half(Q, _ptr(x), _ptr(w)) == 0
    return x, w


def quad_full(Q: int):
    lib = _load()
    x = np.zeros(Q)
    w = np.zeros(Q)
    assert lib.orc_quad_full(Q, _ptr(x), _ptr(w)) == 0
    return x, w


def half_poly(Q: int):
    """(a[0..Q], b[0..Q+1], h[l, s]) of the orthonormal half-range polynomials."""
    lib = _load()
    a = np.zeros(Q + 1)
    b = np.zeros(Q + 2)
    hc = np.zeros((Q + 1) * (Q + 1))
    assert lib.orc_half_poly(Q, _ptr(a), _ptr(b), _ptr(hc)) == 0
    return a, b, hc.reshape(Q + 1, Q + 1)


def kmat_full(Q: int, which: int):
    lib = _load()
    K = np.zeros(Q * Q)
    assert lib.orc_kmat_full(Q, which, _ptr(K)) == 0
    return K.reshape(Q, Q)


def kmat_half(Q: int, which: int):
    lib = _load()
    K = np.zeros(4 * Q * Q)
    assert lib.orc_kmat_half(Q, which, _ptr(K)) == 0
    return K.reshape(2 * Q, 2 * Q)


def geq(half: bool, Q: int, N: int, u: float, T: float):
    lib = _load()
    g = np.zeros(2 * Q if half else Q)
    assert lib.orc_geq(int(half), Q, N, u, T, _ptr(g)) == 0
    return g


def chi(eta: float) -> float:
    return _load().orc_chi(eta)


def prandtl(x: float) -> float:
    return _load().orc_prandtl(x)


def confinement(eta0: float, kn: float) -> float:
    return _load().orc_confinement(eta0, kn)


def knudsen(eta0: float, C: float) -> float:
    return _load().orc_knudsen(eta0, C)


def tau(chi0, kn, L, n, T, chi_, brho) -> float:
    return _load().orc_tau(chi0, kn, L, n, T, chi_, brho)


def vol_sph(s: float, R: float, b: float) -> float:
    return _load().orc_vol_sph(s, R, b)


def vol_slab(s: float, X: float, b: float) -> float:
    return _load().orc_vol_slab(s, X, b)


def vol_cyl(s: float, R: float, b: float) -> float:
    return _load().orc_vol_cyl(s, R, b)


def mf_potential(geometry: int, sigma: float, phi_a: float, r: float, s: float) -> float:
    """Integral of the attractive tail -phi_a (sigma/t)^6 (t > sigma) over the region of radius s
    (ball, infinite cylinder, or the half space x' < s for the plane) seen from radius r."""
    return _load().orc_mf_potential(geometry, sigma, phi_a, r, s)


def fd4(phi: np.ndarray, i: int, dr: float) -> float:
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    return _load().orc_fd4(_ptr(phi), i, len(phi), dr)


def weno5(a, b, c, d, e) -> float:
    return _load().orc_weno5(a, b, c, d, e)


def set_threads(n: int) -> None:
    _load().orc_set_threads(n)


def get_threads() -> int:
    return _load().orc_get_threads()


# ---------------------------------------------------------------- the solver
FIELDS = ("n", "u_r", "u_t1", "u_t2", "T", "q_r", "P_rt1", "nbar", "chi")


def make_params(geometry, r_inner, r_outer, u_wall_inner, t_wall_inner, t_wall_outer, eta0, kn, nr,
                q_radial, q_t1, q_t2, cfl, n_expand=(0, 0, 0), reduced=0, precision=0, phi_a=0.0) -> Params:
    p = Params()
    p.geometry = geometry
    p.r_inner = r_inner
    p.r_outer = r_outer
    p.u_wall_inner = u_wall_inner
    p.t_wall_inner = t_wall_inner
    p.t_wall_outer = t_wall_outer
    p.eta0 = eta0
    p.kn = kn
    p.nr = nr
    p.q_radial = q_radial
    p.q_t1 = q_t1
    p.q_t2 = q_t2
    for a in range(3):
        p.n_expand[a] = n_expand[a]
    p.cfl = cfl
    p.reduced = int(reduced)
    p.phi_a = float(phi_a)
    return p


class Solver:
    """One FDLB solve on the CPU (FP64)."""

    def __init__(self, params: Params | dict, lib=None):
        lib = lib if lib is not None else _load()
        if isinstance(params, dict):
            params = make_params(**params)
        st = ctypes.c_int(0)
        h = lib.orc_create(ctypes.byref(params), ctypes.byref(st))
        if not h:
            raise ValueError(f"oracle rejected the parameters (status {st.value})")
        self._h = h
        self._lib = lib
        info = self.info()
        self.nr = int(info["nr"])
        self.nv = int(info["nv"])
        self.shape = (int(info["n2"]), int(info["n1"]), int(info["n0"]))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_free(h)
            self._h = None

    def info(self) -> dict:
        out = np.zeros(18)
        self._lib.orc_info(self._h, _ptr(out))
        keys = ["nr", "nv", "n0", "n1", "n2", "chi0", "C", "L", "sigma", "rcl", "rcr", "dr", "dt", "steps",
                "last_resid", "N0", "N1", "N2"]
        return dict(zip(keys, out.tolist()))

    def grid(self):
        info = self.info()
        n0, n1, n2 = int(info["n0"]), int(info["n1"]), int(info["n2"])
        pn = np.zeros(n0 + n1 + n2)
        r = np.zeros(self.nr)
        ri = np.zeros(self.nr + 1)
        vol = np.zeros(self.nr)
        self._lib.orc_grid(self._h, _ptr(pn), _ptr(r), _ptr(ri), _ptr(vol))
        return {"p0": pn[:n0], "p1": pn[n0:n0 + n1], "p2": pn[n0 + n1:], "r": r, "ri": ri, "vol": vol}

    def step(self, n: int) -> int:
        return self._lib.orc_step(self._h, n)

    def run_to_steady(self, tol: float, max_steps: int, check_every: int):
        steps = ctypes.c_int64(0)
        res = ctypes.c_double(0)
        rc = self._lib.orc_run_to_steady(self._h, tol, max_steps, check_every, ctypes.byref(steps),
                                         ctypes.byref(res))
        return rc, steps.value, res.value

    def moments(self) -> dict:
        out = np.zeros(9 * self.nr)
        self._lib.orc_moments(self._h, _ptr(out))
        out = out.reshape(9, self.nr)
        return {k: out[i].copy() for i, k in enumerate(FIELDS)}

    def node_coeffs(self) -> dict:
        out = np.zeros(5 * self.nr)
        self._lib.orc_node_coeffs(self._h, _ptr(out))
        out = out.reshape(5, self.nr)
        return {k: out[i].copy() for i, k in enumerate(("tau", "Pr", "brhochi", "q_t1", "q_t2"))}

    def node_grads(self) -> dict:
        """Radial gradients entering J1: d ln(n^2 chi T), d ln T and du of the three components."""
        out = np.zeros(5 * self.nr)
        self._lib.orc_node_grads(self._h, _ptr(out))
        out = out.reshape(5, self.nr)
        return {k: out[i].copy() for i, k in enumerate(("dlog_nnchiT", "dlogT", "du_r", "du_t1", "du_t2"))}

    def rhs(self) -> np.ndarray:
        out = np.zeros(self.nr * self.nv)
        self._lib.orc_rhs(self._h, _ptr(out))
        return out.reshape(self.nr, self.nv)

    def rhs_terms(self) -> dict:
        outs = [np.zeros(self.nr * self.nv) for _ in range(4)]
        self._lib.orc_rhs_terms(self._h, *[_ptr(o) for o in outs])
        return {k: o.reshape(self.nr, self.nv) for k, o in zip(("A", "I", "J0", "J1"), outs)}

    def get_f(self) -> np.ndarray:
        out = np.zeros(self.nr * self.nv)
        self._lib.orc_get_f(self._h, _ptr(out))
        return out.reshape(self.nr, self.nv)

    def set_f(self, f: np.ndarray) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        assert f.size == self.nr * self.nv
        self._lib.orc_set_f(self._h, _ptr(f))

    def W(self) -> np.ndarray:
        out = np.zeros(self.nr * self.nr)
        self._lib.orc_get_W(self._h, _ptr(out))
        return out.reshape(self.nr, self.nr)

    def attraction(self) -> np.ndarray:
        """Mean-field weights A (Phi = A n); zeros without attraction."""
        out = np.zeros(self.nr * self.nr)
        self._lib.orc_get_attraction(self._h, _ptr(out))
        return out.reshape(self.nr, self.nr)

    def mean_field(self):
        """(Phi, F) of the current state: mean-field potential and radial force per node."""
        phi = np.zeros(self.nr)
        F = np.zeros(self.nr)
        self._lib.orc_mean_field(self._h, _ptr(phi), _ptr(F))
        return phi, F

    def mass(self) -> float:
        return self._lib.orc_mass(self._h)
