"""FP64 CPU oracle for the CHFPE hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The product path (the HIP
library and its binding) never calls it.

The arithmetic lives in ``chfpe_oracle.c`` (plain C, FP64, OpenMP over grid
lines); this module marshals arguments with ctypes and adds the spectra of
Eqs. (1DIR_Raman), (2DThz_Raman) and (noncorrelation) as plain discrete
Fourier sums.
It shares no code with the HIP path; inputs come from ``workloads``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborcl.so")

_d3 = ctypes.c_double * 3
_d33 = (ctypes.c_double * 3) * 3
_i3 = ctypes.c_int32 * 3


class Params(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32), ("K", ctypes.c_int32),
        ("Nq", _i3), ("Np", _i3),
        ("Lq", _d3), ("Lp", _d3),
        ("m", _d3), ("omega", _d3), ("g3", _d3), ("g4", _d3),
        ("g2", _d33), ("g21", _d33), ("g12", _d33),
        ("VLL", _d3), ("VSL", _d3),
        ("zeta", _d3), ("gamma", _d3),
        ("beta", ctypes.c_double),
    ]


class Optical(ctypes.Structure):
    _fields_ = [("lin", _d3), ("quad", _d33)]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    src = os.path.join(_HERE, "chfpe_oracle.c")
    if (not os.path.exists(_LIB_PATH)
            or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src)):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER(Params)
    O = ctypes.POINTER(Optical)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.orc_elements.argtypes = [P, ctypes.POINTER(ctypes.c_int)]
    lib.orc_elements.restype = ctypes.c_int
    lib.orc_points.argtypes = [P]
    lib.orc_points.restype = i64
    lib.orc_state_size.argtypes = [P]
    lib.orc_state_size.restype = i64
    lib.orc_potential.argtypes = [P, dp]
    lib.orc_potential.restype = ctypes.c_double
    lib.orc_force.argtypes = [P, dp, ctypes.c_int]
    lib.orc_force.restype = ctypes.c_double
    lib.orc_deriv_line.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
    lib.orc_deriv_line.restype = None
    lib.orc_rhs.argtypes = [P, dp, dp]
    lib.orc_rhs.restype = None
    lib.orc_rhs_point.argtypes = [P, dp, ctypes.c_int, i64]
    lib.orc_rhs_point.restype = ctypes.c_double
    lib.orc_rk4.argtypes = [P, dp, i64, ctypes.c_double]
    lib.orc_rk4.restype = None
    lib.orc_boltzmann.argtypes = [P, dp]
    lib.orc_boltzmann.restype = None
    lib.orc_equilibrate.argtypes = [P, dp, i64, ctypes.c_double]
    lib.orc_equilibrate.restype = None
    lib.orc_perturb.argtypes = [P, O, dp, dp]
    lib.orc_perturb.restype = None
    lib.orc_observe.argtypes = [P, O, dp]
    lib.orc_observe.restype = ctypes.c_double
    lib.orc_moments.argtypes = [P, dp, ctypes.c_int, ctypes.c_int, dp]
    lib.orc_moments.restype = None
    lib.orc_energy.argtypes = [P, dp]
    lib.orc_energy.restype = ctypes.c_double
    lib.orc_response_1d.argtypes = [P, O, dp, i64, ctypes.c_int, ctypes.c_double, dp]
    lib.orc_response_1d.restype = None
    lib.orc_response_2d.argtypes = [P, O, O, O, dp, i64, i64, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.POINTER(i64), i64, dp]
    lib.orc_response_2d.restype = None
    lib.orc_response_3d.argtypes = [P, O, O, O, O, dp, i64, i64, i64, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.POINTER(i64), i64, dp]
    lib.orc_response_3d.restype = None
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def params(w: dict) -> Params:
    """Oracle parameter struct from a workload dict (see ``workloads``)."""
    p = Params()
    M = int(w["M"])
    p.M, p.K = M, int(w["K"])
    for s in range(M):
        p.Nq[s], p.Np[s] = int(w["Nq"][s]), int(w["Np"][s])
        p.Lq[s], p.Lp[s] = float(w["Lq"][s]), float(w["Lp"][s])
        for key in ("m", "omega", "g3", "g4", "VLL", "VSL", "zeta", "gamma"):
            getattr(p, key)[s] = float(w[key][s])
        for t in range(M):
            for key in ("g2", "g21", "g12"):
                getattr(p, key)[s][t] = float(w[key][s][t])
    p.beta = float(w["beta"])
    return p


def optical(X: dict) -> Optical:
    o = Optical()
    for s, v in enumerate(X["lin"]):
        o.lin[s] = float(v)
    for s, row in enumerate(X["quad"]):
        for t, v in enumerate(row):
            o.quad[s][t] = float(v)
    return o


def num_threads() -> int:
    return int(_load().orc_num_threads())


def elements(w: dict) -> np.ndarray:
    """Hierarchy multi-indices n, shape (|N_K|, M), in the oracle's order."""
    lib = _load()
    p = params(w)
    ne = lib.orc_elements(ctypes.byref(p), None)
    out = (ctypes.c_int * (ne * p.M))()
    lib.orc_elements(ctypes.byref(p), out)
    return np.array(list(out), dtype=np.int64).reshape(ne, p.M)


def state_shape(w: dict) -> tuple:
    ne = elements(w).shape[0]
    return (ne,) + tuple(int(x) for x in w["Nq"]) + tuple(int(x) for x in w["Np"])


def _state(w: dict, W) -> np.ndarray:
    a = np.ascontiguousarray(W, dtype=np.float64)
    assert a.shape == state_shape(w), (a.shape, state_shape(w))
    return a


def deriv_line(f, h: float) -> np.ndarray:
    """Compact sixth-order derivative of one line of values (zero outside)."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    y = np.empty_like(f)
    lib.orc_deriv_line(int(f.size), float(h), _ptr(f), _ptr(y))
    return y


def potential(w: dict, q) -> float:
    q = np.ascontiguousarray(q, dtype=np.float64)
    return float(_load().orc_potential(ctypes.byref(params(w)), _ptr(q)))


def force(w: dict, q, s: int) -> float:
    q = np.ascontiguousarray(q, dtype=np.float64)
    return float(_load().orc_force(ctypes.byref(params(w)), _ptr(q), int(s)))


def rhs(w: dict, W) -> np.ndarray:
    """Right-hand side of the hierarchy equation, Eq. (eq:HEOM)."""
    W = _state(w, W)
    out = np.empty_like(W)
    _load().orc_rhs(ctypes.byref(params(w)), _ptr(W), _ptr(out))
    return out


def rhs_point(w: dict, W, e: int, idx: int) -> float:
    W = _state(w, W)
    return float(_load().orc_rhs_point(ctypes.byref(params(w)), _ptr(W), int(e), int(idx)))


def rk4(w: dict, W, nsteps: int, dt: float) -> np.ndarray:
    """nsteps classical RK4 steps; returns a new array."""
    y = _state(w, W).copy()
    _load().orc_rk4(ctypes.byref(params(w)), _ptr(y), int(nsteps), float(dt))
    return y


def boltzmann(w: dict) -> np.ndarray:
    W = np.empty(state_shape(w))
    _load().orc_boltzmann(ctypes.byref(params(w)), _ptr(W))
    return W


def equilibrate(w: dict, nsteps: int, dt: float) -> np.ndarray:
    W = np.empty(state_shape(w))
    _load().orc_equilibrate(ctypes.byref(params(w)), _ptr(W), int(nsteps), float(dt))
    return W


def perturb(w: dict, X: dict, W) -> np.ndarray:
    """Optical excitation X^x applied to every element, Eq. (Opticalexc)."""
    W = _state(w, W)
    out = np.empty_like(W)
    o = optical(X)
    _load().orc_perturb(ctypes.byref(params(w)), ctypes.byref(o), _ptr(W), _ptr(out))
    return out


def observe(w: dict, X: dict, W) -> float:
    W = _state(w, W)
    o = optical(X)
    return float(_load().orc_observe(ctypes.byref(params(w)), ctypes.byref(o), _ptr(W)))


def moments(w: dict, W, e: int, s: int) -> np.ndarray:
    """[int W_e, <q_s>, <p_s>, <q_s^2>, <p_s^2>, <q_s p_s>] (unnormalised)."""
    W = _state(w, W)
    out = np.empty(6)
    _load().orc_moments(ctypes.byref(params(w)), _ptr(W), int(e), int(s), _ptr(out))
    return out


def energy(w: dict, W) -> float:
    W = _state(w, W)
    return float(_load().orc_energy(ctypes.byref(params(w)), _ptr(W)))


def response_1d(w: dict, A: dict, Weq, n_t: int, stride: int, dt: float) -> np.ndarray:
    """R^(1)[j] of Eq. (1Dresponse) at t = j * stride * dt."""
    Weq = _state(w, Weq)
    R = np.empty(int(n_t))
    o = optical(A)
    _load().orc_response_1d(ctypes.byref(params(w)), ctypes.byref(o), _ptr(Weq), int(n_t),
                            int(stride), float(dt), _ptr(R))
    return R


def response_2d(w: dict, A: dict, B: dict, C: dict, Weq, n_t1: int, n_t2: int,
                stride1: int, stride2: int, dt: float, j1_list=None) -> np.ndarray:
    """R^(2)[j2, j1] of Eq. (2Dresponse); shape (n_t2, n_t1), t1 fastest.

    With ``j1_list`` only those t1 columns are computed (others are NaN).
    """
    Weq = _state(w, Weq)
    R = np.full((int(n_t2), int(n_t1)), np.nan)
    oa, ob, oc = optical(A), optical(B), optical(C)
    if j1_list is None:
        jl, nj = None, 0
    else:
        arr = np.ascontiguousarray(sorted(int(j) for j in j1_list), dtype=np.int64)
        jl, nj = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), arr.size
    _load().orc_response_2d(ctypes.byref(params(w)), ctypes.byref(oa), ctypes.byref(ob),
                            ctypes.byref(oc), _ptr(Weq), int(n_t1), int(n_t2), int(stride1),
                            int(stride2), float(dt), jl, int(nj), _ptr(R))
    return R


def response_3d(w: dict, A: dict, B: dict, C: dict, D: dict, Weq, n_t1: int, t2_steps: int, n_t3: int,
                stride1: int, stride3: int, dt: float, j1_list=None) -> np.ndarray:
    """R^(3)[j3, j1] of Eq. (3Dresponse) at the waiting time t2 = t2_steps * dt;
    shape (n_t3, n_t1), t1 fastest.  With ``j1_list`` only those t1 columns
    are computed (others are NaN)."""
    Weq = _state(w, Weq)
    R = np.full((int(n_t3), int(n_t1)), np.nan)
    ops = [optical(X) for X in (A, B, C, D)]
    if j1_list is None:
        jl, nj = None, 0
    else:
        arr = np.ascontiguousarray(sorted(int(j) for j in j1_list), dtype=np.int64)
        jl, nj = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), arr.size
    _load().orc_response_3d(ctypes.byref(params(w)), *[ctypes.byref(o) for o in ops], _ptr(Weq),
                            int(n_t1), int(t2_steps), int(n_t3), int(stride1), int(stride3), float(dt),
                            jl, int(nj), _ptr(R))
    return R


# ---------------------------------------------------------------------------
# spectra, Eqs. (1DIR_Raman), (2DThz_Raman) and (noncorrelation), as plain
# Fourier sums
# ---------------------------------------------------------------------------

def spectrum_1d(R, tau: float):
    """I(omega_k) = omega_k Im{ sum_j tau e^{+i omega_k t_j} R[j] }.

    t_j = j tau, omega_k = 2 pi k / (n tau), k = 0..n-1; rectangle rule with
    weight 1 at t = 0, no window.  Returns (omega, I).
    """
    R = np.asarray(R, dtype=np.float64)
    n = R.size
    j = np.arange(n)
    k = np.arange(n)
    omega = 2.0 * np.pi * k / (n * tau)
    phase = np.exp(1j * 2.0 * np.pi * np.outer(k, j) / n)  # e^{+i omega_k t_j}
    I = omega * np.imag(tau * (phase @ R))
    return omega, I


def spectrum_2d(R, tau1: float, tau2: float):
    """I(omega1, omega2) = Im{ tau1 tau2 sum e^{-i omega1 t1 - i omega2 t2} R(t2, t1) }.

    R has shape (n2, n1) with t1 fastest; the result has the same shape,
    indexed [k2, k1].  Returns (omega1, omega2, I).
    """
    R = np.asarray(R, dtype=np.float64)
    n2, n1 = R.shape
    k1 = np.arange(n1)
    k2 = np.arange(n2)
    E1 = np.exp(-1j * 2.0 * np.pi * np.outer(k1, k1) / n1)  # [k1, j1]
    E2 = np.exp(-1j * 2.0 * np.pi * np.outer(k2, k2) / n2)  # [k2, j2]
    I = np.imag(tau1 * tau2 * (E2 @ R @ E1.T))
    omega1 = 2.0 * np.pi * k1 / (n1 * tau1)
    omega2 = 2.0 * np.pi * k2 / (n2 * tau2)
    return omega1, omega2, I


def spectrum_2dir(R, tau1: float, tau3: float):
    """I(omega3, t2, omega1) = Im{ tau1 tau3 sum e^{-i omega1 t1 + i omega3 t3} R(t3, t1) },
    Eq. (noncorrelation), at the waiting time of R.

    R has shape (n3, n1) with t1 fastest; the result has the same shape,
    indexed [k3, k1].  Returns (omega1, omega3, I).
    """
    R = np.asarray(R, dtype=np.float64)
    n3, n1 = R.shape
    k1 = np.arange(n1)
    k3 = np.arange(n3)
    E1 = np.exp(-1j * 2.0 * np.pi * np.outer(k1, k1) / n1)  # [k1, j1]
    E3 = np.exp(+1j * 2.0 * np.pi * np.outer(k3, k3) / n3)  # [k3, j3]
    I = np.imag(tau1 * tau3 * (E3 @ R @ E1.T))
    omega1 = 2.0 * np.pi * k1 / (n1 * tau1)
    omega3 = 2.0 * np.pi * k3 / (n3 * tau3)
    return omega1, omega3, I
