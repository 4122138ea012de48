"""MI355X (gfx950) solver for the multimode classical hierarchical Fokker-Planck
equations (CHFPE): Python binding of the C ABI in ``include/chfpe.h``.

This module only marshals arguments: every step of the computation runs in
the HIP kernels of ``libchfpe.so``.  PyTorch supplies device memory (the
context workspace) and the stream.  Importing works without a GPU; creating
a ``Solver`` needs the built library and a visible gfx950 device and raises
otherwise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["Params", "Optical", "Solver", "ChfpeError", "lib", "params_from_workload",
           "optical_from_dict", "workspace_bytes", "stream_copy", "stream_mix", "spectrum_1d", "spectrum_2d", "spectrum_2dir",
           "closure_rows", "closure_features", "closure_eval", "closure_grad", "ClosureTrainer",
           "CLOSURE_PARAMS", "LIB_PATH"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchfpe.so")

CHFPE_OK, CHFPE_EINVAL, CHFPE_ENOMEM, CHFPE_EDEVICE, CHFPE_ENONFINITE, CHFPE_ESTATE = 0, -1, -2, -3, -4, -5
CHFPE_FP64, CHFPE_FP32 = 0, 1
CHFPE_BASIS_GRID, CHFPE_BASIS_HERMITE = 0, 1
_CODES = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENONFINITE", -5: "ESTATE"}

_d3 = ctypes.c_double * 3
_d33 = (ctypes.c_double * 3) * 3
_i3 = ctypes.c_int32 * 3


class Params(ctypes.Structure):
    """chfpe_params."""
    _fields_ = [
        ("M", ctypes.c_int32), ("K", ctypes.c_int32),
        ("Nq", _i3), ("Np", _i3), ("Lq", _d3), ("Lp", _d3),
        ("m", _d3), ("omega", _d3), ("g3", _d3), ("g4", _d3),
        ("g2", _d33), ("g21", _d33), ("g12", _d33),
        ("V_LL", _d3), ("V_SL", _d3), ("zeta", _d3), ("gamma", _d3),
        ("beta", ctypes.c_double), ("precision", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("basis", ctypes.c_int32),
    ]


class Optical(ctypes.Structure):
    """chfpe_optical: X(q) = sum lin_s q_s + 1/2 sum quad_ss' q_s q_s'."""
    _fields_ = [("lin", _d3), ("quad", _d33)]


class ChfpeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"chfpe error {code} ({_CODES.get(code, '?')}): {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded libchfpe.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ChfpeError(CHFPE_EDEVICE, f"{LIB_PATH} is missing: run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(Params)
    O = ctypes.POINTER(Optical)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    L.chfpe_workspace_bytes.argtypes = [P]
    L.chfpe_workspace_bytes.restype = ctypes.c_size_t
    L.chfpe_setup.argtypes = [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.chfpe_setup.restype = ctypes.c_int
    L.chfpe_equilibrate.argtypes = [vp, i64, ctypes.c_double]
    L.chfpe_equilibrate.restype = ctypes.c_int
    L.chfpe_propagate.argtypes = [vp, i64, ctypes.c_double]
    L.chfpe_propagate.restype = ctypes.c_int
    L.chfpe_response_1d.argtypes = [vp, O, i64, i32, ctypes.c_double, dp]
    L.chfpe_response_1d.restype = ctypes.c_int
    L.chfpe_response_2d.argtypes = [vp, O, O, O, i64, i64, i32, i32, ctypes.c_double, dp]
    L.chfpe_response_2d.restype = ctypes.c_int
    L.chfpe_response_2d_range.argtypes = [vp, O, O, O, i64, i64, i64, i32, i32, ctypes.c_double, dp]
    L.chfpe_response_2d_range.restype = ctypes.c_int
    L.chfpe_response_3d.argtypes = [vp, O, O, O, O, i64, i64, i64, i32, i32, ctypes.c_double, dp]
    L.chfpe_response_3d.restype = ctypes.c_int
    L.chfpe_state_count.argtypes = [vp]
    L.chfpe_state_count.restype = i64
    L.chfpe_get_state.argtypes = [vp, dp]
    L.chfpe_get_state.restype = ctypes.c_int
    L.chfpe_set_state.argtypes = [vp, dp]
    L.chfpe_set_state.restype = ctypes.c_int
    L.chfpe_use_state_as_equilibrium.argtypes = [vp]
    L.chfpe_use_state_as_equilibrium.restype = ctypes.c_int
    L.chfpe_rhs.argtypes = [vp]
    L.chfpe_rhs.restype = ctypes.c_int
    L.chfpe_perturb.argtypes = [vp, O]
    L.chfpe_perturb.restype = ctypes.c_int
    L.chfpe_observe.argtypes = [vp, O, dp]
    L.chfpe_observe.restype = ctypes.c_int
    L.chfpe_spectrum_1d.argtypes = [dp, i64, ctypes.c_double, dp, dp, vp]
    L.chfpe_spectrum_1d.restype = ctypes.c_int
    L.chfpe_spectrum_2d.argtypes = [dp, i64, i64, ctypes.c_double, ctypes.c_double, dp, vp]
    L.chfpe_spectrum_2d.restype = ctypes.c_int
    L.chfpe_spectrum_2dir.argtypes = [dp, i64, i64, ctypes.c_double, ctypes.c_double, dp, vp]
    L.chfpe_spectrum_2dir.restype = ctypes.c_int
    L.chfpe_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.chfpe_stream_copy.restype = ctypes.c_int
    L.chfpe_stream_mix.argtypes = [vp, vp, vp, vp, i32, ctypes.c_size_t, vp]
    L.chfpe_stream_mix.restype = ctypes.c_int
    L.chfpe_set_kernel_timing.argtypes = [vp, i32]
    L.chfpe_set_kernel_timing.restype = ctypes.c_int
    L.chfpe_kernel_times.argtypes = [vp, i32, ctypes.POINTER(i64), dp, dp, ctypes.POINTER(ctypes.c_char_p)]
    L.chfpe_kernel_times.restype = ctypes.c_int
    L.chfpe_autotune.argtypes = [vp, i32]
    L.chfpe_autotune.restype = ctypes.c_int
    L.chfpe_tile_config.argtypes = [vp, ctypes.POINTER(i32), i32]
    L.chfpe_tile_config.restype = ctypes.c_int
    fp = ctypes.POINTER(ctypes.c_float)
    ip = ctypes.POINTER(i32)
    L.chfpe_closure_rows.argtypes = [P]
    L.chfpe_closure_rows.restype = i32
    L.chfpe_closure_features.argtypes = [P, fp, ip]
    L.chfpe_closure_features.restype = ctypes.c_int
    L.chfpe_closure_moments.argtypes = [vp, dp, dp, dp]
    L.chfpe_closure_moments.restype = ctypes.c_int
    L.chfpe_closure_eval.argtypes = [fp, fp, i32, fp, vp]
    L.chfpe_closure_eval.restype = ctypes.c_int
    L.chfpe_closure_grad.argtypes = [fp, fp, i32, fp, fp, vp]
    L.chfpe_closure_grad.restype = ctypes.c_int
    L.chfpe_closure_train.argtypes = [fp, i32, i32, ip, dp, dp, dp, fp, fp, fp, i32, i32, ctypes.c_float, fp, vp]
    L.chfpe_closure_train.restype = ctypes.c_int
    L.chfpe_set_closure.argtypes = [vp, dp]
    L.chfpe_set_closure.restype = ctypes.c_int
    L.chfpe_last_error.argtypes = [vp]
    L.chfpe_last_error.restype = ctypes.c_char_p
    L.chfpe_destroy.argtypes = [vp]
    L.chfpe_destroy.restype = None
    _lib = L
    return L


def params_from_workload(w: dict, precision=None, batch: int = 0) -> Params:
    """chfpe_params from a workload dict (see ``workloads``); precision
    defaults to the workload's ("f32" -> CHFPE_FP32, else CHFPE_FP64), and
    the p basis to its "basis" entry ("hermite" -> CHFPE_BASIS_HERMITE, Np
    then counting Hermite functions; else the p grid)."""
    if precision is None:
        precision = CHFPE_FP32 if w.get("precision") == "f32" else CHFPE_FP64
    p = Params()
    M = int(w["M"])
    p.M, p.K = M, int(w["K"])
    for s in range(M):
        p.Nq[s], p.Np[s] = int(w["Nq"][s]), int(w["Np"][s])
        p.Lq[s], p.Lp[s] = float(w["Lq"][s]), float(w["Lp"][s])
        p.m[s], p.omega[s] = float(w["m"][s]), float(w["omega"][s])
        p.g3[s], p.g4[s] = float(w["g3"][s]), float(w["g4"][s])
        p.V_LL[s], p.V_SL[s] = float(w["VLL"][s]), float(w["VSL"][s])
        p.zeta[s], p.gamma[s] = float(w["zeta"][s]), float(w["gamma"][s])
        for t in range(M):
            p.g2[s][t] = float(w["g2"][s][t])
            p.g21[s][t] = float(w["g21"][s][t])
            p.g12[s][t] = float(w["g12"][s][t])
    p.beta = float(w["beta"])
    p.precision = int(precision)
    p.batch = int(batch)
    p.basis = CHFPE_BASIS_HERMITE if w.get("basis") == "hermite" else CHFPE_BASIS_GRID
    return p


def optical_from_dict(X: dict) -> Optical:
    o = Optical()
    for s, v in enumerate(X["lin"]):
        o.lin[s] = float(v)
    for s, row in enumerate(X["quad"]):
        for t, v in enumerate(row):
            o.quad[s][t] = float(v)
    return o


def workspace_bytes(p: Params) -> int:
    return int(lib().chfpe_workspace_bytes(ctypes.byref(p)))


def stream_copy(dst, src, nbytes: int, stream=None) -> None:
    """Plain device copy kernel (bandwidth reference); dst/src are torch tensors."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = lib().chfpe_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                 ctypes.c_size_t(nbytes), ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise ChfpeError(rc, "stream copy failed")


def stream_mix(dst, srcs, nbytes: int, stream=None) -> None:
    """Bandwidth reference for read/write mixes: dst = sum of the tensors in
    srcs (0 to 3 of them; FP64 pairs), over nbytes bytes."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    ptr = [ctypes.c_void_p(t.data_ptr()) for t in srcs] + [ctypes.c_void_p(None)] * (3 - len(srcs))
    rc = lib().chfpe_stream_mix(ctypes.c_void_p(dst.data_ptr()), ptr[0], ptr[1], ptr[2], len(srcs),
                                ctypes.c_size_t(nbytes), ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise ChfpeError(rc, "stream mix failed")


def _fptr(a: np.ndarray):
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _iptr(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _lib_check(rc: int):
    if rc != 0:
        raise ChfpeError(rc, lib().chfpe_last_error(None).decode())


CLOSURE_PARAMS = 16 * 32 + 32 + 32 + 1


def closure_rows(p: Params) -> int:
    n = int(lib().chfpe_closure_rows(ctypes.byref(p)))
    if n < 0:
        raise ChfpeError(n, lib().chfpe_last_error(None).decode())
    return n


def closure_features(p: Params):
    """(features rows x 16 float32, axis id of every row)."""
    n = closure_rows(p)
    feat = np.zeros((n, 16), dtype=np.float32)
    axis = np.zeros(n, dtype=np.int32)
    _lib_check(lib().chfpe_closure_features(ctypes.byref(p), _fptr(feat), _iptr(axis)))
    return feat, axis


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def closure_eval(prm, feat, stream=None) -> np.ndarray:
    prm = np.ascontiguousarray(prm, dtype=np.float32)
    feat = np.ascontiguousarray(feat, dtype=np.float32)
    s = np.zeros(feat.shape[0], dtype=np.float32)
    _lib_check(lib().chfpe_closure_eval(_fptr(prm), _fptr(feat), feat.shape[0], _fptr(s), _stream_ptr(stream)))
    return s


def closure_grad(prm, feat, gs, stream=None) -> np.ndarray:
    prm = np.ascontiguousarray(prm, dtype=np.float32)
    feat = np.ascontiguousarray(feat, dtype=np.float32)
    gs = np.ascontiguousarray(gs, dtype=np.float32)
    g = np.zeros(CLOSURE_PARAMS, dtype=np.float32)
    _lib_check(lib().chfpe_closure_grad(_fptr(prm), _fptr(feat), feat.shape[0], _fptr(gs), _fptr(g),
                                        _stream_ptr(stream)))
    return g


class ClosureTrainer:
    """Adam state and parameters of the closure network (FP32 host copies);
    every step runs in chfpe_closure_train."""

    def __init__(self, prm):
        self.prm = np.ascontiguousarray(prm, dtype=np.float32).copy()
        self.m = np.zeros(CLOSURE_PARAMS, dtype=np.float32)
        self.v = np.zeros(CLOSURE_PARAMS, dtype=np.float32)
        self.t = 0

    def train(self, feat, group_start, G, b, ct, n_steps: int, lr: float, stream=None) -> np.ndarray:
        feat = np.ascontiguousarray(feat, dtype=np.float32)
        gst = np.ascontiguousarray(group_start, dtype=np.int32)
        G = np.ascontiguousarray(G, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        ct = np.ascontiguousarray(ct, dtype=np.float64)
        loss = np.zeros(max(1, n_steps), dtype=np.float32)
        _lib_check(lib().chfpe_closure_train(_fptr(feat), feat.shape[0], len(gst) - 1, _iptr(gst), _dptr(G),
                                             _dptr(b), _dptr(ct), _fptr(self.prm), _fptr(self.m), _fptr(self.v),
                                             self.t, int(n_steps), float(lr), _fptr(loss), _stream_ptr(stream)))
        self.t += int(n_steps)
        return loss[:n_steps]


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def spectrum_1d(R, tau: float, stream=None):
    """(omega, I) of Eq. (1DIR_Raman) computed on the device."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    om = np.empty(R.size)
    I = np.empty(R.size)
    rc = lib().chfpe_spectrum_1d(_dptr(R), R.size, float(tau), _dptr(om), _dptr(I), _stream_handle(stream))
    if rc != 0:
        raise ChfpeError(rc, "spectrum_1d failed")
    return om, I


def spectrum_2d(R, tau1: float, tau2: float, stream=None):
    """I(omega1, omega2) of Eq. (2DThz_Raman) on the device; R has shape (n_t2, n_t1)."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    n2, n1 = R.shape
    I = np.empty_like(R)
    rc = lib().chfpe_spectrum_2d(_dptr(R), n1, n2, float(tau1), float(tau2), _dptr(I), _stream_handle(stream))
    if rc != 0:
        raise ChfpeError(rc, "spectrum_2d failed")
    return I


def spectrum_2dir(R, tau1: float, tau3: float, stream=None):
    """I(omega3, t2, omega1) of Eq. (noncorrelation) on the device; R has shape (n_t3, n_t1)."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    n3, n1 = R.shape
    I = np.empty_like(R)
    rc = lib().chfpe_spectrum_2dir(_dptr(R), n1, n3, float(tau1), float(tau3), _dptr(I), _stream_handle(stream))
    if rc != 0:
        raise ChfpeError(rc, "spectrum_2dir failed")
    return I


class Solver:
    """One solver context: workspace allocated by torch on ``device``, work
    issued on a stream of its own (default priority; a non-null stream lets
    the library capture 2D-response waves as HIP graphs).  Calls that return
    host data synchronize that stream; other work on the device can be
    ordered after it with torch.cuda.synchronize() or solver.stream."""

    def __init__(self, params: Params, device: str = "cuda:0"):
        import torch
        L = lib()
        if not torch.cuda.is_available():
            raise ChfpeError(CHFPE_EDEVICE, "no GPU visible to torch")
        self.device = torch.device(device)
        nbytes = workspace_bytes(params)
        if nbytes == 0:
            ctx = ctypes.c_void_p()
            rc = L.chfpe_setup(ctypes.byref(params), None, 0, None, ctypes.byref(ctx))
            raise ChfpeError(rc, L.chfpe_last_error(None).decode())
        with torch.cuda.device(self.device):
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.Stream(self.device)
            # the workspace may be memory that pending work on the current
            # stream still uses: start after it
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._ctx = ctypes.c_void_p()
        rc = L.chfpe_setup(ctypes.byref(params), ctypes.c_void_p(aligned), ctypes.c_size_t(nbytes),
                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._ctx))
        if rc != 0:
            raise ChfpeError(rc, L.chfpe_last_error(None).decode())
        self.params = params
        self._ws_ptr = aligned
        self._ws_bytes = nbytes
        self.count = int(L.chfpe_state_count(self._ctx))

    def rebuild(self):
        """Run chfpe_setup again into the same workspace (tables rebuilt and
        uploaded; the equilibrium is dropped)."""
        L = lib()
        L.chfpe_destroy(self._ctx)
        self._ctx = ctypes.c_void_p()
        rc = L.chfpe_setup(ctypes.byref(self.params), ctypes.c_void_p(self._ws_ptr),
                           ctypes.c_size_t(self._ws_bytes), ctypes.c_void_p(self.stream.cuda_stream),
                           ctypes.byref(self._ctx))
        if rc != 0:
            self._ctx = None
            raise ChfpeError(rc, L.chfpe_last_error(None).decode())

    # -- helpers ---------------------------------------------------------------
    def _check(self, rc: int):
        if rc != 0:
            raise ChfpeError(rc, lib().chfpe_last_error(self._ctx).decode())

    def close(self):
        if getattr(self, "_ctx", None):
            self.stream.synchronize()  # the workspace returns to torch's allocator
            lib().chfpe_destroy(self._ctx)
            self._ctx = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- the C ABI ---------------------------------------------------------------
    def equilibrate(self, n_steps: int, dt: float):
        self._check(lib().chfpe_equilibrate(self._ctx, int(n_steps), float(dt)))

    def propagate(self, n_steps: int, dt: float):
        self._check(lib().chfpe_propagate(self._ctx, int(n_steps), float(dt)))

    def response_1d(self, A: dict, n_t: int, stride: int, dt: float) -> np.ndarray:
        R = np.empty(int(n_t))
        o = optical_from_dict(A)
        self._check(lib().chfpe_response_1d(self._ctx, ctypes.byref(o), int(n_t), int(stride), float(dt),
                                            _dptr(R)))
        return R

    def response_2d(self, A: dict, B: dict, C: dict, n_t1: int, n_t2: int, stride1: int, stride2: int,
                    dt: float) -> np.ndarray:
        R = np.empty((int(n_t2), int(n_t1)))
        oa, ob, oc = optical_from_dict(A), optical_from_dict(B), optical_from_dict(C)
        self._check(lib().chfpe_response_2d(self._ctx, ctypes.byref(oa), ctypes.byref(ob), ctypes.byref(oc),
                                            int(n_t1), int(n_t2), int(stride1), int(stride2), float(dt),
                                            _dptr(R)))
        return R

    def response_2d_range(self, A: dict, B: dict, C: dict, j1_begin: int, j1_end: int, n_t2: int,
                          stride1: int, stride2: int, dt: float) -> np.ndarray:
        R = np.empty((int(n_t2), int(j1_end) - int(j1_begin)))
        oa, ob, oc = optical_from_dict(A), optical_from_dict(B), optical_from_dict(C)
        self._check(lib().chfpe_response_2d_range(self._ctx, ctypes.byref(oa), ctypes.byref(ob), ctypes.byref(oc),
                                                  int(j1_begin), int(j1_end), int(n_t2), int(stride1),
                                                  int(stride2), float(dt), _dptr(R)))
        return R

    def response_3d(self, A: dict, B: dict, C: dict, D: dict, n_t1: int, t2_steps: int, n_t3: int,
                    stride1: int, stride3: int, dt: float) -> np.ndarray:
        """R^(3)[j3, j1] of Eq. (3Dresponse) at t2 = t2_steps * dt; shape (n_t3, n_t1)."""
        R = np.empty((int(n_t3), int(n_t1)))
        ops = [optical_from_dict(X) for X in (A, B, C, D)]
        self._check(lib().chfpe_response_3d(self._ctx, *[ctypes.byref(o) for o in ops], int(n_t1), int(t2_steps),
                                            int(n_t3), int(stride1), int(stride3), float(dt), _dptr(R)))
        return R

    def get_state(self) -> np.ndarray:
        out = np.empty(self.count)
        self._check(lib().chfpe_get_state(self._ctx, _dptr(out)))
        return out

    def set_state(self, W) -> None:
        a = np.ascontiguousarray(W, dtype=np.float64).ravel()
        if a.size != self.count:
            raise ValueError(f"state has {a.size} values, expected {self.count}")
        self._check(lib().chfpe_set_state(self._ctx, _dptr(a)))

    def use_state_as_equilibrium(self):
        self._check(lib().chfpe_use_state_as_equilibrium(self._ctx))

    def rhs(self):
        self._check(lib().chfpe_rhs(self._ctx))

    def perturb(self, X: dict):
        o = optical_from_dict(X)
        self._check(lib().chfpe_perturb(self._ctx, ctypes.byref(o)))

    def observe(self, X: dict) -> float:
        o = optical_from_dict(X)
        v = ctypes.c_double()
        self._check(lib().chfpe_observe(self._ctx, ctypes.byref(o), ctypes.byref(v)))
        return v.value

    def closure_moments(self):
        """chfpe_closure_moments of the current (fine-grid) state:
        (list of G_a, list of b_a, array of (c_a, t_a)) for the 2:1 coarse grid."""
        M = int(self.params.M)
        N = [int(self.params.Nq[s]) // 2 for s in range(M)] + [int(self.params.Np[s]) // 2 for s in range(M)]
        P = [2 * n - 3 for n in N]  # skew entries on two off-diagonals
        G = np.zeros(sum(p * p for p in P))
        b = np.zeros(sum(P))
        ct = np.zeros(2 * 2 * M)
        self._check(lib().chfpe_closure_moments(self._ctx, _dptr(G), _dptr(b), _dptr(ct)))
        Gs, bs, go, bo = [], [], 0, 0
        for p in P:
            Gs.append(G[go:go + p * p].reshape(p, p))
            bs.append(b[bo:bo + p])
            go += p * p
            bo += p
        return Gs, bs, ct.reshape(2 * M, 2)

    def set_closure(self, s):
        """chfpe_set_closure (None restores the plain scheme)."""
        if s is None:
            self._check(lib().chfpe_set_closure(self._ctx, None))
            return
        a = np.ascontiguousarray(s, dtype=np.float64)
        self._check(lib().chfpe_set_closure(self._ctx, _dptr(a)))

    def set_kernel_timing(self, every: int):
        self._check(lib().chfpe_set_kernel_timing(self._ctx, int(every)))

    def autotune(self, n_steps: int = 2) -> dict:
        """chfpe_autotune; returns the tile shapes then in use."""
        self._check(lib().chfpe_autotune(self._ctx, int(n_steps)))
        return self.tile_config()

    def tile_config(self) -> dict:
        """chfpe_tile_config as a dict."""
        out = (ctypes.c_int32 * 15)()
        k = lib().chfpe_tile_config(self._ctx, out, 15)
        if k < 0:
            self._check(k)
        keys = ("pblock_blocks_per_task", "pblock_split_lines", "pblock_threads", "qpass_positions",
                "qpass_acc_positions", "qpass_threads", "request_pblock_blocks",
                "request_split", "request_qpass_positions", "pblock_run", "request_pblock_run", "pcube",
                "pcube_stream", "hcube_chunk", "hcube_ktile")
        return {keys[i]: int(out[i]) for i in range(k)}

    def kernel_times(self) -> dict:
        """{kind: (timed launches, mean ms, mean algorithmic bytes)}."""
        n = 32
        counts = (ctypes.c_int64 * n)()
        means = (ctypes.c_double * n)()
        mbytes = (ctypes.c_double * n)()
        names = (ctypes.c_char_p * n)()
        k = lib().chfpe_kernel_times(self._ctx, n, counts, means, mbytes, names)
        if k < 0:
            self._check(k)
        return {names[i].decode(): (int(counts[i]), float(means[i]), float(mbytes[i])) for i in range(k)}
