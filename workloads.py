"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds parameter sets and seeded array generators only; it holds
none of the method's arithmetic (no grids, no derivatives, no potentials).
Both the CPU oracle (``oracle/``) and the HIP library's Python binding take
their inputs from here and convert them to their own structures.

Parameter sets follow the model of the paper (multimode anharmonic Brownian
oscillators, Sec. II A; hierarchy Sec. II B; optical operators Sec. II C),
with k_B = 1 and every mass 1.  Readings applied where the workload
descriptions are terse (each one is listed in the design doc):

* grid boxes are the one-mode box q, p in [-6, 6] expressed in each mode's
  thermal units: q_s in [-6/omega_s, 6/omega_s], p_s in [-6, 6];
* every grid is uniform and cell-centred (h = 2L/N);
* modes without explicit on-site anharmonicity take the cubic -0.15 and
  quartic 0.02 of the one- and two-mode workloads, and the coupling
  V_s(q) = 1.0 q + 0.3 q^2/2 with beta = 2;
* "q_i^2 q_j 0.02" means g_{s^2 s'} = g_{s s'^2} = 0.02 for every pair;
* mu = sum_s (q_s + 0.1 q_s^2)  ->  mu_s = 1, mu_ss = 0.2 (factor 1/2! in
  the expansion of the dipole); Pi = sum_s q_s + 0.05 sum_{s<s'} q_s q_s'
  ->  Pi_s = 1, Pi_ss' = 0.05 for s != s'.
"""
from __future__ import annotations

import copy
import numpy as np

__all__ = ["WORKLOADS", "workload", "optical", "smooth_state", "noise_state",
           "draw_perturbed", "state_shape"]


def _base(M: int, N: int, K: int) -> dict:
    omegas = [1.0, 1.6, 2.2][:M]
    w = {
        "M": M, "K": K,
        "Nq": [N] * M, "Np": [N] * M,
        "Lq": [6.0 / om for om in omegas], "Lp": [6.0] * M,
        "m": [1.0] * M, "omega": list(omegas),
        "g3": [-0.15] * M, "g4": [0.02] * M,
        "g2": [[0.0] * M for _ in range(M)],
        "g21": [[0.0] * M for _ in range(M)],
        "g12": [[0.0] * M for _ in range(M)],
        "VLL": [1.0] * M, "VSL": [0.3] * M,
        "zeta": [0.3] * M, "gamma": [1.0] * M,
        "beta": 2.0,
        "dt": 0.005, "eq_steps": 4000,
    }
    return w


def _dipole(M: int) -> dict:
    quad = [[0.0] * M for _ in range(M)]
    for s in range(M):
        quad[s][s] = 0.2
    return {"lin": [1.0] * M, "quad": quad}


def _polarizability(M: int) -> dict:
    quad = [[0.05 if s != t else 0.0 for t in range(M)] for s in range(M)]
    return {"lin": [1.0] * M, "quad": quad}


def _make_workloads() -> dict:
    out = {}

    # One mode, 48 x 48 (q, p) grid on [-6, 6]^2, depth 3, 1D linear absorption.
    w = _base(1, 48, 3)
    w.update(kind="1d", n_t=4000, stride=1, A=_dipole(1), precision="f64")
    out["one_mode_48"] = w

    # Two modes, 32^4 grid, bilinear coupling 0.05, depth 3, 2D THz-Raman
    # (THz-Raman-THz ordering) over 64 t1 x 256 t2 samples.
    w = _base(2, 32, 3)
    w["g2"][0][1] = 0.05
    w.update(kind="2d", n_t1=64, n_t2=256, stride1=1, stride2=1,
             A=_dipole(2), B=_polarizability(2), C=_dipole(2), precision="f64")
    out["two_mode_32"] = w

    # Three modes, 24^6 grid, pairwise bilinear 0.05 and cubic 0.02 couplings,
    # depth 2 (10 elements), 2D THz-Raman 64 x 256.
    w = _base(3, 24, 2)
    for s in range(3):
        for t in range(s + 1, 3):
            w["g2"][s][t] = 0.05
            w["g21"][s][t] = 0.02
            w["g12"][s][t] = 0.02
    w.update(kind="2d", n_t1=64, n_t2=256, stride1=1, stride2=1,
             A=_dipole(3), B=_polarizability(3), C=_dipole(3), precision="f64")
    out["three_mode_24"] = w

    # Same model on a 16^6 grid, all 128 t1 branches, FP32 propagated state.
    w = copy.deepcopy(out["three_mode_24"])
    w["Nq"] = [16] * 3
    w["Np"] = [16] * 3
    w.update(n_t1=128, precision="f32")
    out["three_mode_16"] = w

    # Same model on a coarse 12^6 grid (learned-closure workload).
    w = copy.deepcopy(out["three_mode_24"])
    w["Nq"] = [12] * 3
    w["Np"] = [12] * 3
    w.update(precision="f32")
    out["three_mode_12"] = w

    # The three-mode model with the paper's own p discretisation (Hermite
    # functions, Sec. III A): the 24^3 q grid and 12 Hermite functions per
    # mode (Np counts them; Lp is not used).
    w = copy.deepcopy(out["three_mode_24"])
    w["Np"] = [12] * 3
    w.update(basis="hermite")
    out["three_mode_24_hermite"] = w

    # The two-mode model in the Hermite basis: 32^2 q grid, 16 functions per mode.
    w = copy.deepcopy(out["two_mode_32"])
    w["Np"] = [16] * 2
    w.update(basis="hermite")
    out["two_mode_32_hermite"] = w
    return out


WORKLOADS = _make_workloads()


def workload(name: str, **overrides) -> dict:
    """A deep copy of a named workload with optional field overrides."""
    w = copy.deepcopy(WORKLOADS[name])
    for k, v in overrides.items():
        w[k] = copy.deepcopy(v)
    return w


def optical(M: int, lin=None, quad=None) -> dict:
    """An optical operator X(q) = sum_s lin_s q_s + 1/2 sum_ss' quad_ss' q_s q_s'."""
    lin = [0.0] * M if lin is None else list(lin)
    quad = [[0.0] * M for _ in range(M)] if quad is None else [list(r) for r in quad]
    return {"lin": lin, "quad": quad}


def n_elements(M: int, K: int) -> int:
    """Number of multi-indices n in N^M with |n| <= K (a counting fact only)."""
    from math import comb
    return comb(M + K, K)


def state_shape(w: dict) -> tuple:
    """Shape of a state array: (elements, Nq_1..Nq_M, Np_1..Np_M)."""
    return (n_elements(w["M"], w["K"]),) + tuple(w["Nq"]) + tuple(w["Np"])


def smooth_state(w: dict, seed: int, dtype=np.float64) -> np.ndarray:
    """A seeded, smooth, separable-sum array in index space.

    Each element is a sum of three separable products of low-frequency
    cosines in the normalised index u = (i + 1/2)/N, each times a bump
    sin(pi u)^2 that vanishes towards the box edges.  Pure index-space
    construction: no physical coordinate enters.
    """
    rng = np.random.default_rng(seed)
    shape = state_shape(w)
    out = np.zeros(shape, dtype=np.float64)
    ndim = len(shape) - 1
    for e in range(shape[0]):
        for _ in range(3):
            amp = rng.normal()
            term = np.array(amp)
            for d in range(ndim):
                n = shape[1 + d]
                u = (np.arange(n) + 0.5) / n
                f = rng.uniform(0.5, 3.0)
                ph = rng.uniform(0, 2 * np.pi)
                v = np.cos(np.pi * f * u + ph) * np.sin(np.pi * u) ** 2
                term = np.multiply.outer(term, v)
            out[e] += term
    return out.astype(dtype)


def noise_state(w: dict, seed: int, dtype=np.float64) -> np.ndarray:
    """Seeded i.i.d. N(0, 1) values of the state's shape."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(state_shape(w)).astype(dtype)


def draw_perturbed(w: dict, seed: int, rel: float = 0.2) -> dict:
    """A copy of ``w`` with every scalar model parameter scaled by U(1-rel, 1+rel).

    Grids, depth, time step and optical operators are left unchanged.
    """
    rng = np.random.default_rng(seed)
    out = copy.deepcopy(w)
    for key in ("m", "omega", "g3", "g4", "VLL", "VSL", "zeta", "gamma"):
        out[key] = [x * rng.uniform(1 - rel, 1 + rel) for x in out[key]]
    for key in ("g2", "g21", "g12"):
        out[key] = [[x * rng.uniform(1 - rel, 1 + rel) for x in row] for row in out[key]]
    out["beta"] = out["beta"] * rng.uniform(1 - rel, 1 + rel)
    return out


def response_types(w: dict) -> dict:
    """Operator triples (A, B, C) of the second-order responses of Sec. II C:
    the three 2D THz-Raman orderings Raman-THz-THz (A = Pi), THz-Raman-THz
    (B = Pi) and THz-THz-Raman (C = Pi), and the all-dipole second-order
    (THz/IR) response TTT; operators other than Pi are the dipole mu."""
    M = int(w["M"])
    mu, pi = _dipole(M), _polarizability(M)
    return {"RTT": (pi, mu, mu), "TRT": (mu, pi, mu), "TTR": (mu, mu, pi), "TTT": (mu, mu, mu)}
