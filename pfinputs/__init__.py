"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds parameter sets, workload recipes and random test states.
It contains none of the model's arithmetic: no fluxes, no projection, no
stability bound.  Both the oracle and the HIP library receive what it
produces as plain inputs.

The paper's production parameters (Ag-Al-Cu Calphad fits) are not available,
so the parameter set P0 below is synthetic: four phases (three solids S1..S3
and the liquid, index 3), two chemical potentials, nondimensional units with
the eutectic temperature TE = 1 and mu_E = 0 at the four-phase point.
"""
from __future__ import annotations

import copy
import math

import numpy as np

DEFAULT_SEED = 42
LIQ = 3
MASK64 = (1 << 64) - 1


# ------------------------------------------------------------- generators

class SplitMix64:
    """SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) for drawing workload
    shapes; u() = (next >> 11) * 2**-53 in [0, 1)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def u(self) -> float:
        return (self.next() >> 11) * 2.0 ** -53


# ------------------------------------------------------------- parameters

def p0_params(*, solid_height: int, G: float = 1e-3, v: float = 0.01,
              delta_sl: float = 0.0, eps: float = 4.0, TE: float = 1.0,
              dt: float = 0.0, chi1: float = 0.0, gamma3: float = 10.0,
              antitrapping: int = 1, mu_frozen: int = 0) -> dict:
    """Synthetic parameter set P0.

    gamma_ab = 1, tau = 1, eps = 4; diagonal susceptibility 1, 2, 3, 1.5 per
    phase; diffusivity 1e-3 in the solids and 1 in the liquid; solids favoured
    below TE through omega_bar = (T - TE); offsets c0 typical of a ternary
    eutectic; T0 = TE - G * solid_height puts the initial front at TE.
    ``dt <= 0`` asks the library for a quarter of its stability bound.
    """
    chi0 = [[1.0, 1.0], [2.0, 2.0], [3.0, 3.0], [1.5, 1.5]]
    gamma = [[0.0 if a == b else 1.0 for b in range(4)] for a in range(4)]
    delta = [[0.0] * 4 for _ in range(4)]
    for a in range(3):
        delta[a][LIQ] = delta[LIQ][a] = delta_sl
    return {
        "eps": eps,
        "tau": [1.0, 1.0, 1.0, 1.0],
        "gamma": gamma,
        "gamma3": gamma3,
        "delta": delta,
        "chi0": chi0,
        "chi1": [[chi1, chi1] for _ in range(4)],
        "c0": [[0.80, 0.10], [0.10, 0.80], [0.10, 0.10], [1.0 / 3.0, 1.0 / 3.0]],
        "c1": [[0.0, 0.0], [0.0, 0.0], [0.0, 0.0], [0.10, -0.10]],
        "w0": [0.0, 0.0, 0.0, 0.0],
        "w1": [1.0, 1.0, 1.0, 0.0],
        "D": [1e-3, 1e-3, 1e-3, 1.0],
        "TE": TE,
        "T0": TE - G * solid_height,
        "G": G,
        "v": v,
        "zoff": 0.0,
        "dt": dt,
        "antitrapping": antitrapping,
        "mu_frozen": mu_frozen,
    }


def with_dt(p: dict, dt: float) -> dict:
    q = copy.deepcopy(p)
    q["dt"] = float(dt)
    return q


# ------------------------------------------------------------- workloads

def workload(name: str) -> dict:
    """Single-domain workloads: shape (nz, ny, nx), precision, seeding, params.

    c1  32x32x64 FP64, 12 seeds, 16 solid layers, 100 steps (correctness).
    c2  256x256x512 FP64, 64 seeds, 128 solid layers, 1000 steps.
    c3  512x512x1024 FP32 bulk, 96 seeds, 256 solid layers, cubic anisotropy
        0.05 on solid-liquid pairs, 1000 steps.
    """
    if name == "c1":
        nx, ny, nz, seeds, prec, steps, dsl = 32, 32, 64, 12, "fp64", 100, 0.0
    elif name == "c2":
        nx, ny, nz, seeds, prec, steps, dsl = 256, 256, 512, 64, "fp64", 1000, 0.0
    elif name == "c3":
        nx, ny, nz, seeds, prec, steps, dsl = 512, 512, 1024, 96, "fp32", 1000, 0.05
    else:
        raise KeyError(name)
    hs = nz // 4
    return {
        "name": name, "shape": (nz, ny, nx), "prec": prec, "nseeds": seeds,
        "solid_height": hs, "seed": DEFAULT_SEED, "steps": steps,
        "params": p0_params(solid_height=hs, delta_sl=dsl),
    }


def pack_workloads(count: int = 64, seed: int = DEFAULT_SEED) -> list[dict]:
    """Uneven independent domains: lateral L in [32,192], height in [64,384],
    v in [0.005,0.02], G in [5e-4,2e-3]; FP32; seed per domain."""
    r = SplitMix64(seed)
    out = []
    for d in range(count):
        L = 32 + int(161 * r.u())
        nz = 64 + int(321 * r.u())
        v = 0.005 + 0.015 * r.u()
        G = 5e-4 + 1.5e-3 * r.u()
        dseed = r.next()
        nseeds = max(12, round(L * L / 1024))
        hs = nz // 4
        out.append({
            "name": f"pack{d}", "shape": (nz, L, L), "prec": "fp32",
            "nseeds": nseeds, "solid_height": hs, "seed": dseed,
            "params": p0_params(solid_height=hs, G=G, v=v),
        })
    return out


def serving_trace(count: int = 128, rate: float = 20.0, seed: int = DEFAULT_SEED,
                  lateral=(64, 384), steps=(200, 5000)) -> list[dict]:
    """Poisson arrivals of solves: lateral L in [64,384], Nz = 2L,
    steps in [200,5000], FP32 or FP64 with probability 1/2 each."""
    r = SplitMix64(seed)
    t = 0.0
    out = []
    lo, hi = lateral
    slo, shi = steps
    for q in range(count):
        t += -math.log(1.0 - r.u()) / rate
        L = lo + int((hi - lo + 1) * r.u())
        nst = slo + int((shi - slo + 1) * r.u())
        prec = "fp32" if r.u() < 0.5 else "fp64"
        dseed = r.next()
        nz = 2 * L
        hs = nz // 4
        out.append({
            "id": q, "arrival": t, "shape": (nz, L, L), "prec": prec,
            "steps": nst, "nseeds": max(12, round(L * L / 1024)),
            "solid_height": hs, "seed": dseed,
            "params": p0_params(solid_height=hs),
        })
    return out


# ------------------------------------------------------------- test states

def random_state(shape, seed: int, *, interior: bool = True, mu_scale: float = 0.05,
                 spread: float = 1.0):
    """Random phi on the Gibbs simplex (strictly inside when interior=True)
    and random mu, as float64 arrays phi[4,nz,ny,nx], mu[2,nz,ny,nx]."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    w = rng.random((4, nz, ny, nx)) ** spread
    if interior:
        w = w + 0.05
    phi = w / w.sum(axis=0, keepdims=True)
    mu = mu_scale * (2.0 * rng.random((2, nz, ny, nx)) - 1.0)
    return phi, mu


def smooth_interface_state(shape, seed: int, *, width: float = 6.0):
    """Smooth solid/liquid state: a wavy front with three solid lamellae
    below it, so every term of the step (gradients, anti-trapping, driving
    force) is active on many faces."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z = np.arange(nz)[:, None, None] + 0.5
    y = np.arange(ny)[None, :, None] + 0.5
    x = np.arange(nx)[None, None, :] + 0.5
    kx, ky = 2 * np.pi / nx, 2 * np.pi / ny
    ph = rng.random(4) * 2 * np.pi
    front = nz * 0.4 + 0.12 * nz * np.sin(kx * x + ph[0]) * np.cos(ky * y + ph[1])
    solid = 0.5 * (1.0 - np.tanh((z - front) / width))
    ang = (np.sin(kx * x + ph[2]) + np.cos(ky * y + ph[3]) + 2.0) / 4.0  # in [0,1]
    s = np.stack([np.exp(-((ang - c) ** 2) / 0.02) for c in (0.2, 0.5, 0.8)])
    s = s / s.sum(axis=0, keepdims=True)
    phi = np.empty((4, nz, ny, nx))
    phi[:3] = solid[None] * s
    phi[3] = 1.0 - solid
    phi = np.broadcast_to(phi, (4, nz, ny, nx)).copy()
    phi = np.maximum(phi, 0.0)
    phi /= phi.sum(axis=0, keepdims=True)
    mu = 0.02 * np.stack([np.sin(kx * x + 0.3 * z) + 0 * y, np.cos(ky * y - 0.2 * z) + 0 * x])
    mu = np.broadcast_to(mu, (2, nz, ny, nx)).copy()
    return phi, mu
