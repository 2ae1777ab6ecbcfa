"""FP64 CPU oracle of the grand-potential phase-field time step.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library in ``paper_1506_01684_amd``; the two meet only in the
seeded input generators of ``pfinputs``.

Thin ctypes marshalling over ``pf_oracle.c`` (which cites the paper's
equations: Sec. 2 Eqs. (1)-(4), Algorithm 1).  Arrays are numpy float64,
C-contiguous, shaped ``phi[4, nz, ny, nx]`` and ``mu[2, nz, ny, nx]``.
Parameters are the plain dicts produced by ``pfinputs``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_D = C.c_double
_PD = C.POINTER(C.c_double)


class OrcGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("dx", _D)]


class OrcParams(C.Structure):
    _fields_ = [
        ("eps", _D), ("tau", _D * 4), ("gamma", (_D * 4) * 4), ("gamma3", _D),
        ("delta", (_D * 4) * 4), ("chi0", (_D * 2) * 4), ("chi1", (_D * 2) * 4),
        ("c0", (_D * 2) * 4), ("c1", (_D * 2) * 4), ("w0", _D * 4), ("w1", _D * 4),
        ("D", _D * 4), ("TE", _D), ("T0", _D), ("G", _D), ("v", _D), ("zoff", _D),
        ("dt", _D), ("antitrapping", C.c_int32), ("mu_frozen", C.c_int32),
        ("top_dirichlet", C.c_int32), ("pad", C.c_int32), ("mu_top", _D * 2),
    ]


class OrcDiag(C.Structure):
    _fields_ = [
        ("sum_c", _D * 2), ("sum_phi", _D * 4), ("max_simplex_dev", _D),
        ("phi_min", _D), ("phi_max", _D), ("nonfinite", C.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = C.CDLL(path)
        G, P = C.POINTER(OrcGrid), C.POINTER(OrcParams)
        i = C.c_int
        sig = {
            "orc_splitmix64_next": (C.c_uint64, [C.POINTER(C.c_uint64)]),
            "orc_temperature": (_D, [P, G, _D, _D]),
            "orc_stability_bound": (_D, [P, G]),
            "orc_project": (None, [_PD, _PD]),
            "orc_aniso_X": (None, [_PD, _D, _PD]),
            "orc_phi_face": (None, [G, P, _PD, i, i, i, i, _PD, _PD]),
            "orc_phi_rhs": (None, [G, P, _D, _PD, _PD, i, i, i, _PD]),
            "orc_phi_cell": (None, [G, P, _D, _PD, _PD, i, i, i, _PD]),
            "orc_mu_face": (None, [G, P, _D, _PD, _PD, _PD, i, i, i, i, _PD, _PD]),
            "orc_mu_cell": (None, [G, P, _D, _D, _PD, _PD, _PD, i, i, i, _PD]),
            "orc_phi_sweep": (None, [G, P, _D, _PD, _PD, _PD, i]),
            "orc_mu_sweep": (None, [G, P, _D, _D, _PD, _PD, _PD, _PD, i]),
            "orc_run": (i, [G, P, C.c_int64, C.c_int64, _PD, _PD, i]),
            "orc_window_shift": (i, [G, C.c_int32, _PD, _PD, _PD]),
            "orc_run_window": (i, [G, P, C.c_int64, C.c_int64, C.c_int32, _PD,
                                   C.POINTER(C.c_int64), _PD, _PD, i]),
            "orc_init_voronoi": (None, [G, C.c_uint64, C.c_int32, C.c_int32, _PD, _PD, _PD]),
            "orc_diagnostics": (None, [G, P, _D, _PD, _PD, C.POINTER(OrcDiag)]),
            "orc_mesh_phase": (C.c_int64, [G, _PD, C.c_int32, _D, C.POINTER(C.c_float),
                                          C.c_int64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# ------------------------------------------------------------------ helpers

def make_params(p: dict) -> OrcParams:
    s = OrcParams()
    s.eps = p["eps"]
    s.gamma3 = p["gamma3"]
    for a in range(4):
        s.tau[a] = p["tau"][a]
        s.w0[a] = p["w0"][a]
        s.w1[a] = p["w1"][a]
        s.D[a] = p["D"][a]
        for b in range(4):
            s.gamma[a][b] = p["gamma"][a][b]
            s.delta[a][b] = p["delta"][a][b]
        for q in range(2):
            s.chi0[a][q] = p["chi0"][a][q]
            s.chi1[a][q] = p["chi1"][a][q]
            s.c0[a][q] = p["c0"][a][q]
            s.c1[a][q] = p["c1"][a][q]
    for k in ("TE", "T0", "G", "v", "zoff", "dt"):
        setattr(s, k, p[k])
    s.antitrapping = int(p.get("antitrapping", 1))
    s.mu_frozen = int(p.get("mu_frozen", 0))
    s.top_dirichlet = int(p.get("top_bc", 0))
    fill = p.get("mu_fill", (0.0, 0.0))
    s.mu_top[0], s.mu_top[1] = float(fill[0]), float(fill[1])
    return s


def make_grid(shape, dx: float = 1.0) -> OrcGrid:
    """shape = (nz, ny, nx)."""
    nz, ny, nx = shape
    return OrcGrid(nx, ny, nz, dx)


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_PD)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _shape_of(phi: np.ndarray):
    assert phi.ndim == 4 and phi.shape[0] == 4
    return phi.shape[1:]


# --------------------------------------------------------------- functions

def splitmix64(seed: int, count: int) -> list[int]:
    st = C.c_uint64(seed)
    return [lib().orc_splitmix64_next(C.byref(st)) for _ in range(count)]


def temperature(p: dict, shape, zc: float, t: float, dx: float = 1.0) -> float:
    return lib().orc_temperature(C.byref(make_params(p)), C.byref(make_grid(shape, dx)), zc, t)


def stability_bound(p: dict, shape, dx: float = 1.0) -> float:
    return lib().orc_stability_bound(C.byref(make_params(p)), C.byref(make_grid(shape, dx)))


def default_dt(p: dict, shape, dx: float = 1.0) -> float:
    return 0.25 * stability_bound(p, shape, dx)


def project(y) -> np.ndarray:
    y = _f64(y).reshape(4)
    x = np.empty(4)
    lib().orc_project(_ptr(y), _ptr(x))
    return x


def aniso_X(q, delta: float) -> np.ndarray:
    q = _f64(q).reshape(3)
    X = np.empty(3)
    lib().orc_aniso_X(_ptr(q), float(delta), _ptr(X))
    return X


def phi_face(p, phi, i, j, k, d, dx=1.0):
    phi = _f64(phi)
    F, S = np.empty(4), np.empty(4)
    lib().orc_phi_face(C.byref(make_grid(_shape_of(phi), dx)), C.byref(make_params(p)),
                       _ptr(phi), i, j, k, d, _ptr(F), _ptr(S))
    return F, S


def phi_rhs(p, phi, mu, t, i, j, k, dx=1.0):
    phi, mu = _f64(phi), _f64(mu)
    r = np.empty(4)
    lib().orc_phi_rhs(C.byref(make_grid(_shape_of(phi), dx)), C.byref(make_params(p)), t,
                      _ptr(phi), _ptr(mu), i, j, k, _ptr(r))
    return r


def phi_cell(p, phi, mu, t, i, j, k, dx=1.0):
    phi, mu = _f64(phi), _f64(mu)
    r = np.empty(4)
    lib().orc_phi_cell(C.byref(make_grid(_shape_of(phi), dx)), C.byref(make_params(p)), t,
                       _ptr(phi), _ptr(mu), i, j, k, _ptr(r))
    return r


def mu_face(p, phi0, phi1, mu, t, i, j, k, d, dx=1.0):
    phi0, phi1, mu = _f64(phi0), _f64(phi1), _f64(mu)
    P, J = np.empty(2), np.empty(2)
    lib().orc_mu_face(C.byref(make_grid(_shape_of(phi0), dx)), C.byref(make_params(p)), t,
                      _ptr(phi0), _ptr(phi1), _ptr(mu), i, j, k, d, _ptr(P), _ptr(J))
    return P, J


def mu_cell(p, phi0, phi1, mu, t0, t1, i, j, k, dx=1.0):
    phi0, phi1, mu = _f64(phi0), _f64(phi1), _f64(mu)
    r = np.empty(2)
    lib().orc_mu_cell(C.byref(make_grid(_shape_of(phi0), dx)), C.byref(make_params(p)), t0, t1,
                      _ptr(phi0), _ptr(phi1), _ptr(mu), i, j, k, _ptr(r))
    return r


def phi_sweep(p, phi, mu, t, nthreads=None, dx=1.0):
    phi, mu = _f64(phi), _f64(mu)
    out = np.empty_like(phi)
    lib().orc_phi_sweep(C.byref(make_grid(_shape_of(phi), dx)), C.byref(make_params(p)), t,
                        _ptr(phi), _ptr(mu), _ptr(out), nthreads or default_threads())
    return out


def mu_sweep(p, phi0, phi1, mu, t0, t1, nthreads=None, dx=1.0):
    phi0, phi1, mu = _f64(phi0), _f64(phi1), _f64(mu)
    out = np.empty_like(mu)
    lib().orc_mu_sweep(C.byref(make_grid(_shape_of(phi0), dx)), C.byref(make_params(p)), t0, t1,
                       _ptr(phi0), _ptr(phi1), _ptr(mu), _ptr(out), nthreads or default_threads())
    return out


def run(p, phi, mu, nsteps, step0=0, nthreads=None, dx=1.0):
    """nsteps time steps (Algorithm 1) from step index step0; returns copies."""
    phi, mu = _f64(phi).copy(), _f64(mu).copy()
    rc = lib().orc_run(C.byref(make_grid(_shape_of(phi), dx)), C.byref(make_params(p)),
                       int(step0), int(nsteps), _ptr(phi), _ptr(mu),
                       nthreads or default_threads())
    if rc != 0:
        raise MemoryError("oracle run: allocation failed")
    return phi, mu


def window_shift(phi, mu, zw, mu_fill=(0.0, 0.0), dx=1.0):
    """One moving-window check and shift; returns (phi, mu, shifted)."""
    phi, mu = _f64(phi).copy(), _f64(mu).copy()
    m = _f64(mu_fill).reshape(2)
    r = lib().orc_window_shift(C.byref(make_grid(_shape_of(phi), dx)), int(zw), _ptr(m),
                               _ptr(phi), _ptr(mu))
    return phi, mu, bool(r)


def run_window(p, phi, mu, nsteps, zw, mu_fill=(0.0, 0.0), step0=0, shifts=0, nthreads=None,
               dx=1.0):
    """nsteps steps with a moving window at plane zw; returns (phi, mu, shifts)."""
    phi, mu = _f64(phi).copy(), _f64(mu).copy()
    m = _f64(mu_fill).reshape(2)
    sh = C.c_int64(int(shifts))
    rc = lib().orc_run_window(C.byref(make_grid(_shape_of(phi), dx)), C.byref(make_params(p)),
                              int(step0), int(nsteps), int(zw), _ptr(m), C.byref(sh),
                              _ptr(phi), _ptr(mu), nthreads or default_threads())
    if rc != 0:
        raise MemoryError("oracle run: allocation failed")
    return phi, mu, sh.value


def mesh_phase(phi, phase: int, iso: float = 0.5) -> np.ndarray:
    """Marching-cubes mesh of phi[phase] = iso (output path, Sec. 3.2; rules
    in pf_oracle_mesh.c): float32 array [ntri, 3, 3] of triangle vertices in
    cell-index units, in cube order, normals out of the phase.  phi may be
    [4, nz, ny, nx] (or any [k, nz, ny, nx] with phase < k)."""
    phi = _f64(phi)
    g = make_grid(_shape_of(phi))
    n = lib().orc_mesh_phase(C.byref(g), _ptr(phi), int(phase), float(iso), None, 0)
    out = np.empty((max(n, 1), 3, 3), np.float32)
    lib().orc_mesh_phase(C.byref(g), _ptr(phi), int(phase), float(iso),
                         out.ctypes.data_as(C.POINTER(C.c_float)), int(n))
    return out[:n]


def init_voronoi(shape, seed, nseeds, solid_height, mu_init=(0.0, 0.0), dx=1.0):
    nz, ny, nx = shape
    phi = np.empty((4, nz, ny, nx))
    mu = np.empty((2, nz, ny, nx))
    m = _f64(mu_init).reshape(2)
    lib().orc_init_voronoi(C.byref(make_grid(shape, dx)), C.c_uint64(seed), int(nseeds),
                           int(solid_height), _ptr(m), _ptr(phi), _ptr(mu))
    return phi, mu


def diagnostics(p, phi, mu, t, dx=1.0) -> dict:
    phi, mu = _f64(phi), _f64(mu)
    d = OrcDiag()
    lib().orc_diagnostics(C.byref(make_grid(_shape_of(phi), dx)), C.byref(make_params(p)), t,
                          _ptr(phi), _ptr(mu), C.byref(d))
    return {
        "sum_c": list(d.sum_c), "sum_phi": list(d.sum_phi),
        "max_simplex_dev": d.max_simplex_dev, "phi_min": d.phi_min,
        "phi_max": d.phi_max, "nonfinite": d.nonfinite,
    }
