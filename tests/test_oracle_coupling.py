"""Pins of the oracle's diagnostics, of its anisotropic gradient-energy path
end to end, and of the temperature coupling of the phi equation.

  - Diagnostics: every field of the oracle's diagnostics against its
    definition written with numpy, on a crafted state with off-simplex
    cells, and on one with NaN and Inf cells.
  - Anisotropy (Sec. 3.3, sine-shaped interface profile; Sec. 2 Eq. (2),
    gradient term): with the cubic form ac(q) = 1 - delta (3 - 4 sum q_i^4),
    a flat two-phase interface whose normal lies along a lattice axis has
    ac = 1 + delta, and one whose normal lies along (1,1,0) has
    ac = 1 - delta.  The gradient energy is then the isotropic one scaled by
    ac^2, and the stationary profile is 1/2 - 1/2 sin(k d) with
    k = 4 / (pi eps ac) (width pi^2 eps ac / 4), d the distance from the
    interface.
  - Temperature (Sec. 2, frozen temperature T(z,t) = T0 + G(z - v t)): in a
    gradient, a flat front with mu frozen comes to rest at the T_E isotherm
    from either side; and the phi step of time level n uses T(z, t_n), the
    old time level of the explicit Euler step.

The last test compiles copies of the oracle with a planted slip (the
temperature of the phi equation taken at t_{n+1} or half a cell off, the
sign of the anisotropy flipped, one factor ac dropped) and checks that
these pins reject each of them.
"""
import ctypes as C
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
import pfinputs
from tests import modelref

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_DIR = os.path.join(os.path.dirname(HERE), "oracle")


def _params(**kw):
    hs = kw.pop("solid_height", 8)
    return pfinputs.p0_params(solid_height=hs, **kw)


def _oracle_run(phi, mu, p, nsteps, step0=0):
    return oracle.run(p, phi, mu, nsteps, step0=step0, nthreads=1)


# ------------------------------------------------------------- diagnostics

def _diag_state():
    shape = (5, 4, 6)
    p = _params(G=4e-3, v=0.3, chi1=0.4)
    p["c1"][1][0] = 0.05
    phi, mu = pfinputs.random_state(shape, 31, mu_scale=0.2)
    phi[:, 1, 2, 3] *= 1.01          # off the simplex, sum 1.01
    phi[:, 3, 0, 0] = (0.7, 0.4, -0.05, -0.02)  # negative entries, sum 1.03
    phi[:, 4, 3, 5] = (0.2, 0.2, 0.2, 0.3)      # sum 0.9
    return p, phi, mu


def test_diagnostics_fields_match_their_definitions():
    p, phi, mu = _diag_state()
    t = 7 * 0.013
    d = oracle.diagnostics(p, phi, mu, t)
    c = modelref.conc_total_field(p, phi, mu, t)
    for q in range(2):
        ref = math.fsum(c[q].ravel())
        assert abs(d["sum_c"][q] - ref) <= 1e-13 * math.fsum(np.abs(c[q]).ravel())
    for a in range(4):
        ref = math.fsum(phi[a].ravel())
        assert abs(d["sum_phi"][a] - ref) <= 1e-13 * math.fsum(np.abs(phi[a]).ravel())
    dev = np.abs(phi.sum(axis=0) - 1.0).max()
    assert abs(d["max_simplex_dev"] - dev) <= 1e-15
    assert abs(d["max_simplex_dev"] - 0.1) <= 1e-12  # the cell whose sum is 0.9
    assert d["phi_min"] == phi.min() == -0.05
    assert d["phi_max"] == phi.max()
    assert d["nonfinite"] == 0


def test_diagnostics_with_nonfinite_cells():
    """Non-finite values: the count is of cells holding a NaN or Inf in any
    of the six fields; NaN enters no minimum, maximum or deviation (IEEE
    comparisons with NaN are false), Inf does; the sums propagate both."""
    p, phi, mu = _diag_state()
    phi[1, 0, 0, 1] = np.nan
    mu[0, 2, 1, 1] = np.inf
    phi[2, 4, 0, 2] = -np.inf
    mu[1, 4, 0, 2] = np.nan          # same cell as the -inf: counted once
    d = oracle.diagnostics(p, phi, mu, 0.0)
    bad = ~np.isfinite(phi).all(axis=0) | ~np.isfinite(mu).all(axis=0)
    assert d["nonfinite"] == int(bad.sum()) == 3
    assert d["phi_min"] == -np.inf
    assert d["phi_max"] == np.nanmax(phi)
    assert math.isnan(d["sum_phi"][1]) and d["sum_phi"][2] == -np.inf
    for a in (0, 3):
        assert abs(d["sum_phi"][a] - math.fsum(phi[a].ravel())) <= 1e-13 * phi[a].size
    assert d["max_simplex_dev"] == np.inf  # the -inf cell; the NaN cell is skipped
    assert all(math.isnan(v) for v in d["sum_c"])


# ------------------------------------------------------ anisotropic profiles

def _sine(dist, eps, ac):
    k = 4.0 / (math.pi * eps * ac)
    return 0.5 - 0.5 * np.sin(np.clip(k * dist, -math.pi / 2, math.pi / 2))


def _axis_interface(run, eps, nz, steps, delta):
    """Solid 0 below, liquid above, along z; the middle cell starts at 1/2
    so the interface sits on a cell centre (the stable lattice position).
    Returns phi_0 along z and its centre fitted from the solid amount."""
    p = _params(G=0.0, eps=eps, delta_sl=delta)
    p["T0"] = p["TE"]
    p["c0"] = [[0.3, 0.3]] * 4
    p["c1"] = [[0.0, 0.0]] * 4
    p["dt"] = 0.05
    half = nz // 2
    phi = np.zeros((4, nz, 1, 1))
    mu = np.zeros((2, nz, 1, 1))
    phi[0, :half] = 1.0
    phi[3, half + 1:] = 1.0
    phi[0, half] = phi[3, half] = 0.5
    phi, mu = run(phi, mu, p, steps)
    f = phi[0, :, 0, 0]
    # a profile symmetric about z0 with 1 below and 0 above sums to z0 + 1/2
    z0 = float(f.sum()) - 0.5
    return phi, f, np.arange(nz, dtype=float) - z0


def _axis_errors(run, delta=0.05):
    out = []
    for eps0, nz, steps in ((4.0, 80, 6000), (8.0, 160, 12000)):
        eps = eps0 / (1.0 + delta)
        phi, f, dist = _axis_interface(run, eps, nz, steps, delta)
        out.append((float(np.max(np.abs(f - _sine(dist, eps, 1.0 + delta)))),
                    float(np.max(np.abs(f - _sine(dist, eps, 1.0)))), phi))
    return out


def test_anisotropic_axis_interface_relaxes_to_sine_profile():
    """Normal along z: ac = 1 + delta, width pi^2 eps (1+delta)/4.  With
    eps = eps0/(1+delta) the discrete problem is the isotropic one of eps0
    scaled by (1+delta), so the error falls like the isotropic one's as eps0
    doubles; the isotropic width is far off."""
    (e4, w4, phi4), (e8, w8, _) = _axis_errors(_oracle_run)
    assert e4 <= 2.5e-3 and e8 <= 1e-3
    assert e4 / e8 >= 3.0
    assert w4 >= 1e-2 and w8 >= 1e-2
    assert np.all(phi4[1:3] == 0.0)


def _diagonal_stripe(run, delta, eps=4.0, n=64, steps=600):
    """Solid 0 in the stripe n/4 <= (x + y) mod n <= 3n/4 of a 64x64x1
    periodic layer, liquid outside: two flat interfaces with normal
    (1,1,0)/sqrt(2), on lattice lines.  Starts from a profile 10% too wide.
    Returns the error against the ac = 1 - delta and the ac = 1 profiles."""
    p = _params(G=0.0, eps=eps, delta_sl=delta)
    p["T0"] = p["TE"]
    p["c0"] = [[0.3, 0.3]] * 4
    p["c1"] = [[0.0, 0.0]] * 4
    p["dt"] = 0.05
    x = np.arange(n)[None, :]
    y = np.arange(n)[:, None]
    s = (x + y) % n
    dist = np.maximum(n // 4 - s, s - 3 * n // 4) / math.sqrt(2.0)
    f0 = _sine(dist, eps, 1.1)
    phi = np.zeros((4, 1, n, n))
    phi[0, 0] = f0
    phi[3, 0] = 1.0 - f0
    mu = np.zeros((2, 1, n, n))
    phi, _ = run(phi, mu, p, steps)
    f = phi[0, 0]
    return (float(np.max(np.abs(f - _sine(dist, eps, 1.0 - delta)))),
            float(np.max(np.abs(f - _sine(dist, eps, 1.0)))))


def test_anisotropic_diagonal_interface_relaxes_to_sine_profile():
    """Normal along (1,1,0): ac = 1 - delta, so the interface is narrower
    than the isotropic one; the tangential face gradients (4-point
    averages) carry half of every face's normal derivative here."""
    e, wrong = _diagonal_stripe(_oracle_run, 0.05)
    assert e <= 1e-3
    assert wrong >= 1e-2


# ---------------------------------------------------- temperature coupling

def _front_series(run, start, G=0.02, m=32, nz=64, chunks=8, chunk=1250):
    """Solid 0 below `start`, liquid above, mu frozen at 0, equal c0 so
    that only omega_bar = T - T_E drives the front; T = T_E on the face
    between cells m-1 and m.  Returns the solid amount after each chunk."""
    p = _params(G=G, mu_frozen=1)
    p["v"] = 0.0
    p["T0"] = p["TE"] - G * (m - 0.5)
    p["c0"] = [[0.3, 0.3]] * 4
    p["c1"] = [[0.0, 0.0]] * 4
    p["dt"] = 0.05
    phi = np.zeros((4, nz, 1, 1))
    phi[0, :start] = 1.0
    phi[3, start:] = 1.0
    mu = np.zeros((2, nz, 1, 1))
    out = []
    for c in range(chunks):
        phi, _ = run(phi, mu, p, chunk, step0=c * chunk)
        out.append(float(phi[0].sum()))
    return out


def _front_ok(run, m=32):
    lo = _front_series(run, m - 4)
    hi = _front_series(run, m + 4)
    moved = lo[0] > m - 4 + 0.5 and hi[0] < m + 4 - 0.5
    monotone = np.all(np.diff(lo) > -1e-9) and np.all(np.diff(hi) < 1e-9)
    settled = abs(lo[-1] - m) <= 0.05 and abs(hi[-1] - m) <= 0.05
    return moved and monotone and settled, lo, hi


def test_front_comes_to_rest_at_the_eutectic_isotherm_from_both_sides():
    """Below T_E the solids are favoured (omega_bar = T - T_E), above it the
    liquid: a front started four cells below or above the isotherm moves
    toward it and stops there (the solid amount then equals the number of
    cells below the isotherm; the factor T on the interface terms leaves a
    small offset, 0.016 cells at G = 0.02)."""
    ok, lo, hi = _front_ok(_oracle_run)
    assert ok, (lo, hi)


def _time_level_gap(run, s=7):
    """One step from time level s of a run whose temperature moves
    (v != 0), against one step of a run with v = 0 whose temperature field
    is T(z, t_s) (zoff = -v t_s, so z + zoff equals z - v t_s exactly).
    Returns (gap to that run, gap to the run frozen at T(z, t_{s+1}))."""
    shape = (16, 6, 6)
    phi, mu = pfinputs.smooth_interface_state(shape, 3, width=2.0)
    p = _params(G=0.02, v=0.7, chi1=0.3, mu_frozen=1)
    p["T0"] = 0.95
    p["dt"] = 0.01
    moving, _ = run(phi, mu, p, 1, step0=s)
    gaps = []
    for lvl in (s, s + 1):
        q = dict(p)
        q["v"] = 0.0
        q["zoff"] = -(p["v"] * (lvl * p["dt"]))
        frozen, _ = run(phi, mu, q, 1, step0=s)
        gaps.append(float(np.max(np.abs(moving - frozen))))
    return gaps


def test_phi_step_uses_the_temperature_of_the_old_time_level():
    """Explicit Euler (Algorithm 1 with Eq. (1)) evaluates the phi rhs at
    t_n: bitwise the step of the frozen field T(z, t_n), and measurably not
    the one of T(z, t_{n+1})."""
    same, next_level = _time_level_gap(_oracle_run)
    assert same == 0.0
    assert next_level > 1e-9


# ------------------------------------------------------- planted mutations

_MUTANTS = {
    # temperature of the phi rhs one time level late
    "t_next": ("void orc_phi_rhs(", "(double)k, t);", "(double)k, t + p->dt);"),
    # temperature of the phi rhs half a cell up
    "half_cell": ("void orc_phi_rhs(", "(double)k, t);", "(double)k + 0.5, t);"),
    # cubic anisotropy with the wrong sign
    "aniso_sign": ("void orc_aniso_X(", "1.0 - delta * (3.0 - 4.0 * P)",
                   "1.0 + delta * (3.0 - 4.0 * P)"),
    # one factor ac of d(ac^2 |q|^2)/dq dropped
    "aniso_factor": ("void orc_aniso_X(", "X[c] = 2.0 * ac * (ac * q[c]",
                     "X[c] = 2.0 * (ac * q[c]"),
}


def _build_mutant(name, tmpdir):
    anchor, old, new = _MUTANTS[name]
    src = open(os.path.join(ORACLE_DIR, "pf_oracle.c")).read()
    at = src.index(anchor)
    pos = src.index(old, at)
    src = src[:pos] + new + src[pos + len(old):]
    cfile = os.path.join(tmpdir, f"mut_{name}.c")
    with open(cfile, "w") as f:
        f.write(src)
    so = os.path.join(tmpdir, f"libmut_{name}.so")
    subprocess.run(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                    "-fno-fast-math", "-I", ORACLE_DIR, "-o", so, cfile, "-lm"], check=True)
    L = C.CDLL(so)
    L.orc_run.restype = C.c_int
    L.orc_run.argtypes = [C.POINTER(oracle.OrcGrid), C.POINTER(oracle.OrcParams),
                          C.c_int64, C.c_int64, C.POINTER(C.c_double),
                          C.POINTER(C.c_double), C.c_int]

    def run(phi, mu, p, nsteps, step0=0):
        phi = np.ascontiguousarray(phi, dtype=np.float64).copy()
        mu = np.ascontiguousarray(mu, dtype=np.float64).copy()
        g = oracle.make_grid(phi.shape[1:])
        rc = L.orc_run(C.byref(g), C.byref(oracle.make_params(p)), int(step0), int(nsteps),
                       phi.ctypes.data_as(C.POINTER(C.c_double)),
                       mu.ctypes.data_as(C.POINTER(C.c_double)), 1)
        assert rc == 0
        return phi, mu

    return run


@pytest.mark.parametrize("name", sorted(_MUTANTS))
def test_planted_slips_are_rejected(name, tmp_path):
    run = _build_mutant(name, str(tmp_path))
    if name in ("t_next", "half_cell"):
        front_ok = _front_ok(run)[0]
        same, _ = _time_level_gap(run)
        assert not (front_ok and same == 0.0)
    else:
        (e4, _, _), (e8, _, _) = _axis_errors(run)
        axis_ok = e4 <= 2.5e-3 and e8 <= 1e-3 and e4 / e8 >= 3.0
        diag_ok = _diagonal_stripe(run, 0.05)[0] <= 1e-3
        assert not (axis_ok and diag_ok)
