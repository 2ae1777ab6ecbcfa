"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the property it checks and where it comes from.  None of them
re-types the oracle's own update formulas: they use closed forms, brute force,
invariants the paper states (Sec. 2: simplex, bulk regions; Sec. 3.3:
sine-shaped interface; Eq. (3): concentration balance), the energy functional
the phi equation descends, and the literal Eq. (4).
"""
import math
import os

import numpy as np
import pytest

import oracle
import pfinputs
from tests import modelref

HERE = os.path.dirname(os.path.abspath(__file__))


def _params(**kw):
    hs = kw.pop("solid_height", 8)
    p = pfinputs.p0_params(solid_height=hs, **kw)
    return p


# ------------------------------------------------------------ generators

def test_splitmix64_matches_published_vector():
    rows = [l.split()[0] for l in open(os.path.join(HERE, "golden", "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    expect = [int(r, 16) for r in rows]
    assert oracle.splitmix64(0, len(expect)) == expect
    r = pfinputs.SplitMix64(0)
    assert [r.next() for _ in expect] == expect


def test_paper_roofline_example_units():
    """Sec. 5.1.1: 80 GiB/s / 680 B/LUP = 126.3 MLUP/s and 1384 flop x 4.2
    MLUP/s = 5.8 GFLOP/s = 27% of 21.6 GFLOP/s.  Pins the MLUP/s and
    bytes-per-update conventions the benchmark reports in."""
    vals = {}
    for l in open(os.path.join(HERE, "golden", "paper_roofline_example.txt")):
        if l.strip() and not l.startswith("#"):
            k, v = l.split()
            vals[k] = float(v)
    mlups = vals["bandwidth_gib_s"] * 2 ** 30 / vals["bytes_per_lup"] / 1e6
    assert abs(mlups - vals["mlups"]) < 0.05
    gf = vals["flop_per_lup"] * vals["mlups_per_core"] * 1e6 / 1e9
    assert abs(gf - vals["gflops_per_core"]) < 0.05
    assert abs(gf / vals["core_peak_gflops"] - 0.27) < 0.005


# ------------------------------------------------------------ projection

def _project_bruteforce(y):
    """Enumerate all 15 supports; on each the affine projection onto
    {x_S sums to 1, x_else = 0}; keep the feasible point nearest to y."""
    best, bd = None, math.inf
    for mask in range(1, 16):
        S = [a for a in range(4) if mask >> a & 1]
        x = np.zeros(4)
        shift = (sum(y[a] for a in S) - 1.0) / len(S)
        for a in S:
            x[a] = y[a] - shift
        if min(x) < -1e-15:
            continue
        d = float(np.sum((x - y) ** 2))
        if d < bd:
            bd, best = d, x
    return best


def test_projection_matches_bruteforce():
    rng = np.random.default_rng(1)
    ys = [rng.normal(0.25, s, 4) for s in (0.01, 0.1, 0.5, 2.0) for _ in range(2500)]
    ys += [np.array([1.2, -0.1, -0.05, -0.05]), np.array([0.5, 0.5, 0.0, 0.0]),
           np.array([0.25] * 4), np.array([0.3, 0.3, 0.3, 0.3]),
           np.array([1.0, 0.0, 0.0, 0.0]), np.array([2.0, 2.0, -5.0, 0.1])]
    for y in ys:
        x = oracle.project(y)
        xb = _project_bruteforce(y)
        assert np.max(np.abs(x - xb)) <= 1e-15 * max(1.0, np.max(np.abs(y))) * 4
        assert abs(x.sum() - 1.0) <= 4 * np.finfo(float).eps
        assert x.min() >= 0.0


def test_projection_fixes_simplex_points():
    rng = np.random.default_rng(2)
    for _ in range(1000):
        w = rng.random(4)
        x = w / w.sum()
        assert np.max(np.abs(oracle.project(x) - x)) <= 4e-16


# ----------------------------------------------------------- anisotropy

def _A_aniso(q, delta):
    qn = np.linalg.norm(q)
    P = np.sum((q / qn) ** 4)
    ac = 1.0 - delta * (3.0 - 4.0 * P)
    return ac * ac * qn * qn


@pytest.mark.parametrize("delta", [0.0, 0.02, 0.05])
def test_aniso_X_is_gradient_of_pair_energy(delta):
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(200):
        q = rng.normal(size=3) * rng.choice([0.1, 1.0, 5.0])
        X = oracle.aniso_X(q, delta)
        fd = np.zeros(3)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h * max(1.0, np.linalg.norm(q))
            fd[c] = (_A_aniso(q + e, delta) - _A_aniso(q - e, delta)) / (2 * e[c])
        assert np.max(np.abs(fd - X)) <= 1e-8 * max(1.0, np.max(np.abs(X)))


def test_aniso_stiffness_extremes():
    """ac = 1 + delta along <100> (P = 1) and 1 - 5 delta/3 along <111>."""
    d = 0.05
    for q in ([1.0, 0, 0], [0, -2.0, 0]):
        q = np.array(q)
        X = oracle.aniso_X(q, d)
        # along an axis the q_hat^3 - P q_hat term vanishes: X = 2 ac^2 q
        assert np.allclose(X, 2 * (1 + d) ** 2 * q, rtol=1e-15, atol=0)
    q = np.ones(3) / math.sqrt(3)
    X = oracle.aniso_X(q, d)
    assert np.allclose(X, 2 * (1 - 5 * d / 3) ** 2 * q, rtol=1e-14, atol=0)


# ------------------------------------------- phi rhs = energy gradient

@pytest.mark.parametrize("dx", [1.0, 0.7])
def test_phi_rhs_is_gradient_of_discrete_energy(dx):
    """Isotropic, uniform T: rhs_a(P) dx^3 = dE_h/dphi_a(P) (central FD)."""
    shape = (4, 4, 4)
    p = _params(G=0.0, chi1=0.3)
    p["T0"] = 0.93
    p["c1"][0][1] = 0.2
    phi, mu = pfinputs.random_state(shape, 11, mu_scale=0.3)
    T = p["T0"]
    h = 1e-6
    worst = 0.0
    for k in range(4):
        for j in range(4):
            for i in range(4):
                rhs = oracle.phi_rhs(p, phi, mu, 0.0, i, j, k, dx=dx)
                for a in range(4):
                    pp, pm = phi.copy(), phi.copy()
                    pp[a, k, j, i] += h
                    pm[a, k, j, i] -= h
                    fd = (modelref.energy(p, pp, mu, T, dx) - modelref.energy(p, pm, mu, T, dx)) / (2 * h)
                    worst = max(worst, abs(fd - rhs[a] * dx ** 3) / max(1.0, abs(rhs[a] * dx ** 3)))
    assert worst <= 1e-8


def test_phi_rhs_gradient_catches_planted_sign_error():
    """The energy-gradient pin is sharp: flipping the sign of the face share
    S of da/dphi (a plausible slip) moves rhs far outside the FD tolerance."""
    shape = (4, 4, 4)
    p = _params(G=0.0)
    phi, mu = pfinputs.random_state(shape, 12, mu_scale=0.3)
    i, j, k = 1, 2, 1
    rhs = oracle.phi_rhs(p, phi, mu, 0.0, i, j, k)
    bad = rhs.copy()
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        _, Su = oracle.phi_face(p, phi, i, j, k, d)
        _, Sl = oracle.phi_face(p, phi, i - e[0], j - e[1], k - e[2], d)
        bad -= p["eps"] * p["T0"] * (Su + Sl)  # turns +1/2(Su+Sl) into -1/2(Su+Sl)
    h = 1e-6
    a = 0
    pp, pm = phi.copy(), phi.copy()
    pp[a, k, j, i] += h
    pm[a, k, j, i] -= h
    fd = (modelref.energy(p, pp, mu, p["T0"]) - modelref.energy(p, pm, mu, p["T0"])) / (2 * h)
    assert abs(fd - rhs[a]) <= 1e-8 * max(1, abs(fd))
    assert abs(fd - bad[a]) > 1e-3


# ------------------------------------------------------- P5 anisotropy

def test_zero_delta_pairs_match_isotropic_bitwise():
    """With phase 0 absent, turning on anisotropy only on pair (0, liquid)
    leaves every rhs bitwise equal to the isotropic one."""
    shape = (6, 5, 7)
    phi, mu = pfinputs.random_state(shape, 5)
    phi[0] = 0.0
    phi /= phi.sum(axis=0, keepdims=True)
    p_iso = _params()
    p_iso["dt"] = 0.01
    p_an = _params()
    p_an["dt"] = 0.01
    p_an["delta"][0][3] = p_an["delta"][3][0] = 0.05
    out_iso = oracle.phi_sweep(p_iso, phi, mu, 0.0)
    out_an = oracle.phi_sweep(p_an, phi, mu, 0.0)
    assert np.array_equal(out_iso, out_an)
    assert np.max(np.abs(out_iso - phi)) > 1e-4


def test_cubic_symmetry_xy_transpose_and_mirror():
    n = 8
    phi, mu = pfinputs.smooth_interface_state((n, n, n), 7, width=2.0)
    p = _params(delta_sl=0.05)
    p["dt"] = 0.005
    out = oracle.phi_sweep(p, phi, mu, 0.0)
    # x <-> y transpose
    phi_t = np.ascontiguousarray(np.swapaxes(phi, 2, 3))
    mu_t = np.ascontiguousarray(np.swapaxes(mu, 2, 3))
    out_t = oracle.phi_sweep(p, phi_t, mu_t, 0.0)
    assert np.max(np.abs(np.swapaxes(out_t, 2, 3) - out)) <= 1e-14
    # mirror x -> n-1-x
    phi_m = np.ascontiguousarray(phi[..., ::-1])
    mu_m = np.ascontiguousarray(mu[..., ::-1])
    out_m = oracle.phi_sweep(p, phi_m, mu_m, 0.0)
    assert np.max(np.abs(out_m[..., ::-1] - out)) <= 1e-14
    # and the anisotropy actually matters on this state
    out_iso = oracle.phi_sweep(_params(), phi, mu, 0.0)
    assert np.max(np.abs(out_iso - out)) > 1e-6


# ------------------------------------------------ P6 flat interface sine

def _flat_interface(eps, nz, steps, dt):
    p = _params(G=0.0, eps=eps)
    p["T0"] = p["TE"]
    p["c0"] = [[0.3, 0.3]] * 4
    p["c1"] = [[0.0, 0.0]] * 4
    p["dt"] = dt
    phi = np.zeros((4, nz, 1, 1))
    mu = np.zeros((2, nz, 1, 1))
    half = nz // 2
    phi[0, :half] = 1.0
    phi[3, half:] = 1.0
    phi, mu = oracle.run(p, phi, mu, steps, nthreads=1)
    z = np.arange(nz, dtype=float)
    z0 = half - 0.5
    kk = 4.0 / (math.pi * eps)
    arg = np.clip(kk * (z - z0), -math.pi / 2, math.pi / 2)
    exact = 0.5 - 0.5 * np.sin(arg)
    return phi, mu, exact


def test_flat_interface_relaxes_to_sine_profile():
    """Sec. 3.3: the interface profile of the obstacle potential is a sine
    of width pi^2 eps/4; third phases stay exactly zero."""
    phi4, mu4, ex4 = _flat_interface(4.0, 80, 6000, 0.05)
    err4 = np.max(np.abs(phi4[0, :, 0, 0] - ex4))
    assert err4 <= 1e-2
    assert np.all(phi4[1:3] == 0.0)
    assert np.all(mu4 == 0.0)
    phi8, _, ex8 = _flat_interface(8.0, 160, 20000, 0.05)
    err8 = np.max(np.abs(phi8[0, :, 0, 0] - ex8))
    assert err8 <= 1e-2
    assert err4 / err8 >= 3.0


# ------------------------------------------------ P7 Fourier decay of mu

def _liquid(shape):
    nz, ny, nx = shape
    phi = np.zeros((4, nz, ny, nx))
    phi[3] = 1.0
    return phi


def test_fourier_mode_decays_at_discrete_rate():
    shape = (16, 8, 32)
    nz, ny, nx = shape
    p = _params(G=1e-3, v=0.0)
    p["dt"] = 0.05
    mx, mz = 2, 3
    x = np.arange(nx)[None, None, :]
    z = np.arange(nz)[:, None, None]
    mode0 = np.cos(2 * np.pi * mx * x / nx) * np.cos(np.pi * mz * (z + 0.5) / nz) * np.ones((1, ny, 1))
    mode1 = np.cos(2 * np.pi * 1 * x / nx) * np.ones((nz, ny, 1))
    A = 0.01
    phi = _liquid(shape)
    mu = np.stack([A * mode0, -A * mode1])
    n = 40
    phi_n, mu_n = oracle.run(p, phi, mu, n)
    D, dt = p["D"][3], p["dt"]
    r0 = 1 - D * dt * 4 * (math.sin(math.pi * mx / nx) ** 2 + math.sin(math.pi * mz / (2 * nz)) ** 2)
    r1 = 1 - D * dt * 4 * math.sin(math.pi * 1 / nx) ** 2
    assert np.array_equal(phi_n, phi)
    assert np.max(np.abs(mu_n[0] - A * r0 ** n * mode0)) <= 1e-13 * A
    assert np.max(np.abs(mu_n[1] + A * r1 ** n * mode1)) <= 1e-13 * A


def test_mixed_phase_mobility_and_susceptibility():
    """Uniform two-solid/liquid mixture, phi frozen for one mu step:
    the decay factor is 1 - dt (M/chi) 4 sin^2(pi m/N) with
    M = sum D_a phi_a chi_a and chi = sum h_a chi_a."""
    shape = (4, 4, 16)
    nz, ny, nx = shape
    p = _params(G=0.0, v=0.0)
    p["dt"] = 0.05
    p["chi0"] = [[1.0, 2.5], [2.0, 1.2], [3.0, 0.8], [1.5, 1.1]]
    ph = np.array([0.2, 0.1, 0.0, 0.7])
    phi = np.ones((4,) + shape) * ph[:, None, None, None]
    x = np.arange(nx)[None, None, :] * np.ones(shape)
    m = 1
    mode = np.cos(2 * np.pi * m * x / nx)
    mu = np.stack([0.01 * mode, 0.02 * mode])
    out = oracle.mu_sweep(p, phi, phi, mu, 0.0, p["dt"])
    h = ph ** 2 / np.sum(ph ** 2)
    for q in range(2):
        chi = np.array([p["chi0"][a][q] for a in range(4)])
        M = np.sum(np.array(p["D"]) * ph * chi)
        X = np.sum(h * chi)
        r = 1 - p["dt"] * (M / X) * 4 * math.sin(math.pi * m / nx) ** 2
        assert np.max(np.abs(out[q] - r * mu[q])) <= 1e-15


# ------------------------------------------------ P8 conservation of c

def test_total_concentration_conserved_moving_temperature():
    shape = (32, 16, 16)
    p = _params(solid_height=8, G=2e-3, v=0.5, chi1=0.5)
    p["dt"] = oracle.default_dt(p, shape)
    phi, mu = oracle.init_voronoi(shape, 42, 6, 8, (0.01, -0.02))
    c0 = modelref.conc_total_field(p, phi, mu, 0.0).sum(axis=(1, 2, 3))
    n = 600
    phi_n, mu_n = oracle.run(p, phi, mu, n)
    c1 = modelref.conc_total_field(p, phi_n, mu_n, n * p["dt"]).sum(axis=(1, 2, 3))
    assert np.all(np.abs(c1 - c0) <= 1e-12 * np.abs(c0))
    d = oracle.diagnostics(p, phi_n, mu_n, n * p["dt"])
    assert np.allclose(d["sum_c"], c1, rtol=1e-13, atol=0)
    # the run actually evolved phi and mu
    assert np.max(np.abs(phi_n - phi)) > 0.1 and np.max(np.abs(mu_n - mu)) > 1e-3


def test_uniform_cell_source_terms_conserve_local_concentration():
    """With no gradients the flux divergence vanishes, so each cell's c must
    be unchanged by the source terms for any phi^n -> phi^{n+1} and T change."""
    rng = np.random.default_rng(9)
    shape = (3, 3, 3)
    p = _params(G=3e-2, v=2.0, chi1=0.7)
    p["c1"] = [[0.05, -0.02], [0.1, 0.03], [-0.07, 0.02], [0.1, -0.1]]
    p["dt"] = 0.01
    for trial in range(20):
        w0, w1 = rng.random(4) + 0.01, rng.random(4) + 0.01
        w0[rng.integers(4)] = 0.0
        phi0 = np.ones((4,) + shape) * (w0 / w0.sum())[:, None, None, None]
        phi1 = np.ones((4,) + shape) * (w1 / w1.sum())[:, None, None, None]
        mu = np.ones((2,) + shape) * rng.normal(0, 0.1, 2)[:, None, None, None]
        t0, t1 = 7 * p["dt"], 8 * p["dt"]
        out = oracle.mu_sweep(p, phi0, phi1, mu, t0, t1)
        cb = modelref.conc_total_field(p, phi0, mu, t0)
        ca = modelref.conc_total_field(p, phi1, out, t1)
        assert np.max(np.abs(ca - cb)) <= 1e-14


# ------------------------------------------------ P9 bulk invariance

def test_bulk_cells_stay_pure_and_have_no_antitrapping():
    shape = (8, 8, 8)
    p = _params(solid_height=4, G=1e-3, v=0.05)
    p["dt"] = oracle.default_dt(p, shape)
    phi, mu = oracle.init_voronoi(shape, 3, 3, 4)
    phi1 = oracle.phi_sweep(p, phi, mu, 0.0)
    nz, ny, nx = shape
    checked = 0
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                nb = [phi[:, min(max(k + c, 0), nz - 1), (j + b) % ny, (i + a) % nx]
                      for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
                if all(np.array_equal(v, nb[0]) for v in nb):
                    checked += 1
                    assert np.array_equal(phi1[:, k, j, i], phi[:, k, j, i])
                    for d in range(3):
                        _, J = oracle.mu_face(p, phi, phi1, mu, 0.0, i, j, k, d)
                        assert np.all(J == 0.0)
    assert checked > 100


# ------------------------------------------------ P10 energy descent

def test_energy_descends_with_frozen_mu():
    shape = (16, 8, 8)
    p = _params(solid_height=5, G=0.0, mu_frozen=1)
    p["T0"] = 0.97
    p["dt"] = oracle.default_dt(p, shape)
    phi, mu = oracle.init_voronoi(shape, 8, 5, 5, (0.02, -0.01))
    E = [modelref.energy(p, phi, mu, p["T0"])]
    for s in range(25):
        phi, mu2 = oracle.run(p, phi, mu, 1, step0=s)
        assert np.array_equal(mu2, mu)
        E.append(modelref.energy(p, phi, mu, p["T0"]))
    dE = np.diff(E)
    assert np.all(dE <= 1e-12 * abs(E[0]))
    assert E[-1] < E[0] - 1.0


# ------------------------------------------------ P11 driving force sign

@pytest.mark.parametrize("undercool,grows", [(0.05, True), (-0.05, False)])
def test_driving_force_moves_front(undercool, grows):
    nz = 128
    p = _params(G=0.0, mu_frozen=1)
    p["T0"] = p["TE"] - undercool
    p["dt"] = 0.05
    phi = np.zeros((4, nz, 1, 1))
    phi[0, :64] = 1.0
    phi[3, 64:] = 1.0
    mu = np.zeros((2, nz, 1, 1))
    fronts = []
    for s in range(4):
        phi, _ = oracle.run(p, phi, mu, 250, step0=250 * s, nthreads=1)
        fronts.append(phi[0].sum())
    d = np.diff(fronts)
    assert np.all(d > 0) if grows else np.all(d < 0)


# ------------------------------------------------ P12 anti-trapping

def test_antitrapping_matches_literal_dyadic_form():
    shape = (4, 4, 4)
    p = _params(G=5e-3, chi1=0.2)
    p["dt"] = 0.01
    phi0, mu = pfinputs.random_state(shape, 21, mu_scale=0.2)
    phi1, _ = pfinputs.random_state(shape, 22)
    phi1 = 0.9 * phi0 + 0.1 * phi1
    t = 0.3
    worst = 0.0
    for d in range(3):
        for (i, j, k) in [(0, 0, 0), (1, 2, 1), (3, 3, 2), (2, 0, 1)]:
            if d == 2 and k >= shape[0] - 1:
                continue
            Tf = p["T0"] + p["G"] * ((k + (0.5 if d == 2 else 0.0)) - p["v"] * t)
            Jm = modelref.antitrap_matrix_literal(p, phi0, phi1, mu, i, j, k, d, Tf)
            _, J = oracle.mu_face(p, phi0, phi1, mu, t, i, j, k, d)
            worst = max(worst, np.max(np.abs(J - Jm[:, d])))
            assert np.max(np.abs(Jm[:, d])) > 1e-6
    assert worst <= 1e-14


def test_antitrapping_zero_cases_and_direction():
    shape = (4, 4, 4)
    p = _params()
    p["dt"] = 0.01
    phi0, mu = pfinputs.random_state(shape, 31)
    # no liquid -> J = 0
    nol = phi0.copy()
    nol[3] = 0.0
    nol /= nol.sum(axis=0, keepdims=True)
    _, J = oracle.mu_face(p, nol, 0.5 * (nol + pfinputs.random_state(shape, 32)[0]), mu, 0.0, 1, 1, 1, 0)
    assert np.all(J == 0.0)
    # no phi change -> J = 0
    _, J = oracle.mu_face(p, phi0, phi0, mu, 0.0, 1, 1, 1, 2)
    assert np.all(J == 0.0)
    # solidifying S1 front below liquid: component 1 is richer in the liquid
    # (c^l_1 = 1/3 > c^S1_1 = 0.1), so J_z points into the liquid (+z).
    nz = 8
    phi = np.zeros((4, nz, 1, 1))
    prof = np.clip(0.5 - 0.5 * np.sin((np.arange(nz) - 3.5) / 2.0), 0, 1)
    phi[0, :, 0, 0] = prof
    phi[3, :, 0, 0] = 1 - prof
    phin = phi.copy()
    newp = np.clip(prof + 0.01 * (prof * (1 - prof)), 0, 1)
    phin[0, :, 0, 0] = newp
    phin[3, :, 0, 0] = 1 - newp
    mu = np.zeros((2, nz, 1, 1))
    _, J = oracle.mu_face(p, phi, phin, mu, 0.0, 0, 0, 3, 2)
    assert J[1] > 0 and J[0] < 0  # component 0 is richer in S1 -> opposite sign


# ------------------------------------------------ P13 Voronoi

def test_voronoi_matches_exhaustive_search():
    shape = (6, 24, 20)
    nz, ny, nx = shape
    seed, nseeds, hs = 1234, 9, 3
    phi, mu = oracle.init_voronoi(shape, seed, nseeds, hs, (0.1, -0.2))
    r = pfinputs.SplitMix64(seed)
    pts = []
    for s in range(nseeds):
        sx = (r.next() >> 11) * 2.0 ** -53 * nx
        sy = (r.next() >> 11) * 2.0 ** -53 * ny
        pts.append((sx, sy))
    for j in range(ny):
        for i in range(nx):
            d2 = []
            for (sx, sy) in pts:
                ddx = abs(i + 0.5 - sx)
                ddx = min(ddx, nx - ddx)
                ddy = abs(j + 0.5 - sy)
                ddy = min(ddy, ny - ddy)
                d2.append(ddx * ddx + ddy * ddy)
            s = int(np.argmin(d2))  # first minimum = lowest index
            for k in range(nz):
                expect = np.zeros(4)
                expect[s % 3 if k < hs else 3] = 1.0
                assert np.array_equal(phi[:, k, j, i], expect)
    assert np.all(mu[0] == 0.1) and np.all(mu[1] == -0.2)
    # each of the three solids appears
    assert all(phi[a, 0].sum() > 0 for a in range(3))


# ------------------------------------------------ P14 time step bound

def test_stability_bound_closed_form():
    # c1: T_max = 1 - 16e-3 + 63e-3 = 1.047; phase-field bound 1/(12 T_max)
    w = pfinputs.workload("c1")
    assert abs(oracle.default_dt(w["params"], w["shape"]) - 0.25 / (12 * 1.047)) < 1e-15
    assert abs(oracle.default_dt(w["params"], w["shape"]) - 0.0198981) < 1e-7
    w = pfinputs.workload("c2")
    assert abs(oracle.default_dt(w["params"], w["shape"]) - 0.25 / (12 * 1.383)) < 1e-15
    w = pfinputs.workload("c3")  # anisotropy factor (1.05)(1.75)
    assert abs(oracle.default_dt(w["params"], w["shape"]) - 0.25 / (12 * 1.767 * 1.05 * 1.75)) < 1e-15
    # chemistry-limited: D_l = 10 -> dx^2 min(chi) / (6 max(D chi)) = 1/90
    p = pfinputs.p0_params(solid_height=16)
    p["D"][3] = 10.0
    assert abs(oracle.stability_bound(p, (64, 32, 32)) - 1.0 / 90.0) < 1e-15


# ------------------------------------------------ P15 translation, P2

def test_periodic_translation_is_bitwise():
    shape = (10, 12, 16)
    p = _params(solid_height=4, delta_sl=0.05)
    p["dt"] = oracle.default_dt(p, shape)
    phi, mu = pfinputs.smooth_interface_state(shape, 4, width=2.0)
    a_phi, a_mu = oracle.run(p, phi, mu, 3)
    sh = lambda f: np.ascontiguousarray(np.roll(np.roll(f, 5, axis=3), 3, axis=2))
    b_phi, b_mu = oracle.run(p, sh(phi), sh(mu), 3)
    assert np.array_equal(b_phi, sh(a_phi))
    assert np.array_equal(b_mu, sh(a_mu))


def test_thread_count_does_not_change_result():
    w = pfinputs.workload("c1")
    shape = (16, 16, 16)
    p = pfinputs.with_dt(w["params"], oracle.default_dt(w["params"], shape))
    phi, mu = oracle.init_voronoi(shape, 42, 6, 4)
    a = oracle.run(p, phi, mu, 4, nthreads=1)
    b = oracle.run(p, phi, mu, 4, nthreads=5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_simplex_invariants_every_step():
    shape = (24, 12, 12)
    p = _params(solid_height=6, G=1e-3, v=0.01)
    p["dt"] = oracle.default_dt(p, shape)
    phi, mu = oracle.init_voronoi(shape, 42, 6, 6)
    for s in range(30):
        phi, mu = oracle.run(p, phi, mu, 1, step0=s)
        assert np.max(np.abs(phi.sum(axis=0) - 1.0)) <= 4 * np.finfo(float).eps
        assert phi.min() >= 0.0 and phi.max() <= 1.0
