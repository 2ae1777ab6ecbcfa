"""Pins of the oracle's moving window (Sec. 3.3, the moving-window technique
the paper cites for directional solidification).

The window is pinned three ways: the shift itself against its definition
written with numpy slicing; a window run against the same run composed by
hand (numpy check and shift, then one oracle step with the temperature
offset by the shifts made so far); and, physically, against a tall domain
without a window: the front of the window run, counted in the tall domain's
coordinates, follows the tall domain's front."""
import numpy as np
import pytest

import oracle
import pfinputs


def numpy_shift(phi, mu, zw, mu_fill):
    """Definition: if the mean liquid fraction of plane zw is below 1/2,
    drop plane 0, move every plane down by one, and fill the top plane with
    liquid at mu_fill."""
    nx_ny = phi.shape[2] * phi.shape[3]
    if not (float(np.sum(phi[3, zw])) < 0.5 * nx_ny):
        return phi.copy(), mu.copy(), False
    p2 = np.empty_like(phi)
    m2 = np.empty_like(mu)
    p2[:, :-1] = phi[:, 1:]
    m2[:, :-1] = mu[:, 1:]
    p2[:, -1] = 0.0
    p2[3, -1] = 1.0
    m2[0, -1], m2[1, -1] = mu_fill
    return p2, m2, True


def test_shift_matches_definition():
    rng = np.random.default_rng(3)
    shape = (12, 5, 7)
    phi = rng.random((4,) + shape)
    phi /= phi.sum(axis=0, keepdims=True)
    mu = rng.normal(size=(2,) + shape)
    zw = 4
    phi[3, zw] = 0.1  # front has passed plane zw
    a, b, shifted = oracle.window_shift(phi, mu, zw, mu_fill=(0.25, -0.5))
    ea, eb, eshift = numpy_shift(phi, mu, zw, (0.25, -0.5))
    assert shifted and eshift
    assert np.array_equal(a, ea) and np.array_equal(b, eb)
    # liquid plane: no shift, fields untouched
    phi[3, zw] = 0.9
    a, b, shifted = oracle.window_shift(phi, mu, zw)
    assert not shifted and np.array_equal(a, phi) and np.array_equal(b, mu)


def test_threshold_is_strict():
    shape = (6, 2, 2)
    phi = np.zeros((4,) + shape)
    phi[3] = 1.0
    mu = np.zeros((2,) + shape)
    phi[3, 2] = [[0.5, 0.5], [0.5, 0.5]]  # mean exactly 1/2: not passed
    phi[0, 2] = 0.5
    _, _, shifted = oracle.window_shift(phi, mu, 2)
    assert not shifted
    phi[3, 2, 0, 0] = 0.5 - 1e-12
    _, _, shifted = oracle.window_shift(phi, mu, 2)
    assert shifted


def test_window_run_equals_hand_composition():
    shape = (20, 6, 6)
    hs = 8
    p = pfinputs.p0_params(solid_height=hs, G=0.05, v=1.0)
    p["chi1"] = [[0.2, 0.1]] * 4
    p["c1"] = [[0.05, -0.02], [0.1, 0.03], [-0.07, 0.02], [0.1, -0.1]]
    p["dt"] = oracle.default_dt(p, shape)
    phi, mu = oracle.init_voronoi(shape, 11, 3, hs)
    zw, fill = hs - 2, (0.05, -0.02)
    a, b, shifts = oracle.run_window(p, phi, mu, 12, zw=zw, mu_fill=fill, nthreads=2)
    hp, hm, hsh = phi.copy(), mu.copy(), 0
    for s in range(12):
        hp, hm, did = numpy_shift(hp, hm, zw, fill)
        hsh += int(did)
        q = dict(p, zoff=p["zoff"] + hsh * 1.0)
        hp, hm = oracle.run(q, hp, hm, 1, step0=s, nthreads=2)
    assert shifts == hsh == 2  # planes hs-2 and hs-1 start solid
    assert np.array_equal(a, hp) and np.array_equal(b, hm)


@pytest.mark.parametrize("G,v", [(0.05, 1.0)])
def test_window_front_follows_tall_domain(G, v):
    """Lamella of one solid under liquid, front driven by the moving
    isotherm; the window (plane 20 of 40) shifts once the front passes it.
    Front height = sum over z of the mean solid fraction (global planes)."""
    hs, n = 20, 4
    tall, short = (96, n, n), (40, n, n)
    p = pfinputs.p0_params(solid_height=hs, G=G, v=v)
    p["dt"] = min(oracle.default_dt(p, tall), oracle.default_dt(p, short))
    pt, mt = oracle.init_voronoi(tall, 42, 1, hs)
    ps, ms = oracle.init_voronoi(short, 42, 1, hs)
    pt, mt = oracle.run(p, pt, mt, 1200, nthreads=4)
    ps, ms, shifts = oracle.run_window(p, ps, ms, 1200, zw=hs, nthreads=4)

    def front(phi):
        return float(np.sum(1.0 - phi[3].mean(axis=(1, 2))))

    assert shifts >= 1
    assert abs((front(ps) + shifts) - front(pt)) < 0.05
    assert np.abs(pt[:, shifts:shifts + short[0]] - ps).max() < 0.02
