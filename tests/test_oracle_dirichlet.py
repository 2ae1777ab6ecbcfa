"""Pins of the oracle's Dirichlet top boundary (the paper's boundary
handling names Dirichlet conditions beside Neumann and periodic ones, Sec.
3.1; reading: a ghost plane above the top held at liquid, phi = e_liquid,
and mu = mu_top).

With G v = 0 and T-independent coefficients, mu in pure liquid obeys
mu^{n+1} = mu^n + dt D Lap_h mu^n.  With a zero-gradient mirror below plane
0 and mu = 0 in the ghost plane nz, the discrete eigenmodes along z are
cos(theta (k + 1/2)) with theta (nz + 1/2) = pi (m + 1/2), and each decays
by the factor r = 1 - 4 D dt sin^2(theta / 2) / dx^2 per step, exactly."""
import numpy as np
import pytest

import oracle
import pfinputs


def _liquid_params(shape, **kw):
    p = pfinputs.p0_params(solid_height=0, G=0.0, v=0.0)
    p["c1"] = [[0.0, 0.0]] * 4
    p["top_bc"] = 1
    p.update(kw)
    p["dt"] = oracle.default_dt(p, shape)
    return p


@pytest.mark.parametrize("m", [0, 1, 3])
def test_dirichlet_mode_decays_by_the_discrete_factor(m):
    nz, n = 24, 4
    shape = (nz, n, n)
    p = _liquid_params(shape, mu_fill=(0.0, 0.0))
    theta = np.pi * (m + 0.5) / (nz + 0.5)
    k = np.arange(nz) + 0.5
    mode = np.cos(theta * k)
    phi, mu = oracle.init_voronoi(shape, 1, 0, 0)
    mu[0] = 0.3 * mode[:, None, None]
    mu[1] = -0.2 * mode[:, None, None]
    steps = 60
    _, mu_n = oracle.run(p, phi, mu, steps, nthreads=2)
    D, dt = p["D"][3], p["dt"]
    r = 1.0 - 4.0 * D * dt * np.sin(theta / 2) ** 2
    for q, amp in ((0, 0.3), (1, -0.2)):
        want = amp * r ** steps * mode[:, None, None] * np.ones((1, n, n))
        err = np.max(np.abs(mu_n[q] - want)) / np.max(np.abs(want))
        assert err < 1e-12, err


def test_dirichlet_value_is_a_fixed_point_and_mirror_differs():
    shape = (12, 4, 4)
    p = _liquid_params(shape, mu_fill=(0.05, -0.03))
    phi, mu = oracle.init_voronoi(shape, 1, 0, 0, mu_init=(0.05, -0.03))
    a, b = oracle.run(p, phi, mu, 20, nthreads=2)
    assert np.array_equal(b, mu) and np.array_equal(a, phi)
    # a different interior value relaxes towards the Dirichlet value at the
    # top only; with the mirror the uniform state does not move at all
    phi, mu = oracle.init_voronoi(shape, 1, 0, 0, mu_init=(0.0, 0.0))
    _, bd = oracle.run(p, phi, mu, 20, nthreads=2)
    _, bm = oracle.run(dict(p, top_bc=0), phi, mu, 20, nthreads=2)
    assert np.all(bm == 0.0)
    assert bd[0, -1].min() > bd[0, 0].max() >= 0.0  # pulled up from the top
