"""Dirichlet top boundary on the GPU (Sec. 3.1 boundary handling; ghost
plane above the top held at liquid, phi = e_liquid, and mu = mu_fill)
against the oracle, the exact discrete decay of the cosine modes that
vanish at the ghost plane, and together with the moving window."""
import numpy as np
import pytest

import oracle
import pfinputs
from tests.gpu_util import field_errors, gpu_domain, lib, log

pytestmark = pytest.mark.gpu


def _params(shape, hs, **kw):
    p = pfinputs.p0_params(solid_height=hs)
    p["chi1"] = [[0.2, 0.1]] * 4
    p["c1"] = [[0.05, -0.02], [0.1, 0.03], [-0.07, 0.02], [0.1, -0.1]]
    p.update(kw)
    p["dt"] = oracle.default_dt(p, shape)
    return p


@pytest.mark.parametrize("prec,variant,aniso", [("fp64", 1, 0.0), ("fp64", 0, 0.0),
                                                ("fp64", 1, 0.05), ("fp32", 1, 0.05)])
def test_dirichlet_matches_oracle(prec, variant, aniso):
    shape, hs = (24, 20, 36), 16   # front 8 planes below the top
    p = _params(shape, hs, top_bc=1, mu_fill=(0.04, -0.03))
    for a in range(3):
        p["delta"][a][3] = p["delta"][3][a] = aniso
    phi0, mu0 = oracle.init_voronoi(shape, 9, 4, hs)
    log(f"case dirichlet {prec} variant {variant} aniso {aniso}")
    po, mo = oracle.run(p, phi0, mu0, 40)
    d = gpu_domain(shape, p, prec, variant, phi=phi0, mu=mu0)
    d.step(40)
    pg, mg = d.read()
    d.close()
    e = field_errors(pg, mg, po, mo)
    log(f"  errors {max(e):.2e}")
    # the boundary acts: the top plane differs from the mirror run
    pm, mm = oracle.run(dict(p, top_bc=0), phi0, mu0, 40)
    assert np.max(np.abs(mm[:, -1] - mo[:, -1])) > 1e-3
    if prec == "fp64":
        assert max(e) <= 1e-12
    else:
        assert float(np.max(np.abs(pg - po))) <= 2e-4 and max(e[4:]) <= 1e-4


def test_dirichlet_mode_decay_on_gpu():
    nz, n, m = 24, 8, 1
    shape = (nz, n, n)
    p = pfinputs.p0_params(solid_height=0, G=0.0, v=0.0)
    p["c1"] = [[0.0, 0.0]] * 4
    p["top_bc"] = 1
    p["dt"] = oracle.default_dt(p, shape)
    theta = np.pi * (m + 0.5) / (nz + 0.5)
    mode = np.cos(theta * (np.arange(nz) + 0.5))
    phi, mu = oracle.init_voronoi(shape, 1, 0, 0)
    mu[0] = 0.3 * mode[:, None, None]
    mu[1] = -0.2 * mode[:, None, None]
    d = gpu_domain(shape, p, "fp64", 1, phi=phi, mu=mu)
    d.step(60)
    _, mg = d.read()
    d.close()
    r = 1.0 - 4.0 * p["D"][3] * p["dt"] * np.sin(theta / 2) ** 2
    for q, amp in ((0, 0.3), (1, -0.2)):
        want = amp * r ** 60 * mode[:, None, None] * np.ones((1, n, n))
        assert np.max(np.abs(mg[q] - want)) / np.max(np.abs(want)) < 1e-12


def test_dirichlet_with_window_and_pack():
    shape, hs = (40, 24, 72), 12
    p = _params(shape, hs, top_bc=1, window_z=10, mu_fill=(0.05, -0.02))
    phi0, mu0 = oracle.init_voronoi(shape, 5, 3, hs)
    po, mo, sh = oracle.run_window(p, phi0, mu0, 20, zw=10, mu_fill=(0.05, -0.02))
    pf = lib()
    a = gpu_domain(shape, p, "fp64", 1, phi=phi0, mu=mu0)
    b = gpu_domain((24, 16, 16), dict(pfinputs.p0_params(solid_height=8), dt=0.0), "fp64", 1,
                   voronoi=(3, 2, 8))
    pk = pf.Pack("fp64", max_domains=4)
    pk.add(a, 20)
    pk.add(b, 20)
    pk.step(20)
    pk.sync()
    pg, mg = a.read()
    assert a.diagnostics()["window_shifts"] == sh == 2
    assert max(field_errors(pg, mg, po, mo)) <= 1e-12
    pk.close()
    a.close()
    b.close()


def test_top_bc_validated():
    pf = lib()
    shape = (16, 8, 8)
    d = pf.Domain(shape, "fp64")
    with pytest.raises(pf.PfError) as e:
        d.set_params(dict(_params(shape, 4), top_bc=2))
    assert "INVALID_ARG" in str(e.value)
    d.close()
