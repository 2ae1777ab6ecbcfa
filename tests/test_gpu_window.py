"""Moving window on the GPU (Sec. 3.3 moving-window technique) against the
oracle's window run: same shift count, fields within the parity bound;
packs carry windowed domains bitwise; invalid window planes are rejected."""
import numpy as np
import pytest

import oracle
import pfinputs
from tests.gpu_util import field_errors, gpu_domain, lib, log

pytestmark = pytest.mark.gpu


def _params(shape, hs, G=1e-3, v=0.01, **kw):
    p = pfinputs.p0_params(solid_height=hs, G=G, v=v)
    p["chi1"] = [[0.2, 0.1]] * 4
    p["c1"] = [[0.05, -0.02], [0.1, 0.03], [-0.07, 0.02], [0.1, -0.1]]
    p.update(kw)
    p["dt"] = oracle.default_dt(p, shape)
    return p


@pytest.mark.parametrize("prec,shape,hs,zw,steps,G,v,fill", [
    ("fp64", (40, 24, 72), 12, 10, 20, 1e-3, 0.01, (0.05, -0.02)),   # two shifts at once
    ("fp64", (40, 8, 8), 20, 20, 1000, 0.04, 1.0, (0.0, 0.0)),       # front passes the plane
    ("fp32", (40, 24, 72), 12, 10, 20, 1e-3, 0.01, (0.05, -0.02)),
])
def test_window_matches_oracle(prec, shape, hs, zw, steps, G, v, fill):
    p = _params(shape, hs, G=G, v=v, window_z=zw, mu_fill=fill)
    phi0, mu0 = oracle.init_voronoi(shape, 5, 3, hs)
    log(f"case window {prec} {shape} zw={zw} steps={steps}")
    po, mo, sh = oracle.run_window(p, phi0, mu0, steps, zw=zw, mu_fill=fill)
    d = gpu_domain(shape, p, prec, 1, phi=phi0, mu=mu0)
    d.step(steps)
    pg, mg = d.read()
    dg = d.diagnostics()
    d.close()
    e = field_errors(pg, mg, po, mo)
    log(f"  shifts gpu {dg['window_shifts']} oracle {sh}; errors {max(e):.2e}")
    assert dg["window_shifts"] == sh and sh >= 1
    if prec == "fp64":
        assert max(e) <= 1e-12
    else:
        assert float(np.max(np.abs(pg - po))) <= 2e-4 and max(e[4:]) <= 1e-4


def test_window_in_pack_is_bitwise_alone():
    shape, hs = (40, 24, 72), 12
    p = _params(shape, hs, window_z=10, mu_fill=(0.05, -0.02))
    phi0, mu0 = oracle.init_voronoi(shape, 5, 3, hs)
    pf = lib()
    alone = gpu_domain(shape, p, "fp32", 1, phi=phi0, mu=mu0)
    alone.step(12)
    ref = alone.read()
    alone.close()
    other = pfinputs.p0_params(solid_height=8)
    a = gpu_domain(shape, p, "fp32", 1, phi=phi0, mu=mu0)
    b = gpu_domain((24, 16, 16), dict(other, dt=0.0), "fp32", 1, voronoi=(3, 2, 8))
    pk = pf.Pack("fp32", max_domains=4)
    pk.add(a, 12)
    pk.add(b, 12)
    pk.step(12)
    pk.sync()
    got = a.read()
    assert a.diagnostics()["window_shifts"] == 2
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    pk.close()
    a.close()
    b.close()


def test_window_plane_validated():
    pf = lib()
    shape = (16, 8, 8)
    p = _params(shape, 4)
    d = pf.Domain(shape, "fp64")
    for bad in (-1, shape[0] - 1, shape[0]):
        with pytest.raises(pf.PfError) as e:
            d.set_params(dict(p, window_z=bad))
        assert "INVALID_ARG" in str(e.value)
    d.set_params(dict(p, window_z=shape[0] - 2))
    d.close()
