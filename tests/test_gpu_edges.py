"""Edge cases of the decomposition and the boundaries: one-cell axes,
one or two planes, ragged tiles in both tile shapes, and both precisions,
each against the oracle."""
import numpy as np
import pytest

import oracle
import pfinputs
from tests.gpu_util import field_errors, gpu_domain, log, params_full

pytestmark = pytest.mark.gpu

SHAPES = [(1, 8, 8), (2, 5, 7), (20, 1, 1), (3, 1, 40), (6, 33, 1), (7, 9, 97), (5, 70, 65),
          (4, 4, 129)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_edge_shapes_against_oracle(shape, prec):
    log(f"case edge shape={shape} {prec}")
    p = params_full(shape, max(1, shape[0] // 3), G=2e-3, v=0.05, delta_sl=0.05)
    phi, mu = pfinputs.smooth_interface_state(shape, 3, width=1.5)
    d = gpu_domain(shape, p, prec, 1, phi, mu)
    d.step(3)
    phi_g, mu_g = d.read()
    d.close()
    phi_o, mu_o = oracle.run(p, phi, mu, 3)
    if prec == "fp64":
        e = field_errors(phi_g, mu_g, phi_o, mu_o)
        log("rel errors " + " ".join(f"{v:.1e}" for v in e))
        assert max(e) <= 1e-12
    else:
        dphi = float(np.max(np.abs(phi_g - phi_o)))
        dmu = float(np.max(np.abs(mu_g - mu_o))) / max(float(np.max(np.abs(mu_o))), 1e-30)
        log(f"fp32: phi {dphi:.1e} mu rel {dmu:.1e}")
        assert dphi <= 1e-5 and dmu <= 1e-4
    assert np.all(np.isfinite(phi_g)) and np.all(np.isfinite(mu_g))
