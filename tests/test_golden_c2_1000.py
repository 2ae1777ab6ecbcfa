"""Checks of the stored 1000-step oracle sample of the 256x256x512 FP64
workload (tests/golden/c2_fp64_1000.npz, written by
tests/golden/make_c2_1000.py from the oracle alone), on the CPU:

  - it belongs to the workload's current parameters and time step;
  - the total concentration of its final state equals that of the initial
    Voronoi state up to rounding: the mu update is exactly conservative for
    periodic x/y and zero-flux z at any T(t) (Eq. (3) discretised with the
    exact-difference sources), so only the rounding of 3.4e7 cell updates
    per step, over 1000 steps, moves it.  On this domain that drift is about
    1e-11 relative (9.5e-12 after 475 steps), so the bound is 1e-10, well
    below any real flux or source error (a single unbalanced face flux of
    one cell per step would move it by more than 1e-9);
  - the sample is the one the script draws (cells in range, no repeats) and
    holds interface cells, so the GPU comparison sees the front.
"""
import os

import numpy as np
import pytest

import oracle
import pfinputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_fp64_1000.npz")

pytestmark = pytest.mark.skipif(not os.path.exists(GOLDEN),
                                reason="tests/golden/c2_fp64_1000.npz has not been written")


def test_golden_belongs_to_the_workload():
    from tests.golden.make_c2_1000 import params_digest, sample_cells

    z = np.load(GOLDEN)
    w = pfinputs.workload("c2")
    assert str(z["params_sha256"]) == params_digest(w["params"])
    assert float(z["dt"]) == oracle.default_dt(w["params"], w["shape"])
    assert int(z["steps"]) == 1000
    cells = z["cells"]
    assert np.array_equal(cells, sample_cells(w["shape"], w["solid_height"]))
    nz, ny, nx = w["shape"]
    assert cells[:, 0].max() < nx and cells[:, 1].max() < ny and cells[:, 2].max() < nz
    assert len({tuple(c) for c in cells.tolist()}) == len(cells)
    phi = z["phi"]
    assert np.all(np.abs(phi.sum(axis=1) - 1.0) <= 1e-12)
    assert np.all(phi >= 0.0) and np.all(phi <= 1.0)
    assert np.any((phi > 1e-3) & (phi < 1 - 1e-3))  # interface cells in the sample
    assert np.all(np.abs(phi).max(axis=0) <= z["maxabs_phi"])
    assert np.all(np.abs(z["mu"]).max(axis=0) <= z["maxabs_mu"])


def test_golden_conserves_the_total_concentration():
    z = np.load(GOLDEN)
    w = pfinputs.workload("c2")
    p = pfinputs.with_dt(w["params"], float(z["dt"]))
    phi0, mu0 = oracle.init_voronoi(w["shape"], w["seed"], w["nseeds"], w["solid_height"])
    d0 = oracle.diagnostics(p, phi0, mu0, 0.0)
    for q in range(2):
        rel = abs(float(z["sum_c"][q]) - d0["sum_c"][q]) / abs(d0["sum_c"][q])
        assert rel <= 1e-10, (q, rel)
