"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (tiled variant, the runtime's own tiling):

  - 256x256x512 FP64 and 512x512x1024 FP32 anisotropic: one step from the
    Voronoi state, sampled cells against the oracle's per-cell functions
    (the oracle computes phi^{n+1} itself wherever the mu update needs it);
  - properties that hold at any size: conservation of the total
    concentration, the simplex constraint, finiteness;
  - the FP32 path against the GPU FP64 path after 1000 steps on the
    512x512x1024 domain (phi max-abs <= 2e-4, mu relative <= 1e-4).
"""
import os

import numpy as np
import pytest

import oracle
import pfinputs
from tests.gpu_util import lib, log

pytestmark = pytest.mark.gpu


def _sample_cells(shape, solid_height, rng, n_random=600):
    nz, ny, nx = shape
    cells = set()
    for _ in range(n_random):
        cells.add((int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))))
    # columns through the solid-liquid front, all boundary planes, tile edges
    for _ in range(12):
        i, j = int(rng.integers(nx)), int(rng.integers(ny))
        for k in range(max(0, solid_height - 3), min(nz, solid_height + 3)):
            cells.add((i, j, k))
    for k in (0, 1, nz - 2, nz - 1):
        for _ in range(20):
            cells.add((int(rng.integers(nx)), int(rng.integers(ny)), k))
    for i in (0, 63, 64, nx - 1):
        for j in (0, 3, 4, ny - 1):
            cells.add((i, j, solid_height - 1))
            cells.add((i, j, solid_height))
    return sorted(cells)


def _oracle_samples(p, phi0, mu0, cells, t0=0.0):
    """phi^{n+1} and mu^{n+1} of the sampled cells, one cell at a time, for
    the step that starts at time t0."""
    nz, ny, nx = phi0.shape[1:]
    dt = p["dt"]
    phi1 = phi0.copy()
    need = set()
    for (i, j, k) in cells:
        need.add((i, j, k))
        for (a, b, c) in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            kk = k + c
            if 0 <= kk < nz:
                need.add(((i + a) % nx, (j + b) % ny, kk))
    for (i, j, k) in need:
        phi1[:, k, j, i] = oracle.phi_cell(p, phi0, mu0, t0, i, j, k)
    out_phi, out_mu = [], []
    for (i, j, k) in cells:
        out_phi.append(phi1[:, k, j, i].copy())
        out_mu.append(oracle.mu_cell(p, phi0, phi1, mu0, t0, t0 + dt, i, j, k))
    return np.array(out_phi), np.array(out_mu)


def _one_step_sampled(name, tol_phi, tol_mu_rel):
    pf = lib()
    pf.set_variant(1)
    w = pfinputs.workload(name)
    shape = w["shape"]
    p = pfinputs.with_dt(w["params"], oracle.default_dt(w["params"], shape))
    log(f"case {name} full size one step: init")
    phi0, mu0 = oracle.init_voronoi(shape, w["seed"], w["nseeds"], w["solid_height"])
    d = pf.Domain(shape, w["prec"])
    d.set_params(p)
    d.init_voronoi(w["seed"], w["nseeds"], w["solid_height"])
    d.step(1)
    phi_g, mu_g = d.read()
    d.close()
    rng = np.random.default_rng(7)
    cells = _sample_cells(shape, w["solid_height"], rng)
    log(f"case {name}: oracle on {len(cells)} sampled cells")
    ph_o, mu_o = _oracle_samples(p, phi0, mu0, cells)
    idx = tuple(np.array(cells).T)  # (i, j, k)
    ph_g = np.stack([phi_g[a][idx[2], idx[1], idx[0]] for a in range(4)], axis=1)
    mu_gs = np.stack([mu_g[q][idx[2], idx[1], idx[0]] for q in range(2)], axis=1)
    e_phi = float(np.max(np.abs(ph_g - ph_o)))
    scale = max(float(np.max(np.abs(mu_o))), 1e-300)
    e_mu = float(np.max(np.abs(mu_gs - mu_o))) / scale
    log(f"{name}: phi max-abs {e_phi:.2e}, mu rel {e_mu:.2e} (max |mu| {scale:.2e})")
    assert e_phi <= tol_phi and e_mu <= tol_mu_rel
    # the front actually moved and mu actually changed on the sample
    assert np.max(np.abs(ph_o - np.stack([phi0[a][idx[2], idx[1], idx[0]] for a in range(4)], 1))) > 1e-3
    assert scale > 0


def test_c2_fullsize_one_step_fp64_sampled():
    _one_step_sampled("c2", 1e-12, 1e-12)


def test_c3_fullsize_one_step_fp32_sampled():
    _one_step_sampled("c3", 5e-6, 1e-4)


def test_c2_fullsize_step_with_tile_shortcuts_sampled():
    """A later step of the 256x256x512 FP64 domain, when the bulk phi chunks
    and the pure mu items are in use: the state before the step is read back
    and the oracle evaluates the step's sampled cells from it (the liquid
    far above the front, where those shortcuts act, included)."""
    pf = lib()
    pf.set_variant(1)
    w = pfinputs.workload("c2")
    shape = w["shape"]
    p = pfinputs.with_dt(w["params"], oracle.default_dt(w["params"], shape))
    d = pf.Domain(shape, w["prec"])
    d.set_params(p)
    d.init_voronoi(w["seed"], w["nseeds"], w["solid_height"])
    n = 5
    d.step(n)
    phi0, mu0 = d.read()
    d.step(1)
    phi_g, mu_g = d.read()
    dg = d.diagnostics()
    d.close()
    log(f"c2 step {n + 1}: kept {dg['fixed_items']}, pure mu {dg['mu_pure_items']}, "
        f"light {dg['light_items']} of {dg['work_items']}")
    assert dg["fixed_items"] > dg["work_items"] // 2 and dg["mu_pure_items"] > dg["work_items"] // 2
    rng = np.random.default_rng(11)
    cells = _sample_cells(shape, w["solid_height"], rng)
    nz, ny, nx = shape
    for _ in range(200):  # the pure liquid far above the front
        cells.append((int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz // 2, nz))))
    cells = sorted(set(cells))
    ph_o, mu_o = _oracle_samples(p, phi0, mu0, cells, t0=n * p["dt"])
    idx = tuple(np.array(cells).T)
    ph_g = np.stack([phi_g[a][idx[2], idx[1], idx[0]] for a in range(4)], axis=1)
    mu_gs = np.stack([mu_g[q][idx[2], idx[1], idx[0]] for q in range(2)], axis=1)
    e_phi = float(np.max(np.abs(ph_g - ph_o)))
    scale = max(float(np.max(np.abs(mu_o))), 1e-300)
    e_mu = float(np.max(np.abs(mu_gs - mu_o))) / scale
    log(f"c2 step {n + 1} on {len(cells)} cells: phi max-abs {e_phi:.2e}, mu rel {e_mu:.2e}")
    assert e_phi <= 1e-12 and e_mu <= 1e-12
    assert float(np.max(np.abs(mu_gs - np.stack([mu0[q][idx[2], idx[1], idx[0]] for q in range(2)], 1)))) > 0


def test_c2_fullsize_invariants_over_200_steps():
    pf = lib()
    pf.set_variant(1)
    w = pfinputs.workload("c2")
    d = pf.Domain(w["shape"], "fp64")
    d.set_params(w["params"])
    d.init_voronoi(w["seed"], w["nseeds"], w["solid_height"])
    d0 = d.diagnostics()
    d.step(200)
    d1 = d.diagnostics()
    d.close()
    drift = [abs(d1["sum_c"][q] - d0["sum_c"][q]) / abs(d0["sum_c"][q]) for q in range(2)]
    log(f"c2 200 steps: sum c drift {drift}, simplex dev {d1['max_simplex_dev']:.1e}, "
        f"phi in [{d1['phi_min']}, {d1['phi_max']}]")
    assert max(drift) <= 1e-12
    assert d1["max_simplex_dev"] <= 1e-14 and d1["nonfinite"] == 0
    assert d1["phi_min"] >= 0.0 and d1["phi_max"] <= 1.0
    assert d1["step"] == 200


def test_c3_fp32_vs_fp64_after_1000_steps():
    """512x512x1024, anisotropic: the FP32 path (FP64 temperature, time,
    projection and sums) stays within phi max-abs 2e-4 and mu relative
    1e-4 of the FP64 path after 1000 steps."""
    pf = lib()
    pf.set_variant(1)
    w = pfinputs.workload("c3")
    res = {}
    for prec in ("fp64", "fp32"):
        log(f"case c3 1000 steps {prec}")
        d = pf.Domain(w["shape"], prec)
        d.set_params(w["params"])
        d.init_voronoi(w["seed"], w["nseeds"], w["solid_height"])
        d.step(1000)
        res[prec] = (d.read(), d.diagnostics())
        d.close()
    (p64, m64), g64 = res["fp64"]
    (p32, m32), g32 = res["fp32"]
    dphi = float(np.max(np.abs(p32 - p64)))
    dmu = max(float(np.max(np.abs(m32[q] - m64[q]))) / float(np.max(np.abs(m64[q]))) for q in range(2))
    del p64, p32, m64, m32
    drift = [abs(g32["sum_c"][q] - g64["sum_c"][q]) / abs(g64["sum_c"][q]) for q in range(2)]
    log(f"c3 after 1000 steps: phi max-abs {dphi:.2e}, mu rel {dmu:.2e}, "
        f"sum c fp32 vs fp64 {drift}")
    assert dphi <= 2e-4 and dmu <= 1e-4
    assert g32["nonfinite"] == 0 and g64["nonfinite"] == 0


GOLDEN_C2 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_fp64_1000.npz")


@pytest.mark.parametrize("shortcuts", [1, 0])
def test_c2_1000_steps_fp64_against_oracle(shortcuts):
    """The 256x256x512 FP64 workload over its 1000 steps against the
    oracle's state after 1000 steps (tests/golden/c2_fp64_1000.npz, written
    by tests/golden/make_c2_1000.py from the oracle alone): about 4900
    sampled cells (whole columns, front columns, boundary planes, tile and
    chunk edges, liquid and solid interiors) at rel-inf <= 1e-12 per field
    (max error over the sample / max |value| of the whole field), and the
    total concentration of the whole domain."""
    from tests.golden.make_c2_1000 import params_digest

    if not os.path.exists(GOLDEN_C2):
        pytest.skip("tests/golden/c2_fp64_1000.npz has not been written")
    z = np.load(GOLDEN_C2)
    w = pfinputs.workload("c2")
    assert str(z["params_sha256"]) == params_digest(w["params"])
    steps = int(z["steps"])
    p = pfinputs.with_dt(w["params"], float(z["dt"]))
    pf = lib()
    pf.set_variant(1)
    log(f"case c2 {steps} steps FP64 shortcuts={shortcuts}")
    d = pf.Domain(w["shape"], "fp64")
    d.set_params(dict(p, shortcuts=shortcuts))
    d.init_voronoi(w["seed"], w["nseeds"], w["solid_height"])
    d.step(steps)
    phi_g, mu_g = d.read()
    dg = d.diagnostics()
    d.close()
    i, j, k = z["cells"][:, 0], z["cells"][:, 1], z["cells"][:, 2]
    ph = np.stack([phi_g[a][k, j, i] for a in range(4)], axis=1)
    mu = np.stack([mu_g[q][k, j, i] for q in range(2)], axis=1)
    del phi_g, mu_g
    e_phi = [float(np.max(np.abs(ph[:, a] - z["phi"][:, a]))) / float(z["maxabs_phi"][a])
             for a in range(4)]
    e_mu = [float(np.max(np.abs(mu[:, q] - z["mu"][:, q]))) / float(z["maxabs_mu"][q])
            for q in range(2)]
    e_c = [abs(dg["sum_c"][q] - float(z["sum_c"][q])) / abs(float(z["sum_c"][q])) for q in range(2)]
    log(f"c2 {steps} steps, {len(i)} cells: phi rel {max(e_phi):.2e}, mu rel {max(e_mu):.2e}, "
        f"sum c rel {max(e_c):.2e}; kept {dg['fixed_items']}, pure mu {dg['mu_pure_items']}")
    # Sum c of the whole domain: each side drifts from the initial value by
    # the rounding of its own cell updates (about 1e-11 relative over these
    # 1000 steps on this domain; both sides conserve it exactly in exact
    # arithmetic), so the two agree to that, not to the per-cell 1e-12.
    assert max(e_phi) <= 1e-12 and max(e_mu) <= 1e-12 and max(e_c) <= 1e-10
    assert dg["step"] == steps and dg["nonfinite"] == 0
    # the sample holds interface cells whose state the run changed
    assert np.any((z["phi"] > 1e-3) & (z["phi"] < 1 - 1e-3))
