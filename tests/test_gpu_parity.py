"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
identical seeded inputs.

Bar: FP64 path within 1e-12 of the oracle, relative to each field's max
(max|a-b| / max|b| per field); FP32 path within 2e-4 absolute on phi and
1e-4 relative on mu of the GPU FP64 path; integer-like state (initial
fields, pure bulk cells) bitwise.
"""
import os

import numpy as np
import pytest

import oracle
import pfinputs
from tests.gpu_util import field_errors, gpu_domain, lib, log, params_full, rel_inf

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
VARIANTS = [int(v) for v in os.environ.get("PF_TEST_VARIANTS", "0,1").split(",")]
DEFAULT_VARIANT = VARIANTS[-1]


def _oracle_run(p, phi, mu, n, step0=0):
    return oracle.run(p, phi, mu, n, step0=step0)


def _assert_close64(phi_g, mu_g, phi_o, mu_o, tol=TOL64, what=""):
    e = field_errors(phi_g, mu_g, phi_o, mu_o)
    log(f"{what} rel errors phi0..3 mu0..1: " + " ".join(f"{v:.2e}" for v in e))
    assert max(e) <= tol, e


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("shape", [(8, 12, 16), (9, 17, 70), (5, 3, 2)])
def test_one_step_smooth_state_fp64(variant, shape):
    log(f"case one_step_smooth variant={variant} shape={shape}")
    p = params_full(shape, 3, G=2e-3, v=0.05)
    phi, mu = pfinputs.smooth_interface_state(shape, 5, width=2.0)
    d = gpu_domain(shape, p, "fp64", variant, phi, mu)
    assert abs(d.dt - p["dt"]) <= 1e-15 * p["dt"]
    d.set_time(3)
    d.step(1)
    phi_g, mu_g = d.read()
    phi_o, mu_o = _oracle_run(p, phi, mu, 1, step0=3)
    _assert_close64(phi_g, mu_g, phi_o, mu_o, what="one step")
    d.close()


@pytest.mark.parametrize("variant", VARIANTS)
def test_one_step_anisotropic_fp64(variant):
    shape = (10, 12, 20)
    log(f"case one_step_aniso variant={variant}")
    p = params_full(shape, 3, G=2e-3, v=0.05, delta_sl=0.05)
    p["delta"][0][1] = p["delta"][1][0] = 0.02
    phi, mu = pfinputs.smooth_interface_state(shape, 6, width=2.0)
    d = gpu_domain(shape, p, "fp64", variant, phi, mu)
    d.step(2)
    phi_g, mu_g = d.read()
    phi_o, mu_o = _oracle_run(p, phi, mu, 2)
    _assert_close64(phi_g, mu_g, phi_o, mu_o, what="aniso 2 steps")
    d.close()


@pytest.mark.parametrize("variant", VARIANTS)
def test_switches_mu_frozen_and_no_antitrapping(variant):
    shape = (8, 8, 8)
    for kw in ({"mu_frozen": 1}, {"antitrapping": 0}):
        log(f"case switches variant={variant} {kw}")
        p = params_full(shape, 3, **kw)
        phi, mu = pfinputs.smooth_interface_state(shape, 8, width=2.0)
        d = gpu_domain(shape, p, "fp64", variant, phi, mu)
        d.step(3)
        phi_g, mu_g = d.read()
        phi_o, mu_o = _oracle_run(p, phi, mu, 3)
        _assert_close64(phi_g, mu_g, phi_o, mu_o, what=str(kw))
        if kw.get("mu_frozen"):
            assert np.array_equal(mu_g, mu)
        d.close()


def test_voronoi_init_bitwise_equals_oracle():
    w = pfinputs.workload("c1")
    shape = w["shape"]
    for prec in ("fp64", "fp32"):
        log(f"case voronoi_init {prec}")
        p = pfinputs.with_dt(w["params"], 0.0)
        d = gpu_domain(shape, p, prec, DEFAULT_VARIANT,
                       voronoi=(w["seed"], w["nseeds"], w["solid_height"]))
        phi_g, mu_g = d.read()
        phi_o, mu_o = oracle.init_voronoi(shape, w["seed"], w["nseeds"], w["solid_height"])
        assert np.array_equal(phi_g, phi_o) and np.array_equal(mu_g, mu_o)
        assert abs(d.dt - oracle.default_dt(w["params"], shape)) <= 1e-16
        d.close()


@pytest.mark.parametrize("variant", VARIANTS)
def test_c1_100_steps_fp64(variant):
    """32x32x64, 12 Voronoi seeds, 100 steps at a quarter of the bound."""
    w = pfinputs.workload("c1")
    shape = w["shape"]
    log(f"case c1_100 variant={variant}")
    p = pfinputs.with_dt(w["params"], oracle.default_dt(w["params"], shape))
    d = gpu_domain(shape, p, "fp64", variant, voronoi=(w["seed"], w["nseeds"], w["solid_height"]))
    d.step(w["steps"])
    phi_g, mu_g = d.read()
    dg = d.diagnostics()
    phi0, mu0 = oracle.init_voronoi(shape, w["seed"], w["nseeds"], w["solid_height"])
    phi_o, mu_o = _oracle_run(p, phi0, mu0, w["steps"])
    _assert_close64(phi_g, mu_g, phi_o, mu_o, what="c1 100 steps")
    do = oracle.diagnostics(p, phi_o, mu_o, w["steps"] * p["dt"])
    assert dg["step"] == w["steps"]
    for q in range(2):
        assert abs(dg["sum_c"][q] - do["sum_c"][q]) <= 1e-12 * abs(do["sum_c"][q])
    for a in range(4):
        assert abs(dg["sum_phi"][a] - do["sum_phi"][a]) <= 1e-12 * max(1.0, abs(do["sum_phi"][a]))
    assert dg["nonfinite"] == 0 and dg["max_simplex_dev"] <= 1e-15
    assert dg["phi_min"] >= 0.0 and dg["phi_max"] <= 1.0
    d.close()


@pytest.mark.skipif(len(VARIANTS) < 2, reason="needs both kernel variants")
def test_variants_agree_on_c1():
    w = pfinputs.workload("c1")
    shape = w["shape"]
    out = []
    for variant in VARIANTS:
        d = gpu_domain(shape, w["params"], "fp64", variant,
                       voronoi=(w["seed"], w["nseeds"], w["solid_height"]))
        d.step(20)
        out.append(d.read())
        d.close()
    e = field_errors(out[1][0], out[1][1], out[0][0], out[0][1])
    log("variant 1 vs 0: " + " ".join(f"{v:.1e}" for v in e))
    assert max(e) <= 1e-13


@pytest.mark.parametrize("variant", VARIANTS)
def test_translation_is_bitwise(variant):
    shape = (12, 20, 70)  # ragged against 64x4 tiles
    p = params_full(shape, 4, delta_sl=0.05)
    phi, mu = pfinputs.smooth_interface_state(shape, 9, width=2.0)

    def sh(f):
        return np.ascontiguousarray(np.roll(np.roll(f, 37, axis=3), 5, axis=2))

    log(f"case translation variant={variant}")
    a = gpu_domain(shape, p, "fp64", variant, phi, mu)
    b = gpu_domain(shape, p, "fp64", variant, sh(phi), sh(mu))
    a.step(3)
    b.step(3)
    pa, ma = a.read()
    pb, mb = b.read()
    assert np.array_equal(pb, sh(pa)) and np.array_equal(mb, sh(ma))
    a.close()
    b.close()


def test_fp32_tracks_fp64_on_c1():
    """FP32 bulk (FP64 projection, temperature and sums) vs the GPU FP64 run."""
    w = pfinputs.workload("c1")
    shape = w["shape"]
    res = {}
    for prec in ("fp64", "fp32"):
        d = gpu_domain(shape, w["params"], prec, DEFAULT_VARIANT,
                       voronoi=(w["seed"], w["nseeds"], w["solid_height"]))
        d.step(w["steps"])
        res[prec] = d.read()
        d.close()
    dphi = np.max(np.abs(res["fp32"][0] - res["fp64"][0]))
    dmu = max(rel_inf(res["fp32"][1][q], res["fp64"][1][q]) for q in range(2))
    log(f"fp32 vs fp64 after 100 steps: phi max-abs {dphi:.2e}, mu rel {dmu:.2e}")
    assert dphi <= 2e-4 and dmu <= 1e-4


def test_error_paths():
    pf = lib()
    shape = (8, 8, 8)
    p = params_full(shape, 2)
    d = pf.Domain(shape, "fp64")
    with pytest.raises(pf.PfError) as e:
        d.step(1)
    assert "STATE" in str(e.value)
    bad = dict(p)
    bad["dt"] = 10.0
    with pytest.raises(pf.PfError) as e:
        d.set_params(bad)
    assert "UNSTABLE" in str(e.value)
    bad = dict(p)
    bad["delta"] = [[0.0, 0.0, 0.0, 0.1], [0.0] * 4, [0.0] * 4, [0.1, 0.0, 0.0, 0.0]]
    with pytest.raises(pf.PfError) as e:
        d.set_params(bad)
    assert "INVALID_ARG" in str(e.value)
    d.set_params(p)
    with pytest.raises(pf.PfError):
        d.step(1)  # fields not initialised
    phi, mu = pfinputs.random_state(shape, 1)
    phi[0, 2, 3, 4] = np.nan
    d.init_host(phi, mu)
    with pytest.raises(pf.PfError) as e:
        d.diagnostics()
    assert "NONFINITE" in str(e.value)
    d.close()
    with pytest.raises(pf.PfError):
        pf.Domain((0, 4, 4))
    # a refused initialisation leaves the domain as it was
    d = pf.Domain(shape, "fp64")
    d.set_params(p)
    d.init_voronoi(3, 4, 2)
    d.step(3)
    before = d.read()
    with pytest.raises(pf.PfError) as e:
        d.init_voronoi(3, -1, 2)
    assert "INVALID_ARG" in str(e.value)
    assert d.step_index == 3
    after = d.read()
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    d.close()


@pytest.mark.parametrize("prec,aniso,nucleating", [("fp64", False, False), ("fp32", True, False),
                                                   ("fp64", True, True), ("fp32", False, True)])
def test_shortcuts_are_bitwise_exact(prec, aniso, nucleating):
    """Skipping exactly-known work (zero-gradient faces, pure fixed-point
    cells) leaves every value bitwise unchanged.  With a tiny gamma_01 and a
    fast tau_1, phase 1 nucleates inside pure phase 0, so pure cells are
    not fixed points and must still be computed."""
    shape = (40, 48, 70)
    p = pfinputs.p0_params(solid_height=10, delta_sl=0.05 if aniso else 0.0)
    if nucleating:
        p["gamma"][0][1] = p["gamma"][1][0] = 0.01
        p["tau"] = [1.0, 0.1, 1.0, 1.0]
    p["dt"] = oracle.default_dt(p, shape)
    out = {}
    for sc in (0, 1):
        q = dict(p)
        q["shortcuts"] = sc
        d = gpu_domain(shape, q, prec, 1, voronoi=(17, 9, 10))
        d.step(15)
        out[sc] = d.read()
        d.close()
    log(f"shortcuts {prec} aniso={aniso} nucleating={nucleating}: "
        f"max |diff| {np.max(np.abs(out[0][0] - out[1][0])):.1e}")
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    if nucleating:  # the nucleation really happens inside the pure solid
        solid0 = out[1][0][0, 2] > 0.5
        assert out[1][0][1, 2][solid0].max() > 0.0
