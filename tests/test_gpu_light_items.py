"""GPU tests of the FP64 mu-sweep split by work-item class: an item whose
faces cannot carry the anti-trapping current (Eq. 4 weights each solid by
its product with the liquid, so no liquid, or only liquid, around the item
means none) is evaluated by a lighter kernel when such items are the large
majority of a step; the result is bitwise the one of the full kernel."""
import numpy as np
import pytest

import oracle
import pfinputs
from tests.gpu_util import gpu_domain, lib, log

pytestmark = pytest.mark.gpu


def _run(shape, p, prec, steps, shortcuts, voronoi, variant=1):
    q = dict(p)
    q["shortcuts"] = shortcuts
    d = gpu_domain(shape, q, prec, variant, voronoi=voronoi)
    d.step(steps)
    out = d.read()
    dg = d.diagnostics()
    d.close()
    return out, dg


@pytest.mark.parametrize("hs,aniso", [(4, False), (4, True), (40, False), (24, False)])
def test_split_is_bitwise_exact(hs, aniso):
    """Mostly liquid (hs = 4): most items are light and the split runs, and
    the top chunks take the mu-from-mu-alone path inside the light kernel;
    mostly solid (hs = 40 of 64): liquid films along the lamella boundaries
    make most items heavy; half liquid (hs = 24): too few light items for
    the split, so the full kernel takes the pure top chunks too.  Either way
    shortcuts on equals shortcuts off."""
    shape = (64, 40, 70)
    p = pfinputs.p0_params(solid_height=hs, delta_sl=0.05 if aniso else 0.0)
    p["dt"] = oracle.default_dt(p, shape)
    a, da = _run(shape, p, "fp64", 12, 1, (5, 9, hs))
    b, db = _run(shape, p, "fp64", 12, 0, (5, 9, hs))
    frac = da["light_items"] / da["work_items"]
    log(f"split hs={hs} aniso={aniso}: light items {da['light_items']} of {da['work_items']} "
        f"({frac:.2f}), mu from mu alone {da['mu_pure_items']}, "
        f"max |dmu| {np.max(np.abs(a[1] - b[1])):.1e}")
    assert db["light_items"] == 0 and db["mu_pure_items"] == 0
    if hs == 4:
        assert frac >= 0.6  # the light kernel really ran
        assert da["mu_pure_items"] > 0
    if hs == 24:
        assert frac < 0.6 and da["mu_pure_items"] > 0
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_light_items_reported_only_for_the_fp64_tiled_sweep():
    pf = lib()
    shape = (32, 24, 40)
    p = pfinputs.p0_params(solid_height=3)
    p["dt"] = oracle.default_dt(p, shape)
    d = gpu_domain(shape, p, "fp64", 1, voronoi=(3, 4, 3))
    assert d.diagnostics()["light_items"] == 0  # no step yet
    d.step(2)
    dg = d.diagnostics()
    assert 0 < dg["light_items"] <= dg["work_items"]
    d.close()
    try:
        for prec, var in (("fp32", 1), ("fp64", 0)):
            _, dg = _run(shape, p, prec, 2, 1, (3, 4, 3), variant=var)
            assert dg["light_items"] == 0, (prec, var)
    finally:
        pf.set_variant(1)


@pytest.mark.parametrize("prec,aniso,top_bc", [("fp64", False, 0), ("fp32", True, 0),
                                               ("fp64", True, 1)])
def test_bulk_chunks_are_copied_exactly(prec, aniso, top_bc):
    """Chunks that hold one pure phase, with all their neighbours, at a fixed
    point are copied by the phi bulk shortcut: most of a tall liquid column
    is; the mu-sweep of a chunk that, with all its neighbours, holds one
    pure phase before and after the phi-sweep reads mu alone.  The result equals the shortcuts-off run bitwise (with the
    Dirichlet top too, whose liquid ghost allows only liquid chunks at the
    top)."""
    shape = (96, 24, 70)
    p = pfinputs.p0_params(solid_height=10, delta_sl=0.05 if aniso else 0.0)
    p["top_bc"] = top_bc
    p["dt"] = oracle.default_dt(p, shape)
    a, da = _run(shape, p, prec, 10, 1, (4, 7, 10))
    b, db = _run(shape, p, prec, 10, 0, (4, 7, 10))
    log(f"bulk {prec} aniso={aniso} top_bc={top_bc}: fixed items {da['fixed_items']} of "
        f"{da['work_items']}, mu from mu alone {da['mu_pure_items']}")
    assert da["fixed_items"] > da["work_items"] // 3 and db["fixed_items"] == 0
    # chunks pure, with all their neighbours, before and after the phi-sweep:
    # mu from mu alone
    assert 0 < da["mu_pure_items"] <= da["work_items"] and db["mu_pure_items"] == 0
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_bulk_flags_survive_variant_switches_and_window_shifts():
    """Flags are only trusted when the tiled sweep wrote them for the state at
    hand: switching to the direct variant and back, and moving-window shifts,
    must not let a stale flag copy a chunk that changed."""
    pf = lib()
    shape = (64, 16, 40)
    p = pfinputs.p0_params(solid_height=20, G=0.04, v=1.0)
    p.update(window_z=12)  # below the front: shifts in the first steps
    p["dt"] = oracle.default_dt(p, shape)
    out = {}
    try:
        for sc in (0, 1):
            q = dict(p, shortcuts=sc)
            d = gpu_domain(shape, q, "fp64", 1, voronoi=(2, 5, 20))
            for var, n in ((1, 6), (0, 3), (1, 6), (0, 1), (1, 8)):
                pf.set_variant(var)
                d.step(n)
            out[sc] = (d.read(), d.diagnostics())
            d.close()
    finally:
        pf.set_variant(1)
    (a, da), (b, db) = out[1], out[0]
    log(f"switches: shifts {da['window_shifts']}, fixed items {da['fixed_items']}")
    assert da["window_shifts"] > 0 and da["window_shifts"] == db["window_shifts"]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_bulk_skip_survives_a_checkpoint_save():
    """A bulk chunk kept for two steps is not copied again (both field copies
    hold it); saving a checkpoint uses the second copy as staging, so the
    flags must be withdrawn: stepping on after a save equals the
    shortcuts-off run bitwise."""
    import os
    import tempfile

    shape = (96, 24, 70)
    p = pfinputs.p0_params(solid_height=10)
    p["dt"] = oracle.default_dt(p, shape)
    out = {}
    with tempfile.TemporaryDirectory() as tmp:
        for sc in (0, 1):
            q = dict(p, shortcuts=sc)
            d = gpu_domain(shape, q, "fp64", 1, voronoi=(4, 7, 10))
            d.step(6)
            d.save_checkpoint(os.path.join(tmp, f"s{sc}.pfc"))
            d.step(5)
            out[sc] = (d.read(), d.diagnostics())
            d.close()
    (a, da), (b, _) = out[1], out[0]
    assert da["fixed_items"] > 0 and da["mu_pure_items"] > 0
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("prec,top_bc", [("fp64", 0), ("fp32", 1)])
def test_bulk_skip_survives_host_reads(prec, top_bc):
    """pf_read_fields stages each field in the copy that does not hold the
    state, which the bulk shortcut may take for equal to the current one:
    reading the fields to the host between steps, then stepping on, equals
    the shortcuts-off run bitwise (with a Dirichlet top too, whose ghost
    planes the staging covers), and each read equals the other run's."""
    shape = (96, 24, 70)
    p = pfinputs.p0_params(solid_height=10)
    p["top_bc"] = top_bc
    p["dt"] = oracle.default_dt(p, shape)
    out = {}
    for sc in (0, 1):
        q = dict(p, shortcuts=sc)
        d = gpu_domain(shape, q, prec, 1, voronoi=(4, 7, 10))
        reads = []
        for n in (6, 1, 4):
            d.step(n)
            reads.append(d.read())
        out[sc] = (reads, d.diagnostics())
        d.close()
    (ra, da), (rb, _) = out[1], out[0]
    log(f"host reads {prec} top_bc={top_bc}: fixed items {da['fixed_items']}, "
        f"copied {da['copied_items']}")
    assert da["fixed_items"] > 0
    for a, b in zip(ra, rb):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def _chunk_layout(shape, prec):
    """Tile and z chunk of the tiled sweeps (the rule the library applies:
    FP64 tiles are always 32x8, FP32 tiles 64x4 unless nx < 48)."""
    nz, ny, nx = shape
    tx = 64 if nx >= 48 and prec != "fp64" else 32
    ty = 256 // tx
    ntx, nty = -(-nx // tx), -(-ny // ty)
    zc = min(32, max(8, nz * ntx * nty // 2048), nz)
    return tx, ty, zc


def _chunk_purity(phi, tx, ty, zc):
    """Per chunk [iz, iy, ix]: the phase all its cells hold purely, and the
    same for its first and its last plane (-1: none)."""
    nz, ny, nx = phi.shape[1:]
    cell = np.full((nz, ny, nx), -1)
    for a in range(4):
        others = np.ones((nz, ny, nx), bool)
        for b in range(4):
            if b != a:
                others &= phi[b] == 0.0
        cell[(phi[a] == 1.0) & others] = a

    def common(block):
        v = np.unique(block)
        return int(v[0]) if len(v) == 1 and v[0] >= 0 else -1
    shp = (-(-nz // zc), -(-ny // ty), -(-nx // tx))
    whole, first, last = (np.full(shp, -1) for _ in range(3))
    for iz, iy, ix in np.ndindex(*shp):
        z0, y0, x0 = iz * zc, iy * ty, ix * tx
        z1 = min(z0 + zc, nz)
        blk = cell[z0:z1, y0:y0 + ty, x0:x0 + tx]
        whole[iz, iy, ix] = common(blk)
        first[iz, iy, ix] = common(blk[0])
        last[iz, iy, ix] = common(blk[-1])
    return whole, first, last


def _expected_pure_items(before, after, top_bc):
    """Items whose chunk and the cells its stencils read around it hold one
    phase purely before and after the step: the chunk and its lateral
    neighbours whole, the chunks below by their last plane, those above by
    their first (periodic in x and y; outside the domain in z the chunk
    itself), liquid only at a Dirichlet top."""
    nzc, nty, ntx = before[0].shape
    n = 0
    for iz, iy, ix in np.ndindex(nzc, nty, ntx):
        a = after[0][iz, iy, ix]
        if a < 0 or (iz == nzc - 1 and top_bc and a != 3):
            continue
        ok = True
        for whole, first, last in (before, after):
            for dz, dy, dx in np.ndindex(3, 3, 3):
                jz = iz + dz - 1
                jz = iz if jz < 0 or jz >= nzc else jz
                j = (jz, (iy + dy - 1) % nty, (ix + dx - 1) % ntx)
                v = (last, whole, first)[dz][j]
                ok = ok and v == a
        n += ok
    return n


@pytest.mark.parametrize("prec,aniso,top_bc", [("fp64", False, 0), ("fp32", True, 1)])
def test_pure_item_count_matches_the_fields(prec, aniso, top_bc):
    """The mu-sweep's pure items of one step are exactly the chunks that the
    fields before and after the step make pure, end planes included (a
    count from the fields read back, computed here)."""
    shape = (96, 24, 70)
    p = pfinputs.p0_params(solid_height=10, delta_sl=0.05 if aniso else 0.0)
    p["top_bc"] = top_bc
    p["dt"] = oracle.default_dt(p, shape)
    d = gpu_domain(shape, p, prec, 1, voronoi=(4, 7, 10))
    d.step(8)
    phi0, _ = d.read()
    d.step(1)
    phi1, _ = d.read()
    dg = d.diagnostics()
    d.close()
    tx, ty, zc = _chunk_layout(shape, prec)
    want = _expected_pure_items(_chunk_purity(phi0, tx, ty, zc), _chunk_purity(phi1, tx, ty, zc), top_bc)
    log(f"pure items {prec} top_bc={top_bc}: {dg['mu_pure_items']} (fields: {want}) of {dg['work_items']}")
    assert 0 < want < dg["work_items"]
    assert dg["mu_pure_items"] == want


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kw", [{"antitrapping": 0}, {"mu_frozen": 1}])
def test_shortcuts_exact_without_antitrapping_or_with_frozen_mu(prec, kw):
    """Without the anti-trapping current every FP64 item is light, and with
    mu frozen no item may take a pure or light mu body: in both cases the
    tile shortcuts still equal shortcuts off bitwise."""
    shape = (96, 24, 70)
    p = pfinputs.p0_params(solid_height=10)
    p.update(kw)
    p["dt"] = oracle.default_dt(p, shape)
    a, da = _run(shape, p, prec, 10, 1, (4, 7, 10))
    b, _ = _run(shape, p, prec, 10, 0, (4, 7, 10))
    log(f"{prec} {kw}: fixed {da['fixed_items']}, light {da['light_items']}, "
        f"pure {da['mu_pure_items']} of {da['work_items']}")
    assert da["fixed_items"] > 0
    if kw.get("mu_frozen"):
        assert da["mu_pure_items"] == 0 and da["light_items"] == 0
    else:
        assert da["mu_pure_items"] > 0
        if prec == "fp64":
            assert da["light_items"] == da["work_items"]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
