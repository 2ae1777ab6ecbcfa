"""GPU tests of the output path (Sec. 3.2, Input/Output): FP32 checkpoints
of the state and the marching-cubes interface mesh of each phase, checked
against the oracle's mesh triangle by triangle."""
import os
import tempfile

import numpy as np
import pytest

import oracle
import pfinputs
from tests.gpu_util import gpu_domain, lib, log

pytestmark = pytest.mark.gpu


def _canon(tris):
    """Triangles as a sorted array: each rotated (winding kept) to start at
    its smallest vertex, then ordered lexicographically."""
    t = np.asarray(tris, np.float32).reshape(-1, 3, 3)
    if len(t) == 0:
        return t.reshape(0, 9)
    order = np.lexsort((t[:, :, 2], t[:, :, 1], t[:, :, 0]), axis=1)[:, 0]  # smallest vertex
    rot = np.stack([t[np.arange(len(t)), (order + k) % 3] for k in range(3)], axis=1)
    flat = rot.reshape(-1, 9)
    return flat[np.lexsort(flat.T[::-1])]


def _state(shape, prec, steps, hs, seed=7, nseeds=9, aniso=0.0, **over):
    p = pfinputs.p0_params(solid_height=hs, delta_sl=aniso)
    p.update(over)
    p["dt"] = oracle.default_dt(p, shape)
    d = gpu_domain(shape, p, prec, 1, voronoi=(seed, nseeds, hs))
    d.step(steps)
    return d, p


@pytest.mark.parametrize("shape,prec,steps", [((40, 33, 70), "fp64", 12), ((24, 20, 36), "fp32", 20),
                                              ((16, 8, 8), "fp64", 0)])
def test_mesh_matches_oracle_exactly(shape, prec, steps):
    d, _ = _state(shape, prec, steps, hs=shape[0] // 3)
    phi, _ = d.read()
    log(f"mesh {shape} {prec} after {steps} steps")
    for phase in range(4):
        for iso in (0.5, 0.3):
            got = d.mesh(phase, iso)
            ref = oracle.mesh_phase(phi, phase, iso)
            log(f"  phase {phase} iso {iso}: {len(got)} triangles (oracle {len(ref)})")
            assert len(got) == len(ref)
            assert np.array_equal(_canon(got), _canon(ref))
    d.close()


def test_mesh_at_full_size_matches_oracle():
    """The 256x256x512 FP64 workload after 20 steps: the liquid's interface
    (front and the films along the lamella boundaries) and one solid."""
    d, _ = _state((512, 256, 256), "fp64", 20, hs=128, seed=42, nseeds=64)
    phi, _ = d.read()
    for phase in (3, 0):
        got = d.mesh(phase, 0.5)
        ref = oracle.mesh_phase(phi, phase, 0.5)
        log(f"full size phase {phase}: {len(got)} triangles")
        assert len(got) == len(ref) and len(got) > 100000
        assert np.array_equal(_canon(got), _canon(ref))
    d.close()


def test_mesh_buffer_too_small_reports_the_total():
    import ctypes as C

    import torch

    pf = lib()
    from paper_1506_01684_amd import _capi as A

    d, _ = _state((20, 16, 24), "fp64", 3, hs=6)
    n = C.c_int64()
    empty = A.PfDeviceBuffer(None, 0)
    st = pf.load().pf_mesh_phase(d.handle, 3, 0.5, C.byref(empty), C.byref(n))
    total = n.value
    assert st == A.PF_ERR_INVALID_ARG and total > 10
    buf = torch.zeros(9 * 10, dtype=torch.float32, device="cuda")
    small = A.PfDeviceBuffer(C.c_void_p(buf.data_ptr()), 36 * 10)
    st = pf.load().pf_mesh_phase(d.handle, 3, 0.5, C.byref(small), C.byref(n))
    assert st == A.PF_ERR_INVALID_ARG and n.value == total
    part = buf.cpu().numpy().reshape(-1, 3, 3)
    full = {tuple(r) for r in _canon(d.mesh(3, 0.5))}
    assert all(tuple(r) in full for r in _canon(part))  # the first ten are real triangles
    for bad in (-1, 4):
        assert pf.load().pf_mesh_phase(d.handle, bad, 0.5, C.byref(empty), C.byref(n)) == \
            A.PF_ERR_INVALID_ARG
    assert pf.load().pf_mesh_phase(d.handle, 0, float("nan"), C.byref(empty), C.byref(n)) == \
        A.PF_ERR_INVALID_ARG
    d.close()


def _read_ckpt(path):
    raw = open(path, "rb").read()
    h = np.frombuffer(raw[:64], np.uint8)
    magic = bytes(h[:8])
    nx, ny, nz, prec = np.frombuffer(raw[8:24], "<i4")
    step, shifts = np.frombuffer(raw[24:40], "<i8")
    dx, dt = np.frombuffer(raw[40:56], "<f8")
    data = np.frombuffer(raw[64:], "<f4").reshape(6, nz, ny, nx)
    return magic, (int(nx), int(ny), int(nz), int(prec)), int(step), int(shifts), (dx, dt), data


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_checkpoint_round_trip_and_resume(prec):
    shape = (30, 20, 36)
    hs = 10
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "state.pfc")
        d, p = _state(shape, prec, 7, hs)
        phi0, mu0 = d.read()
        d.save_checkpoint(path)
        magic, dims, step, shifts, (dx, dt), data = _read_ckpt(path)
        assert magic == b"PFCKPT01" and dims == (36, 20, 30, 0 if prec == "fp64" else 1)
        assert step == 7 and shifts == 0 and dx == 1.0 and dt == p["dt"]
        assert np.array_equal(data[:4], phi0.astype(np.float32))
        assert np.array_equal(data[4:], mu0.astype(np.float32))
        # the domain that wrote it goes on unchanged
        assert np.array_equal(d.read()[0], phi0)
        d.step(9)
        cont = d.read()
        d.close()
        e = lib().Domain(shape, prec)
        e.set_params(p)
        e.load_checkpoint(path)
        assert e.step_index == 7
        phi1, mu1 = e.read()
        assert np.array_equal(phi1, phi0.astype(np.float32).astype(np.float64))
        assert np.array_equal(mu1, mu0.astype(np.float32).astype(np.float64))
        e.step(9)
        res = e.read()
        e.close()
    if prec == "fp32":  # the checkpoint holds the FP32 state exactly
        assert np.array_equal(res[0], cont[0]) and np.array_equal(res[1], cont[1])
    else:
        # loading is exactly a restart from the rounded state at step 7 ...
        f = lib().Domain(shape, prec)
        f.set_params(p)
        f.init_host(phi0.astype(np.float32).astype(np.float64),
                    mu0.astype(np.float32).astype(np.float64))
        f.set_time(7)
        f.step(9)
        ref = f.read()
        f.close()
        assert np.array_equal(res[0], ref[0]) and np.array_equal(res[1], ref[1])
        # ... which stays close to the run that was never rounded
        dphi = np.max(np.abs(res[0] - cont[0]))
        dmu = np.max(np.abs(res[1] - cont[1])) / np.max(np.abs(cont[1]))
        log(f"checkpoint fp64 resume after 9 steps: phi {dphi:.1e}, mu rel {dmu:.1e}")
        assert dphi < 1e-6 and dmu < 1e-3


def test_checkpoint_keeps_window_shifts_and_dirichlet_top():
    shape = (40, 8, 8)
    p = pfinputs.p0_params(solid_height=20, G=0.04, v=1.0)
    p.update(window_z=16, top_bc=1, mu_fill=(0.01, -0.02))
    p["dt"] = oracle.default_dt(p, shape)
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "w.pfc")
        d = gpu_domain(shape, p, "fp32", 1, voronoi=(3, 2, 20))
        d.step(60)
        sh = d.diagnostics()["window_shifts"]
        assert sh > 0
        d.save_checkpoint(path)
        d.step(40)
        cont, dg = d.read(), d.diagnostics()
        d.close()
        e = lib().Domain(shape, "fp32")
        e.set_params(p)
        e.load_checkpoint(path)
        assert e.diagnostics()["window_shifts"] == sh and e.step_index == 60
        e.step(40)
        res, eg = e.read(), e.diagnostics()
        e.close()
    assert eg["window_shifts"] == dg["window_shifts"]
    assert np.array_equal(res[0], cont[0]) and np.array_equal(res[1], cont[1])


def test_checkpoint_errors():
    pf = lib()
    shape = (12, 8, 10)
    p = pfinputs.p0_params(solid_height=4)
    p["dt"] = oracle.default_dt(p, shape)
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "a.pfc")
        d = gpu_domain(shape, p, "fp64", 1, voronoi=(1, 3, 4))
        d.save_checkpoint(path)
        other = pf.Domain((12, 8, 12), "fp64")
        other.set_params(p)
        with pytest.raises(pf.PfError) as e:
            other.load_checkpoint(path)
        assert "INVALID_ARG" in str(e.value)
        with pytest.raises(pf.PfError) as e:
            d.load_checkpoint(os.path.join(tmp, "missing.pfc"))
        assert "IO" in str(e.value)
        junk = os.path.join(tmp, "junk.pfc")
        open(junk, "wb").write(b"x" * 200)
        with pytest.raises(pf.PfError) as e:
            d.load_checkpoint(junk)
        assert "INVALID_ARG" in str(e.value)
        short = os.path.join(tmp, "short.pfc")
        open(short, "wb").write(open(path, "rb").read()[:1000])
        before = d.read()
        with pytest.raises(pf.PfError) as e:
            d.load_checkpoint(short)
        assert "IO" in str(e.value)
        after = d.read()  # a truncated file leaves the state alone
        assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
        fresh = pf.Domain(shape, "fp64")
        with pytest.raises(pf.PfError) as e:
            fresh.load_checkpoint(path)  # no parameters yet
        assert "STATE" in str(e.value)
        with pytest.raises(pf.PfError) as e:
            fresh.save_checkpoint(path)  # no state yet
        assert "STATE" in str(e.value)
        with pytest.raises(pf.PfError) as e:
            d.save_checkpoint(os.path.join(tmp, "no", "such", "dir.pfc"))
        assert "IO" in str(e.value)
        for x in (d, other, fresh):
            x.close()
