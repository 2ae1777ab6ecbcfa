"""Host-side pieces of bench.py: the device-source digest that guards the
recorded counter traffic, and the parsing of the committed summary."""
import json
import os
import shutil

import bench


def _fake_root(tmp_path, digest):
    root = tmp_path / "repo"
    csrc = root / "paper_1506_01684_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in bench.STEP_SOURCES:
        shutil.copy(os.path.join(bench.ROOT, "paper_1506_01684_amd", "csrc", name), csrc / name)
    (root / "profiles").mkdir()
    rec = {"kernel_source_sha256": digest, "fetch_scale": 2.0, "write_scale": 1.0,
           "kernels": {"c2": {"mu_tiled_f64": {"fetch_kib": 100.0, "write_kib": 50.0}}}}
    (root / "profiles" / "hbm_traffic.md").write_text(
        "# HBM traffic\n\ntext\n\n```json\n" + json.dumps(rec) + "\n```\n")
    return root


def test_traffic_is_used_only_for_matching_sources(tmp_path, monkeypatch):
    digest = bench.kernel_source_digest()
    root = _fake_root(tmp_path, digest)
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.kernel_source_digest() == digest
    assert bench.recorded_traffic("mu_tiled_f64", "c2") == (100.0 * 2.0 + 50.0) * 1024.0
    assert bench.recorded_traffic("phi_tiled_f64", "c2") is None
    # a changed device source invalidates the record
    src = root / "paper_1506_01684_amd" / "csrc" / "pf_tiled.hip"
    src.write_text(src.read_text() + "\n// changed\n")
    assert bench.kernel_source_digest() != digest
    assert bench.recorded_traffic("mu_tiled_f64", "c2") is None


def test_committed_summary_parses():
    path = os.path.join(bench.ROOT, "profiles", "hbm_traffic.md")
    text = open(path).read()
    rec = json.loads(text.split("```json\n", 1)[1].split("\n```", 1)[0])
    assert rec["fetch_scale"] > 0 and rec["write_scale"] > 0
    assert "c2" in rec["kernels"] and "c3" in rec["kernels"]


def test_owed_bytes_follow_the_item_classes():
    """Bytes a sweep owes per step: evaluated phi items 10 values per cell,
    kept items nothing (8 values when copied); mu items 12 values per cell,
    pure items 4.  With the shortcuts off (or the direct variant) every
    item is evaluated."""
    cells, es = 4096 * 8192, 8
    d0 = {"work_items": 4096, "fixed_items": 2000, "copied_items": 10, "mu_pure_items": 2500,
          "light_items": 3000}
    d1 = dict(d0, fixed_items=2100, copied_items=0, mu_pure_items=2600)
    o = bench.owed_bytes(d0, d1, cells, es, 1, 1)
    cpi = 8192
    assert o["phi"] == ((4096 - 2050) * 10 + 5 * 8) * cpi * es
    assert o["mu"] == ((4096 - 2550) * 12 + 2550 * 4) * cpi * es
    assert o["items"]["fixed"] == 2050 and o["items"]["mu_pure"] == 2550
    for sc, var in ((0, 1), (1, 0)):
        o = bench.owed_bytes(d0, d1, cells, es, sc, var)
        assert o["phi"] == 10 * cells * es and o["mu"] == 12 * cells * es


def test_valu_counts_are_used_only_for_matching_sources(tmp_path, monkeypatch):
    digest = bench.kernel_source_digest()
    root = _fake_root(tmp_path, digest)
    rec = {"kernel_source_sha256": digest,
           "kernels": {"c3": {"mu_pure_f32": {"valu_insts": 10.0, "grbm_gui_active": 1.0},
                              "mu_tiled_f32": {"valu_insts": 32.0, "grbm_gui_active": 1.0}}}}
    (root / "profiles" / "sq_counters.md").write_text(
        "# SQ\n\n```json\n" + json.dumps(rec) + "\n```\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.recorded_valu("mu_pure_f32+mu_tiled_f32", "c3") == 42.0
    assert bench.recorded_valu("mu_tiled_f64", "c3") is None
    src = root / "paper_1506_01684_amd" / "csrc" / "pf_device.h"
    src.write_text(src.read_text() + "\n// changed\n")
    assert bench.recorded_valu("mu_pure_f32+mu_tiled_f32", "c3") is None


def test_valu_peaks_follow_the_published_rates():
    # 64 lanes x 2 flops per FMA wave instruction
    assert abs(bench.VALU_PEAK_WIPS["double"] * 128 / 1e12 - 78.6) < 0.1
    assert abs(bench.VALU_PEAK_WIPS["float"] * 128 / 1e12 - 157.3) < 0.1


def test_pcie_inclusive_rate_counts_both_copies_and_the_steps():
    # 1e6 cells, 1000 steps of 1 ms, 0.5 s in and 0.5 s out: 1e9 LUP in 2 s
    hc = {"init_s": 0.5, "read_s": 0.5}
    assert abs(bench.pcie_inclusive_mlups(1_000_000, 1000, 1.0, hc) - 500.0) < 1e-9
    # without host copies it is the step rate itself
    assert abs(bench.pcie_inclusive_mlups(1_000_000, 1000, 1.0, {"init_s": 0, "read_s": 0})
               - 1000.0) < 1e-9
