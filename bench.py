"""Benchmark of the phase-field time step (phi-sweep + mu-sweep) on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c3|c1]
                    [--variant 0|1] [--shortcuts 0|1] [--no-cpu] [--no-fp32]
                    [--no-plain] [--no-fp32-error] [--no-pack] [--no-serve]

Headline: the FP64 256x256x512 domain (64 Voronoi seeds, 128 solid layers,
synthetic parameter set P0, dt a quarter of the stability bound).  One step
is the prologue, the phi-sweep and the mu-sweep (Algorithm 1 of the paper)
with fields resident in HBM.  Exact shortcuts are on by default (their
results are bitwise identical to evaluating everything); the same workload
with them off is reported as "plain".  Also reported: the FP32 512x512x1024
anisotropic domain with its error against the FP64 path after 1000 steps,
the pack of 64 uneven FP32 domains, a serving trace, and the FP64 CPU
oracle timed on a bounded sample of the headline workload on the host's
cores.

Prints one JSON line.  MLUP/s = cells * steps / seconds / 1e6 (the paper's
unit, Sec. 5).  Roofline: the bytes the dominant sweep owes per launch,
divided by its average HIP-event duration, against 8 TB/s.  What a sweep
owes follows from the work it does: an item the phi-sweep evaluates reads
phi^n and mu^n and writes phi^{n+1} (10 values per cell), an item the bulk
shortcut keeps owes nothing, or 8 values per cell when it has to be copied;
an item the mu-sweep evaluates in full reads phi^n, phi^{n+1}, mu^n and
writes mu^{n+1} (12 values per cell), a pure item reads mu^n and writes
mu^{n+1} (4 values).  With the shortcuts off every item is evaluated, so the
owed bytes are the dense ones.  The item counts come from the library's
diagnostics (the step before and the last step of the timed run,
averaged).  The dense bytes over the same time are reported beside it as
"effective_gbs".  "traffic" is the HBM bytes per launch that rocprofv3
counted for the same kernel sources.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALUES_PER_CELL = {"phi": 10, "mu": 12}
# VALU issue peaks from the published vector rates and the unit counts
# (256 CUs at 2.4 GHz, 64 lanes per wave instruction, two flops per lane of
# an FMA): FP64 78.6 TFLOP/s is 78.6e12 / 128 = 6.144e11 wave instructions/s,
# one per clock per CU; FP32 157.3 TFLOP/s is twice that.  The counts are of
# every VALU instruction (address arithmetic, moves and selects included),
# so the fraction is an issue-rate utilisation.
VALU_PEAK_WIPS = {"double": 256 * 2.4e9, "float": 2 * 256 * 2.4e9}


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_gpu(workload: str, steps: int, warmup: int, variant: int, shortcuts: int = 1,
            solid_height: int | None = None, over: dict | None = None) -> dict:
    import torch

    import paper_1506_01684_amd as pf
    import pfinputs

    w = pfinputs.workload(workload)
    if solid_height is not None:  # same domain, front placed at another height
        dsl = w["params"]["delta"][0][3]
        w = dict(w, solid_height=solid_height,
                 params=pfinputs.p0_params(solid_height=solid_height, delta_sl=dsl))
    nz, ny, nx = w["shape"]
    cells = nx * ny * nz
    pf.set_variant(variant)
    d = pf.Domain(w["shape"], w["prec"])
    d.set_params(dict(w["params"], shortcuts=shortcuts, **(over or {})))
    d.init_voronoi(w["seed"], w["nseeds"], w["solid_height"])
    _log(f"[bench] {workload}: {nx}x{ny}x{nz} {w['prec']} shortcuts={shortcuts} "
         f"dt={d.dt:.6g} warmup {warmup}")
    d.step(warmup)
    d.sync()
    before = d.diagnostics()
    torch.cuda.synchronize()
    _log(f"[bench] {workload}: timing {steps} steps")
    t0 = time.perf_counter()
    phi_ms, mu_ms = d.step_timed(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    diag = d.diagnostics()
    d.close()
    esize = 8 if w["prec"] == "fp64" else 4
    out = {
        "workload": workload, "shape": [nx, ny, nz], "prec": w["prec"], "cells": cells,
        "steps": steps, "wall_s": wall, "ms_per_step": 1e3 * wall / steps,
        "mlups": cells * steps / wall / 1e6,
        "phi_ms": phi_ms / steps, "mu_ms": mu_ms / steps,
        "nonfinite": diag["nonfinite"], "max_simplex_dev": diag["max_simplex_dev"],
        "window_shifts": diag["window_shifts"],
    }
    owed = owed_bytes(before, diag, cells, esize, shortcuts, variant)
    out["items"] = owed["items"]
    for k in ("phi", "mu"):
        dense = VALUES_PER_CELL[k] * esize * cells
        sec = out[f"{k}_ms"] * 1e-3
        out[f"{k}_bytes_per_launch"] = owed[k]
        out[f"{k}_gbs"] = owed[k] / sec / 1e9
        out[f"{k}_dense_bytes"] = dense
        out[f"{k}_effective_gbs"] = dense / sec / 1e9
    step_dense = (VALUES_PER_CELL["phi"] + VALUES_PER_CELL["mu"]) * esize * cells
    step_s = wall / steps
    out["step_hbm_frac"] = (owed["phi"] + owed["mu"]) / step_s / 1e9 / HBM_PEAK_GBS
    out["step_effective_hbm_frac"] = step_dense / step_s / 1e9 / HBM_PEAK_GBS
    return out


def owed_bytes(before: dict, after: dict, cells: int, esize: int, shortcuts: int,
               variant: int) -> dict:
    """Bytes each sweep owes per step from the work it does (see the module
    docstring), from the item counts of the library's diagnostics: the mean
    of the step before the timed run and its last step.  Items are counted
    at the mean cells per item (every item of the benchmark's domains is
    whole)."""
    items = after["work_items"]
    cpi = cells / items

    def mean(k):
        return 0.5 * (before[k] + after[k])

    if shortcuts and variant == 1:
        fixed, copied, pure = mean("fixed_items"), mean("copied_items"), mean("mu_pure_items")
    else:
        fixed = copied = pure = 0.0
    phi = ((items - fixed) * VALUES_PER_CELL["phi"] + copied * 8) * cpi * esize
    mu = ((items - pure) * VALUES_PER_CELL["mu"] + pure * 4) * cpi * esize
    return {"phi": phi, "mu": mu,
            "items": {"work": items, "fixed": fixed, "copied": copied, "mu_pure": pure,
                      "light": mean("light_items")}}


def sweep_kernels(sweep: str, real: str, aniso: bool) -> str:
    """Kernel names of one sweep as rocprofv3 lists them, joined by '+'.  The
    mu-sweep is two launches (FP64: pure and light items, then the rest;
    FP32: pure items, then the rest), the phi-sweep the bulk shortcut's
    launch and the tiled sweep; with the shortcuts off the first launch of
    each sweep finds no item and returns at once."""
    if sweep == "mu":
        return "mu_light_f64+mu_tiled_f64" if real == "double" else "mu_pure_f32+mu_tiled_f32"
    return (f"phi_bulk_kernel<{real}>+phi_tiled_f{64 if real == 'double' else 32}"
            f"{'_aniso' if aniso else ''}")


def sweep_rooflines(run: dict, real: str, aniso: bool, workload: str, variant: int,
                    plain: bool = False) -> dict:
    """Per-sweep roofline of one timed run: the bytes the sweep owes per
    launch over its HIP-event time, against the HBM peak; the counter bytes
    of the same kernels when a matching rocprofv3 record exists."""
    out = {}
    for k in ("phi", "mu"):
        kn = sweep_kernels(k, real, aniso)
        tr = recorded_traffic(kn, workload + ("_plain" if plain else "")) if variant == 1 else None
        out[k] = {"kernel": kn, "ms": round(run[f"{k}_ms"], 4),
                  "bytes_per_launch": round(run[f"{k}_bytes_per_launch"]),
                  "achieved": round(run[f"{k}_gbs"], 1),
                  "frac": round(run[f"{k}_gbs"] / HBM_PEAK_GBS, 4),
                  "effective_gbs": round(run[f"{k}_effective_gbs"], 1),
                  "traffic": None if tr is None else round(tr)}
        # the ALU side of the same sweep: recorded VALU wave instructions per
        # launch (shortcuts on only; none recorded for the plain runs) over
        # the live sweep time, against the issue peak
        va = recorded_valu(kn, workload) if variant == 1 and not plain else None
        if va is not None:
            wips, peak = va / (run[f"{k}_ms"] * 1e-3), VALU_PEAK_WIPS[real]
            out[k]["alu"] = {"bound": "alu", "valu_wave_insts_per_launch": round(va),
                             "achieved": round(wips / 1e9, 2), "peak": round(peak / 1e9, 1),
                             "unit": "G wave-instructions/s", "frac": round(wips / peak, 4)}
    return out


def run_scenarios(steps: int, variant: int) -> dict:
    """The headline domain with the solid/liquid front at half height, and
    entirely solid or liquid (solid height Nz/2, Nz, 0), with the exact
    shortcuts on and off."""
    import pfinputs

    nz = pfinputs.workload("c2")["shape"][0]
    out = {}
    for name, hs in (("interface", nz // 2), ("solid", nz), ("liquid", 0)):
        r1 = run_gpu("c2", steps, 5, variant, 1, solid_height=hs)
        r0 = run_gpu("c2", steps, 5, variant, 0, solid_height=hs)
        out[name] = {"solid_height": hs, "mlups": round(r1["mlups"], 1),
                     "plain_mlups": round(r0["mlups"], 1),
                     "phi_ms": round(r1["phi_ms"], 4), "mu_ms": round(r1["mu_ms"], 4),
                     "plain_phi_ms": round(r0["phi_ms"], 4), "plain_mu_ms": round(r0["mu_ms"], 4)}
    return out


def run_window(steps: int, variant: int) -> dict:
    """Moving window on the headline domain: with the window plane far
    above the front (the per-step check only), and with it below the front
    so that every timed step starts with a shift (one plane of the whole
    state copied down)."""
    import pfinputs

    nz = pfinputs.workload("c2")["shape"][0]
    chk = run_gpu("c2", steps, 5, variant, 1, over={"window_z": nz - 64})
    n = min(steps, 48)
    sh = run_gpu("c2", n, 5, variant, 1, over={"window_z": 64})
    return {"check_only": {"window_z": nz - 64, "mlups": round(chk["mlups"], 1),
                           "ms_per_step": round(chk["ms_per_step"], 4),
                           "shifts": chk["window_shifts"]},
            "every_step_shifts": {"window_z": 64, "steps": n, "mlups": round(sh["mlups"], 1),
                                  "ms_per_step": round(sh["ms_per_step"], 4),
                                  "shifts": sh["window_shifts"]}}


def run_output(steps: int = 20, reps: int = 5) -> dict:
    """Output path on the headline domain after `steps` steps: the
    marching-cubes mesh of each phase (extraction into a device buffer,
    counted and synchronised, per call) and one FP32 checkpoint save/load
    through a file in /tmp."""
    import ctypes as C
    import tempfile

    import torch

    import paper_1506_01684_amd as pf
    from paper_1506_01684_amd import _capi as A
    import pfinputs

    w = pfinputs.workload("c2")
    nz, ny, nx = w["shape"]
    pf.set_variant(1)
    d = pf.Domain(w["shape"], "fp64")
    d.set_params(w["params"])
    d.init_voronoi(w["seed"], w["nseeds"], w["solid_height"])
    d.step(steps)
    d.sync()
    lib = pf.load()
    out = {"steps": steps, "phases": []}
    n = C.c_int64()
    for phase in range(4):
        empty = A.PfDeviceBuffer(None, 0)
        lib.pf_mesh_phase(d.handle, phase, 0.5, C.byref(empty), C.byref(n))
        buf = torch.empty(max(n.value, 1) * 9, dtype=torch.float32, device="cuda")
        dev = A.PfDeviceBuffer(C.c_void_p(buf.data_ptr()), n.value * 36)
        lib.pf_mesh_phase(d.handle, phase, 0.5, C.byref(dev), C.byref(n))  # warm-up
        t0 = time.perf_counter()
        for _ in range(reps):
            st = lib.pf_mesh_phase(d.handle, phase, 0.5, C.byref(dev), C.byref(n))
        ms = (time.perf_counter() - t0) / reps * 1e3
        if st != A.PF_OK:
            raise RuntimeError(f"mesh phase {phase}: status {st}")
        out["phases"].append({"phase": phase, "triangles": n.value, "ms": round(ms, 3),
                              "phi_read_gbs": round(8.0 * nx * ny * nz / (ms * 1e-3) / 1e9, 1)})
        del buf
    with tempfile.TemporaryDirectory(dir="/tmp") as tmp:
        path = os.path.join(tmp, "c2.pfc")
        t0 = time.perf_counter()
        d.save_checkpoint(path)
        t1 = time.perf_counter()
        d.load_checkpoint(path)
        t2 = time.perf_counter()
        out["checkpoint"] = {"bytes": os.path.getsize(path), "save_s": round(t1 - t0, 3),
                             "load_s": round(t2 - t1, 3)}
    # the host side of the boundary: all six fields to host memory as FP64
    # (pf_read_fields) and back (pf_init_fields from host arrays)
    t0 = time.perf_counter()
    phi, mu = d.read()
    t1 = time.perf_counter()
    d.init_host(phi, mu)
    d.sync()
    t2 = time.perf_counter()
    out["host_copy"] = {"field_bytes": 6 * 8 * nx * ny * nz, "read_s": round(t1 - t0, 3),
                        "init_s": round(t2 - t1, 3)}
    d.close()
    return out


def pcie_inclusive_mlups(cells: int, steps: int, ms_per_step: float, host_copy: dict) -> float:
    """Rate of a whole job that starts from host arrays and ends in host
    arrays: one pf_init_fields from the host, `steps` steps, one
    pf_read_fields (never the bench value, which starts from HBM)."""
    t = host_copy["init_s"] + host_copy["read_s"] + steps * ms_per_step * 1e-3
    return cells * steps / t / 1e6


def run_stream(nbytes: int = 2 << 30, reps: int = 10) -> dict:
    """STREAM-style device bandwidth with torch kernels on FP32 arrays of
    nbytes each: copy (b = a, 2 nbytes per pass) and add (b = a + c,
    3 nbytes per pass), event-timed over `reps` passes."""
    import torch

    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    c = torch.ones_like(a)
    b = torch.empty_like(a)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    copy = 2 * nbytes / timed(lambda: b.copy_(a)) / 1e9
    add = 3 * nbytes / timed(lambda: torch.add(a, c, out=b)) / 1e9
    del a, b, c
    return {"bytes_per_array": nbytes, "copy_gbs": round(copy, 1), "add_gbs": round(add, 1)}


def run_fp32_error(steps: int) -> dict:
    """The FP32-bulk path against the FP64 path on the 512x512x1024
    anisotropic domain after `steps` steps from the same initial state:
    max-abs error of phi and max over mu_i of max|dmu_i| / max|mu_i|."""
    import numpy as np

    import paper_1506_01684_amd as pf
    import pfinputs

    w = pfinputs.workload("c3")
    res = {}
    for prec in ("fp64", "fp32"):
        _log(f"[bench] c3 {prec}: {steps} steps for the FP32 error")
        d = pf.Domain(w["shape"], prec)
        d.set_params(w["params"])
        d.init_voronoi(w["seed"], w["nseeds"], w["solid_height"])
        d.step(steps)
        res[prec] = d.read()
        d.close()
    (p64, m64), (p32, m32) = res["fp64"], res["fp32"]
    dphi = float(np.max(np.abs(p32 - p64)))
    dmu = max(float(np.max(np.abs(m32[q] - m64[q]))) / float(np.max(np.abs(m64[q])))
              for q in range(2))
    return {"steps": steps, "phi_max_abs": dphi, "mu_rel": dmu,
            "tolerance": {"phi_max_abs": 2e-4, "mu_rel": 1e-4},
            "within": bool(dphi <= 2e-4 and dmu <= 1e-4)}


STEP_SOURCES = ("pf_device.h", "pf_kernels.hip", "pf_kernels_common.h", "pf_launch.h",
                "pf_runtime.hip", "pf_tiled.hip")


def kernel_source_digest() -> str:
    """SHA-256 over the sources of the step's kernels and their launch
    setup; a recorded counter measurement is used only while this digest is
    unchanged."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1506_01684_amd", "csrc")
    for name in STEP_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def recorded_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` (several kernels joined by '+' are
    summed: one sweep made of several launches) on `workload` from the
    committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary
    (profiles/hbm_traffic.md), each counter scaled by what it reads for a copy
    of known size; None when no summary matches the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_source_sha256") != kernel_source_digest():
        return None
    total = 0.0
    for name in kernel.split("+"):
        k = rec.get("kernels", {}).get(workload, {}).get(name)
        if not k:
            return None
        total += (k["fetch_kib"] * rec["fetch_scale"] + k["write_kib"] * rec["write_scale"]) * 1024.0
    return total


def recorded_valu(kernel: str, workload: str):
    """VALU wave instructions per launch of `kernel` (several joined by '+'
    are summed) on `workload`, from the committed rocprofv3 SQ summary
    (profiles/sq_counters.md); None when no summary matches the current
    kernel sources."""
    path = os.path.join(ROOT, "profiles", "sq_counters.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_source_sha256") != kernel_source_digest():
        return None
    total = 0.0
    for name in kernel.split("+"):
        k = rec.get("kernels", {}).get(workload, {}).get(name)
        if not k:
            return None
        total += k["valu_insts"]
    return total


def fp32_error(p32, m32, p64, m64) -> tuple[float, float]:
    """FP32 result against its FP64 twin: max-abs error of phi and, per mu
    component, max|dmu| / max|mu| (the larger of the two)."""
    import numpy as np

    dphi = float(np.max(np.abs(p32 - p64)))
    dmu = max(float(np.max(np.abs(m32[q] - m64[q]))) / max(float(np.max(np.abs(m64[q]))), 1e-300)
              for q in range(2))
    return dphi, dmu


def run_pack(count: int, steps: int, warmup: int) -> dict:
    """64 uneven FP32 domains: one pack (one launch per kernel per step over
    all domains, step captured in a HIP graph) vs looping single-domain
    launches over the same domains; then the same domains as an FP64 pack,
    whose results give the FP32 pack's error."""
    import torch

    import paper_1506_01684_amd as pf
    import pfinputs

    ws = pfinputs.pack_workloads(count)
    cells = sum(w["shape"][0] * w["shape"][1] * w["shape"][2] for w in ws)

    def make(prec="fp32"):
        doms = []
        for w in ws:
            d = pf.Domain(w["shape"], prec)
            d.set_params(w["params"])
            d.init_voronoi(w["seed"], w["nseeds"], w["solid_height"])
            doms.append(d)
        return doms

    def packed(prec):
        doms = make(prec)
        pk = pf.Pack(prec, max_domains=count)
        for d in doms:
            pk.add(d, warmup + steps)
        pk.step(warmup)
        pk.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pk.step(steps)
        pk.sync()
        t = time.perf_counter() - t0
        return pk, doms, t

    pk32, doms32, t_pack = packed("fp32")
    _log("[bench] pack: FP64 twin")
    pk64, doms64, t_pack64 = packed("fp64")
    dphi = dmu = 0.0
    for a, b in zip(doms32, doms64):
        e = fp32_error(*a.read(), *b.read())
        dphi, dmu = max(dphi, e[0]), max(dmu, e[1])
    for pk, doms in ((pk32, doms32), (pk64, doms64)):
        pk.close()
        for d in doms:
            d.close()
    _log("[bench] pack: looped single-domain launches")
    doms = make()
    for d in doms:
        d.step(warmup)
    for d in doms:
        d.sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        for d in doms:
            d.step(1)
    for d in doms:
        d.sync()
    t_loop = time.perf_counter() - t0
    for d in doms:
        d.close()
    return {
        "workload": f"{count} FP32 domains, lateral 32-192, height 64-384, {cells} cells",
        "steps": steps, "pack_mlups": round(cells * steps / t_pack / 1e6, 1),
        "loop_mlups": round(cells * steps / t_loop / 1e6, 1),
        "speedup": round(t_loop / t_pack, 3),
        "fp64_pack_mlups": round(cells * steps / t_pack64 / 1e6, 1),
        "error_vs_fp64": {"steps": warmup + steps, "phi_max_abs": dphi, "mu_rel": dmu,
                          "tolerance": {"phi_max_abs": 2e-4, "mu_rel": 1e-4},
                          "within": bool(dphi <= 2e-4 and dmu <= 1e-4)},
    }


def run_serving(count: int, lateral, steps_rng, rate: float, budget: float, serial: bool,
                policies=("fifo", "sjf"), progress: bool = False, fp32_twins: int = 0) -> dict:
    """Poisson arrivals of Voronoi solves of mixed size, step count and
    precision through the continuous-batching server; the serial baseline
    runs the same trace first come, first served with single-domain
    launches.  For the `fp32_twins` smallest FP32 requests the server keeps
    the fields (read back when the request finishes), and each is solved
    again in FP64 afterwards for the FP32 error."""
    import pfinputs
    from paper_1506_01684_amd import serving as S

    trace = pfinputs.serving_trace(count=count, rate=rate, lateral=lateral, steps=steps_rng)
    twins = sorted((t for t in trace if t["prec"] == "fp32"),
                   key=lambda t: t["shape"][0] * t["shape"][1] * t["shape"][2])[:fp32_twins]
    twin_ids = {t["id"] for t in twins}
    out = {
        "workload": f"{count} requests, Poisson {rate}/s, lateral {lateral[0]}-{lateral[1]}, "
                    f"Nz = 2L, steps {steps_rng[0]}-{steps_rng[1]}, fp32/fp64 half each, "
                    f"budget {budget / 1e9:.0f} GB",
        "lups": sum(t["shape"][0] * t["shape"][1] * t["shape"][2] * t["steps"] for t in trace),
    }
    kept = {}
    for pol in policies:
        _log(f"[bench] serving with policy {pol}")
        reqs = [S.request_from_trace(t, keep_fields=t["id"] in twin_ids) for t in trace]
        be = S.GpuBackend(max_domains=256)
        kw = {} if pol == "fifo" else dict(policy="sjf", target_cells=32e6, rate=2e10)
        srv = S.Server(be, budget_bytes=budget, max_slots=256, round_steps=25,
                       log=_log if progress else None, **kw)
        res = srv.run(reqs)
        be.shutdown()
        if pol == "fifo":
            out["server"] = dict(S.summarize(res), policy="arrival order, every request "
                                                          "admitted that fits")
        else:
            out["server_sjf"] = dict(S.summarize(res), policy="shortest expected job first "
                                                              "with aging, packs held to 32M cells")
        for r in res:
            if r.id in twin_ids and r.fields is not None:
                kept[r.id] = r.fields
    if serial:
        _log("[bench] serving: serial FIFO")
        out["serial_fifo"] = S.summarize(S.run_serial_gpu(
            [S.request_from_trace(t) for t in trace]))
    if twins:
        import paper_1506_01684_amd as pf

        errs = []
        for t in twins:
            if t["id"] not in kept:
                continue
            d = pf.Domain(t["shape"], "fp64")
            d.set_params(t["params"])
            d.init_voronoi(t["seed"], t["nseeds"], t["solid_height"])
            d.step(t["steps"])
            e = fp32_error(*kept[t["id"]], *d.read())
            d.close()
            errs.append({"id": t["id"], "shape": list(t["shape"]), "steps": t["steps"],
                         "phi_max_abs": e[0], "mu_rel": e[1],
                         "within": bool(e[0] <= 2e-4 and e[1] <= 1e-4)})
        out["fp32_error_vs_fp64"] = {
            "note": f"the {len(errs)} smallest FP32 requests, solved again in FP64 alone",
            "requests": errs, "tolerance": {"phi_max_abs": 2e-4, "mu_rel": 1e-4}}
    return out


def run_cpu_baseline(workload: str, budget_s: float = 20.0) -> dict:
    """The FP64 oracle (as it stands) on the host's cores, on a bounded sample:
    full steps of the headline domain from its Voronoi initial state."""
    import oracle
    import pfinputs

    w = pfinputs.workload(workload)
    shape = w["shape"]
    p = pfinputs.with_dt(w["params"], oracle.default_dt(w["params"], shape))
    threads = oracle.default_threads()
    phi, mu = oracle.init_voronoi(shape, w["seed"], w["nseeds"], w["solid_height"])
    cells = shape[0] * shape[1] * shape[2]
    n = 0
    t0 = time.perf_counter()
    while True:
        phi, mu = oracle.run(p, phi, mu, 1, step0=n, nthreads=threads)
        n += 1
        el = time.perf_counter() - t0
        if el * (n + 1) / n > budget_s:
            break
    # the host CPU as /proc/cpuinfo describes its first processor (a
    # virtual machine may report only the vendor's product line by name)
    host = {"cpu": "unknown"}
    keys = {"model name": "cpu", "cpu family": "family", "model": "model", "stepping": "stepping",
            "cpu MHz": "mhz", "cache size": "cache"}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break
                k, _, v = line.partition(":")
                if k.strip() in keys:
                    host[keys[k.strip()]] = v.strip()
    except OSError:
        pass
    host["nproc"] = os.cpu_count()
    host["usable_cpus"] = len(os.sched_getaffinity(0))
    # the small workload in full (100 steps), on one thread and on all
    w1 = pfinputs.workload("c1")
    s1 = w1["shape"]
    p1 = pfinputs.with_dt(w1["params"], oracle.default_dt(w1["params"], s1))
    c1_cells = s1[0] * s1[1] * s1[2]
    c1 = {}
    for nt in (1, threads):
        ph1, mu1 = oracle.init_voronoi(s1, w1["seed"], w1["nseeds"], w1["solid_height"])
        t1 = time.perf_counter()
        oracle.run(p1, ph1, mu1, 100, nthreads=nt)
        c1[nt] = c1_cells * 100 / (time.perf_counter() - t1) / 1e6
    return {
        "value": cells * n / el / 1e6, "unit": "MLUP/s", "cores": threads, "kind": "oracle",
        "sample": f"{n} full step(s) of the {shape[2]}x{shape[1]}x{shape[0]} FP64 domain "
                  f"from its Voronoi state, z planes split over {threads} threads, {el:.1f} s",
        "small_workload_full": {
            "workload": f"{s1[2]}x{s1[1]}x{s1[0]} FP64, 100 steps from its Voronoi state",
            "one_thread_mlups": round(c1[1], 3), "all_threads_mlups": round(c1[threads], 3),
            "threads": threads},
        "host": host,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3"])
    ap.add_argument("--variant", type=int, default=1)
    ap.add_argument("--fp32-steps", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-pack", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the timing with shortcuts off")
    ap.add_argument("--no-fp32-error", action="store_true",
                    help="skip the 1000-step FP32-vs-FP64 error run")
    ap.add_argument("--shortcuts", type=int, default=1, choices=[0, 1])
    ap.add_argument("--no-window", action="store_true",
                    help="skip the moving-window timings of the headline domain")
    ap.add_argument("--no-scenarios", action="store_true",
                    help="skip the interface/solid/liquid timings of the headline domain")
    ap.add_argument("--no-output", action="store_true",
                    help="skip the mesh and checkpoint timings of the headline domain")
    ap.add_argument("--pack-steps", type=int, default=500)
    ap.add_argument("--serve-count", type=int, default=24)
    ap.add_argument("--full-serving", action="store_true",
                    help="only run the full serving trace: 128 requests, lateral 64-384, "
                         "steps 200-5000, 200 GB budget (long)")
    ap.add_argument("--serve-policy", default="sjf", choices=["fifo", "sjf"],
                    help="scheduling policy of the --full-serving run")
    ap.add_argument("--serve-rate", type=float, default=20.0,
                    help="mean Poisson arrival rate (1/s) of the --full-serving run")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes 5 times "
                         "(reference for the FETCH_SIZE/WRITE_SIZE counter scale)")
    args = ap.parse_args()
    if args.calibrate_copy > 0:
        import torch

        a = torch.ones(args.calibrate_copy, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.calibrate_copy, "repeats": 5}))
        return
    if args.full_serving:
        r = run_serving(128, (64, 384), (200, 5000), args.serve_rate, 200e9, serial=False,
                        policies=(args.serve_policy,), progress=True)
        print(json.dumps({"metric": "served-solve latency (p50/p99)", "serving": r}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this benchmark runs on one GPU; --gpus must be 1 "
              "(sharding over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    main_run = run_gpu(args.workload, args.steps, args.warmup, args.variant, args.shortcuts)
    dom = "mu" if main_run["mu_ms"] >= main_run["phi_ms"] else "phi"
    achieved = main_run[f"{dom}_gbs"]
    real = "double" if main_run["prec"] == "fp64" else "float"
    aniso = "true" if args.workload == "c3" else "false"
    kname = sweep_kernels(dom, real, aniso == "true")
    traffic = recorded_traffic(kname, args.workload) if args.variant == 1 else None
    line = {
        "metric": "MLUP/s of phi+mu step (FP32 vs FP64) + %HBM peak",
        "value": round(main_run["mlups"], 1),
        "unit": "MLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_run["prec"] == "fp64" else "f32",
        "data": "synthetic (Voronoi-seeded solid lamellae under liquid, parameter set P0)",
        "config": {
            "workload": f"{args.workload}: {'x'.join(map(str, main_run['shape']))} cells, "
                        f"{main_run['prec']}, N=4 phases, K-1=2 mu",
            "cells": main_run["cells"], "variant": args.variant, "shortcuts": args.shortcuts,
            # bytes the two sweeps owe for the work they do, per step time
            "hbm_frac_step": round(main_run["step_hbm_frac"], 4),
            # dense bytes (22 values per cell) per step time
            "effective_hbm_frac_step": round(main_run["step_effective_hbm_frac"], 4),
            "phi_sweep_ms": round(main_run["phi_ms"], 4), "mu_sweep_ms": round(main_run["mu_ms"], 4),
            "items": main_run["items"],
        },
        "roofline": {
            "bound": "hbm", "kernel": kname,
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic),
            "bytes_per_launch": round(main_run[f"{dom}_bytes_per_launch"]),
            "effective_gbs": round(main_run[f"{dom}_effective_gbs"], 1),
            "dense_bytes_per_launch": main_run[f"{dom}_dense_bytes"],
            "sweeps": sweep_rooflines(main_run, real, aniso == "true", args.workload, args.variant),
        },
    }
    if not args.no_plain and args.shortcuts == 1:
        rp = run_gpu(args.workload, args.steps, args.warmup, args.variant, shortcuts=0)
        line["plain"] = {
            "note": "same workload with every face and cell evaluated (shortcuts off; "
                    "results are bitwise identical)",
            "mlups": round(rp["mlups"], 1), "ms_per_step": round(rp["ms_per_step"], 4),
            "phi_sweep_ms": round(rp["phi_ms"], 4), "mu_sweep_ms": round(rp["mu_ms"], 4),
            "hbm_frac_step": round(rp["step_hbm_frac"], 4),
            "roofline": sweep_rooflines(rp, real, aniso == "true", args.workload, args.variant,
                                        plain=True),
        }
    stream = run_stream()
    best = max(stream["copy_gbs"], stream["add_gbs"])
    line["roofline"]["stream"] = stream
    line["roofline"]["frac_of_stream"] = round(achieved / best, 4)
    if not args.no_scenarios and args.workload == "c2":
        _log("[bench] interface / solid / liquid scenarios")
        line["scenarios"] = run_scenarios(args.steps // 2, args.variant)
    if not args.no_window and args.workload == "c2":
        _log("[bench] moving window")
        line["window"] = run_window(args.steps // 2, args.variant)
    if not args.no_output and args.workload == "c2":
        _log("[bench] output path: meshes and checkpoint")
        line["output"] = run_output()
        hc = line["output"]["host_copy"]
        hc["pcie_inclusive_mlups_1000_steps"] = round(
            pcie_inclusive_mlups(main_run["cells"], 1000, main_run["ms_per_step"], hc), 1)
    if not args.no_fp32 and args.workload == "c2":
        r32 = run_gpu("c3", args.fp32_steps, 5, args.variant, args.shortcuts)
        line["fp32"] = {
            "workload": "c3: 512x512x1024 cells, fp32 bulk, cubic anisotropy 0.05",
            "mlups": round(r32["mlups"], 1), "ms_per_step": round(r32["ms_per_step"], 4),
            "hbm_frac_step": round(r32["step_hbm_frac"], 4),
            "effective_hbm_frac_step": round(r32["step_effective_hbm_frac"], 4),
            "phi_sweep_ms": round(r32["phi_ms"], 4), "mu_sweep_ms": round(r32["mu_ms"], 4),
            "items": r32["items"],
            "roofline": sweep_rooflines(r32, "float", True, "c3", args.variant),
            "steps": args.fp32_steps,
        }
        if not args.no_plain and args.shortcuts == 1:
            rp = run_gpu("c3", args.fp32_steps, 5, args.variant, shortcuts=0)
            line["fp32"]["plain"] = {
                "mlups": round(rp["mlups"], 1), "ms_per_step": round(rp["ms_per_step"], 4),
                "hbm_frac_step": round(rp["step_hbm_frac"], 4),
                "phi_sweep_ms": round(rp["phi_ms"], 4), "mu_sweep_ms": round(rp["mu_ms"], 4),
                "roofline": sweep_rooflines(rp, "float", True, "c3", args.variant, plain=True),
            }
        if not args.no_fp32_error:
            line["fp32"]["error_vs_fp64"] = run_fp32_error(1000)
    if not args.no_pack and args.workload == "c2":
        _log("[bench] pack of 64 domains")
        line["pack"] = run_pack(64, args.pack_steps, 5)
    if not args.no_serve and args.workload == "c2":
        _log("[bench] serving trace")
        line["serving"] = run_serving(args.serve_count, (64, 384), (200, 5000), 20.0, 200e9,
                                      serial=True, fp32_twins=3)
    if not args.no_cpu:
        _log("[bench] timing the CPU oracle")
        line["cpu_baseline"] = run_cpu_baseline(args.workload)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
