"""Write tests/golden/c2_fp64_1000.npz: sampled cells of the 256x256x512 FP64
workload after 1000 time steps of the CPU oracle (Sec. 2 Eqs. (1)-(4),
Algorithm 1), with the per-field maxima and the diagnostics of the whole
final state.

Calls only ``oracle`` and ``pfinputs``; nothing here comes from the HIP
library.  Command that wrote the committed file (about four hours on eight
cores of the build host; the oracle's results do not depend on the thread
count):

    python -m tests.golden.make_c2_1000 --threads 7 --state /path/to/state.npz

``--state`` keeps the oracle state every ``--every`` steps so that an
interrupted run resumes where it stopped.  The sample: three whole columns
(bottom to top), 16 columns through the front at the initial solid height,
cells on the four boundary planes, cells on tile and chunk edges of the
256x256 lateral grid, and random cells deep in the liquid and in the solid,
all drawn with numpy's default_rng(20150601).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import time

import numpy as np

import oracle
import pfinputs

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "c2_fp64_1000.npz")
STEPS = 1000
SAMPLE_SEED = 20150601


def params_digest(p: dict) -> str:
    """SHA-256 of the parameter dict (sorted JSON), so that a test can refuse
    a golden file written for other parameters."""
    return hashlib.sha256(json.dumps(p, sort_keys=True).encode()).hexdigest()


def sample_cells(shape, solid_height) -> np.ndarray:
    nz, ny, nx = shape
    rng = np.random.default_rng(SAMPLE_SEED)
    cells = set()
    for _ in range(3):  # whole columns: solid, front, liquid, both z ends
        i, j = int(rng.integers(nx)), int(rng.integers(ny))
        cells.update((i, j, k) for k in range(nz))
    for _ in range(16):  # columns through the front
        i, j = int(rng.integers(nx)), int(rng.integers(ny))
        cells.update((i, j, k) for k in range(solid_height - 8, solid_height + 8))
    for k in (0, 1, nz - 2, nz - 1):  # boundary planes
        for _ in range(64):
            cells.add((int(rng.integers(nx)), int(rng.integers(ny)), k))
    xs = [0, 31, 32, 63, 64, 127, 128, 191, 192, nx - 1]
    ys = [0, 3, 4, 7, 8, 127, 128, ny - 1]
    zs = [solid_height - 1, solid_height, solid_height + 1, 31, 32, 159, 160, 255, 256]
    for i in xs:  # tile and z-chunk edges
        for j in ys:
            for k in zs:
                cells.add((i, j, k))
    while len(cells) < 4900:  # interiors
        i, j = int(rng.integers(nx)), int(rng.integers(ny))
        if rng.random() < 0.6:
            k = int(rng.integers(solid_height + 8, nz))
        else:
            k = int(rng.integers(0, solid_height - 8))
        cells.add((i, j, k))
    return np.array(sorted(cells, key=lambda c: (c[2], c[1], c[0])), dtype=np.int32)


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    ap.add_argument("--state", default="", help="resumable state file (npz)")
    ap.add_argument("--every", type=int, default=50)
    args = ap.parse_args()

    w = pfinputs.workload("c2")
    shape = w["shape"]
    p = pfinputs.with_dt(w["params"], oracle.default_dt(w["params"], shape))
    step = 0
    if args.state and os.path.exists(args.state):
        z = np.load(args.state)
        phi, mu, step = z["phi"], z["mu"], int(z["step"])
        print(f"resumed at step {step}", flush=True)
    else:
        phi, mu = oracle.init_voronoi(shape, w["seed"], w["nseeds"], w["solid_height"])
    while step < STEPS:
        n = min(args.every, STEPS - step)
        t0 = time.time()
        phi, mu = oracle.run(p, phi, mu, n, step0=step, nthreads=args.threads)
        step += n
        print(f"step {step}/{STEPS}: {time.time() - t0:.1f} s", flush=True)
        if args.state and step < STEPS:
            tmp = args.state + ".tmp.npz"
            np.savez(tmp, phi=phi, mu=mu, step=step)
            os.replace(tmp, args.state)

    cells = sample_cells(shape, w["solid_height"])
    i, j, k = cells[:, 0], cells[:, 1], cells[:, 2]
    diag = oracle.diagnostics(p, phi, mu, STEPS * p["dt"])
    np.savez_compressed(
        OUT,
        cells=cells,
        phi=np.stack([phi[a][k, j, i] for a in range(4)], axis=1),
        mu=np.stack([mu[q][k, j, i] for q in range(2)], axis=1),
        maxabs_phi=np.array([np.max(np.abs(phi[a])) for a in range(4)]),
        maxabs_mu=np.array([np.max(np.abs(mu[q])) for q in range(2)]),
        sum_c=np.array(diag["sum_c"]),
        sum_phi=np.array(diag["sum_phi"]),
        dt=np.float64(p["dt"]),
        steps=np.int64(STEPS),
        params_sha256=np.array(params_digest(w["params"])),
    )
    print(f"wrote {OUT}: {len(cells)} cells", flush=True)


if __name__ == "__main__":
    main()
