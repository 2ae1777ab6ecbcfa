"""The oracle's C code under the address and undefined-behaviour sanitizers:
a small driver (oracle/check_driver.c) steps a ragged grid with and without
the moving window and the Dirichlet top, takes the diagnostics and the
mesh of every phase; any out-of-bounds access, leak or undefined operation
fails the run."""
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle
import pfinputs

HERE = os.path.dirname(os.path.abspath(oracle.__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_runs_clean_under_asan_and_ubsan():
    p = pfinputs.p0_params(solid_height=6, delta_sl=0.05)
    p["G"], p["v"] = 0.02, 0.5
    p["dt"] = oracle.default_dt(p, (14, 9, 11))
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "check")
        cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
               "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-o", exe, os.path.join(HERE, "check_driver.c"), os.path.join(HERE, "pf_oracle.c"),
               os.path.join(HERE, "pf_oracle_mesh.c"), "-lm"]
        subprocess.run(cmd, check=True, capture_output=True)
        par = os.path.join(tmp, "params.bin")
        open(par, "wb").write(bytes(oracle.make_params(p)))
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
        r = subprocess.run([exe, par], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stderr[-3000:]
        word, shifts, triangles, _ = r.stdout.split()
        assert word == "ok" and int(shifts) > 0 and int(triangles) > 0
