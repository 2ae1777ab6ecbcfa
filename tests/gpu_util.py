"""Helpers for the GPU tests: build domains through the C ABI, compare with
the oracle on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle
import pfinputs


def lib():
    import paper_1506_01684_amd as pf

    pf.load()
    return pf


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_inf(a, b) -> float:
    """max|a-b| / max|b| over one field (b is the reference)."""
    den = float(np.max(np.abs(b)))
    return float(np.max(np.abs(a - b))) / (den if den > 0 else 1.0)


def field_errors(phi_g, mu_g, phi_o, mu_o):
    e = [rel_inf(phi_g[a], phi_o[a]) for a in range(4)]
    e += [rel_inf(mu_g[q], mu_o[q]) for q in range(2)]
    return e


def gpu_domain(shape, p, prec="fp64", variant=1, phi=None, mu=None, voronoi=None):
    pf = lib()
    pf.set_variant(variant)
    d = pf.Domain(shape, prec)
    d.set_params(p)
    if voronoi is not None:
        seed, nseeds, hs = voronoi
        d.init_voronoi(seed, nseeds, hs)
    else:
        d.init_host(phi, mu)
    return d


def params_full(shape, solid_height, **kw):
    """P0 with every T-dependent term switched on, dt resolved by the oracle."""
    p = pfinputs.p0_params(solid_height=solid_height, **kw)
    p["chi1"] = [[0.3, 0.2], [0.1, 0.4], [0.2, 0.2], [0.5, 0.3]]
    p["c1"] = [[0.05, -0.02], [0.1, 0.03], [-0.07, 0.02], [0.1, -0.1]]
    p["dt"] = oracle.default_dt(p, shape)
    return p
