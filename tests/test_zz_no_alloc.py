"""pf_diag_fields_noalloc: diagnostics of caller-held device fields with the
scratch in a static device array, against pf_read_fields' diagnostics of
the same state (the existing entry point, which keeps its scratch in the
domain's allocation).

Both run the same kernel arithmetic over the same grid and cell order, so
the FP64 sums must agree bit for bit (stricter than the 1e-12 FP64 bar).
Two calls in a row, the second on a smaller domain, check that the array
keeps nothing a later call depends on.
"""
import ctypes as C

import numpy as np
import pytest

import pfinputs
from tests.gpu_util import gpu_domain, lib, log, params_full

pytestmark = pytest.mark.gpu

KEYS = ("sum_c", "sum_phi", "max_simplex_dev", "phi_min", "phi_max", "nonfinite")


def _fields_tensor(d, prec):
    import torch

    phi, mu = d.read()
    host = np.concatenate([phi, mu], axis=0)
    dt = torch.float64 if prec == "fp64" else torch.float32
    # FP32 domains widen exactly on read, so the cast back is exact
    return torch.from_numpy(host).to(dtype=dt, device="cuda").contiguous()


def _compare(ref, got, what):
    log(f"{what}: sum_c {got['sum_c']} vs {ref['sum_c']}, nonfinite {got['nonfinite']}")
    for k in KEYS:
        assert got[k] == ref[k], (what, k, got[k], ref[k])
    assert got["step"] == -1 and got["t"] == ref["t"]


def _case(shape, prec, steps, nseeds, hs):
    pf = lib()
    p = params_full(shape, hs, G=2e-3, v=0.05)
    d = gpu_domain(shape, p, prec, 1, voronoi=(42, nseeds, hs))
    d.step(steps)
    ref = d.diagnostics()
    fields = _fields_tensor(d, prec)
    got = pf.diag_fields_noalloc(fields, p, ref["t"])
    d.close()
    return ref, got, fields, p


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_diag_matches_domain_diag(prec):
    log(f"case noalloc diag prec={prec}: 72x24x40 then 12x8x16")
    ref, got, _, _ = _case((40, 24, 72), prec, 7, 6, 10)
    _compare(ref, got, f"{prec} first call 72x24x40")
    ref2, got2, _, _ = _case((16, 8, 12), prec, 3, 3, 4)  # smaller: fewer cells than blocks x threads
    _compare(ref2, got2, f"{prec} second call 12x8x16")


def test_noalloc_diag_counts_nonfinite_and_rejects_bad_args():
    import torch

    pf = lib()
    from paper_1506_01684_amd import _capi as A

    log("case noalloc diag: planted NaN, invalid arguments")
    ref, got, fields, p = _case((20, 16, 16), "fp64", 2, 4, 5)
    _compare(ref, got, "fp64 16x16x20")
    bad = fields.clone()
    bad[4, 3, 2, 1] = float("nan")
    bad[0, 7, 5, 9] = float("inf")
    got_bad = pf.diag_fields_noalloc(bad, p, ref["t"], raise_nonfinite=False)
    assert got_bad["nonfinite"] == 2
    with pytest.raises(pf.PfError) as e:
        pf.diag_fields_noalloc(bad, p, ref["t"])
    assert e.value.status == A.PF_ERR_NONFINITE
    # argument errors are caught on the host, before any launch
    desc = A.PfDomainDesc(0, 16, 20, A.PF_FP64, 1.0)
    ps = pf.params_struct(p)
    dg = A.PfDiag()
    st = pf.load().pf_diag_fields_noalloc(C.byref(desc), C.byref(ps),
                                          C.c_void_p(fields.data_ptr()), 0.0, None, C.byref(dg))
    assert st == A.PF_ERR_INVALID_ARG
    desc = A.PfDomainDesc(16, 16, 20, A.PF_FP64, 1.0)
    st = pf.load().pf_diag_fields_noalloc(C.byref(desc), C.byref(ps),
                                          C.c_void_p(fields.data_ptr() + 4), 0.0, None,
                                          C.byref(dg))
    assert st == A.PF_ERR_INVALID_ARG
    st = pf.load().pf_diag_fields_noalloc(C.byref(desc), C.byref(ps),
                                          C.c_void_p(fields.data_ptr()), float("nan"), None,
                                          C.byref(dg))
    assert st == A.PF_ERR_INVALID_ARG
    # the array is left as the last call wrote it; a clean call after the
    # failed ones still matches
    again = pf.diag_fields_noalloc(fields, p, ref["t"])
    _compare(ref, again, "fp64 16x16x20 again")
    torch.cuda.synchronize()
