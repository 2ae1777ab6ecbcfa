"""The largest field plane the layout admits, against the oracle.

The tiled sweeps address a cell inside its field plane with a 32-bit byte
offset, so a plane (padded row bytes times ny) must stay below 4 GiB; the
layout rejects anything larger (tests/test_abi.py).  This test runs a domain
whose planes take 2^32 - 1024 bytes, so that the offsets of its last rows
lie just below 2^32 and those past the middle above 2^31: 1 x 33554424 x 16
cells in FP64 (16 doubles = one 128-byte row), about 103 GB of HBM for both
copies and 26 GB of host memory for each of the input and output arrays.

The state is periodic in y with period 8 (a smooth mixed state of an 8-row
domain, repeated 4194303 times), so after two steps every 8-row block must
equal, bit for bit, the first one, and the first one must equal the oracle's
8-row domain after two steps (periodic x/y, and one plane: no z faces), to
the FP64 bound of the other parity tests (1e-12 relative per field).  A
wrong or wrapped offset anywhere in the plane breaks the periodicity.
"""
import numpy as np
import pytest

import oracle
import pfinputs
from tests.gpu_util import field_errors, lib, log, params_full

pytestmark = pytest.mark.gpu

SMALL = (1, 8, 16)
REPEAT = 4194303
BIG = (1, 8 * REPEAT, 16)


def test_largest_plane_is_periodic_and_matches_the_oracle():
    assert BIG[1] * 128 == 2 ** 32 - 1024
    log(f"case maxsize shape={BIG} fp64 steps=2")
    pf = lib()
    pf.set_variant(1)
    p = params_full(SMALL, 1, G=2e-3, v=0.05, delta_sl=0.05)
    assert oracle.default_dt(p, BIG) == p["dt"]  # dt depends on nz only
    phi_s, mu_s = pfinputs.smooth_interface_state(SMALL, 11, width=1.5)
    phi_o, mu_o = oracle.run(p, phi_s, mu_s, 2)

    d = pf.Domain(BIG, "fp64")
    try:
        d.set_params(p)
        phi_b = np.tile(phi_s, (1, 1, REPEAT, 1))
        mu_b = np.tile(mu_s, (1, 1, REPEAT, 1))
        log("maxsize: init")
        d.init_host(phi_b, mu_b)
        del phi_b, mu_b
        log("maxsize: 2 steps")
        d.step(2)
        d.sync()
        log("maxsize: read")
        phi_g, mu_g = d.read()
    finally:
        d.close()

    blocks = [(phi_g.reshape(4, REPEAT, 8, 16), phi_g[:, 0, :8, :]),
              (mu_g.reshape(2, REPEAT, 8, 16), mu_g[:, 0, :8, :])]
    e = field_errors(blocks[0][1][:, None], blocks[1][1][:, None], phi_o, mu_o)
    log("block 0 against the oracle: " + " ".join(f"{v:.1e}" for v in e))
    assert max(e) <= 1e-12
    step = 1 << 16
    for full, first in blocks:
        for i in range(0, REPEAT, step):
            part = full[:, i:i + step]
            if not np.array_equal(part, np.broadcast_to(first[:, None], part.shape)):
                bad = np.nonzero(np.any(part != first[:, None], axis=(0, 2, 3)))[0]
                raise AssertionError(f"blocks {i + bad[:5]} differ from block 0")
    log("maxsize: every block equals block 0")
