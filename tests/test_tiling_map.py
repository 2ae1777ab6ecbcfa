"""Host-side check of the work decomposition: for the tile shapes the runtime
chooses, the block -> (tile x, tile y, z chunk) map used by the sweeps
covers every tile exactly once, puts each domain's first block on XCD 0,
and (in y-slab order) keeps every XCD inside its own rows.  The map is
restated here from its definition (blocks walk x fastest, then y, then z,
inside the XCD's slab of rs tile rows)."""
import pytest

KTHREADS, KXCD = 256, 8


def tiling(nx, ny, nz, prec="fp32"):
    # FP64 tiles are always 32x8; FP32 tiles 64x4 unless nx < 48
    tx = 64 if nx >= 48 and prec != "fp64" else 32
    ty = KTHREADS // tx
    ntx, nty = -(-nx // tx), -(-ny // ty)
    cols = nz * ntx * nty
    zc = min(32, max(8, cols // 2048))
    zc = min(zc, nz)
    nzc = -(-nz // zc)
    rs = -(-nty // 8)
    xmode = 1 if (8 * rs - nty) * 8 <= 8 * rs else 0
    blocks = 8 * rs * ntx * nzc if xmode else -(-(ntx * nty * nzc) // 8) * 8
    return dict(ntx=ntx, nty=nty, nzc=nzc, xmode=xmode, rs=rs, blocks=blocks)


def decode(t, lb):
    if t["xmode"]:
        j, p = lb % KXCD, lb // KXCD
        y_lo = j * t["rs"]
        rows = min(t["rs"], t["nty"] - y_lo)
        if rows <= 0:
            return None
        per_z = rows * t["ntx"]
        iz, rem = divmod(p, per_z)
        if iz >= t["nzc"]:
            return None
        return (rem % t["ntx"], y_lo + rem // t["ntx"], iz)
    ix = lb % t["ntx"]
    r = lb // t["ntx"]
    iy, iz = r % t["nty"], r // t["nty"]
    return (ix, iy, iz) if iz < t["nzc"] else None


@pytest.mark.parametrize("shape", [(512, 256, 256), (1024, 512, 512), (64, 32, 32), (20, 1, 1),
                                   (80, 70, 100), (300, 190, 33), (9, 17, 70), (128, 96, 96)])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_blocks_cover_each_tile_once(shape, prec):
    nz, ny, nx = shape
    t = tiling(nx, ny, nz, prec)
    assert t["blocks"] % 8 == 0
    seen = {}
    for lb in range(t["blocks"]):
        tile = decode(t, lb)
        if tile is None:
            continue
        assert tile not in seen
        seen[tile] = lb
        if t["xmode"]:  # the XCD owns the tile's row
            assert tile[1] // t["rs"] == lb % KXCD
    assert len(seen) == t["ntx"] * t["nty"] * t["nzc"]
    idle = t["blocks"] - len(seen)
    assert idle <= max(7, t["blocks"] // 8)
    if shape in ((512, 256, 256), (1024, 512, 512)):
        assert t["xmode"] == 1 and idle == 0
