"""The C-ABI library loads and exports every symbol include/pfsolve.h
declares; host-only calls validate their arguments (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

import paper_1506_01684_amd as pf
from paper_1506_01684_amd import _capi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pfsolve.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(A.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = pf.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_required_bytes_layout_and_validation():
    b64 = pf.required_bytes((64, 32, 32), "fp64")
    b32 = pf.required_bytes((64, 32, 32), "fp32")
    cells = 64 * 32 * 32
    assert b64 >= 2 * 6 * cells * 8 and b32 >= 2 * 6 * cells * 4
    assert b64 < 2 * 6 * cells * 8 * 1.2
    # 512x512x1024 FP32 fits easily in one GPU's HBM
    big = pf.required_bytes((1024, 512, 512), "fp32")
    assert 12.8e9 < big < 13.5e9
    for bad in [(0, 4, 4), (4, -1, 4), (4, 4, 0)]:
        with pytest.raises(pf.PfError) as e:
            pf.required_bytes(bad)
        assert "INVALID_ARG" in str(e.value)
    with pytest.raises(pf.PfError):
        pf.required_bytes((4, 4, 4), "fp64", dx=0.0)


@pytest.mark.parametrize("prec,nx", [("fp64", 16), ("fp32", 32), ("fp64", 20)])
def test_required_bytes_caps_a_field_plane_below_4_gib(prec, nx):
    # rows are padded to a multiple of 128 bytes; with 128-byte rows the
    # largest plane is 2^32 - 128 bytes (2^25 - 1 rows) and one more row
    # reaches 2^32; nx = 20 FP64 pads to 32 elements (256-byte rows)
    row = -(-nx * (8 if prec == "fp64" else 4) // 128) * 128
    ny_max = (2 ** 32 - 1) // row
    big = pf.required_bytes((1, ny_max, nx), prec)
    assert big >= 2 * 6 * ny_max * row
    with pytest.raises(pf.PfError) as e:
        pf.required_bytes((1, ny_max + 1, nx), prec)
    assert "INVALID_ARG" in str(e.value)


def test_variant_switch_validates():
    with pytest.raises(pf.PfError):
        pf.set_variant(7)
    pf.set_variant(1)


def test_product_path_has_no_oracle_dependency():
    """The package never imports the oracle or reads the paper."""
    pkg = os.path.join(ROOT, "paper_1506_01684_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "pf_oracle" not in text and "/root/reference" not in text, f


def test_struct_layout_matches_header(tmp_path):
    """ctypes mirrors of the ABI structs have the C compiler's size and
    field offsets (compiled from include/pfsolve.h with gcc)."""
    structs = {"pf_params": A.PfParams, "pf_diag": A.PfDiag, "pf_init": A.PfInit,
               "pf_domain_desc": A.PfDomainDesc, "pf_device_buffer": A.PfDeviceBuffer}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pfsolve.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            c, f, v = line.split()
            got[(c, f)] = int(v)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
