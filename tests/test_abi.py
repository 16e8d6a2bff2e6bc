"""The C-ABI library loads without a GPU and exports every declared symbol."""

import ctypes
import os

import pytest

import paper_1412_3510_amd as rp


def test_library_built_and_exports_header_symbols():
    if not os.path.exists(rp.LIB_PATH):
        pytest.fail("librpca.so is not built (python -m paper_1412_3510_amd.build)")
    lib = rp.load()
    names = rp.header_symbols()
    assert "rpca_svd" in names and "rpca_eig_psd" in names and "rpca_spectral_err" in names
    missing = [s for s in names if not hasattr(lib, s)]
    assert not missing, missing


def test_status_strings_and_struct_layout():
    lib = rp.load()
    assert lib.rpca_status_str(0) == b"ok"
    assert lib.rpca_status_str(5).startswith(b"matrix not")
    # rpca_matrix: 2 int32 + 14 eight-byte fields
    assert ctypes.sizeof(rp.Matrix) == 8 + 14 * 8
    assert ctypes.sizeof(rp.Stats) == 16 * 8
    assert ctypes.sizeof(rp.Problem) == 80
    assert ctypes.sizeof(rp.TuneResult) == 6 * 4 + 3 * 8


def test_null_context_rejected():
    lib = rp.load()
    assert lib.rpca_destroy(None) == 1
    assert lib.rpca_set_timing(None, 1) == 1
    assert lib.rpca_svd(None, None, 1, 1, 0, 0, 0, None, 1, None, None, 1) == 1


def test_flag_values_match_the_header():
    import re
    text = open(rp.HEADER).read()
    enum = text[text.index("/* flags */"):]
    enum = enum[:enum.index("};")]
    vals = {name: int(v) for name, v in re.findall(r"RPCA_(\w+)\s*=\s*(\d+)u", enum)}
    want = {"CENTER": rp.CENTER, "SYNC": rp.SYNC, "DETERMINISTIC": rp.DETERMINISTIC,
            "RENORM_ORTH": rp.RENORM_ORTH, "RENORM_LU": rp.RENORM_LU,
            "OMEGA_UNIFORM": rp.OMEGA_UNIFORM, "NYSTROM_SQRT": rp.NYSTROM_SQRT,
            "FUSED_ATA": rp.FUSED_ATA}
    assert vals == want
    # one bit each
    assert all(v & (v - 1) == 0 for v in vals.values()) and len(set(vals.values())) == len(vals)
