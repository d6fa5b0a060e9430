"""The C-ABI library loads on the CPU host and exports every entry point that
include/he.h declares; the Python binding covers the same set.  No compute call
is made here (there is no GPU on this host)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "he.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(he_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2207_04620_amd import he
    if not os.path.exists(he.LIB_PATH):
        from paper_2207_04620_amd import build
        build.build()
    return he.LIB_PATH


def test_header_declares_the_hot_path_calls():
    names = declared()
    for n in ("he_ctx_create", "he_encrypt", "he_matmul", "he_rotate", "he_sign_approx", "he_decrypt",
              "he_matmul_batch", "he_ct_export", "he_ct_import", "he_encrypt_coeffs", "he_serve_start"):
        assert n in names


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.check_output(["nm", "-D", "--defined-only", libpath], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binding_covers_header(libpath):
    from paper_2207_04620_amd import he
    L = he.lib()
    for n in declared():
        assert hasattr(L, n)
    assert sorted(he.SIGNATURES) == declared()
    assert L.he_status_string(6) == b"bad matrix shape"


def test_oracle_and_library_share_no_code():
    """the GPU library never includes or names the oracle, and vice versa"""
    csrc = os.path.join(ROOT, "paper_2207_04620_amd", "csrc")
    for f in os.listdir(csrc):
        txt = open(os.path.join(csrc, f)).read()
        assert "oracle" not in txt.lower() and "orc_" not in txt
    for f in ("he.py", "build.py", "inputs.py"):
        txt = open(os.path.join(ROOT, "paper_2207_04620_amd", f)).read()
        assert "import oracle" not in txt and "from oracle" not in txt
    otxt = open(os.path.join(ROOT, "oracle", "ckks_oracle.c")).read()
    assert "he_internal" not in otxt and "modarith" not in otxt


def test_pack_beta_layout(libpath):
    """he_pack_beta (host memory only, App. E's iota_beta): entry (i, j) of matrix m at slot
    beta (h i + j) + m, against the layout written out index by index; and its argument checks"""
    import numpy as np
    from paper_2207_04620_amd import he
    rng = np.random.default_rng(5)
    for beta, h, t in ((1, 4, 4), (2, 4, 4), (4, 8, 2)):
        mats = [rng.standard_normal((t, h)) for _ in range(beta)]
        v = he.pack_beta(mats)
        want = np.empty(beta * t * h)
        for m in range(beta):
            for i in range(t):
                for j in range(h):
                    want[beta * (h * i + j) + m] = mats[m][i, j]
        assert np.array_equal(v, want)
    import ctypes as C
    out = (C.c_double * 4)()
    assert he.lib().he_pack_beta(0, 4, None, out) == 1
    assert he.lib().he_pack_beta(1, 4, None, out) == 1
