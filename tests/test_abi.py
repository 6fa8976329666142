"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/spid.h, and validates descriptors on the host."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "spid.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(spid_[a-z_A-Z]+)\s*\(", txt)))


def test_header_declares_the_four_stages():
    names = _declared()
    for n in ("spid_sketch_update", "spid_select", "spid_coeffs", "spid_reconstruct"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2103_01380_amd as sp
    lib = sp.load_library()
    out = subprocess.run(["nm", "-D", "--defined-only", sp.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (spid_\w+)", out))
    for name in _declared():
        assert name in exported, name
        assert hasattr(lib, name)
    assert set(sp.EXPORTS) <= exported


def test_binding_names_match_header():
    import paper_2103_01380_amd as sp
    for name in _declared():
        assert callable(getattr(sp, name)), name


def _bytes(**kw):
    import paper_2103_01380_amd as sp
    args = dict(m=[4096, 3000], n=[64, 40], l=18, k_max=8)
    args.update(kw)
    d = sp.make_desc(**args)
    return sp.spid_workspace_bytes(d), sp.spid_last_error()


def test_workspace_size_for_valid_descriptor():
    nb, _ = _bytes()
    assert nb > 0 and nb % 256 == 0
    nb2, _ = _bytes(m=[4096, 3000, 100], n=[64, 40, 30])
    assert nb2 > nb


@pytest.mark.parametrize("kw,msg", [
    (dict(l=0), "l must be"),
    (dict(l=129), "l must be"),
    (dict(k_max=0), "k_max"),
    (dict(k_max=97, l=120, n=[128, 128]), "k_max"),
    (dict(k_max=50), "fixed rank"),               # k_max > n_b=40
    (dict(m=[0, 10]), "m must be"),
    (dict(n=[64, 2000]), "n must be"),
    (dict(tol=-1.0), "tol"),
    (dict(a_dtype=7), "a_dtype"),
    (dict(prec=1, lp_terms=0), "lp_terms"),
])
def test_invalid_descriptors_are_rejected(kw, msg):
    nb, err = _bytes(**kw)
    assert nb == 0
    assert msg in err


def test_tolerance_mode_allows_k_max_above_n():
    nb, err = _bytes(k_max=50, l=60, tol=1e-4)
    assert nb > 0, err


def test_workspace_scales_with_batch():
    import paper_2103_01380_amd as sp
    m = np.full(512, 12288)
    n = np.full(512, 256)
    d = sp.make_desc(m, n, 42, 32, tol=1e-8)
    nb = sp.spid_workspace_bytes(d)
    # sketch (FP64) + R (FP64) dominate: 512*256*(42+32)*8 bytes
    assert 512 * 256 * (42 + 32) * 8 <= nb < 4 * 512 * 256 * (42 + 32) * 8
