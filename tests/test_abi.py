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


def _tuned_bytes(tuning, **kw):
    import paper_2103_01380_amd as sp
    args = dict(m=[4096, 3000], n=[256, 40], l=18, k_max=8)
    args.update(kw)
    d = sp.make_desc(**args)
    return sp.spid_workspace_bytes_tuned(d, sp.make_tuning(tuning)), sp.spid_last_error()


@pytest.mark.parametrize("tuning", [
    None, {}, dict(sk_tn=1, sk_nw=4), dict(sk_tn=2, sk_nw=8, sk_items=1024),
    dict(sk_items=64), dict(sk_items=65536), dict(rc_rpi=1), dict(rc_rpi=16),
    dict(st_groups=1), dict(st_groups=16),
])
def test_valid_launch_shapes_are_accepted(tuning):
    nb, err = _tuned_bytes(tuning)
    assert nb > 0 and nb % 256 == 0, err


@pytest.mark.parametrize("tuning,kw,msg", [
    (dict(sk_tn=3), {}, "sk_tn"),
    (dict(sk_tn=4), {}, "FP64 sketch"),                       # FP64: at most 2 tiles
    (dict(sk_tn=2), dict(l=70), "FP64 sketch"),               # FP64 2 tiles only for l <= 64
    (dict(sk_tn=4), dict(l=100, prec=1, a_dtype=1, lp_terms=2), "BF16 sketch"),
    (dict(sk_tn=2), dict(prec=2, a_dtype=1, lp_terms=3), "FP8 sketch"),
    (dict(sk_nw=6), {}, "sk_nw"),
    (dict(sk_nw=4, sk_tn=2), {}, "sk_nw=4 requires sk_tn=1"),
    (dict(sk_items=10), {}, "sk_items"),
    (dict(rc_rpi=17), {}, "rc_rpi"),
    (dict(rc_rpi=-1), {}, "rc_rpi"),
    (dict(st_groups=17), {}, "st_groups"),
    (dict(st_groups=-2), {}, "st_groups"),
])
def test_invalid_launch_shapes_are_rejected(tuning, kw, msg):
    nb, err = _tuned_bytes(tuning, **kw)
    assert nb == 0
    assert msg in err


def test_more_sketch_items_split_blocks_further():
    """A larger work-item target splits blocks along their rows: more split partials."""
    a, _ = _tuned_bytes(dict(sk_items=64), m=[1 << 16] * 4, n=[64] * 4)
    b, _ = _tuned_bytes(dict(sk_items=4096), m=[1 << 16] * 4, n=[64] * 4)
    assert b > a


def test_autotune_candidates_respect_instantiated_shapes():
    from paper_2103_01380_amd import autotune as at
    for prec, l in (("f64", 42), ("f64", 96), ("bf16", 48), ("bf16", 96), ("fp8", 96)):
        for c in at.sketch_candidates(prec, l, 384):
            nb, err = _tuned_bytes(c, l=l, n=[384, 384], m=[4096, 4096],
                                   prec={"f64": 0, "bf16": 1, "fp8": 2}[prec],
                                   a_dtype=0 if prec == "f64" else 1,
                                   lp_terms=1 if prec == "f64" else 2)
            assert nb > 0, (prec, l, c, err)
    assert at.recon_candidates("f32", "bf16") == [{}]
    assert all("rc_rpi" in c for c in at.recon_candidates("f64", "f64"))


def test_autotune_signature_separates_batches():
    from paper_2103_01380_amd import autotune as at
    s1 = at.signature([100, 200], [10, 20], 18, 8, 0.0, "f64", "f64", 1)
    s2 = at.signature([100, 201], [10, 20], 18, 8, 0.0, "f64", "f64", 1)
    s3 = at.signature([100, 200], [10, 20], 18, 8, 0.0, "f64", "f64", 1, stream_columns=True)
    assert len({s1, s2, s3}) == 3


def test_coarse_grid_descriptor_validation():
    import paper_2103_01380_amd as sp
    g = np.array([[16, 16, 16, 3, 7, 7, 7]], dtype=np.int32)
    ok = sp.make_desc([12288], [64], 81, 8, prec=sp.SK_SUBSAMPLE, grids=g)
    assert sp.spid_workspace_bytes(ok) > 0
    short = sp.make_desc([12288], [64], 80, 8, prec=sp.SK_SUBSAMPLE, grids=g)
    assert sp.spid_workspace_bytes(short) == 0 and "coarse rows" in sp.spid_last_error()
    wrong_m = sp.make_desc([12000], [64], 81, 8, prec=sp.SK_SUBSAMPLE, grids=g)
    assert sp.spid_workspace_bytes(wrong_m) == 0 and "grid has" in sp.spid_last_error()
    no_grid = sp.make_desc([12288], [64], 81, 8, prec=sp.SK_SUBSAMPLE)
    assert sp.spid_workspace_bytes(no_grid) == 0 and "h_grid" in sp.spid_last_error()
    bad = sp.make_desc([12288], [64], 81, 8, prec=sp.SK_SUBSAMPLE,
                       grids=np.array([[16, 16, 16, 3, 0, 7, 7]], dtype=np.int32))
    assert sp.spid_workspace_bytes(bad) == 0 and ">= 1" in sp.spid_last_error()
    # tall coarse grids: allowed beyond the 128 rows of the Gaussian sketch, and the
    # global-memory selection needs a working copy of the sketch
    tall = sp.make_desc([12288], [64], 648, 8, prec=sp.SK_SUBSAMPLE,
                        grids=np.array([[16, 16, 16, 3, 3, 3, 3]], dtype=np.int32))
    assert sp.spid_workspace_bytes(tall) >= 2 * 648 * 64 * 8
    gauss = sp.make_desc([12288], [64], 648, 8)
    assert sp.spid_workspace_bytes(gauss) == 0


def test_two_stage_descriptor_validation():
    import paper_2103_01380_amd as sp
    ok = sp.make_desc([3000], [64], 24, 16, tol=1e-5, ts_windows=4, ts_k1=8)
    assert sp.spid_workspace_bytes(ok) > sp.spid_workspace_bytes(sp.make_desc([3000], [64], 24, 16, tol=1e-5))
    too_many = sp.make_desc([3000], [64], 24, 16, tol=1e-5, ts_windows=65, ts_k1=1)
    assert sp.spid_workspace_bytes(too_many) == 0 and "windows exceed" in sp.spid_last_error()
    wide = sp.make_desc([3000], [1024], 24, 16, tol=1e-5, ts_windows=64, ts_k1=32)
    assert sp.spid_workspace_bytes(wide) == 0 and "1024" in sp.spid_last_error()
    no_k1 = sp.make_desc([3000], [64], 24, 16, tol=1e-5, ts_windows=4, ts_k1=0)
    assert sp.spid_workspace_bytes(no_k1) == 0 and "ts_k1" in sp.spid_last_error()
    mixed = sp.make_desc([3000], [64], 24, 16, tol=1e-5, a_dtype=sp.A_F32, prec=sp.SK_BF16,
                         ts_windows=4, ts_k1=8)
    assert sp.spid_workspace_bytes(mixed) == 0 and "split-bfloat16" in sp.spid_last_error()
