"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/godec.h declares, validates arguments, and its host-side A1
generator matches the oracle's independent implementation bit for bit."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1309_0302_amd import binding as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "godec.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(godec_[A-Za-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(b.LIB_PATH):
        pytest.fail("libgodec.so is not built (run python -m paper_1309_0302_amd.build)")
    return b.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", b.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (godec_[A-Za-z0-9_]+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)


def test_binding_covers_every_entry_point():
    assert set(declared_functions()) <= set(b._SIG)


def test_version_string(lib):
    assert b"gfx950" in lib.godec_version()


# the last case is large enough for the draw to be split over threads
@pytest.mark.parametrize("seed,n,r", [(0, 7, 3), (1234567, 50, 4), (2 ** 63 + 5, 33, 1),
                                      (99, 3301, 20)])
def test_host_a1_matches_oracle_bitwise(seed, n, r):
    from oracle.rng_ref import a1_gaussian
    got = b.godec_draw_a1(seed, n, r)
    ref = a1_gaussian(seed, n, r)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def _ws(m, n, r, k, q, dtype=b.GODEC_F32, opts=None):
    return b.godec_workspace_size(m, n, r, k, q, dtype, opts)


def test_workspace_size_grows_with_problem(lib):
    a = _ws(100, 80, 4, 100, 1)
    c = _ws(1000, 800, 4, 10000, 1)
    assert 0 < a < c
    # the f32 working copy alone: m * round_up(n, 16) * 4 bytes
    assert c >= 1000 * 800 * 4
    o, _ = b.make_opts(prec=b.GODEC_PREC_BF16_REFINE)
    assert _ws(1000, 800, 4, 10000, 1, opts=o) >= c + 1000 * 800 * 2


@pytest.mark.parametrize("args,code", [
    ((0, 10, 1, 1, 1), 1), ((10, 0, 1, 1, 1), 1),
    ((10, 10, 0, 1, 1), 1), ((10, 8, 9, 1, 1), 1),
    ((100, 100, 33, 1, 1), 6), ((10, 10, 2, 101, 1), 1),
    ((10, 10, 2, -1, 1), 1), ((10, 10, 2, 5, -1), 1),
])
def test_workspace_size_rejects_bad_arguments(lib, args, code):
    with pytest.raises(b.GodecError) as ei:
        _ws(*args)
    assert ei.value.status == code
    assert lib.godec_last_error()


def test_bf16_mode_needs_f32(lib):
    o, _ = b.make_opts(prec=b.GODEC_PREC_BF16_REFINE)
    with pytest.raises(b.GodecError) as ei:
        _ws(100, 100, 4, 10, 1, dtype=b.GODEC_F64, opts=o)
    assert ei.value.status == 1


def test_opts_size_checked(lib):
    o, _ = b.make_opts()
    o.size = 3
    with pytest.raises(b.GodecError):
        _ws(100, 100, 4, 10, 1, opts=o)


def test_lstep_checked(lib):
    o, _ = b.make_opts(lstep=1)
    assert _ws(100, 100, 4, 10, 1, opts=o) == _ws(100, 100, 4, 10, 1)
    o, _ = b.make_opts(lstep=2)
    with pytest.raises(b.GodecError) as ei:
        _ws(100, 100, 4, 10, 1, opts=o)
    assert ei.value.status == 1


def test_warm_start_checked(lib):
    o, _ = b.make_opts(warm_start=1)
    assert _ws(100, 100, 4, 10, 1, opts=o) > 0
    o, _ = b.make_opts(warm_start=3)
    with pytest.raises(b.GodecError) as ei:
        _ws(100, 100, 4, 10, 1, opts=o)
    assert ei.value.status == 1


def test_redraw_a1_checked(lib):
    o, _ = b.make_opts(redraw_a1=1)
    # plus two device slots of four n x r FP64 draws
    assert _ws(100, 100, 4, 10, 1, opts=o) >= _ws(100, 100, 4, 10, 1) + 2 * 4 * 100 * 4 * 8
    for kw in ({"redraw_a1": 2}, {"redraw_a1": 1, "warm_start": 1},
               {"redraw_a1": 1, "a1": np.zeros((100, 4))}):
        o, _keep = b.make_opts(**kw)
        with pytest.raises(b.GodecError) as ei:
            _ws(100, 100, 4, 10, 1, opts=o)
        assert ei.value.status == 1


def test_k_extremes_accepted(lib):
    assert _ws(20, 10, 2, 0, 0) > 0
    assert _ws(20, 10, 2, 200, 0) > 0


def test_init_rejects_null_pointers_without_touching_the_gpu(lib):
    ctx = ctypes.c_void_p()
    st = lib.godec_init(ctypes.byref(ctx), None, 1, 10, 10, 10, 2, 5, 1, 0,
                        None, 0, None)
    assert st == 1
    st = lib.godec_init(ctypes.byref(ctx), 4096, 1, 10, 10, 9, 2, 5, 1, 0,
                        4096, 1 << 20, None)
    assert st == 1                       # ldx < n
    st = lib.godec_init(ctypes.byref(ctx), 4096, 1, 10, 10, 10, 2, 5, 1, 0,
                        4096 + 16, 1 << 20, None)
    assert st == 1                       # workspace misaligned


@pytest.mark.parametrize("args,code", [
    ((0, 10, 1), 1), ((10, 0, 1), 1), ((10, 10, 0), 1), ((10, 8, 9), 1),
    ((100, 100, 33), 6),
])
def test_grebsmo_workspace_size_rejects_bad_arguments(lib, args, code):
    with pytest.raises(b.GodecError) as ei:
        b.godec_grebsmo_workspace_size(*args, b.GODEC_F32)
    assert ei.value.status == code


def test_grebsmo_workspace_size_grows(lib):
    a = b.godec_grebsmo_workspace_size(100, 80, 4, b.GODEC_F32)
    c = b.godec_grebsmo_workspace_size(1000, 800, 4, b.GODEC_F32)
    assert 0 < a < c
    # D and R, both m x round_up(n, 128) in the dtype of X
    assert c >= 2 * 1000 * 896 * 4
    assert b.godec_grebsmo_workspace_size(1000, 800, 4, b.GODEC_F64) > c


@pytest.mark.parametrize("dr,power,lam", [(0, 2, 0.1), (1, 0, 0.1), (1, 2, -1.0),
                                          (1, 2, float("nan")), (1, 2, float("inf"))])
def test_grebsmo_init_rejects_bad_parameters_without_touching_the_gpu(lib, dr, power, lam):
    h = ctypes.c_void_p()
    st = lib.godec_grebsmo_init(ctypes.byref(h), 4096, 1, 10, 10, 10, 2, dr, power, lam, 0,
                                None, 4096, 1 << 20, None)
    assert st == 1 and not h.value


def test_grebsmo_init_rejects_null_and_misaligned(lib):
    h = ctypes.c_void_p()
    assert lib.godec_grebsmo_init(ctypes.byref(h), None, 1, 10, 10, 10, 2, 1, 2, 0.1, 0,
                                  None, 4096, 1 << 20, None) == 1
    assert lib.godec_grebsmo_init(ctypes.byref(h), 4096, 1, 10, 10, 9, 2, 1, 2, 0.1, 0,
                                  None, 4096, 1 << 20, None) == 1       # ldx < n
    assert lib.godec_grebsmo_init(ctypes.byref(h), 4096, 1, 10, 10, 10, 2, 1, 2, 0.1, 0,
                                  None, 4096 + 16, 1 << 20, None) == 1  # workspace misaligned
    assert lib.godec_grebsmo_init(ctypes.byref(h), 4096, 1, 10, 10, 10, 2, 1, 2, 0.1, 0,
                                  None, 4096, 64, None) == 2            # workspace too small


def test_product_path_has_no_oracle_dependency():
    """The package never imports the oracle (it is test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_1309_0302_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f


# ---- MSE training: host-side argument checks (no device work) ---------------

def _mse_status(n, p, labels, ranks, K, dtype=b.GODEC_F32):
    import ctypes as C
    lptr, rows, rk = b._label_arrays(labels, ranks)
    ctx = C.c_void_p()
    # fake, aligned, non-null pointers: every check below fails before any
    # device access
    return b.load().godec_mse_init(C.byref(ctx), 256, dtype, n, p, p, len(labels),
                                   rk.ctypes.data, lptr.ctypes.data, rows.ctypes.data, K, 1,
                                   256, 1 << 40, None)


def test_mse_rejects_bad_arguments():
    ok = [np.arange(0, 10, 2), np.arange(5)]
    assert b.STATUS[_mse_status(20, 16, [np.array([3, 1])], [2], 5)] == "GODEC_E_INVAL"
    assert b.STATUS[_mse_status(20, 16, [np.array([1, 1])], [2], 5)] == "GODEC_E_INVAL"
    assert b.STATUS[_mse_status(20, 16, [np.array([25])], [2], 5)] == "GODEC_E_INVAL"
    assert b.STATUS[_mse_status(20, 16, ok, [2, 9], 5)] == "GODEC_E_UNSUPPORTED"
    assert b.STATUS[_mse_status(20, 16, ok, [2, 0], 5)] == "GODEC_E_INVAL"
    assert b.STATUS[_mse_status(20, 600, ok, [2, 2], 5)] == "GODEC_E_UNSUPPORTED"
    assert b.STATUS[_mse_status(20, 300, ok, [2, 2], 5, b.GODEC_F64)] == "GODEC_E_UNSUPPORTED"
    assert b.STATUS[_mse_status(20, 16, ok, [2, 2], 20 * 16 + 1)] == "GODEC_E_INVAL"


def test_mse_workspace_size_grows_with_rows():
    a = b.godec_mse_workspace_size(1000, 100, [np.arange(10)], [2], 50, b.GODEC_F32)
    c = b.godec_mse_workspace_size(1000, 100, [np.arange(900)], [2], 50, b.GODEC_F32)
    assert c > a > 1000 * 100 * 4
