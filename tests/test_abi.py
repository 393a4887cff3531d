"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_2303_02608_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "esim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(esim_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libesim.so not built")
    return B.load()


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ("esim_wlr_threshold", "esim_wlr_regress", "esim_events", "esim_wlr_backward"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.SIGNATURES), set(names) ^ set(B.SIGNATURES)


def test_status_strings(lib):
    assert lib.esim_status_string(0) == b"ok"
    assert lib.esim_status_string(-1) == b"invalid argument"
    assert b"gfx950" in lib.esim_build_info()


def test_invalid_arguments_fail_before_any_launch(lib):
    out = ctypes.c_void_p()
    assert lib.esim_plan_create(None, None, None, 1, ctypes.byref(out)) == B.E_INVAL
    assert b"null" in lib.esim_last_error()
    assert lib.esim_plan_create(None, None, None, 1, None) == B.E_INVAL
    assert lib.esim_log_brightness(None, None, -1, 1e-3, None) == B.E_INVAL
    assert lib.esim_log_brightness(None, None, 10, 1e-3, None) == B.E_INVAL
    assert lib.esim_log_brightness(None, None, 0, 1e-3, None) == B.OK
    assert lib.esim_wlr_threshold(None, 1, None, None, None, None) == B.E_INVAL
    assert lib.esim_wlr_regress(None, 0, None, None, 0, None, None, None, None, None) == B.E_INVAL
    assert lib.esim_events(None, 0, 1, None, None, None, None, None, 0, None, None) == B.E_INVAL
    assert lib.esim_wlr_backward(None, None, 1, None, None, None, None, 0, None) == B.E_INVAL
    assert lib.esim_log_variance(None, None, 4, None, 10, 1e-3, None) == B.E_INVAL
    assert lib.esim_log_variance(None, None, 0, None, 0, 1e-3, None) == B.E_INVAL    # spp < 1
    assert lib.esim_log_variance(None, None, 4, None, 0, 1e-3, None) == B.OK
    hs = (ctypes.c_double * 1)(1.0)
    assert lib.esim_wlr_regress_bandwidth(None, 0, None, None, 1, None, hs, 1, None, None, None, None,
                                          None) == B.E_INVAL
    assert lib.esim_plan_pixels(None) == -1
    assert lib.esim_plan_set_schedule(None, 4, 16, 4) == B.E_INVAL


def test_bad_shapes_and_params_are_rejected(lib):
    """Plan validation runs on the host before any device allocation."""
    F = 7
    clip = B.esim_clip(64, 64, 4, F, B.F32, 1, 1)     # dummy non-null pointers
    good = B.Params(r=5, tr=0, C=0.2)
    out = ctypes.c_void_p()

    def create(c, p):
        return lib.esim_plan_create(ctypes.byref(c), ctypes.byref(p), None, 1, ctypes.byref(out))

    bad_clip = B.esim_clip(0, 64, 4, F, B.F32, 1, 1)
    assert create(bad_clip, good.struct(F)) == B.E_INVAL
    assert create(B.esim_clip(64, 64, 4, 13, B.F32, 1, 1), good.struct(F)) == B.E_UNSUPPORTED
    assert create(B.esim_clip(64, 64, 4, F, B.F32, None, 1), good.struct(F)) == B.E_INVAL
    for p in (B.Params(r=0, tr=0, C=0.2), B.Params(r=5, tr=-1, C=0.2), B.Params(r=5, tr=0, C=0.0),
              B.Params(r=5, tr=0, C=0.2, h=0.0), B.Params(r=5, tr=0, C=0.2, ridge=-1.0),
              B.Params(r=5, tr=0, C=0.2, b=[1.0] * 8 + [0.0]),
              B.Params(r=5, tr=0, C=0.2, precision=7), B.Params(r=5, tr=0, C=0.2, threshold=3),
              B.Params(r=5, tr=0, C=0.2, threshold=-1), B.Params(r=5, tr=0, C=0.2, dt=0.0),
              B.Params(r=5, tr=0, C=0.2, dt=float("inf")), B.Params(r=5, tr=0, C=0.2, dt=float("nan"))):
        assert create(clip, p.struct(F)) == B.E_INVAL, vars(p)
    # mixed F across clips of one plan
    clips = (B.esim_clip * 2)(clip, B.esim_clip(64, 64, 4, 3, B.F32, 1, 1))
    pars = (B.esim_params * 2)(good.struct(F), good.struct(F))
    assert lib.esim_plan_create(clips, pars, None, 2, ctypes.byref(out)) == B.E_UNSUPPORTED
    # the threshold form is one per plan
    pars = (B.esim_params * 2)(good.struct(F),
                               B.Params(r=5, tr=0, C=0.2, threshold=B.THRESHOLD_NEW_WINDOW).struct(F))
    clips = (B.esim_clip * 2)(clip, clip)
    assert lib.esim_plan_create(clips, pars, None, 2, ctypes.byref(out)) == B.E_UNSUPPORTED
    # 2^31 pixels or more over the clips (each clip alone is valid: 1.07 G
    # pixels, one FP16 feature, windows below 4 GiB)
    big = B.esim_clip(32768, 32767, 1, 1, B.F16, 1, 1)
    one = B.Params(r=5, tr=0, C=0.2).struct(1)
    clips = (B.esim_clip * 3)(big, big, big)
    pars = (B.esim_params * 3)(one, one, one)
    assert lib.esim_plan_create(clips, pars, None, 3, ctypes.byref(out)) == B.E_UNSUPPORTED
    assert b"2^31" in lib.esim_last_error()


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """No CPU fallback: without the built library every entry point raises."""
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(ImportError, match="not built"):
        B.load(str(tmp_path / "libesim.so"))
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "libesim.so"))
    monkeypatch.setattr(B.load, "__defaults__", (str(tmp_path / "libesim.so"),))
    with pytest.raises(ImportError, match="not built"):
        B.log_brightness(__import__("torch").zeros(4))


def test_product_code_never_reaches_the_oracle():
    """The package imports nothing from the oracle, and the benchmark only in
    its CPU-baseline leg."""
    import ast
    pkg = os.path.join(ROOT, "paper_2303_02608_amd")
    for name in sorted(os.listdir(pkg)):
        if not name.endswith(".py"):
            continue
        tree = ast.parse(open(os.path.join(pkg, name)).read())
        for node in ast.walk(tree):
            mods = ([a.name for a in node.names] if isinstance(node, ast.Import)
                    else [node.module or ""] if isinstance(node, ast.ImportFrom) else [])
            assert not any(m == "oracle" or m.startswith("oracle.") for m in mods), name
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    users = set()
    for fn in ast.walk(tree):
        if isinstance(fn, ast.FunctionDef):
            for node in ast.walk(fn):
                if isinstance(node, (ast.Import, ast.ImportFrom)):
                    mods = ([a.name for a in node.names] if isinstance(node, ast.Import) else [node.module or ""])
                    if any(m == "oracle" or m.startswith("oracle.") for m in mods):
                        users.add(fn.name)
    top = [n for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))]
    assert not any((isinstance(n, ast.Import) and any(a.name.startswith("oracle") for a in n.names)) or
                   (isinstance(n, ast.ImportFrom) and (n.module or "").startswith("oracle")) for n in top)
    assert users and all("cpu" in u for u in users), users
