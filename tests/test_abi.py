"""The C-ABI library loads and exports every entry point include/ugkwp.h
declares; argument validation that needs no device.  No GPU required."""
import ctypes as C
import os
import re

import pytest

from paper_2312_16981_amd import ugkwp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "ugkwp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ugkwp_[a-z_0-9]+)\s*\(", src)))


def test_header_lists_the_required_entry_points():
    names = header_functions()
    for required in ("ugkwp_init_mesh", "ugkwp_set_opacity", "ugkwp_step", "ugkwp_get_fields"):
        assert required in names
    assert set(names) == set(ugkwp.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(ugkwp.LIB_PATH):
        pytest.skip("libugkwp.so not built")
    L = ugkwp.load()
    for name in header_functions():
        assert hasattr(L, name), name


def test_invalid_parameters_are_rejected_without_a_device():
    if not os.path.exists(ugkwp.LIB_PATH):
        pytest.skip("libugkwp.so not built")
    L = ugkwp.load()
    h = C.c_void_p()
    for bad in (dict(dt=0.0), dict(dt=-1.0), dict(c=0.0), dict(eps=-1.0), dict(si_max_iters=0),
                dict(pool_capacity=-5), dict(n_cap=1 << 40)):
        p = ugkwp.make_params(**bad)
        assert L.ugkwp_create(C.byref(h), C.byref(p), None) == ugkwp.EINVAL
    assert L.ugkwp_step(None, 1) == ugkwp.EINVAL
    assert L.ugkwp_init_mesh(None, 1, 10, 1, None, None, None, None, 4, None, 0, 1.0) == ugkwp.EINVAL
    d = ugkwp.Diag()
    assert L.ugkwp_get_diag(None, C.byref(d)) == ugkwp.EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(ugkwp, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(ugkwp, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        ugkwp.load()


def test_batch_rejects_instances_that_differ_in_shared_parameters():
    """A context shares dt, the opacity law and the flags: a batch whose
    instances differ there is refused before any device call."""
    from paper_2312_16981_amd import ugkwp, workloads as W
    probs = [W.larsen(nx=40), W.larsen(nx=60)]             # dt = dx / c differs
    with pytest.raises(ValueError, match="dt"):
        ugkwp.from_batch(probs)
    with pytest.raises(ValueError, match="opacity_stim"):
        ugkwp.from_batch([W.larsen(nx=40), W.larsen(nx=40, opacity_stim=0)])
