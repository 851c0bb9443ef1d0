"""The C ABI library loads, exports every symbol include/rbe.h declares, and
rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2110_14362_amd import rbe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "rbe.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rbe_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_binding_exports():
    assert declared_symbols() == sorted(rbe.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = rbe.load_library()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_version_and_empty_error():
    lib = rbe.load_library()
    assert lib.rbe_version().decode().startswith("rbe-gfx950")
    assert isinstance(lib.rbe_last_error(), bytes)


def _init(cfg, box=(10.0, 10.0, 10.0)):
    lib = rbe.load_library()
    boxarr = (ctypes.c_double * 3)(*box)
    ctx = ctypes.c_void_p()
    dummy = ctypes.c_void_p(0x1000)      # never dereferenced: validation fails first
    st = lib.rbe_init(ctypes.byref(cfg), dummy, boxarr, None, ctypes.byref(ctx))
    return st, lib.rbe_last_error().decode()


def good_cfg(**kw):
    c = dict(n=10, p=4, box_mode=0, precision=1, p_pressure=0, alpha=0.09, coulomb=1.0,
             seed=1, system_id=0)
    c.update(kw)
    return rbe.Config(**c)


@pytest.mark.parametrize("field,value,msg", [("n", 0, "n ="), ("p", 0, "p ="), ("p", 70000, "p ="),
                                             ("alpha", -1.0, "alpha"), ("coulomb", 0.0, "coulomb"),
                                             ("box_mode", 7, "box_mode"), ("precision", 5, "precision"),
                                             ("p_pressure", 3, "p_pressure"),
                                             ("p_pressure", 70000, "p_pressure")])
def test_init_rejects_bad_config(field, value, msg):
    st, err = _init(good_cfg(**{field: value}))
    assert st == 1 and msg in err


@pytest.mark.parametrize("box,msg", [((10.0, -1.0, 10.0), "box[1]"), ((10.0, 10.0, float("nan")), "box[2]"),
                                     ((10.0, 11.0, 10.0), "cubic")])
def test_init_rejects_bad_box(box, msg):
    st, err = _init(good_cfg(), box)
    assert st == 1 and msg in err


def test_semiiso_needs_square_xy():
    st, err = _init(good_cfg(box_mode=1), (10.0, 11.0, 12.0))
    assert st == 1 and "lx == ly" in err


def test_table_capacity_limit():
    st, err = _init(good_cfg(alpha=100.0), (100.0, 100.0, 100.0))
    assert st == 1 and "too large" in err


def test_null_context_calls_fail_cleanly():
    lib = rbe.load_library()
    assert lib.rbe_sample_k(None, 0) == 1
    assert lib.rbe_check(None) == 1
    assert lib.rbe_forces_pressure(None, None, None, None, None, None, None, 0, None, None) == 1
    lib.rbe_destroy(None)
