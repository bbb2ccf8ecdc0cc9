"""The C-ABI library loads and exports what the header declares (CPU only).

No compute call is made here; only argument validation that fails before any
HIP call is exercised.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "htsvt.h")
LIB = os.path.join(ROOT, "paper_2506_09594_amd", "libhtsvt.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ht_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2506_09594_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = _declared()
    assert "ht_gnhtsvt" in names and "ht_plan_create" in names and "ht_admm_iterate" in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), f"{name} declared in htsvt.h but not exported"


def test_binding_covers_header(lib):
    from paper_2506_09594_amd import htsvt
    assert sorted(htsvt.EXPORTS) == _declared()
    assert htsvt.version() == 200


def test_invalid_descriptions_rejected_before_device_work(lib):
    from paper_2506_09594_amd import htsvt
    d = htsvt._PlanDesc()
    h = ctypes.c_void_p()
    d.order = 1
    assert lib.ht_plan_create(ctypes.byref(d), ctypes.byref(h)) == htsvt.ERR_INVALID_ARG
    assert b"order" in htsvt._lib.ht_last_error()
    d.order, d.precision = 3, 7
    assert lib.ht_plan_create(ctypes.byref(d), ctypes.byref(h)) == htsvt.ERR_INVALID_ARG
    d.precision, d.r = 1, 0
    assert lib.ht_plan_create(ctypes.byref(d), ctypes.byref(h)) == htsvt.ERR_INVALID_ARG
    d.r, d.dims[0], d.dims[1], d.dims[2] = 5, 0, 4, 4
    assert lib.ht_plan_create(ctypes.byref(d), ctypes.byref(h)) == htsvt.ERR_INVALID_ARG
    assert lib.ht_plan_create(None, ctypes.byref(h)) == htsvt.ERR_INVALID_ARG
    assert lib.ht_gnhtsvt(None, None, None, ctypes.c_double(1.0), None, 0, None, 0, None, None, None) \
        == htsvt.ERR_INVALID_ARG


def test_batch_descriptions_rejected_before_device_work(lib):
    from paper_2506_09594_amd import htsvt
    h = ctypes.c_void_p()
    descs = (htsvt._PlanDesc * 2)()
    for d in descs:
        d.order, d.r, d.p, d.q, d.precision = 3, 4, 2, 1, 1
        d.dims[0], d.dims[1], d.dims[2] = 8, 8, 4
    assert lib.ht_batch_plan_create(0, descs, ctypes.byref(h)) == htsvt.ERR_INVALID_ARG
    assert lib.ht_batch_plan_create(2, None, ctypes.byref(h)) == htsvt.ERR_INVALID_ARG
    descs[1].precision = 2  # precision must agree across a batch
    assert lib.ht_batch_plan_create(2, descs, ctypes.byref(h)) == htsvt.ERR_INVALID_ARG
    assert b"agree" in htsvt._lib.ht_last_error()
    descs[1].precision, descs[1].q = 1, 2  # and q
    assert lib.ht_batch_plan_create(2, descs, ctypes.byref(h)) == htsvt.ERR_INVALID_ARG
    assert lib.ht_plan_set_tuning(None, 64, 0) == htsvt.ERR_INVALID_ARG
    assert lib.ht_plan_graph_enable(None, 1) == htsvt.ERR_INVALID_ARG
