"""The C-ABI library loads and exports what the header declares (CPU only).

No compute call is made here; only argument validation that fails before any
HIP call is exercised.
"""
import ctypes
import os
import re

import numpy as np

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
    assert htsvt.version() == 300


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


def test_error_codes_reachable_without_a_gpu(lib):
    """Every error code but NONFINITE (which needs a computed slice; see the GPU
    tests) comes back through the ABI with a message, before or at the first
    device call."""
    from paper_2506_09594_amd import htsvt
    lib = htsvt._lib  # with argument types (size_t and double arguments)
    h = ctypes.c_void_p()
    d = htsvt._make_desc((20, 20, 4), ["dct2"], 4, 2, 1, "fp32", 0, 0, None, [])
    # a valid description: the device tables cannot be allocated without a GPU
    assert lib.ht_plan_create(ctypes.byref(d), ctypes.byref(h)) == htsvt.ERR_ALLOC
    # a valid request this build does not take: sketch width above HT_MAX_WIDTH
    d = htsvt._make_desc((200, 200, 4), ["dct2"], 70, 10, 1, "fp32", 0, 0, None, [])
    assert lib.ht_plan_create(ctypes.byref(d), ctypes.byref(h)) == htsvt.ERR_UNSUPPORTED
    assert b"HT_MAX_WIDTH" in htsvt._lib.ht_last_error()
    # a DFT mode next to a real one
    d = htsvt._make_desc((20, 20, 4, 4), ["dct2", "dft_unnormalized"], 4, 2, 1, "fp32", 0, 0, None, [])
    assert lib.ht_plan_create(ctypes.byref(d), ctypes.byref(h)) == htsvt.ERR_UNSUPPORTED
    fake = ctypes.c_void_p(0x1000)
    # a misaligned workspace
    assert lib.ht_mlp_grad(fake, fake, fake, 1, fake, None, ctypes.c_void_p(0x1001), 1 << 20, None) \
        == htsvt.ERR_WORKSPACE
    assert b"aligned" in htsvt._lib.ht_last_error()
    # too small a workspace
    assert lib.ht_mlp_grad(fake, fake, fake, 1, fake, None, ctypes.c_void_p(0x1000), 16, None) \
        == htsvt.ERR_WORKSPACE
    # the HIP runtime's own failure (no device here) is reported as HIP
    assert lib.ht_mlp_forward(fake, fake, fake, 1, None) == htsvt.ERR_HIP
    assert b"kernel launch failed" in htsvt._lib.ht_last_error()
    # invalid arguments
    assert lib.ht_mlp_train_step(fake, fake, fake, 0, fake, fake, 1, ctypes.c_float(1e-3), ctypes.c_float(0.9),
                                 ctypes.c_float(0.999), ctypes.c_float(1e-8), None, fake, 1 << 20, None) \
        == htsvt.ERR_INVALID_ARG
    assert lib.ht_plan_status(None, fake, None, None) == htsvt.ERR_INVALID_ARG
    assert lib.ht_plan_device(None, None) == htsvt.ERR_INVALID_ARG
    assert lib.ht_admm_set_truth(None, None) == htsvt.ERR_INVALID_ARG


def _fake_plan(htsvt, precision="fp32", N=24):
    """A Plan object without a device plan behind it: the binding's argument
    checks run before any call into the library."""
    p = htsvt.Plan.__new__(htsvt.Plan)
    p._h = None
    p.precision, p.N = precision, N
    p.workspace_bytes = p.admm_workspace_bytes = 1024
    p.n_slices, p.width = 2, 3
    return p


def test_binding_rejects_misuse_before_the_library(lib):
    import torch
    from paper_2506_09594_amd import htsvt
    p = _fake_plan(htsvt)
    good = torch.zeros(24, dtype=torch.float32)
    ws = torch.zeros(2048, dtype=torch.uint8)
    cases = [
        (torch.zeros(24, dtype=torch.float64), "float32"),          # an FP64 tensor on an FP32 plan
        (torch.zeros(23, dtype=torch.float32), "elements"),         # too short
        (torch.zeros(48, dtype=torch.float32)[::2], "contiguous"),  # strided
        (good, "CUDA"),                                             # host memory
        (np.zeros(24, dtype=np.float32), "torch tensor"),
    ]
    for X, msg in cases:
        with pytest.raises(ValueError, match=msg):
            p.gnhtsvt(X, 1.0, out=good, workspace=ws)
        with pytest.raises(ValueError, match=msg):
            p.transform(X)
    with pytest.raises(ValueError, match="float64"):
        _fake_plan(htsvt, "fp64").gnhtsvt(good, 1.0)
    adm = htsvt.Admm.__new__(htsvt.Admm)
    adm.plan = p
    with pytest.raises(ValueError, match="L must be"):
        adm.init(torch.zeros(24, dtype=torch.float64), good, good, ws)
    with pytest.raises(ValueError, match="L holds"):
        adm.iterate(good, torch.zeros(24, dtype=torch.uint8), torch.zeros(3, dtype=torch.float32), good, good, 1, ws)
    with pytest.raises(ValueError, match="workspace must be torch.uint8"):
        htsvt.check_tensor(torch.zeros(8, dtype=torch.float32), "workspace", torch.uint8, 0)
    with pytest.raises(ValueError, match="truth"):
        adm.set_truth(torch.zeros(2, dtype=torch.float32))


def test_binding_exposes_new_kinds(lib):
    from paper_2506_09594_amd import htsvt
    assert htsvt.TRANSFORMS["dft_unnormalized"] == 3
    assert htsvt.PENALTIES["firm"] == 5
    assert htsvt.REGIONS["status"] == 21
