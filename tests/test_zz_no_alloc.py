"""The allocation-free t-SVT (ht_gnhtsvt_noalloc) against ht_gnhtsvt.

Both calls run the same kernels on the same inputs and sketch draws; the only
difference is where the workspace lives (the library's device scratch or a
caller-provided buffer).  Two calls in a row on different plans, the second
smaller, check that the shared scratch carries nothing from one call into the
next.  Tolerance as for the oracle parity: 1e-10 (FP64) and 1e-5 (FP32) in the
relative Frobenius norm; in practice the outputs agree bit for bit.
"""
import numpy as np
import pytest

from workloads import synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


@pytest.fixture(scope="module")
def ht():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2506_09594_amd import htsvt
    return htsvt


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _pair(ht, dims, kinds, rank, r, p, q, prec, seed, tau, pen):
    import torch
    X = synth.lowrank_tensor(dims, rank, kinds, seed=seed, noise_std=1e-3)
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision=prec, seed=500 + seed)
    dX = ht.to_device(X, plan.torch_dtype)
    sig = torch.empty(plan.n_slices * plan.width, dtype=torch.float64, device="cuda")
    kept = torch.empty(plan.n_slices, dtype=torch.int32, device="cuda")
    got = plan.gnhtsvt_noalloc(dX, tau, pen, call_index=3, stats=(sig, kept))
    ref, rsig, rkept = plan.gnhtsvt(dX, tau, pen, call_index=3, stats=True)
    torch.cuda.synchronize()
    return plan, ht.from_device(got, dims), ht.from_device(ref, dims), sig.cpu().numpy(), \
        rsig.cpu().numpy().ravel(), kept.cpu().numpy(), rkept.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_workspace_call_twice(ht, prec):
    # first a larger tensor (two modes of 16 for FP32: the per-wavefront transform and the
    # streaming product), then a smaller one of another shape on the same scratch
    cases = [((200, 96, 16, 16), ["dct2", "dct2"], 8, 8, 6, 2, ("mcp", (60.0,)), 30.0),
             ((60, 50, 20), ["dct2"], 5, 5, 5, 1, ("l1", ()), 5.0)]
    for i, (dims, kinds, rank, r, p, q, pen, tau) in enumerate(cases):
        plan, got, ref, sig, rsig, kept, rkept = _pair(ht, dims, kinds, rank, r, p, q, prec, 11 + i, tau, pen)
        print(f"noalloc {prec} {dims}: workspace {plan.workspace_bytes} B, rel diff {_rel(got, ref):.3e}",
              flush=True)
        assert _rel(got, ref) <= TOL[prec]
        assert np.abs(sig - rsig).max() <= TOL[prec] * max(1.0, np.abs(rsig).max())
        assert np.array_equal(kept, rkept)


def test_noalloc_rejects_what_it_cannot_hold(ht):
    import torch
    # 512 x 512 x 32 x 8 FP32: 256 slices of 1 MiB, workspace above the 256 MiB scratch
    dims = (512, 512, 32, 8)
    plan = ht.Plan(dims, ["dct2", "dct2"], r=10, p=5, q=1, precision="fp32", seed=1)
    assert plan.workspace_bytes > 256 << 20
    X = torch.zeros(plan.N, dtype=torch.float32, device="cuda")
    with pytest.raises(ht.HtError) as e:
        plan.gnhtsvt_noalloc(X, 1.0)
    assert e.value.code == ht.ERR_WORKSPACE
    # batch plans and plans with graph replay are refused before any launch
    small = ht.Plan((40, 30, 4), ["dct2"], r=3, p=2, q=1, precision="fp32", seed=2)
    Xs = torch.zeros(small.N, dtype=torch.float32, device="cuda")
    small.graph(True)
    with pytest.raises(ht.HtError) as e:
        small.gnhtsvt_noalloc(Xs, 1.0)
    assert e.value.code == ht.ERR_UNSUPPORTED
    small.graph(False)
    small.gnhtsvt_noalloc(Xs, 1.0)
    torch.cuda.synchronize()
