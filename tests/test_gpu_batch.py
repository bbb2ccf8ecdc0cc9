"""Batches of uneven tensors in one plan (one launch per stage over every slice
of every tensor), tile tuning, the autotuner and graph replay, against the FP64
oracle run tensor by tensor.

Tolerances (relative Frobenius error of each tensor's output): FP64 1e-10,
FP32 1e-5, BF16-mixed 2e-2.  Tensor t of a batch draws its sketch from the
Philox stream stream_id + t; the oracle is given the same draws (rounded to
FP32 for the FP32 and BF16-mixed plans, whose sketch matrices are stored in FP32).
"""
import numpy as np
import pytest

from oracle import transforms as otr, tsvt as otsvt
from workloads import synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16": 2e-2}
MCP = ("mcp", (40.0,))
SHAPES = [(70, 50, 4), (64, 96, 2, 3), (33, 130, 2, 2, 2), (128, 64), (96, 96, 3)]
RANKS = [5, 8, 3, 10, 6]
PS = [5, 4, 6, 2, 10]
TAUS = [2.0, 3.0, 1.0, 4.0, 0.5]


@pytest.fixture(scope="module")
def ht():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2506_09594_amd import htsvt
    return htsvt


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _kinds(shape):
    return ["dct2"] * (len(shape) - 2)


def _inputs(shapes, ranks, prec, seed=11):
    xs = []
    for t, (s, r) in enumerate(zip(shapes, ranks)):
        X = synth.lowrank_tensor(s, r, _kinds(s), seed=seed + t, noise_std=1e-2)
        xs.append(X.astype(np.float64 if prec == "fp64" else np.float32).astype(np.float64))
    return xs


def _oracle(xs, shapes, ranks, ps, q, taus, pen, seed, stream_id, call, prec):
    outs = []
    for t, (X, s) in enumerate(zip(xs, shapes)):
        om = otsvt.omegas(s, _kinds(s), ranks[t], ps[t], seed=seed, call=call, stream=stream_id + t,
                          round_to=None if prec == "fp64" else np.float32)
        outs.append(otsvt.tsvt_randomized(X, taus[t], pen, otr.build_transforms(s, _kinds(s)), ranks[t], ps[t], q,
                                          om))
    return outs


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_batch_matches_oracle(ht, prec):
    import torch
    q, seed, sid = 1, 4242, 7
    xs = _inputs(SHAPES, RANKS, prec)
    plan = ht.BatchPlan(SHAPES, r=RANKS, p=PS, q=q, precision=prec, seed=seed, stream_id=sid)
    assert plan.n_slices == sum(int(np.prod(s[2:])) for s in SHAPES)
    out = plan.gnhtsvt(plan.pack(xs), TAUS, MCP, call_index=3)
    torch.cuda.synchronize()
    got = plan.unpack(out)
    ref = _oracle(xs, SHAPES, RANKS, PS, q, TAUS, MCP, seed, sid, 3, prec)
    for t in range(len(SHAPES)):
        assert _rel(got[t], ref[t]) < TOL[prec], f"tensor {t} shape {SHAPES[t]}"


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_width_classes_match_oracle(ht, prec):
    """Widths 10, 26, 42, 58, 74: one slice class per launch of the
    orthonormalization and the small SVD (classes up to 16, 32, 48, 64, 76)."""
    import torch
    shapes = [(96, 96, 3), (80, 90, 2, 2), (128, 100, 2), (90, 120, 2), (100, 96, 3)]
    ranks, ps = [5, 20, 36, 50, 66], [5, 6, 6, 8, 8]
    taus = [1.0, 2.0, 3.0, 2.5, 1.5]
    q, seed, sid = 1, 777, 2
    xs = _inputs(shapes, ranks, prec, seed=5)
    plan = ht.BatchPlan(shapes, r=ranks, p=ps, q=q, precision=prec, seed=seed, stream_id=sid)
    assert plan.widths == [10, 26, 42, 58, 74]
    out = plan.gnhtsvt(plan.pack(xs), taus, MCP, call_index=1)
    torch.cuda.synchronize()
    got = plan.unpack(out)
    ref = _oracle(xs, shapes, ranks, ps, q, taus, MCP, seed, sid, 1, prec)
    for t in range(len(shapes)):
        assert _rel(got[t], ref[t]) < TOL[prec], f"tensor {t} shape {shapes[t]}"


def test_batch_of_one_equals_single_plan(ht):
    import torch
    dims, kinds = (96, 80, 4, 4), ["dct2", "dct2"]
    X = synth.lowrank_tensor(dims, 8, kinds, seed=3).astype(np.float32)
    single = ht.Plan(dims, kinds, r=8, p=6, q=2, precision="fp32", seed=9, stream_id=5)
    batch = ht.BatchPlan([dims], r=[8], p=[6], q=2, precision="fp32", seed=9, stream_id=5)
    a = single.gnhtsvt(ht.to_device(X, torch.float32), 4.0, MCP, call_index=2)
    b = batch.gnhtsvt(batch.pack([X]), [4.0], MCP, call_index=2)
    torch.cuda.synchronize()
    assert torch.equal(a, b[: single.N])


@pytest.mark.parametrize("rows,kib", [(64, 32), (128, 32), (64, 128), (128, 64)])
def test_batch_tile_choices(ht, rows, kib):
    import torch
    q, seed, sid = 2, 99, 0
    xs = _inputs(SHAPES, RANKS, "fp32", seed=21)
    plan = ht.BatchPlan(SHAPES, r=RANKS, p=PS, q=q, precision="fp32", seed=seed, stream_id=sid)
    plan.set_tuning(prod_rows=rows, transform_lds_kib=kib)
    assert plan.tuning() == {"prod_rows": rows, "transform_lds_kib": kib}
    out = plan.gnhtsvt(plan.pack(xs), TAUS, ("l1", ()), call_index=0)
    torch.cuda.synchronize()
    ref = _oracle(xs, SHAPES, RANKS, PS, q, TAUS, ("l1", ()), seed, sid, 0, "fp32")
    for t, g in enumerate(plan.unpack(out)):
        assert _rel(g, ref[t]) < TOL["fp32"]


def test_autotune_then_parity(ht):
    import torch
    q, seed = 1, 5
    xs = _inputs(SHAPES, RANKS, "bf16", seed=31)
    plan = ht.BatchPlan(SHAPES, r=RANKS, p=PS, q=q, precision="bf16", seed=seed)
    X = plan.pack(xs)
    tuning, ms = plan.autotune(X, repeats=2)
    assert tuning["prod_rows"] in (64, 128) and tuning["transform_lds_kib"] in (32, 64, 128)
    assert 0.0 < ms < 1e3
    out = plan.gnhtsvt(X, TAUS, MCP, call_index=1)
    torch.cuda.synchronize()
    ref = _oracle(xs, SHAPES, RANKS, PS, q, TAUS, MCP, seed, 0, 1, "bf16")
    for t, g in enumerate(plan.unpack(out)):
        assert _rel(g, ref[t]) < TOL["bf16"]


def test_graph_replay_matches_eager(ht):
    """The recorded graph replays with a new call index each time and gives the
    eager result bit for bit; eager work and synchronizations run between replays."""
    import torch
    xs = _inputs(SHAPES, RANKS, "fp32", seed=41)
    plan = ht.BatchPlan(SHAPES, r=RANKS, p=PS, q=2, precision="fp32", seed=17)
    X = plan.pack(xs)
    ws = plan.alloc_workspace()
    tau = torch.tensor(TAUS, dtype=torch.float64, device="cuda")
    out = torch.zeros_like(X)  # gaps between the packed tensors are never written
    eager = []
    for call in range(3):
        plan.gnhtsvt(X, tau, MCP, call_index=call, out=out, workspace=ws)
        eager.append(out.clone())
    torch.cuda.synchronize()
    plan.graph(True)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for rep, call in enumerate([0, 1, 2, 1]):
            out.fill_(0.0)
            plan.gnhtsvt(X, tau, MCP, call_index=call, out=out, workspace=ws)
            torch.cuda.synchronize()
            assert torch.equal(out, eager[call]), f"replay {rep} (call {call})"
            junk = (X * 2.0).sum()  # eager work between replays
            torch.cuda.synchronize()
            del junk
        tau2 = tau * 0.5  # new tau array pointer: records a new graph
        plan.gnhtsvt(X, tau2, MCP, call_index=0, out=out, workspace=ws)
        torch.cuda.synchronize()
    ref = _oracle(xs, SHAPES, RANKS, PS, 2, [t * 0.5 for t in TAUS], MCP, 17, 0, 0, "fp32")
    for t, g in enumerate(plan.unpack(out)):
        assert _rel(g, ref[t]) < TOL["fp32"]
    plan.graph(False)


def test_single_plan_graph_replay(ht):
    import torch
    dims, kinds = (60, 50, 20), ["dct2"]
    X = synth.lowrank_tensor(dims, 5, kinds, seed=4, noise_std=1e-3)
    plan = ht.Plan(dims, kinds, r=5, p=5, q=1, precision="fp64", seed=3)
    dX = ht.to_device(X, torch.float64)
    ws = plan.alloc_workspace()
    out = torch.empty_like(dX)
    eager = []
    for call in range(2):
        plan.gnhtsvt(dX, 2.0, ("l1", ()), call_index=call, out=out, workspace=ws)
        eager.append(out.clone())
    torch.cuda.synchronize()
    plan.graph(True)
    with pytest.raises(ht.HtError):  # the null stream cannot be captured
        plan.gnhtsvt(dX, 2.0, ("l1", ()), call_index=0, out=out, workspace=ws)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for call in (1, 0, 1):
            plan.gnhtsvt(dX, 2.0, ("l1", ()), call_index=call, out=out, workspace=ws)
            torch.cuda.synchronize()
            assert torch.equal(out, eager[call])
    plan.graph(False)


def test_random_batch_bf16(ht):
    """A seeded batch drawn like the uneven-batch workload, at reduced sizes:
    orders 3-5, modes in {2, 4}, n1, n2 in [40, 160], ranks in [5, 40], p = 10, q = 2."""
    import torch
    spec = synth.batch_shapes(12, seed=8, modes=(2, 4), n_range=(40, 160))
    shapes = [s for s, _ in spec]
    ranks = [r for _, r in spec]
    ps = [10] * len(spec)
    taus = [1.0 + 0.25 * t for t in range(len(spec))]
    xs = []
    for t, (s, r) in enumerate(spec):
        xs.append(synth.lowrank_tensor(s, r, _kinds(s), seed=100 + t, noise_std=1e-2).astype(np.float32)
                  .astype(np.float64))
    plan = ht.BatchPlan(shapes, r=ranks, p=ps, q=2, precision="bf16", seed=123)
    out, sig, kept = plan.gnhtsvt(plan.pack(xs), taus, MCP, call_index=0, stats=True)
    torch.cuda.synchronize()
    got = plan.unpack(out)
    ref = _oracle(xs, shapes, ranks, ps, 2, taus, MCP, 123, 0, 0, "bf16")
    for t in range(len(spec)):
        assert _rel(got[t], ref[t]) < TOL["bf16"], f"tensor {t} {shapes[t]}"
    # per-slice stats rows are padded with zeros past each tensor's width
    sig = sig.cpu().numpy()
    for t in range(len(spec)):
        f, w = plan.first_slice[t], plan.widths[t]
        assert np.all(sig[f, w:] == 0.0) and np.all(sig[f, :w] >= 0.0)
