"""Parity on the code paths the larger workloads take, against the FP64 oracle:
length-8 transformed modes at the learned-width workload's full shape
(128x128x8x8x8, l = 74), the generic transform tile with a length-16 mode on
the matrix cores next to a length-8 mode, 4096 face slices in one tile list
(16x16x16 modes), a seeded batch of uneven tensors with modes in {4, 8, 16},
and one ADMM iteration at the per-iteration tolerances.

Tolerances (relative Frobenius): FP64 1e-10, FP32 1e-5, BF16-mixed 2e-2.
"""
import numpy as np
import pytest

from oracle import solver as osolver, transforms as otr, tsvt as otsvt
from workloads import synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16": 2e-2}
MCP = ("mcp", (40.0,))


@pytest.fixture(scope="module")
def ht():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2506_09594_amd import htsvt
    return htsvt


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _np(prec):
    return np.float64 if prec == "fp64" else np.float32


def _tsvt_case(ht, X, dims, kinds, r, p, q, prec, tau, pen, seed, call=0):
    import torch
    Xs = X.astype(_np(prec)).astype(np.float64)
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision=prec, seed=seed)
    out = plan.gnhtsvt(ht.to_device(Xs, plan.torch_dtype), tau, pen, call_index=call)
    torch.cuda.synchronize()
    om = otsvt.omegas(dims, kinds, r, p, seed=seed, call=call, round_to=None if prec == "fp64" else np.float32)
    ref = otsvt.tsvt_randomized(Xs, tau, pen, otr.build_transforms(dims, kinds), r, p, q, om)
    return ht.from_device(out, dims), ref, plan


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_learned_workload_shape_length8_modes_width74(ht, prec):
    """128x128x8x8x8 (512 slices, three modes of 8 on the vector units), per-slice
    rank uniform in [4, 64], fixed r = 64, p = 10 (l = 74: the wide
    orthonormalization and the 80-wide small SVD), q = 2."""
    dims, kinds = (128, 128, 8, 8, 8), ["dct2"] * 3
    ranks = synth.rng(5, "ranks").integers(4, 65, size=512)
    X = synth.slice_rank_tensor(dims, ranks, kinds, 5) + 1e-2 * synth.rng(5, "noise").standard_normal(dims)
    got, ref, plan = _tsvt_case(ht, X, dims, kinds, 64, 10, 2, prec, 30.0, MCP, seed=55)
    assert plan.width == 74 and plan.n_slices == 512
    assert _rel(got, ref) < TOL[prec]


@pytest.mark.parametrize("dims", [(40, 36, 16, 8), (40, 36, 8, 16), (52, 44, 16, 3)])
def test_generic_transform_tile_with_a_mode_of_16(ht, dims):
    """FP32 tensors whose transformed modes are not exactly two of 16: the
    generic tile runs the length-16 mode on the matrix cores and the others on
    the vector units (forward, inverse and a whole t-SVT)."""
    import torch
    kinds = ["dct2"] * (len(dims) - 2)
    rng = np.random.default_rng(3)
    X = rng.standard_normal(dims).astype(np.float32).astype(np.float64)
    plan = ht.Plan(dims, kinds, r=4, p=4, q=1, precision="fp32")
    dX = ht.to_device(X, torch.float32)
    fwd = plan.transform(dX)
    back = plan.transform(fwd, inverse=True)
    torch.cuda.synchronize()
    T = otr.build_transforms(dims, kinds)
    assert _rel(ht.from_device(fwd, dims), otr.forward(X, T)) < 1e-6
    assert _rel(ht.from_device(back, dims), X) < 1e-6
    Xl = synth.lowrank_tensor(dims, 5, kinds, seed=9, noise_std=1e-2)
    got, ref, _ = _tsvt_case(ht, Xl, dims, kinds, 5, 5, 2, "fp32", 2.0, MCP, seed=19)
    assert _rel(got, ref) < TOL["fp32"]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp64"])
def test_order5_4096_slices(ht, prec):
    """Modes 16 x 16 x 16: 4096 face slices (8 tube positions per transform tile
    at 128 KiB), every per-slice launch over 4096 slices."""
    dims, kinds = (24, 20, 16, 16, 16), ["dct2"] * 3
    X = synth.lowrank_tensor(dims, 3, kinds, seed=4, noise_std=1e-2)
    got, ref, plan = _tsvt_case(ht, X, dims, kinds, 3, 3, 1, prec, 1.0, MCP, seed=23)
    assert plan.n_slices == 4096
    assert _rel(got, ref) < TOL[prec]


def _kinds(shape):
    return ["dct2"] * (len(shape) - 2)


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_seeded_batch_modes_4_8_16(ht, prec):
    """Eight uneven tensors drawn like the batched workload (orders 3-5, every
    transformed mode in {4, 8, 16}, ranks in [5, 40], p = 10, q = 2) at
    n1, n2 in [64, 128]: 4,416 slices of eight shapes in one plan."""
    import torch
    spec = synth.batch_shapes(8, seed=3, modes=(4, 8, 16), n_range=(64, 128))
    shapes = [s for s, _ in spec]
    ranks = [r for _, r in spec]
    ps = [10] * len(spec)
    taus = [2.0 + 0.5 * t for t in range(len(spec))]
    xs = [synth.lowrank_tensor(s, r, _kinds(s), seed=300 + t, noise_std=1e-2).astype(np.float32).astype(np.float64)
          for t, (s, r) in enumerate(spec)]
    plan = ht.BatchPlan(shapes, r=ranks, p=ps, q=2, precision=prec, seed=77, stream_id=2)
    assert plan.n_slices == sum(int(np.prod(s[2:])) for s in shapes)
    out = plan.gnhtsvt(plan.pack(xs), taus, MCP, call_index=4)
    torch.cuda.synchronize()
    got = plan.unpack(out)
    for t, (X, s) in enumerate(zip(xs, shapes)):
        om = otsvt.omegas(s, _kinds(s), ranks[t], ps[t], seed=77, call=4, stream=2 + t, round_to=np.float32)
        ref = otsvt.tsvt_randomized(X, taus[t], MCP, otr.build_transforms(s, _kinds(s)), ranks[t], ps[t], 2, om)
        assert _rel(got[t], ref) < TOL[prec], f"tensor {t} shape {s}"


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("model", ["completion", "rpca"])
def test_admm_one_iteration_at_tight_tolerance(ht, prec, model):
    """One iteration of the pure-L ADMM (t-SVT of M - E + Y/mu, then the E, Y
    and mu updates) matches the oracle at the per-iteration tolerances on L, E
    and Y, and the stopping terms match."""
    import torch
    dims, kinds, rank = (60, 50, 20), ["dct2"], 5
    Lt = synth.lowrank_tensor(dims, rank, kinds, seed=4, noise_std=1e-3)
    mask = synth.observation_mask(dims, 0.3 if model == "completion" else 0.5, 4)
    S = synth.outliers(dims, 0.05, 4) * 3.0 if model == "rpca" else 0.0
    M = np.where(mask, Lt + S, 0.0).astype(_np(prec)).astype(np.float64)
    r, p, q, seed = 5, 5, 1, 78
    mu0 = 1.0 / synth.max_slice_norm(M, kinds)
    lam = 2.0 / np.sqrt(max(dims[0], dims[1]) * dims[2])
    pen = MCP if model == "completion" else ("l1", ())
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision=prec, seed=seed)
    adm = ht.Admm(plan, model, phi=pen, psi=("l1", ()), lam=lam, mu0=mu0, vartheta=1.2, mu_max=1e10)
    dt = plan.torch_dtype
    dL, dE, dY = (torch.empty(plan.N, dtype=dt, device="cuda") for _ in range(3))
    ws = plan.alloc_workspace(admm=True)
    adm.init(dL, dE, dY, ws)
    adm.iterate(ht.to_device(M, dt), ht.to_device(mask.astype(np.uint8), torch.uint8), dL, dE, dY, 1, ws)
    st = adm.stats(ws)
    T = otr.build_transforms(dims, kinds)
    rnd = lambda X, tau, t: otsvt.tsvt_randomized(
        X, tau, pen, T, r, p, q,
        otsvt.omegas(dims, kinds, r, p, seed=seed, call=t, round_to=None if prec == "fp64" else np.float32))
    Lr, Er, Yr, hist = osolver.admm(M, mask, model, pen, ("l1", ()), lam, mu0, 1.2, 1e10, 1, rnd)
    tol = TOL[prec]
    assert _rel(ht.from_device(dL, dims), Lr) < tol
    assert _rel(ht.from_device(dE, dims), Er) < tol
    assert _rel(ht.from_device(dY, dims), Yr) < tol
    assert st["iteration"] == 1
    for key in ("dL", "dE", "resid"):
        assert st[key] == pytest.approx(hist[0][key], rel=1e-9 if prec == "fp64" else 1e-4)
