"""BF16 mixed-precision path (through the C-ABI) against the FP64 oracle.

The transformed slices are stored in BF16 and the sketch products run on the
BF16 matrix cores with FP32 accumulation; everything else is FP32 with FP64
Gram/Cholesky/eigen work.  Tolerance: relative Frobenius error 2e-2 of the
whole output against the FP64 oracle run on the FP32 input with the FP32-rounded
sketch matrices.
"""
import numpy as np
import pytest

from oracle import solver as osolver, transforms as otr, tsvt as otsvt
from workloads import synth

pytestmark = pytest.mark.gpu

TOL_BF16 = 2e-2
PEN = {"l1": ("l1", ()), "mcp": ("mcp", (40.0,)), "scad": ("scad", (3.7, 6.0))}


@pytest.fixture(scope="module")
def ht():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2506_09594_amd import htsvt
    return htsvt


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _run(ht, dims, kinds, rank, r, p, q, tau, pen, seed=1, noise=0.0, call=0):
    import torch
    X = synth.lowrank_tensor(dims, rank, kinds, seed=seed, noise_std=noise).astype(np.float32).astype(np.float64)
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision="bf16", seed=1000 + seed)
    out = plan.gnhtsvt(ht.to_device(X, plan.torch_dtype), tau, PEN[pen], call_index=call)
    torch.cuda.synchronize()
    got = ht.from_device(out, dims)
    om = otsvt.omegas(dims, kinds, r, p, seed=1000 + seed, call=call, round_to=np.float32)
    ref = otsvt.tsvt_randomized(X, tau, PEN[pen], otr.build_transforms(dims, kinds), r, p, q, om)
    return got, ref


@pytest.mark.parametrize("dims", [(96, 80, 4, 4), (36, 20, 16, 16)])
def test_bf16_transformed_slices_are_rounded_transform(ht, dims):
    import torch
    kinds = ["dct2", "dct2"]
    X = synth.lowrank_tensor(dims, 8, kinds, seed=2).astype(np.float32).astype(np.float64)
    plan = ht.Plan(dims, kinds, r=8, p=6, q=1, precision="bf16", seed=5)
    ws = plan.alloc_workspace()
    plan.gnhtsvt(ht.to_device(X, plan.torch_dtype), 1.0, PEN["l1"], workspace=ws)
    torch.cuda.synchronize()
    A = plan.region(ws, "A", dtype=torch.bfloat16)[: plan.N].double().cpu().numpy()
    ref = otr.to_slices(otr.forward(X, otr.build_transforms(dims, kinds))).reshape(-1, order="F")
    # every value is a BF16 neighbour of the exact transform: within the unit
    # roundoff of 8 significant bits (2^-8 relative) plus the FP32 transform's error
    assert np.all(np.abs(A - ref) <= 2.0 ** -8 * np.abs(ref) * (1 + 1e-4) + 1e-6 * np.abs(ref).max())
    # and almost always the round-to-nearest-even value of the FP32 transform
    rne = torch.from_numpy(ref.astype(np.float32)).to(torch.bfloat16).double().numpy()
    assert np.mean(A == rne) > 0.99


@pytest.mark.parametrize("pen", ["l1", "mcp", "scad"])
@pytest.mark.parametrize("dims,kinds,rank,r,p,q", [
    ((96, 80, 4, 4), ["dct2", "dct2"], 8, 8, 6, 2),        # 16-byte aligned columns
    ((130, 70, 3, 2, 2), ["dct2"] * 3, 6, 6, 10, 1),       # columns not 8-aligned: scalar loads
    ((132, 100, 3, 2), ["dct2", "dct2"], 30, 30, 20, 1),   # l = 50: two 32-column blocks
    ((200, 160, 2, 2), ["dct2", "dct2"], 50, 60, 10, 2),   # l = 70: three blocks
])
def test_tsvt_bf16(ht, pen, dims, kinds, rank, r, p, q):
    got, ref = _run(ht, dims, kinds, rank, r, p, q, tau=5.0, pen=pen)
    assert _rel(got, ref) < TOL_BF16


@pytest.mark.parametrize("dims,kinds,rank,r,p,q", [
    ((40, 30), [], 3, 3, 2, 1),              # order 2: one slice, no transform
    ((9, 7, 3), ["dct2"], 2, 5, 10, 1),      # l clamped to min(n1, n2)
    ((1, 6, 4), ["dct2"], 1, 1, 2, 0),       # n1 = 1
    ((257, 129, 3), ["dct2"], 4, 4, 4, 2),   # ragged tiles everywhere
    ((260, 36, 3), ["dct2"], 10, 10, 6, 2),  # tall
    ((36, 300, 3), ["dct2"], 10, 12, 4, 1),  # wide
])
def test_tsvt_bf16_edge_shapes(ht, dims, kinds, rank, r, p, q):
    got, ref = _run(ht, dims, kinds, rank, r, p, q, tau=1.0, pen="l1")
    assert _rel(got, ref) < TOL_BF16


def test_tsvt_bf16_full_size_config(ht):
    """256x256x16x16, rank 20 under DCT on modes 3 and 4, r=20 p=10 q=2, MCP."""
    got, ref = _run(ht, (256, 256, 16, 16), ["dct2", "dct2"], 20, 20, 10, 2, tau=50.0, pen="mcp", seed=2)
    assert _rel(got, ref) < TOL_BF16


def test_admm_completion_bf16(ht):
    """Twelve solver iterations in BF16-mixed stay within the BF16 tolerance of the
    FP64 oracle run, and recover the low-rank tensor as well as it does."""
    import torch
    dims, kinds, rank = (60, 50, 20), ["dct2"], 5
    Ltrue = synth.lowrank_tensor(dims, rank, kinds, seed=4, noise_std=1e-3)
    mask = synth.observation_mask(dims, 0.3, 4)
    M = np.where(mask, Ltrue, 0.0).astype(np.float32).astype(np.float64)
    r, p, q, seed = 5, 5, 1, 77
    mu0 = 1.0 / synth.max_slice_norm(M, kinds)
    vartheta, mu_max, n_iter = 1.2, 1e10, 12
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision="bf16", seed=seed)
    adm = ht.Admm(plan, "completion", phi=PEN["mcp"], psi=PEN["l1"], lam=0.0, mu0=mu0, vartheta=vartheta,
                  mu_max=mu_max)
    dt = plan.torch_dtype
    dM, dmask = ht.to_device(M, dt), ht.to_device(mask.astype(np.uint8), torch.uint8)
    dL, dE, dY = (torch.empty(plan.N, dtype=dt, device="cuda") for _ in range(3))
    ws = plan.alloc_workspace(admm=True)
    adm.init(dL, dE, dY, ws)
    adm.iterate(dM, dmask, dL, dE, dY, n_iter, ws)
    torch.cuda.synchronize()
    T = otr.build_transforms(dims, kinds)
    rnd = lambda X, tau, t: otsvt.tsvt_randomized(
        X, tau, PEN["mcp"], T, r, p, q, otsvt.omegas(dims, kinds, r, p, seed=seed, call=t, round_to=np.float32))
    Lr, _, _, _ = osolver.admm(M, mask, "completion", PEN["mcp"], PEN["l1"], 0.0, mu0, vartheta, mu_max, n_iter, rnd)
    got = ht.from_device(dL, dims)
    assert _rel(got, Lr) < TOL_BF16
    assert osolver.rse(got, Ltrue) < 1.5 * osolver.rse(Lr, Ltrue) + 1e-3
