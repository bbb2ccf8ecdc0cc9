"""Unitary DFT on modes 3..d (complex transformed slices) against the FP64
oracle's complex randomized t-SVT.

Only one slice of each conjugate pair is sketched (the output of its partner
is the conjugate, so the result is real); the complex slice is sketched with
the real Gaussian Omega the oracle uses (keyed by the canonical member of the
pair), every product complex, CholeskyQR and the Hermitian eigensolver in
complex FP64.  Tolerances as for the real transforms: FP64 1e-10, FP32 1e-5,
BF16-mixed 2e-2 (relative Frobenius).
"""
import numpy as np
import pytest

from oracle import solver as osolver, transforms as otr, tsvt as otsvt
from workloads import synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16": 2e-2}


@pytest.fixture(scope="module")
def ht():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2506_09594_amd import htsvt
    return htsvt


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _case(ht, dims, rank, r, p, q, prec, tau, pen, seed=1, noise=1e-2):
    import torch
    kinds = ["dft"] * (len(dims) - 2)
    X = synth.lowrank_tensor(dims, rank, kinds, seed=seed, noise_std=noise)
    Xs = X.astype(np.float64 if prec == "fp64" else np.float32).astype(np.float64)
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision=prec, seed=50 + seed)
    out = plan.gnhtsvt(ht.to_device(Xs, plan.torch_dtype), tau, pen, call_index=2)
    torch.cuda.synchronize()
    om = otsvt.omegas(dims, kinds, r, p, seed=50 + seed, call=2, round_to=None if prec == "fp64" else np.float32)
    ref = otsvt.tsvt_randomized(Xs, tau, pen, otr.build_transforms(dims, kinds), r, p, q, om)
    return ht.from_device(out, dims), ref, plan


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("noise", [0.0, 1e-6, 1e-3])
def test_tsvt_dft_repeated_singular_values(ht, prec, noise):
    """Every transformed slice of X = sum_i u_i v_i^T c (u, v orthonormal, c a
    real tube) is c_hat_j U V^T: its nonzero singular values are |c_hat_j|,
    repeated rank times.  Noise splits them into tight clusters (and fills
    the zero ones).  All repeated values are kept (rank <= r)."""
    import torch
    dims, kinds, rank, r, p, q = (40, 36, 8, 2), ["dft", "dft"], 4, 6, 4, 1
    rng = np.random.default_rng(5)
    U = np.linalg.qr(rng.standard_normal((dims[0], rank)))[0]
    V = np.linalg.qr(rng.standard_normal((dims[1], rank)))[0]
    c = rng.standard_normal(dims[2:])
    X = np.einsum("ar,br,jk->abjk", U, V, c) + noise * rng.standard_normal(dims)
    Xs = X.astype(np.float64 if prec == "fp64" else np.float32).astype(np.float64)
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision=prec, seed=61)
    tau, pen = 0.05, ("mcp", (30.0,))
    out = plan.gnhtsvt(ht.to_device(Xs, plan.torch_dtype), tau, pen, call_index=4)
    torch.cuda.synchronize()
    om = otsvt.omegas(dims, kinds, r, p, seed=61, call=4, round_to=None if prec == "fp64" else np.float32)
    ref = otsvt.tsvt_randomized(Xs, tau, pen, otr.build_transforms(dims, kinds), r, p, q, om)
    assert _rel(ht.from_device(out, dims), ref) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("dims,rank,r,p,q", [
    ((40, 30, 4, 3), 5, 5, 5, 1),    # even mode: self-conjugate slices at index 0 and n/2
    ((33, 20, 5), 4, 6, 4, 2),       # odd mode, ragged rows
    ((35, 27, 6), 4, 6, 4, 2),       # odd row and column counts in both thin blocks
    ((24, 64, 2, 2, 2), 3, 8, 8, 1), # order 5, all slices self-conjugate
    ((40, 36, 4, 16, 2), 5, 6, 4, 1),  # order 5: first mode 2, last 16, a mode of 4 between
    ((64, 48, 6), 10, 12, 6, 2),     # columns aligned for 16-byte loads
    ((136, 100, 4, 2), 30, 40, 10, 2),  # width 50: three 64-row tiles with a ragged last one
    ((64, 70, 3, 3), 20, 54, 10, 1),    # width 64, the largest complex width
    ((48, 40, 8, 16), 6, 8, 4, 1),      # FFT modes of 8 and 16
    ((36, 28, 32), 5, 8, 4, 1),         # FFT mode of 32
    ((520, 512, 2, 2), 6, 8, 4, 1),     # more transform tiles than resident workgroups; tiles across columns
])
def test_tsvt_dft_matches_oracle(ht, prec, dims, rank, r, p, q):
    got, ref, plan = _case(ht, dims, rank, r, p, q, prec, 2.0, ("mcp", (30.0,)))
    assert _rel(got, ref) < TOL[prec]
    # one slot per conjugate pair
    P = int(np.prod(dims[2:]))
    canon = {otr.canonical_slice(j, dims, ["dft"] * (len(dims) - 2)) for j in range(P)}
    assert plan.n_slices == len(canon)


def test_dft_low_rank_recovered_exactly(ht):
    """tau = 0 on an exactly low-rank tensor: the output is the input (to rounding)."""
    import torch
    dims, kinds = (30, 26, 6), ["dft"]
    X = synth.lowrank_tensor(dims, 4, kinds, seed=3)
    plan = ht.Plan(dims, kinds, r=4, p=4, q=1, precision="fp64", seed=1)
    out = plan.gnhtsvt(ht.to_device(X, torch.float64), 0.0, ("l1", ()))
    torch.cuda.synchronize()
    assert _rel(ht.from_device(out, dims), X) < 1e-11


def test_dft_stats_are_the_complex_singular_values(ht):
    import torch
    dims, kinds = (40, 30, 5), ["dft"]
    X = synth.lowrank_tensor(dims, 6, kinds, seed=4, noise_std=1e-2)
    plan = ht.Plan(dims, kinds, r=6, p=4, q=1, precision="fp64", seed=1)
    out, sig, kept = plan.gnhtsvt(ht.to_device(X, torch.float64), 1.0, ("l1", ()), stats=True)
    torch.cuda.synchronize()
    sig = sig.cpu().numpy()
    assert plan.width == 10 and sig.shape[1] == 10
    LX = otr.to_slices(otr.forward(X, otr.build_transforms(dims, kinds)))
    s_true = np.linalg.svd(LX[:, :, 1], compute_uv=False)[:6]
    slot = sorted({otr.canonical_slice(j, dims, kinds) for j in range(5)}).index(1)
    assert np.allclose(sig[slot, :6], s_true, rtol=1e-8)
    assert np.all(kept.cpu().numpy() == 6)


def test_rpca_dft_matches_oracle(ht):
    """Robust completion (pure-L ADMM) under the unitary DFT, FP32, 10 iterations."""
    import torch
    dims, kinds, rank = (40, 32, 4, 2), ["dft", "dft"], 4
    L = synth.lowrank_tensor(dims, rank, kinds, seed=8, noise_std=1e-3)
    mask = synth.observation_mask(dims, 0.6, 8)
    S = synth.outliers(dims, 0.05, 8)
    M = np.where(mask, L + S, 0.0).astype(np.float32).astype(np.float64)
    r, p, q, seed, n_iter = 4, 4, 1, 21, 10
    mu0 = 1.0 / synth.max_slice_norm(M, kinds)
    lam = 1.0 / np.sqrt(max(dims[0], dims[1]) * 8)
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision="fp32", seed=seed)
    adm = ht.Admm(plan, "rpca", phi=("l1", ()), psi=("l1", ()), lam=lam, mu0=mu0, vartheta=1.15, mu_max=1e10)
    dL, dE, dY = (torch.empty(plan.N, dtype=torch.float32, device="cuda") for _ in range(3))
    ws = plan.alloc_workspace(admm=True)
    adm.init(dL, dE, dY, ws)
    adm.iterate(ht.to_device(M, torch.float32), ht.to_device(mask.astype(np.uint8), torch.uint8), dL, dE, dY,
                n_iter, ws)
    torch.cuda.synchronize()
    T = otr.build_transforms(dims, kinds)
    rnd = lambda X, tau, t: otsvt.tsvt_randomized(
        X, tau, ("l1", ()), T, r, p, q, otsvt.omegas(dims, kinds, r, p, seed=seed, call=t, round_to=np.float32))
    Lr, Er, _, _ = osolver.admm(M, mask, "rpca", ("l1", ()), ("l1", ()), lam, mu0, 1.15, 1e10, n_iter, rnd)
    assert _rel(ht.from_device(dL, dims), Lr) < 1e-4
    assert _rel(ht.from_device(dE, dims), Er) < 1e-4


def test_dft_unsupported_combinations(ht):
    with pytest.raises(ht.HtError):  # mixed real and DFT modes
        ht.Plan((20, 20, 4, 4), ["dct2", "dft"], r=4, p=4)
    with pytest.raises(ht.HtError) as e:  # complex widths stop at 64
        ht.Plan((100, 100, 4), ["dft"], r=60, p=10)
    assert e.value.code == ht.ERR_UNSUPPORTED
    ht.Plan((100, 100, 4), ["dft"], r=50, p=10)  # l = 60: the large robust-PCA width


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("shapes", [
    [(40, 32, 8, 4), (36, 24, 4, 8), (24, 20, 4, 4, 4)],  # one first-mode length: fused transform across tensors
    [(40, 32, 8, 4), (30, 20, 6)],                         # mixed mode lengths: the general transform
])
def test_batch_of_dft_tensors_matches_oracle(ht, prec, shapes):
    """Uneven DFT tensors in one batched plan (Philox stream stream_id + t for
    tensor t) against the oracle tensor by tensor."""
    import torch
    n = len(shapes)
    ranks, ps, taus = [4, 5, 3][:n], [4, 3, 5][:n], [2.0, 1.5, 1.0][:n]
    q, seed, sid = 1, 99, 3
    kinds = [["dft"] * (len(s) - 2) for s in shapes]
    xs = [synth.lowrank_tensor(s, ranks[t], kinds[t], seed=20 + t, noise_std=1e-2).astype(np.float32)
          .astype(np.float64) for t, s in enumerate(shapes)]
    plan = ht.BatchPlan(shapes, transforms=kinds, r=ranks, p=ps, q=q, precision=prec, seed=seed, stream_id=sid)
    out = plan.gnhtsvt(plan.pack(xs), taus, ("mcp", (30.0,)), call_index=2)
    torch.cuda.synchronize()
    got = plan.unpack(out)
    for t, s in enumerate(shapes):
        om = otsvt.omegas(s, kinds[t], ranks[t], ps[t], seed=seed, call=2, stream=sid + t, round_to=np.float32)
        ref = otsvt.tsvt_randomized(xs[t], taus[t], ("mcp", (30.0,)), otr.build_transforms(s, kinds[t]), ranks[t],
                                    ps[t], q, om)
        assert _rel(got[t], ref) < TOL[prec], f"tensor {t} shape {s}"
