"""Boundary features of the C-ABI on the GPU, against the FP64 oracle: the
unnormalized DFT (alpha = n, the FFT of the experiments), the FIRM penalty,
non-finite detection (HT_ERR_NONFINITE) and the solver's RSE against a
registered ground truth.  Tolerances: FP64 1e-10, FP32 1e-5 (relative
Frobenius)."""
import numpy as np
import pytest

from oracle import solver as osolver, transforms as otr, tsvt as otsvt
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


def _np(prec):
    return np.float64 if prec == "fp64" else np.float32


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,kinds,rank,r,p,q,tau", [
    ((40, 30, 6), ["dft_unnormalized"], 5, 5, 5, 1, 6.0),
    ((36, 28, 4, 3), ["dft_unnormalized", "dft_unnormalized"], 4, 6, 4, 2, 8.0),
    ((36, 28, 4, 3), ["dft", "dft_unnormalized"], 4, 6, 4, 1, 4.0),   # the two DFT kinds mixed across modes
])
def test_unnormalized_dft_matches_oracle(ht, prec, dims, kinds, rank, r, p, q, tau):
    """F without the 1/sqrt(n) (alpha = n): the transformed slices are sqrt(n)
    larger per mode and tau applies to them unscaled."""
    import torch
    X = synth.lowrank_tensor(dims, rank, ["dft"] * (len(dims) - 2), seed=3, noise_std=1e-2)
    Xs = X.astype(_np(prec)).astype(np.float64)
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision=prec, seed=71)
    out = plan.gnhtsvt(ht.to_device(Xs, plan.torch_dtype), tau, ("mcp", (50.0,)), call_index=3)
    torch.cuda.synchronize()
    om = otsvt.omegas(dims, kinds, r, p, seed=71, call=3, round_to=None if prec == "fp64" else np.float32)
    ref = otsvt.tsvt_randomized(Xs, tau, ("mcp", (50.0,)), otr.build_transforms(dims, kinds), r, p, q, om)
    assert _rel(ht.from_device(out, dims), ref) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("a", [1.5, 4.0])
def test_firm_penalty_matches_oracle(ht, prec, a):
    import torch
    dims, kinds = (60, 50, 20), ["dct2"]
    X = synth.lowrank_tensor(dims, 5, kinds, seed=5, noise_std=1e-2)
    Xs = X.astype(_np(prec)).astype(np.float64)
    plan = ht.Plan(dims, kinds, r=5, p=5, q=1, precision=prec, seed=9)
    out = plan.gnhtsvt(ht.to_device(Xs, plan.torch_dtype), 20.0, ("firm", (a,)))
    torch.cuda.synchronize()
    om = otsvt.omegas(dims, kinds, 5, 5, seed=9, round_to=None if prec == "fp64" else np.float32)
    ref = otsvt.tsvt_randomized(Xs, 20.0, ("firm", (a,)), otr.build_transforms(dims, kinds), 5, 5, 1, om)
    assert _rel(ht.from_device(out, dims), ref) < TOL[prec]


def test_firm_rejects_ratio_at_most_one(ht):
    import torch
    plan = ht.Plan((20, 16, 3), ["dct2"], r=3, p=2, q=1, precision="fp64")
    X = torch.zeros(plan.N, dtype=torch.float64, device="cuda")
    with pytest.raises(ht.HtError) as e:
        plan.gnhtsvt(X, 1.0, ("firm", (1.0,)))
    assert e.value.code == ht.ERR_INVALID_ARG


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nonfinite_input_is_reported(ht, prec):
    """A NaN (and separately an infinity) in one tube of the tensor reaches
    every slice under the DCT; the status call reports the slices and returns
    HT_ERR_NONFINITE; a finite call on the same workspace clears it."""
    import torch
    dims, kinds = (48, 40, 6), ["dct2"]
    X = synth.lowrank_tensor(dims, 4, kinds, seed=2)
    plan = ht.Plan(dims, kinds, r=4, p=4, q=1, precision=prec, seed=1)
    ws = plan.alloc_workspace()
    dX = ht.to_device(X, plan.torch_dtype)
    plan.gnhtsvt(dX, 1.0, ("l1", ()), workspace=ws)
    assert plan.status(ws) == 0
    for bad in (float("nan"), float("inf")):
        Xb = dX.clone()
        Xb[7 + 48 * 11] = bad
        plan.gnhtsvt(Xb, 1.0, ("l1", ()), workspace=ws)
        with pytest.raises(ht.HtError) as e:
            plan.status(ws)
        assert e.value.code == ht.ERR_NONFINITE
        assert "slice" in str(e.value)
    plan.gnhtsvt(dX, 1.0, ("l1", ()), workspace=ws)
    assert plan.status(ws) == 0


def test_solver_reports_nonfinite_and_rse(ht):
    """Completion on 60x50x20: with a registered ground truth the solver state
    carries ||L - L*|| / ||L*|| of the GPU iterate (FP64 sums); a NaN in the
    observations makes the stopping terms NaN (not dropped) and the stats call
    returns HT_ERR_NONFINITE."""
    import torch
    dims, kinds = (60, 50, 20), ["dct2"]
    Lt = synth.lowrank_tensor(dims, 5, kinds, seed=4)
    mask = synth.observation_mask(dims, 0.3, 4)
    M = np.where(mask, Lt, 0.0)
    plan = ht.Plan(dims, kinds, r=5, p=5, q=1, precision="fp64", seed=3)
    adm = ht.Admm(plan, "completion", phi=("mcp", (40.0,)), mu0=1.0 / synth.max_slice_norm(M, kinds),
                  vartheta=1.2, mu_max=1e10)
    dM, dmask = ht.to_device(M, torch.float64), ht.to_device(mask.astype(np.uint8), torch.uint8)
    dL, dE, dY = (torch.empty(plan.N, dtype=torch.float64, device="cuda") for _ in range(3))
    ws = plan.alloc_workspace(admm=True)
    adm.init(dL, dE, dY, ws)
    adm.iterate(dM, dmask, dL, dE, dY, 3, ws)
    st = adm.stats(ws)
    assert np.isnan(st["rse"])  # no ground truth registered
    truth = ht.to_device(Lt, torch.float64)
    adm.set_truth(truth)
    adm.iterate(dM, dmask, dL, dE, dY, 5, ws)
    st = adm.stats(ws)
    assert st["iteration"] == 8
    assert st["rse"] == pytest.approx(osolver.rse(ht.from_device(dL, dims), Lt), rel=1e-12)
    assert st["rse"] < 1.0
    adm.set_truth(None)
    Mb = dM.clone()
    Mb[int(np.flatnonzero(mask.ravel(order="F"))[0])] = float("nan")
    adm.init(dL, dE, dY, ws)
    adm.iterate(Mb, dmask, dL, dE, dY, 2, ws)
    with pytest.raises(ht.HtError) as e:
        adm.stats(ws)
    assert e.value.code == ht.ERR_NONFINITE


def test_plan_records_its_device(ht):
    import torch
    plan = ht.Plan((20, 16, 3), ["dct2"], r=3, p=2, q=1, precision="fp32")
    assert plan.device() == torch.cuda.current_device()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("model", ["rpca_tube", "rpca_slice"])
def test_group_sparse_models_match_oracle(ht, prec, model):
    """Robust completion with tube-wise and slice-wise GNHTT on the sparse part
    (structured outliers: whole corrupted tubes or slices), one and eight
    iterations against the oracle at the per-iteration tolerances."""
    import torch
    dims, kinds, rank = (40, 30, 6, 4), ["dct2", "dct2"], 4
    Lt = synth.lowrank_tensor(dims, rank, kinds, seed=5, noise_std=1e-3)
    rng = np.random.default_rng(5)
    S = np.zeros(dims)
    if model == "rpca_tube":
        for _ in range(60):  # corrupted tubes
            S[rng.integers(dims[0]), rng.integers(dims[1]), :, :] = rng.uniform(-2, 2, dims[2:])
    else:
        for j in rng.choice(24, 3, replace=False):  # corrupted slices
            S[:, :, j % 6, j // 6] = rng.uniform(-1, 1, dims[:2])
    mask = synth.observation_mask(dims, 0.7, 5)
    M = np.where(mask, Lt + S, 0.0).astype(np.float64 if prec == "fp64" else np.float32).astype(np.float64)
    r, p, q, seed = 4, 4, 1, 31
    mu0 = 1.0 / synth.max_slice_norm(M, kinds)
    lam = 0.5 / np.sqrt(max(dims[0], dims[1]) * 24)
    phi, psi = ("mcp", (40.0,)), ("l1", ())
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision=prec, seed=seed)
    dt = plan.torch_dtype
    T = otr.build_transforms(dims, kinds)
    for n_iter in (1, 8):
        adm = ht.Admm(plan, model, phi=phi, psi=psi, lam=lam, mu0=mu0, vartheta=1.2, mu_max=1e10)
        dL, dE, dY = (torch.empty(plan.N, dtype=dt, device="cuda") for _ in range(3))
        ws = plan.alloc_workspace(admm=True)
        adm.init(dL, dE, dY, ws)
        adm.iterate(ht.to_device(M, dt), ht.to_device(mask.astype(np.uint8), torch.uint8), dL, dE, dY, n_iter, ws)
        torch.cuda.synchronize()
        rnd = lambda X, tau, t: otsvt.tsvt_randomized(
            X, tau, phi, T, r, p, q,
            otsvt.omegas(dims, kinds, r, p, seed=seed, call=t, round_to=None if prec == "fp64" else np.float32))
        Lr, Er, Yr, _ = osolver.admm(M, mask, model, phi, psi, lam, mu0, 1.2, 1e10, n_iter, rnd)
        # one iteration at the per-iteration tolerance; eight at ten times it (rounding of the
        # storage type feeds the next iteration's sketch input)
        tol = TOL[prec] * (1 if n_iter == 1 else 10)
        for name, g, ref in (("L", dL, Lr), ("E", dE, Er), ("Y", dY, Yr)):
            e = _rel(ht.from_device(g, dims), ref)
            assert e < tol, f"{model} {prec} {n_iter} iterations: {name} rel err {e:.3e}"
