"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances (relative Frobenius norm of the whole output):
  FP64 path  1e-10
  FP32 path  1e-5
Inputs: seeded synthetic low-tubal-rank tensors (workloads.synth); the oracle
runs on exactly the values the GPU receives (rounded to the storage type) and
on the same sketch matrices (Philox draws rounded to the storage type).
"""
import numpy as np
import pytest

from oracle import philox, solver as osolver, transforms as otr, tsvt as otsvt
from workloads import synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}
PEN = {"l1": ("l1", ()), "mcp": ("mcp", (40.0,)), "scad": ("scad", (3.7, 6.0)), "log": ("log", (5.0,)),
       "capped_l1": ("capped_l1", (30.0,)), "firm": ("firm", (2.5,))}


@pytest.fixture(scope="module")
def ht():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2506_09594_amd import htsvt
    return htsvt


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _np_dtype(prec):
    return np.float64 if prec == "fp64" else np.float32


def _run_case(ht, dims, kinds, rank, r, p, q, prec, tau, pen, seed=1, noise=0.0, call=0):
    import torch
    X = synth.lowrank_tensor(dims, rank, kinds, seed=seed, noise_std=noise)
    Xs = X.astype(_np_dtype(prec)).astype(np.float64)
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision=prec, seed=1000 + seed)
    dX = ht.to_device(Xs, plan.torch_dtype)
    out = plan.gnhtsvt(dX, tau, PEN[pen], call_index=call)
    torch.cuda.synchronize()
    got = ht.from_device(out, dims)
    T = otr.build_transforms(dims, kinds)
    om = otsvt.omegas(dims, kinds, r, p, seed=1000 + seed, call=call,
                      round_to=_np_dtype(prec) if prec != "fp64" else None)
    ref = otsvt.tsvt_randomized(Xs, tau, PEN[pen], T, r, p, q, om)
    return got, ref, plan


def test_omega_matches_oracle_generator(ht):
    import torch
    dims = (37, 29, 3, 2)
    plan = ht.Plan(dims, ["dct2", "dct2"], r=7, p=4, q=1, precision="fp64", seed=0xDEADBEEF12345, stream_id=3)
    for call in (0, 5):
        dev = plan.omega_fp64(call).cpu().numpy()
        torch.cuda.synchronize()
        l = plan.width
        for j in range(plan.n_slices):
            ref = philox.omega(dims[1], l, j, call, 3, 0xDEADBEEF12345)
            got = dev[j * dims[1] * l:(j + 1) * dims[1] * l].reshape((dims[1], l), order="F")
            assert np.abs(got - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,kinds", [((60, 50, 20), ["dct2"]), ((33, 17, 5, 3), ["dct2", "dct2"]),
                                        ((20, 9, 4, 3, 2), ["dct2", "dct2", "dct2"]), ((70, 65, 33), ["dct2"]),
                                        # two modes of 16: 45 groups of 16 tube positions (a ragged last item
                                        # and a partly filled last workgroup), and an even count
                                        ((36, 20, 16, 16), ["dct2", "dct2"]), ((48, 40, 16, 16), ["dct2", "dct2"])])
def test_transform_matches_oracle(ht, prec, dims, kinds):
    import torch
    rng = np.random.default_rng(0)
    X = rng.standard_normal(dims).astype(_np_dtype(prec)).astype(np.float64)
    plan = ht.Plan(dims, kinds, r=2, p=1, q=0, precision=prec)
    dX = ht.to_device(X, plan.torch_dtype)
    fwd = plan.transform(dX)
    back = plan.transform(fwd, inverse=True)
    torch.cuda.synchronize()
    T = otr.build_transforms(dims, kinds)
    assert _rel(ht.from_device(fwd, dims), otr.forward(X, T)) < (1e-14 if prec == "fp64" else 1e-6)
    assert _rel(ht.from_device(back, dims), X) < (1e-14 if prec == "fp64" else 1e-6)


def test_custom_transform_nonunitary(ht):
    import torch
    rng = np.random.default_rng(1)
    Qm, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    U = 1.7 * Qm
    dims = (12, 10, 6)
    X = rng.standard_normal(dims)
    plan = ht.Plan(dims, ["custom"], r=3, p=2, q=1, precision="fp64", custom=[U])
    fwd = plan.transform(ht.to_device(X, plan.torch_dtype))
    torch.cuda.synchronize()
    T = otr.build_transforms(dims, [("custom", U)])
    assert _rel(ht.from_device(fwd, dims), otr.forward(X, T)) < 1e-14


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_custom_transform_two_modes_of_16(ht, prec):
    """Different non-symmetric matrices with U U^T = alpha I (alpha 2.89 and 0.36) on
    modes 3 and 4 (length 16): a transposed or swapped mode matrix, or a wrong
    inverse, fails."""
    import torch
    rng = np.random.default_rng(5)
    U3 = 1.7 * np.linalg.qr(rng.standard_normal((16, 16)))[0]
    U4 = 0.6 * np.linalg.qr(rng.standard_normal((16, 16)))[0]
    dims = (32, 24, 16, 16)
    X = rng.standard_normal(dims).astype(_np_dtype(prec)).astype(np.float64)
    plan = ht.Plan(dims, ["custom", "custom"], r=3, p=2, q=1, precision=prec, custom=[U3, U4])
    dX = ht.to_device(X, plan.torch_dtype)
    fwd = plan.transform(dX)
    back = plan.transform(fwd, inverse=True)
    torch.cuda.synchronize()
    T = otr.build_transforms(dims, [("custom", U3), ("custom", U4)])
    tol = 1e-13 if prec == "fp64" else 2e-6
    assert _rel(ht.from_device(fwd, dims), otr.forward(X, T)) < tol
    assert _rel(ht.from_device(back, dims), X) < tol


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tsvt_repeated_singular_values(ht, prec):
    """Transformed slices with clusters of equal singular values (6 x 8, 6 x 5, 4 x 2):
    inside a cluster the singular vectors are arbitrary, so the rotations the
    small SVD skips (threshold 1e-10 relative for FP32 output, 1e-15 for FP64) must
    leave K' = U diag(w) U^T unchanged; the shrink weights differ between clusters
    (MCP) and the last cluster falls below tau."""
    import torch
    dims, kinds = (96, 80, 4, 4), ["dct2", "dct2"]
    n1, n2, P = dims[0], dims[1], 16
    g = np.random.default_rng(21)
    sv = np.array([8.0] * 6 + [5.0] * 6 + [2.0] * 4)
    S = np.zeros((n1, n2, P))
    for j in range(P):
        U = np.linalg.qr(g.standard_normal((n1, sv.size)))[0]
        V = np.linalg.qr(g.standard_normal((n2, sv.size)))[0]
        S[:, :, j] = (U * sv) @ V.T
    T = otr.build_transforms(dims, kinds)
    X = otr.inverse(S.reshape(dims, order="F"), T)
    Xs = X.astype(_np_dtype(prec)).astype(np.float64)
    r, p, q, tau, seed = 16, 8, 2, 3.0, 4
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision=prec, seed=seed)
    out = plan.gnhtsvt(ht.to_device(Xs, plan.torch_dtype), tau, PEN["mcp"])
    torch.cuda.synchronize()
    om = otsvt.omegas(dims, kinds, r, p, seed=seed, round_to=_np_dtype(prec) if prec != "fp64" else None)
    ref = otsvt.tsvt_randomized(Xs, tau, PEN["mcp"], T, r, p, q, om)
    assert _rel(ht.from_device(out, dims), ref) < TOL[prec]


@pytest.mark.parametrize("pen", list(PEN))
def test_tsvt_fp64_config_small(ht, pen):
    """60x50x20 under DCT on mode 3, tubal rank 5 plus noise std 1e-3, r=5 p=5 q=1."""
    got, ref, _ = _run_case(ht, (60, 50, 20), ["dct2"], 5, 5, 5, 1, "fp64", tau=20.0, pen=pen, noise=1e-3)
    assert _rel(got, ref) < TOL["fp64"]


@pytest.mark.parametrize("q", [0, 1, 2])
def test_tsvt_fp64_exact_rank_deflation(ht, q):
    """Noise-free rank 5 with l = 10: the sketch is rank deficient and must deflate."""
    got, ref, _ = _run_case(ht, (60, 50, 20), ["dct2"], 5, 5, 5, q, "fp64", tau=5.0, pen="mcp")
    assert _rel(got, ref) < TOL["fp64"]
    T = otr.build_transforms((60, 50, 20), ["dct2"])
    X = synth.lowrank_tensor((60, 50, 20), 5, ["dct2"], seed=1)
    assert _rel(got, otsvt.gnhtsvt_exact(X, 5.0, PEN["mcp"], T)) < 1e-10


@pytest.mark.parametrize("pen", ["l1", "mcp", "scad"])
@pytest.mark.parametrize("dims,kinds,rank,r,p,q", [
    ((96, 80, 4, 4), ["dct2", "dct2"], 8, 8, 6, 2),
    ((130, 70, 3, 2, 2), ["dct2"] * 3, 6, 6, 10, 1),
    ((64, 200, 5), ["dct2"], 12, 12, 8, 2),
])
def test_tsvt_fp32(ht, pen, dims, kinds, rank, r, p, q):
    got, ref, _ = _run_case(ht, dims, kinds, rank, r, p, q, "fp32", tau=8.0, pen=pen)
    assert _rel(got, ref) < TOL["fp32"]


@pytest.mark.parametrize("dims,kinds,rank,r,p,q", [
    ((132, 100, 3, 2), ["dct2", "dct2"], 30, 30, 20, 1),   # l = 50: two 32-column blocks
    ((200, 160, 2, 2), ["dct2", "dct2"], 50, 60, 10, 2),   # l = 70: three 32-column blocks
    ((260, 36, 3), ["dct2"], 10, 10, 6, 2),                # tall, short rows of A^T
    ((36, 300, 3), ["dct2"], 10, 12, 4, 1),                # wide
])
def test_tsvt_fp32_matrix_core_shapes(ht, dims, kinds, rank, r, p, q):
    got, ref, _ = _run_case(ht, dims, kinds, rank, r, p, q, "fp32", tau=5.0, pen="mcp")
    assert _rel(got, ref) < TOL["fp32"]


@pytest.mark.parametrize("dims,kinds,rank,r,p,q", [
    ((260, 300, 3, 2), ["dct2", "dct2"], 10, 10, 6, 2),   # streaming nn: a 256-row tile and a 4-row one, l = 16
    ((448, 96, 5), ["dct2"], 30, 30, 10, 1),               # streaming nn: l = 40 (two column blocks), short reduction
    ((256, 256, 4), ["dct2"], 20, 20, 10, 2),              # streaming nn at the headline slice size
])
def test_tsvt_fp32_streaming_product(ht, dims, kinds, rank, r, p, q):
    """Slices of at least 192 rows take the streaming nn product (A read straight
    into the matrix-core operands, Gram partials per 64 rows)."""
    got, ref, _ = _run_case(ht, dims, kinds, rank, r, p, q, "fp32", tau=6.0, pen="mcp", noise=1e-2)
    assert _rel(got, ref) < TOL["fp32"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("r,p", [(8, 5), (6, 1), (20, 3)])
def test_tsvt_odd_widths(ht, prec, r, p):
    """Odd sketch widths l = r + p run the Jacobi sweeps with a zero padding row
    and column for the idle player of the round-robin schedule."""
    got, ref, plan = _run_case(ht, (70, 64, 6), ["dct2"], r, r, p, 1, prec, tau=4.0, pen="scad", noise=1e-2)
    assert plan.width % 2 == 1
    assert _rel(got, ref) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,kinds,rank,r,p,q", [
    ((40, 30), [], 3, 3, 2, 1),              # order 2: one slice, no transform
    ((9, 7, 3), ["dct2"], 2, 5, 10, 1),      # l clamped to min(n1, n2) = 7
    ((5, 80, 2, 2), ["dct2", "dct2"], 2, 2, 2, 1),  # n1 < l_requested
    ((1, 6, 4), ["dct2"], 1, 1, 2, 0),       # n1 = 1
    ((257, 129, 3), ["dct2"], 4, 4, 4, 2),   # ragged tiles in every kernel
])
def test_tsvt_edge_shapes(ht, prec, dims, kinds, rank, r, p, q):
    got, ref, _ = _run_case(ht, dims, kinds, rank, r, p, q, prec, tau=1.0, pen="l1")
    assert _rel(got, ref) < TOL[prec]


def test_tsvt_tau_zero_identity_on_low_rank(ht):
    got, ref, _ = _run_case(ht, (48, 40, 6), ["dct2"], 4, 4, 4, 1, "fp64", tau=0.0, pen="l1")
    X = synth.lowrank_tensor((48, 40, 6), 4, ["dct2"], seed=1)
    assert _rel(got, X) < 1e-12
    assert _rel(got, ref) < 1e-12


def test_intermediates_q_orthonormal_and_stats(ht):
    import torch
    dims, kinds = (96, 80, 4, 4), ["dct2", "dct2"]
    X = synth.lowrank_tensor(dims, 8, kinds, seed=2)
    plan = ht.Plan(dims, kinds, r=8, p=6, q=2, precision="fp32", seed=5)
    ws = plan.alloc_workspace()
    out, sig, kept = plan.gnhtsvt(ht.to_device(X, plan.torch_dtype), 8.0, PEN["l1"], workspace=ws, stats=True)
    torch.cuda.synchronize()
    l, P = plan.width, plan.n_slices
    Q = plan.region(ws, "Q")[: P * dims[0] * l].double().cpu().numpy()
    T = otr.build_transforms(dims, kinds)
    LX = otr.to_slices(otr.forward(X.astype(np.float32).astype(np.float64), T))
    A = plan.region(ws, "A")[: plan.N].double().cpu().numpy().reshape((dims[0], dims[1], P), order="F")
    assert _rel(A, LX) < 1e-6
    sig = sig.cpu().numpy()
    for j in range(P):
        Qj = Q[j * dims[0] * l:(j + 1) * dims[0] * l].reshape((dims[0], l), order="F")
        nz = np.linalg.norm(Qj, axis=0) > 0.5
        assert nz.sum() >= 8  # rank-8 slices keep at least 8 directions
        G = Qj[:, nz].T @ Qj[:, nz]
        assert np.abs(G - np.eye(nz.sum())).max() < 1e-5
        s_true = np.linalg.svd(LX[:, :, j], compute_uv=False)[:8]
        assert np.allclose(sig[j, :8], s_true, rtol=1e-5)
    assert np.all(kept.cpu().numpy() <= 8)


def test_tsvt_full_size_fp32_config(ht):
    """256x256x16x16, rank 20 under DCT on modes 3 and 4, r=20 p=10 q=2: every slice."""
    got, ref, plan = _run_case(ht, (256, 256, 16, 16), ["dct2", "dct2"], 20, 20, 10, 2, "fp32", tau=50.0,
                               pen="mcp", seed=2)
    assert _rel(got, ref) < TOL["fp32"]


def test_call_index_changes_draw_but_not_low_rank_result(ht):
    dims, kinds = (60, 50, 20), ["dct2"]
    a, ref, _ = _run_case(ht, dims, kinds, 5, 5, 5, 1, "fp64", tau=3.0, pen="l1", noise=1e-3, call=0)
    b, refb, _ = _run_case(ht, dims, kinds, 5, 5, 5, 1, "fp64", tau=3.0, pen="l1", noise=1e-3, call=7)
    assert _rel(b, refb) < TOL["fp64"]
    assert 0 < _rel(a, b) < 1e-4  # different sketches, same dominant subspace


def test_deterministic_repeat(ht):
    import torch
    dims, kinds = (96, 80, 4, 4), ["dct2", "dct2"]
    X = synth.lowrank_tensor(dims, 8, kinds, seed=3)
    plan = ht.Plan(dims, kinds, r=8, p=6, q=2, precision="fp32", seed=9)
    dX = ht.to_device(X, plan.torch_dtype)
    o1 = plan.gnhtsvt(dX, 4.0, PEN["scad"]).clone()
    o2 = plan.gnhtsvt(dX, 4.0, PEN["scad"])
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)


@pytest.mark.parametrize("prec,model", [("fp64", "completion"), ("fp64", "rpca"), ("fp32", "completion")])
def test_admm_matches_oracle(ht, prec, model):
    import torch
    dims, kinds, rank = (60, 50, 20), ["dct2"], 5
    L = synth.lowrank_tensor(dims, rank, kinds, seed=4, noise_std=1e-3)
    mask = synth.observation_mask(dims, 0.3 if model == "completion" else 0.5, 4)
    S = synth.outliers(dims, 0.05, 4) * 3.0 if model == "rpca" else 0.0
    M = np.where(mask, L + S, 0.0).astype(_np_dtype(prec)).astype(np.float64)
    r, p, q, seed = 5, 5, 1, 77
    mu0 = 1.0 / synth.max_slice_norm(M, kinds)
    lam = 2.0 / np.sqrt(max(dims[0], dims[1]) * dims[2])
    vartheta, mu_max, n_iter = 1.2, 1e10, 12
    pen = PEN["mcp"] if model == "completion" else PEN["l1"]
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision=prec, seed=seed)
    adm = ht.Admm(plan, model, phi=pen, psi=PEN["l1"], lam=lam, mu0=mu0, vartheta=vartheta, mu_max=mu_max)
    dt = plan.torch_dtype
    dM, dmask = ht.to_device(M, dt), ht.to_device(mask.astype(np.uint8), torch.uint8)
    dL, dE, dY = (torch.empty(plan.N, dtype=dt, device="cuda") for _ in range(3))
    ws = plan.alloc_workspace(admm=True)
    adm.init(dL, dE, dY, ws)
    adm.iterate(dM, dmask, dL, dE, dY, n_iter, ws)
    st = adm.stats(ws)
    T = otr.build_transforms(dims, kinds)
    rnd = lambda X, tau, t: otsvt.tsvt_randomized(
        X, tau, pen, T, r, p, q,
        otsvt.omegas(dims, kinds, r, p, seed=seed, call=t, round_to=_np_dtype(prec) if prec != "fp64" else None))
    Lr, Er, Yr, hist = osolver.admm(M, mask, model, pen, PEN["l1"], lam, mu0, vartheta, mu_max, n_iter, rnd)
    tol = 1e-9 if prec == "fp64" else 1e-4
    assert _rel(ht.from_device(dL, dims), Lr) < tol
    assert _rel(ht.from_device(dE, dims), Er) < tol
    assert _rel(ht.from_device(dY, dims), Yr) < tol
    assert st["iteration"] == n_iter
    assert st["mu"] == pytest.approx(min(mu_max, mu0 * vartheta ** n_iter), rel=1e-12)
    assert st["resid"] == pytest.approx(hist[-1]["resid"], rel=1e-6 if prec == "fp64" else 1e-2)


@pytest.mark.parametrize("model", ["completion", "rpca"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_admm_one_iteration_matches_oracle(ht, prec, model):
    """One recovery iteration (t-SVT of the current input, then the E / Y / mu
    updates of Sec. V) at the per-operator bounds: 1e-10 (FP64), 1e-5 (FP32)."""
    import torch
    dims, kinds, rank = (60, 50, 20), ["dct2"], 5
    L = synth.lowrank_tensor(dims, rank, kinds, seed=6, noise_std=1e-3)
    mask = synth.observation_mask(dims, 0.3 if model == "completion" else 0.5, 6)
    S = synth.outliers(dims, 0.05, 6) * 3.0 if model == "rpca" else 0.0
    M = np.where(mask, L + S, 0.0).astype(_np_dtype(prec)).astype(np.float64)
    r, p, q, seed = 5, 5, 1, 31
    # tau = 1 / mu0 = a quarter of the largest transformed-slice norm: the first
    # t-SVT keeps part of the spectrum (at 1 / max norm it would zero all of L)
    mu0 = 4.0 / synth.max_slice_norm(M, kinds)
    lam = 2.0 / np.sqrt(max(dims[0], dims[1]) * dims[2])
    vartheta, mu_max = 1.2, 1e10
    pen = PEN["mcp"] if model == "completion" else PEN["l1"]
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision=prec, seed=seed)
    adm = ht.Admm(plan, model, phi=pen, psi=PEN["l1"], lam=lam, mu0=mu0, vartheta=vartheta, mu_max=mu_max)
    dt = plan.torch_dtype
    dM, dmask = ht.to_device(M, dt), ht.to_device(mask.astype(np.uint8), torch.uint8)
    dL, dE, dY = (torch.empty(plan.N, dtype=dt, device="cuda") for _ in range(3))
    ws = plan.alloc_workspace(admm=True)
    adm.init(dL, dE, dY, ws)
    adm.iterate(dM, dmask, dL, dE, dY, 1, ws)
    T = otr.build_transforms(dims, kinds)
    rnd = lambda X, tau, t: otsvt.tsvt_randomized(
        X, tau, pen, T, r, p, q,
        otsvt.omegas(dims, kinds, r, p, seed=seed, call=t, round_to=_np_dtype(prec) if prec != "fp64" else None))
    Lr, Er, Yr, _ = osolver.admm(M, mask, model, pen, PEN["l1"], lam, mu0, vartheta, mu_max, 1, rnd)
    tol = TOL[prec]
    assert _rel(ht.from_device(dL, dims), Lr) < tol
    assert _rel(ht.from_device(dE, dims), Er) < tol
    assert _rel(ht.from_device(dY, dims), Yr) < tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tsvt_wide_sketch_with_deflation(ht, prec):
    """Sketch width 70 (> 64: the factor-once orthonormalization path) on
    rank-5 slices, so most sketch columns deflate; and a full-rank case."""
    for rank, tau in ((5, 1.0), (80, 20.0)):
        got, ref, _ = _run_case(ht, (100, 90, 3), ["dct2"], rank, 60, 10, 2, prec, tau=tau, pen="l1")
        assert _rel(got, ref) < TOL[prec], f"rank {rank}"
