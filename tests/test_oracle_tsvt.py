"""Pins of the oracle's GNHTSVT, exact and randomized (CPU only)."""
import numpy as np
import pytest

from oracle import philox, transforms as tr, tsvt
from workloads import synth

PENALTIES = [("l1", ()), ("mcp", (4.0,)), ("scad", (3.7, 1.5)), ("log", (1.0,)), ("capped_l1", (2.0,))]


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


@pytest.mark.parametrize("kinds", [["dct2"], ["dft", "dft"]])
def test_l1_subgradient_condition(kinds):
    """Convex case: A - G in tau * subdifferential of the nuclear norm, slice-wise."""
    rng = np.random.default_rng(0)
    dims = (6, 5) + tuple([4, 3][: len(kinds)])
    T = tr.build_transforms(dims, kinds)
    A = rng.standard_normal(dims)
    tau = 0.8
    G = tsvt.gnhtsvt_exact(A, tau, ("l1", ()), T)
    LA, LG = tr.to_slices(tr.forward(A, T)), tr.to_slices(tr.forward(G, T))
    for j in range(LA.shape[2]):
        u, s, vh = np.linalg.svd(LG[:, :, j], full_matrices=False)
        k = int(np.sum(s > 1e-10))
        Uk, Vk = u[:, :k], vh[:k, :].conj().T
        W = (LA[:, :, j] - LG[:, :, j]) / tau - Uk @ Vk.conj().T
        assert np.linalg.norm(W, 2) <= 1 + 1e-10
        assert np.abs(Uk.conj().T @ W).max() < 1e-10
        assert np.abs(W @ Vk).max() < 1e-10


@pytest.mark.parametrize("penalty", PENALTIES)
@pytest.mark.parametrize("kinds", [["dct2"], [("dft_unnormalized")]])
def test_theorem_optimality_against_perturbations(penalty, kinds):
    """Thm. 4.1: D_{Phi,tau}(A) attains the lowest objective among nearby points."""
    rng = np.random.default_rng(1)
    dims = (4, 3, 4)
    T = tr.build_transforms(dims, kinds)
    A = 2.0 * rng.standard_normal(dims)
    tau = 1.1
    G = tsvt.gnhtsvt_exact(A, tau, penalty, T)
    f0 = tsvt.objective(G, A, tau, penalty, T)
    for scale in (1e-3, 1e-2, 1e-1, 1.0):
        for _ in range(250):
            f = tsvt.objective(G + scale * rng.standard_normal(dims), A, tau, penalty, T)
            assert f0 <= f + 1e-10
    # and against the trivial candidates 0 and A
    assert f0 <= tsvt.objective(np.zeros(dims), A, tau, penalty, T) + 1e-12
    assert f0 <= tsvt.objective(A, A, tau, penalty, T) + 1e-12


@pytest.mark.parametrize("kinds,dims", [(["dct2"], (14, 11, 6)), (["dct2", "dct2"], (12, 10, 3, 4)),
                                         (["dft", "dft"], (12, 10, 4, 3)), (["dft"], (10, 9, 5))])
@pytest.mark.parametrize("penalty", PENALTIES)
@pytest.mark.parametrize("q", [0, 1, 2])
def test_randomized_exact_for_low_rank(kinds, dims, penalty, q):
    """rank(L(A)^<j>) <= k  =>  the sketch captures the range exactly."""
    rank, r, p = 3, 4, 3
    X = synth.lowrank_tensor(dims, rank, kinds, seed=3)
    T = tr.build_transforms(dims, kinds)
    om = tsvt.omegas(dims, kinds, r, p, seed=17, call=0)
    tau = 2.0
    got = tsvt.tsvt_randomized(X, tau, penalty, T, r, p, q, om)
    ref = tsvt.gnhtsvt_exact(X, tau, penalty, T)
    assert _rel(got, ref) < 1e-10


def test_randomized_full_width_is_exact():
    """l = min(n1, n2) and k = l: randomized equals the exact operator on any input."""
    rng = np.random.default_rng(4)
    dims = (9, 6, 5)
    T = tr.build_transforms(dims, ["dct2"])
    X = rng.standard_normal(dims)
    om = tsvt.omegas(dims, ["dct2"], 6, 0, seed=5)
    for penalty in PENALTIES:
        got = tsvt.tsvt_randomized(X, 0.9, penalty, T, 6, 0, 1, om)
        assert _rel(got, tsvt.gnhtsvt_exact(X, 0.9, penalty, T)) < 1e-12


def test_tau_zero_returns_input_for_rank_le_r():
    dims = (20, 16, 4, 2)
    X = synth.lowrank_tensor(dims, 5, ["dct2", "dct2"], seed=8)
    T = tr.build_transforms(dims, ["dct2", "dct2"])
    om = tsvt.omegas(dims, ["dct2", "dct2"], 5, 5, seed=9)
    assert _rel(tsvt.tsvt_randomized(X, 0.0, ("l1", ()), T, 5, 5, 1, om), X) < 1e-12


def test_q_orthonormal_and_energy_identity():
    rng = np.random.default_rng(10)
    for n1, n2, l, q in [(50, 40, 10, 0), (64, 64, 20, 2), (30, 70, 12, 1)]:
        A = rng.standard_normal((n1, n2)) @ np.diag(np.linspace(1, 0.01, n2))
        Om = philox.omega(n2, l, 0, 0, 0, 123)
        Q, B = tsvt.sketch_slice(A, Om, q)
        assert np.linalg.norm(Q.T @ Q - np.eye(l), 2) <= 10 * l * np.finfo(float).eps
        lhs = np.linalg.norm(A - Q @ (Q.T @ A)) ** 2
        rhs = np.linalg.norm(A) ** 2 - np.linalg.norm(B) ** 2
        assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(A) ** 2


def test_halko_martinsson_tropp_expected_error_bound():
    """E||A - QQ^T A||_F <= sqrt(1 + k/(p-1)) * (sum_{j>k} s_j^2)^(1/2)  (q = 0)."""
    rng = np.random.default_rng(11)
    n1, n2, k, p = 80, 60, 8, 4
    s = 1.0 / (1.0 + np.arange(n2)) ** 1.0
    U, _ = np.linalg.qr(rng.standard_normal((n1, n2)))
    V, _ = np.linalg.qr(rng.standard_normal((n2, n2)))
    A = (U * s) @ V.T
    bound = np.sqrt(1 + k / (p - 1)) * np.sqrt(np.sum(s[k:] ** 2))
    errs = []
    for seed in range(200):
        Q, _B = tsvt.sketch_slice(A, philox.omega(n2, k + p, 0, 0, 0, seed), 0)
        errs.append(np.linalg.norm(A - Q @ (Q.T @ A)))
    assert np.mean(errs) <= bound
    # power iterations only improve the captured subspace (on average)
    errs_q = [np.linalg.norm(A - (lambda Q: Q @ (Q.T @ A))(tsvt.sketch_slice(
        A, philox.omega(n2, k + p, 0, 0, 0, seed), 2)[0])) for seed in range(50)]
    assert np.mean(errs_q) < np.mean(errs)
    assert np.mean(errs_q) >= np.sqrt(np.sum(s[k + p:] ** 2)) - 1e-12  # optimal rank-l error


def test_randomized_stats_and_truncation():
    """k = min(r, l) values are shrunk; values beyond k are dropped (truncate, then prox)."""
    rng = np.random.default_rng(12)
    dims = (12, 10, 3)
    T = tr.build_transforms(dims, ["dct2"])
    X = rng.standard_normal(dims)
    om = tsvt.omegas(dims, ["dct2"], 3, 7, seed=1)
    st = {}
    got = tsvt.tsvt_randomized(X, 0.0, ("l1", ()), T, 3, 7, 0, om, stats=st)
    assert st["k"] == 3 and st["sigma"].shape == (3, 10)
    # with tau = 0 and l = n2 the output is the best rank-3 approximation per slice
    LX = tr.to_slices(tr.forward(X, T))
    ref = np.zeros_like(LX)
    for j in range(3):
        u, s, vh = np.linalg.svd(LX[:, :, j], full_matrices=False)
        ref[:, :, j] = (u[:, :3] * s[:3]) @ vh[:3]
    assert _rel(got, tr.inverse(tr.from_slices(ref, dims), T)) < 1e-12
    assert np.all(st["kept"] == 3)


def test_per_slice_widths_reduce_to_the_fixed_method():
    """With every slice at the plan's width and kept count, the per-slice-width
    routine is the fixed-width routine; with a full-width sketch of an exactly
    low-rank slice the result does not depend on the width either."""
    dims, kinds = (20, 16, 6), ["dct2"]
    X = synth.lowrank_tensor(dims, 3, kinds, seed=5)
    T = tr.build_transforms(dims, kinds)
    om = tsvt.omegas(dims, kinds, 6, 4, seed=1, call=0)
    a = tsvt.tsvt_randomized(X, 0.5, ("l1", ()), T, 6, 4, 1, om)
    b = tsvt.tsvt_randomized_widths(X, 0.5, ("l1", ()), T, [10] * 6, [6] * 6, 1, om)
    assert np.array_equal(a, b)
    # rank-3 slices: any width >= 3 with k >= 3 reproduces the exact operator
    c = tsvt.tsvt_randomized_widths(X, 0.5, ("l1", ()), T, [3, 4, 5, 6, 8, 10], [3, 3, 4, 5, 6, 6], 1, om)
    ex = tsvt.gnhtsvt_exact(X, 0.5, ("l1", ()), T)
    assert np.linalg.norm(c - ex) <= 1e-10 * np.linalg.norm(ex)
