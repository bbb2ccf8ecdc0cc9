"""Pins of the oracle's pure-L ADMM solver (CPU only)."""
import numpy as np
import pytest

from oracle import solver, transforms as tr, tsvt
from workloads import synth


def _problem(dims, rank, kinds, sr, seed, outlier_frac=0.0):
    L = synth.lowrank_tensor(dims, rank, kinds, seed=seed)
    mask = synth.observation_mask(dims, sr, seed)
    S = synth.outliers(dims, outlier_frac, seed) if outlier_frac else np.zeros(dims)
    M = np.where(mask, L + S, 0.0)
    return L, S, mask, M


def test_mask_and_outlier_counts():
    dims = (7, 6, 5)
    assert synth.observation_mask(dims, 0.3, 1).sum() == round(0.3 * 210)
    S = synth.outliers(dims, 0.1, 1)
    assert np.count_nonzero(S) == 21 and np.abs(S).max() <= 1.0


@pytest.mark.parametrize("penalty", [("l1", ()), ("mcp", (50.0,))])
def test_completion_recovers_low_rank(penalty):
    dims, kinds = (24, 20, 6), ["dct2"]
    L, _S, mask, M = _problem(dims, 2, kinds, 0.6, seed=2)
    T = tr.build_transforms(dims, kinds)
    mu0 = 1.0 / synth.max_slice_norm(M, kinds)
    fn = lambda X, tau, t: tsvt.gnhtsvt_exact(X, tau, penalty, T)
    Lh, E, Y, hist = solver.admm(M, mask, "completion", penalty, None, 0.0, mu0, 1.2, 1e10, 80, fn)
    assert solver.rse(Lh, L) < 1e-4
    # Thm. 4.2 behaviour: constraint residual and successive differences decay
    assert hist[-1]["resid"] < 1e-4 * hist[0]["resid"]
    assert hist[-1]["dL"] < 1e-3 * hist[1]["dL"]
    # completion: E vanishes on Omega and L matches the data there
    assert np.all(E[mask] == 0.0)
    assert np.abs((Lh - M)[mask]).max() < 1e-4 * np.abs(M).max()
    # the multiplier lives on Omega only
    assert np.all(Y[~mask] == 0.0)


def test_completion_randomized_matches_exact_on_low_rank():
    dims, kinds = (20, 18, 4, 2), ["dct2", "dct2"]
    L, _S, mask, M = _problem(dims, 2, kinds, 0.7, seed=3)
    T = tr.build_transforms(dims, kinds)
    mu0 = 1.0 / synth.max_slice_norm(M, kinds)
    pen = ("l1", ())
    ex = lambda X, tau, t: tsvt.gnhtsvt_exact(X, tau, pen, T)
    rnd = lambda X, tau, t: tsvt.tsvt_randomized(X, tau, pen, T, 2, 4, 1,
                                                 tsvt.omegas(dims, kinds, 2, 4, seed=5, call=t))
    Le = solver.admm(M, mask, "completion", pen, None, 0.0, mu0, 1.2, 1e10, 40, ex)[0]
    Lr = solver.admm(M, mask, "completion", pen, None, 0.0, mu0, 1.2, 1e10, 40, rnd)[0]
    assert solver.rse(Lr, L) < 1e-3
    assert solver.rse(Le, L) < 1e-3


def test_rpca_separates_outliers():
    dims, kinds = (20, 16, 4), ["dct2"]
    L, S, mask, M = _problem(dims, 2, kinds, 0.8, seed=4, outlier_frac=0.05)
    S = S * 5.0
    M = np.where(mask, L + S, 0.0)
    T = tr.build_transforms(dims, kinds)
    mu0 = 1.0 / synth.max_slice_norm(M, kinds)
    # lambda = xi / sqrt(max(n1, n2) * n3 ... nd), xi from the paper's tuning grid
    lam = 4.0 / np.sqrt(max(dims[0], dims[1]) * dims[2])
    fn = lambda X, tau, t: tsvt.gnhtsvt_exact(X, tau, ("l1", ()), T)
    Lh, E, _Y, hist = solver.admm(M, mask, "rpca", ("l1", ()), ("l1", ()), lam, mu0, 1.1, 1e10, 80, fn)
    naive = solver.rse(M, L)
    assert solver.rse(Lh, L) < 1e-4 * naive
    # the outliers land in E on Omega
    assert np.abs(E[mask] - S[mask]).max() < 1e-3
    assert hist[-1]["resid"] < 1e-3 * hist[0]["resid"]
