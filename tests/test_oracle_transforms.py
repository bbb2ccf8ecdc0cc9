"""Pins of the oracle's transforms and t-product algebra (CPU only)."""
import itertools

import numpy as np
import pytest
import scipy.fft as sfft

from oracle import transforms as tr
from workloads import synth


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 8, 16, 32])
def test_dct2_matches_scipy(n):
    ref = sfft.dct(np.eye(n), type=2, norm="ortho", axis=0)
    assert np.allclose(tr.dct2_matrix(n), ref, atol=1e-14)
    C = tr.dct2_matrix(n)
    assert np.allclose(C @ C.T, np.eye(n), atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 16])
def test_dft_matches_numpy(n):
    ref = np.fft.fft(np.eye(n), axis=0) / np.sqrt(n)
    assert np.allclose(tr.dft_matrix(n), ref, atol=1e-14)


def test_mode_product_matches_loops():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((3, 4, 5, 2))
    U = rng.standard_normal((6, 5))
    Y = tr.mode_product(X, U, 2)
    assert Y.shape == (3, 4, 6, 2)
    ref = np.zeros_like(Y)
    for a, b, c, d in itertools.product(range(3), range(4), range(6), range(2)):
        ref[a, b, c, d] = sum(U[c, e] * X[a, b, e, d] for e in range(5))
    assert np.allclose(Y, ref, atol=1e-13)


@pytest.mark.parametrize("dims,kinds", [((5, 4, 6), ["dct2"]), ((3, 4, 4, 3), ["dft", "dft"]),
                                        ((4, 3, 2, 3, 4), ["dct2", "dft_unnormalized", "dft"])])
def test_forward_slice_matches_full_forward(dims, kinds):
    """One transformed slice from the Kronecker coefficients equals that slice
    of the mode-by-mode transform, for every slice index."""
    rng = np.random.default_rng(7)
    X = rng.standard_normal(dims)
    T = tr.build_transforms(dims, kinds)
    LX = tr.to_slices(tr.forward(X, T))
    for j in range(LX.shape[2]):
        assert np.allclose(tr.forward_slice(X, T, j), LX[:, :, j], atol=1e-13)


def test_forward_matches_scipy_per_axis():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((4, 3, 5, 6))
    T = tr.build_transforms(X.shape, ["dct2", "dft"])
    ref = sfft.fft(sfft.dct(X, type=2, norm="ortho", axis=2), norm="ortho", axis=3)
    assert np.allclose(tr.forward(X, T), ref, atol=1e-13)


@pytest.mark.parametrize("kinds", [["dct2"], ["dft"], ["dct2", "dft"], ["dft", "dft"],
                                   ["dft_unnormalized", "dct2"]])
def test_invertibility(kinds):
    rng = np.random.default_rng(2)
    dims = (5, 4) + tuple([4, 3][: len(kinds)])
    X = rng.standard_normal(dims)
    T = tr.build_transforms(dims, kinds)
    back = tr.inverse(tr.forward(X, T), T)
    assert np.abs(back - X).max() < 1e-13


def test_custom_nonunitary_alpha():
    rng = np.random.default_rng(3)
    Qm, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    U = np.sqrt(2.5) * Qm
    T = tr.build_transforms((3, 3, 4), [("custom", U)])
    assert abs(T[0][1] - 2.5) < 1e-13
    X = rng.standard_normal((3, 3, 4))
    assert np.abs(tr.inverse(tr.forward(X, T), T) - X).max() < 1e-13
    # ||L(X)||_F^2 = rho ||X||_F^2
    assert np.isclose(np.linalg.norm(tr.forward(X, T)) ** 2, 2.5 * np.linalg.norm(X) ** 2)


@pytest.mark.parametrize("kinds", [["dct2", "dct2"], ["dft", "dft"]])
def test_parseval_alpha_one(kinds):
    rng = np.random.default_rng(4)
    X = rng.standard_normal((6, 5, 4, 3))
    T = tr.build_transforms(X.shape, kinds)
    assert np.isclose(np.linalg.norm(tr.forward(X, T)), np.linalg.norm(X), rtol=1e-14)


def test_slice_index_formula():
    dims = (2, 3, 4, 5, 2)
    X = np.arange(np.prod(dims), dtype=float).reshape(dims)
    S = tr.to_slices(X)
    for i3, i4, i5 in itertools.product(range(4), range(5), range(2)):
        j1 = (i5 + 1 - 1) * 4 * 5 + (i4 + 1 - 1) * 4 + (i3 + 1)  # 1-based formula
        j = tr.slice_index((i3, i4, i5), dims)
        assert j == j1 - 1
        assert np.array_equal(S[:, :, j], X[:, :, i3, i4, i5])
    assert np.array_equal(tr.from_slices(S, dims), X)


def test_conjugate_partner_dft():
    rng = np.random.default_rng(5)
    dims = (3, 4, 4, 3)
    X = rng.standard_normal(dims)
    T = tr.build_transforms(dims, ["dft", "dft"])
    S = tr.to_slices(tr.forward(X, T))
    for j in range(12):
        p = tr.conjugate_partner(j, dims)
        assert np.allclose(S[:, :, p], np.conj(S[:, :, j]), atol=1e-13)
        assert tr.conjugate_partner(p, dims) == j


def test_tproduct_identities():
    rng = np.random.default_rng(6)
    tail = (4, 3)
    T = tr.build_transforms((1, 1) + tail, ["dct2", "dct2"])
    X = rng.standard_normal((3, 4) + tail)
    Y = rng.standard_normal((4, 2) + tail)
    Z = rng.standard_normal((2, 5) + tail)
    lhs = tr.t_product(tr.t_product(X, Y, T), Z, T)
    rhs = tr.t_product(X, tr.t_product(Y, Z, T), T)
    assert np.allclose(lhs, rhs, atol=1e-12)
    Ident = tr.t_identity(3, tail, T)
    assert np.allclose(tr.t_product(Ident, X, T), X, atol=1e-12)
    # (X * Y)^T = Y^T * X^T, and for a real orthogonal transform the t-transpose
    # is the plain transpose of every spatial face slice
    XY = tr.t_product(X, Y, T)
    assert np.allclose(tr.t_transpose(XY, T), tr.t_product(tr.t_transpose(Y, T), tr.t_transpose(X, T), T),
                       atol=1e-12)
    assert np.allclose(tr.t_transpose(X, T), np.swapaxes(X, 0, 1), atol=1e-13)


@pytest.mark.parametrize("kinds", [["dct2"], ["dft", "dft"]])
def test_tsvd_factorization(kinds):
    rng = np.random.default_rng(7)
    dims = (5, 4) + tuple([4, 3][: len(kinds)])
    T = tr.build_transforms(dims, kinds)
    X = rng.standard_normal(dims)
    U, S, V = tr.t_svd(X, T)
    rec = tr.t_product(tr.t_product(U, S, T), tr.t_transpose(V, T), T)
    assert np.allclose(rec, X, atol=1e-12)
    UtU = tr.t_product(tr.t_transpose(U, T), U, T)
    assert np.allclose(UtU, tr.t_identity(5, dims[2:], T), atol=1e-12)


@pytest.mark.parametrize("kinds,dims,rank", [(["dct2"], (12, 10, 6), 3),
                                             (["dct2", "dct2"], (9, 8, 4, 3), 2),
                                             (["dft", "dft"], (9, 8, 4, 3), 4)])
def test_synthetic_tensor_tubal_rank(kinds, dims, rank):
    X = synth.lowrank_tensor(dims, rank, kinds, seed=11)
    T = tr.build_transforms(dims, kinds)
    assert tr.tsvd_rank(X, T) == rank
    # the t-product of the same factors through the oracle gives the same tensor
    A = synth.rng(11, "factor_a").standard_normal((dims[0], rank) + dims[2:])
    B = synth.rng(11, "factor_b").standard_normal((rank, dims[1]) + dims[2:])
    assert np.allclose(tr.t_product(A, B, T).real, X, atol=1e-11)
