"""Transforms along modes 3..d, face slices, t-product and T-SVD (Sec. II).

Tensors are numpy arrays indexed (i1, i2, i3, ..., id) with 0-based indices.
Memory order is irrelevant here; at the library boundary the tensor is stored in
Fortran order (i1 fastest), which makes every face slice a contiguous
column-major n1 x n2 block.

Definitions followed:
  * face slice X^<j> = X(:, :, i3, ..., id) with j = i3 + n3*(i4 + n4*(...))
    (0-based form of the slice index of Sec. II);
  * mode-k product: (X x_k U)_(k) = U X_(k) (Kolda-Bader unfolding convention);
  * L(X) = X x_3 U_3 x_4 ... x_d U_d with U U^H = U^H U = alpha I, and
    L^{-1}(X) = X x_d U_d^{-1} ... x_3 U_3^{-1}  (eq. for L and its inverse);
  * t-product C = L^{-1}(L(X) face-wise-times L(Y))  (Def. of the T-product);
  * T-SVD X = U * S * V^T, T-SVD rank = number of nonzero tubes S(i,i,:,...,:)
    (Def. of the T-SVD factorization and rank).

Pins: invertibility, Parseval for alpha = 1, DCT/DFT matrices against scipy/numpy
FFT routines, the mode product against explicit loops, the slice index against
its formula, and the t-product identities (tests/test_oracle_transforms.py).
"""
import numpy as np


# ----------------------------------------------------------------------------
# transform matrices
# ----------------------------------------------------------------------------

def dct2_matrix(n):
    """Orthonormal DCT-II: C[k, m] = sqrt(2/n) c_k cos(pi (2m+1) k / (2n)), c_0 = 1/sqrt 2."""
    k = np.arange(n)[:, None].astype(np.float64)
    m = np.arange(n)[None, :].astype(np.float64)
    c = np.cos(np.pi * (2.0 * m + 1.0) * k / (2.0 * n)) * np.sqrt(2.0 / n)
    c[0, :] *= 1.0 / np.sqrt(2.0)
    return c


def dft_matrix(n):
    """Unitary DFT: F[k, m] = exp(-2 pi i k m / n) / sqrt(n)."""
    k = np.arange(n)[:, None].astype(np.float64)
    m = np.arange(n)[None, :].astype(np.float64)
    return np.exp(-2j * np.pi * k * m / n) / np.sqrt(n)


def transform_matrix(kind, n, custom=None, alpha=None):
    """Return (U, alpha) for one mode.

    kind: "dct2" (alpha = 1), "dft" (unitary, alpha = 1), "dft_unnormalized"
    (alpha = n, the plain FFT matrix), or "custom" (U given; alpha checked or
    derived from U U^H = alpha I).
    """
    if kind == "dct2":
        return dct2_matrix(n), 1.0
    if kind == "dft":
        return dft_matrix(n), 1.0
    if kind == "dft_unnormalized":
        return dft_matrix(n) * np.sqrt(n), float(n)
    if kind == "custom":
        U = np.asarray(custom)
        a = float(np.real(np.trace(U @ U.conj().T)) / n) if alpha is None else float(alpha)
        return U, a
    raise ValueError(f"unknown transform kind {kind!r}")


def build_transforms(dims, kinds):
    """List of (U_k, alpha_k) for modes 3..d.  kinds: one entry per mode 3..d."""
    if len(kinds) != len(dims) - 2:
        raise ValueError("need one transform per mode 3..d")
    out = []
    for n, kind in zip(dims[2:], kinds):
        if isinstance(kind, tuple):
            out.append(transform_matrix(kind[0], n, *kind[1:]))
        else:
            out.append(transform_matrix(kind, n))
    return out


# ----------------------------------------------------------------------------
# mode products and the transform pair
# ----------------------------------------------------------------------------

def mode_product(X, U, axis):
    """X x_k U along the given 0-based axis: Y[..., a, ...] = sum_b U[a, b] X[..., b, ...]."""
    Y = np.tensordot(U, X, axes=([1], [axis]))
    return np.moveaxis(Y, 0, axis)


def forward(X, transforms):
    """L(X) = X x_3 U_3 x_4 U_4 ... x_d U_d."""
    Y = X
    for k, (U, _a) in enumerate(transforms):
        Y = mode_product(Y, U, k + 2)
    return Y


def inverse(X, transforms):
    """L^{-1}(X) = X x_d U_d^{-1} ... x_3 U_3^{-1}, with U^{-1} = U^H / alpha."""
    Y = X
    for k in reversed(range(len(transforms))):
        U, a = transforms[k]
        Y = mode_product(Y, U.conj().T / a, k + 2)
    return Y


def forward_slice(X, transforms, j):
    """Transformed face slice j of L(X) alone, by the definition of the mode
    products: L(X)^<j> = sum_{j'} (prod_k U_k[i_k, i'_k]) X^<j'>, with j and j'
    split into mode indices as in slice_index.  The coefficient vector over j'
    is the Kronecker product of the rows U_d[i_d], ..., U_3[i_3] (i_3 fastest)."""
    dims = X.shape
    idx = np.unravel_index(int(j), dims[2:], order="F")
    coef = np.ones(1, dtype=np.complex128)
    for k in reversed(range(len(transforms))):
        coef = np.kron(coef, transforms[k][0][idx[k], :])
    P = int(np.prod(dims[2:]))
    S = np.asarray(X).reshape((dims[0], dims[1], P), order="F")
    if not np.iscomplexobj(S):  # real data: the real and imaginary coefficients apart
        return np.tensordot(S, coef.real, axes=([2], [0])) + 1j * np.tensordot(S, coef.imag, axes=([2], [0]))
    return np.tensordot(S, coef, axes=([2], [0]))


def rho(transforms):
    """rho = alpha_3 * ... * alpha_d."""
    r = 1.0
    for _U, a in transforms:
        r *= a
    return r


# ----------------------------------------------------------------------------
# face slices
# ----------------------------------------------------------------------------

def slice_index(idx, dims):
    """0-based face-slice index of (i3, ..., id): i3 + n3*(i4 + n4*(...))."""
    j = 0
    for a in reversed(range(2, len(dims))):
        j = j * dims[a] + idx[a - 2]
    return j


def to_slices(X):
    """View X as (n1, n2, P) with the face-slice index on the last axis."""
    n1, n2 = X.shape[:2]
    return X.reshape((n1, n2, -1), order="F")


def from_slices(S, dims):
    return S.reshape(tuple(dims), order="F")


def conjugate_partner(j, dims):
    """Slice index of the conjugate partner under the DFT on every mode 3..d.

    For real X, L(X)^<partner(j)> = conj(L(X)^<j>) with unitary DFTs, where
    partner negates every transform-domain index modulo n_k.
    """
    idx = []
    rem = j
    for n in dims[2:]:
        idx.append(rem % n)
        rem //= n
    pidx = [(-i) % n for i, n in zip(idx, dims[2:])]
    return slice_index(pidx, dims)


def canonical_slice(j, dims, kinds):
    """Key slice of j's conjugate pair under all-DFT transforms; j itself otherwise."""
    if all(k in ("dft", "dft_unnormalized") for k in kinds):
        return min(j, conjugate_partner(j, dims))
    return j


# ----------------------------------------------------------------------------
# t-product algebra
# ----------------------------------------------------------------------------

def facewise(A, B):
    """Face-wise product: (A tri B)^<j> = A^<j> B^<j>."""
    SA, SB = to_slices(A), to_slices(B)
    P = SA.shape[2]
    out = np.stack([SA[:, :, j] @ SB[:, :, j] for j in range(P)], axis=2)
    return from_slices(out, (SA.shape[0], SB.shape[1]) + tuple(A.shape[2:]))


def t_product(X, Y, transforms):
    """C = X *_L Y = L^{-1}(L(X) tri L(Y))."""
    return inverse(facewise(forward(X, transforms), forward(Y, transforms)), transforms)


def t_transpose(X, transforms):
    """Tensor with L(X^T)^<j> = (L(X)^<j>)^H for every slice."""
    LX = to_slices(forward(X, transforms))
    LT = np.conj(np.transpose(LX, (1, 0, 2)))
    dims = (X.shape[1], X.shape[0]) + tuple(X.shape[2:])
    return inverse(from_slices(LT, dims), transforms)


def t_identity(n, tail_dims, transforms):
    """Identity tensor: every transformed face slice is I_n."""
    P = int(np.prod(tail_dims)) if len(tail_dims) else 1
    S = np.repeat(np.eye(n)[:, :, None], P, axis=2).astype(np.complex128)
    return inverse(from_slices(S, (n, n) + tuple(tail_dims)), transforms)


def t_svd(X, transforms):
    """T-SVD: per transformed slice SVD; returns (U, S, V) in the spatial domain."""
    n1, n2 = X.shape[:2]
    tail = tuple(X.shape[2:])
    LX = to_slices(forward(X, transforms))
    P = LX.shape[2]
    LU = np.zeros((n1, n1, P), dtype=np.complex128)
    LS = np.zeros((n1, n2, P), dtype=np.complex128)
    LV = np.zeros((n2, n2, P), dtype=np.complex128)
    for j in range(P):
        u, s, vh = np.linalg.svd(LX[:, :, j])
        LU[:, :, j] = u
        LV[:, :, j] = vh.conj().T
        m = len(s)
        LS[np.arange(m), np.arange(m), j] = s
    U = inverse(from_slices(LU, (n1, n1) + tail), transforms)
    S = inverse(from_slices(LS, (n1, n2) + tail), transforms)
    V = inverse(from_slices(LV, (n2, n2) + tail), transforms)
    return U, S, V


def tsvd_rank(X, transforms, rtol=1e-10):
    """Number of i with a nonzero tube S(i, i, :, ..., :) (relative tolerance rtol)."""
    LX = to_slices(forward(X, transforms))
    svals = np.stack([np.linalg.svd(LX[:, :, j], compute_uv=False) for j in range(LX.shape[2])])
    scale = svals.max() if svals.size else 0.0
    return int(np.sum(np.any(svals > rtol * scale, axis=0)))
