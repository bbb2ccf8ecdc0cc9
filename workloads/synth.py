"""Seeded synthetic tensors for the completion / robust-PCA workloads.

The paper's real datasets (hyperspectral, MRI, video, ...) are not available;
these generators stand in for them with tensors of prescribed tubal rank, built
the way the workloads are specified:

  * low-tubal-rank part: X = A *_L B with Gaussian N(0,1) factors A (n1 x r x
    n3 x ... x nd) and B (r x n2 x n3 x ... x nd), i.e. the face-wise product of
    the transformed factors followed by the inverse transform;
  * optional i.i.d. Gaussian noise of a given standard deviation;
  * observation set: exactly round(SR * N) positions drawn uniformly without
    replacement (the sampling convention of the experiments section);
  * outliers: exactly round(frac * N) positions, values uniform in [-1, 1],
    added to the data.

Random streams come from numpy's PCG64 seeded with (master seed, stream id), so
each ingredient is reproducible on its own.  The transforms here are scipy's
DCT-II / FFT routines with orthonormal scaling.
"""
import numpy as np
import scipy.fft as sfft

STREAMS = {
    "factor_a": 1, "factor_b": 2, "noise": 3, "mask": 4, "outlier_pos": 5,
    "outlier_val": 6, "shapes": 7, "ranks": 8, "mlp_init": 9, "shuffle": 10,
}


def rng(seed, stream):
    return np.random.Generator(np.random.PCG64([int(seed), STREAMS[stream]]))


def _fwd(X, kinds):
    for ax, kind in enumerate(kinds, start=2):
        if kind == "dct2":
            X = sfft.dct(X, type=2, norm="ortho", axis=ax)
        elif kind == "dft":
            X = sfft.fft(X, norm="ortho", axis=ax)
        else:
            raise ValueError(kind)
    return X


def _inv(X, kinds):
    for ax, kind in reversed(list(enumerate(kinds, start=2))):
        if kind == "dct2":
            X = sfft.idct(X, type=2, norm="ortho", axis=ax)
        elif kind == "dft":
            X = sfft.ifft(X, norm="ortho", axis=ax)
        else:
            raise ValueError(kind)
    return X


def _facewise(LA, LB):
    n1, r = LA.shape[:2]
    n2 = LB.shape[1]
    tail = LA.shape[2:]
    P = int(np.prod(tail)) if tail else 1
    a = np.moveaxis(LA.reshape((n1, r, P), order="F"), 2, 0)
    b = np.moveaxis(LB.reshape((r, n2, P), order="F"), 2, 0)
    c = np.moveaxis(np.matmul(a, b), 0, 2)
    return c.reshape((n1, n2) + tuple(tail), order="F")


def lowrank_tensor(dims, rank, kinds, seed, noise_std=0.0):
    """Tubal-rank-`rank` tensor from Gaussian t-product factors, plus noise."""
    dims = tuple(int(d) for d in dims)
    tail = dims[2:]
    A = rng(seed, "factor_a").standard_normal((dims[0], rank) + tail)
    B = rng(seed, "factor_b").standard_normal((rank, dims[1]) + tail)
    X = _inv(_facewise(_fwd(A, kinds), _fwd(B, kinds)), kinds)
    if np.iscomplexobj(X):
        X = X.real
    X = np.ascontiguousarray(X)
    if noise_std > 0.0:
        X = X + noise_std * rng(seed, "noise").standard_normal(dims)
    return X


def slice_rank_tensor(dims, ranks, kinds, seed):
    """Tensor whose transformed slice j has rank ranks[j] (built in the transform domain)."""
    dims = tuple(int(d) for d in dims)
    n1, n2 = dims[:2]
    P = int(np.prod(dims[2:]))
    ga, gb = rng(seed, "factor_a"), rng(seed, "factor_b")
    S = np.zeros((n1, n2, P))
    for j in range(P):
        r = int(ranks[j])
        S[:, :, j] = ga.standard_normal((n1, r)) @ gb.standard_normal((r, n2))
    X = _inv(S.reshape(dims, order="F"), kinds)
    return np.ascontiguousarray(X.real if np.iscomplexobj(X) else X)


def observation_mask(dims, sr, seed):
    """Boolean mask with exactly round(sr * N) True entries, uniform without replacement."""
    N = int(np.prod(dims))
    m = int(round(sr * N))
    idx = rng(seed, "mask").choice(N, size=m, replace=False)
    mask = np.zeros(N, dtype=bool)
    mask[idx] = True
    return mask.reshape(tuple(dims), order="F")


def outliers(dims, frac, seed):
    """Sparse tensor with round(frac * N) entries uniform in [-1, 1]."""
    N = int(np.prod(dims))
    m = int(round(frac * N))
    pos = rng(seed, "outlier_pos").choice(N, size=m, replace=False)
    val = rng(seed, "outlier_val").uniform(-1.0, 1.0, size=m)
    S = np.zeros(N)
    S[pos] = val
    return S.reshape(tuple(dims), order="F")


def max_slice_norm(X, kinds):
    """max_j ||L(X)^<j>||_2 (spectral norm of every transformed face slice)."""
    LX = _fwd(np.asarray(X, dtype=np.float64), kinds)
    n1, n2 = LX.shape[:2]
    S = LX.reshape((n1, n2, -1), order="F")
    return float(max(np.linalg.norm(S[:, :, j], 2) for j in range(S.shape[2])))


def to_fortran_flat(X):
    """Flatten in Fortran order (i1 fastest): the library's storage layout."""
    return np.asarray(X).ravel(order="F")


def from_fortran_flat(flat, dims):
    return np.asarray(flat).reshape(tuple(dims), order="F")


def batch_shapes(n_tensors, seed, orders=(3, 4, 5), modes=(4, 8, 16), n_range=(64, 512), r_range=(5, 40)):
    """Shapes and target ranks of a batch of uneven tensors: order uniform over
    `orders`, every transformed mode uniform over `modes`, n1 and n2 uniform
    integers in n_range, rank uniform in r_range (all bounds inclusive)."""
    g = rng(seed, "shapes")
    out = []
    for _ in range(n_tensors):
        d = int(g.choice(orders))
        n1, n2 = (int(v) for v in g.integers(n_range[0], n_range[1] + 1, size=2))
        rest = tuple(int(v) for v in g.choice(modes, size=d - 2))
        r = int(g.integers(r_range[0], r_range[1] + 1))
        out.append(((n1, n2) + rest, r))
    return out
