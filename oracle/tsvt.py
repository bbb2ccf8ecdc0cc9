"""GNHTSVT: the exact operator and its per-slice randomized approximation.

Exact operator (Def. 4.3 and the deterministic branch of Alg. 4):
    D_{Phi,tau}(A, L) = L^{-1}( slice-wise  U_j diag(Prox_{Phi,tau}(sigma_j)) V_j^H ),
with [U_j, sigma_j, V_j] the SVD of the transformed face slice L(A)^<j>.  By
Thm. 4.1 it minimizes tau*||G||_{Phi,L} + ||G - A||_F^2 / 2, where
||G||_{Phi,L} = (1/rho) sum_ij Phi(sigma_ij) and rho = alpha_3 ... alpha_d.

Randomized approximation (the sketch-per-transformed-slice route): for every
slice, with l = min(r + p, n1, n2) and k = min(r, l),
    Y = A_j Omega_j,  Q = orth(Y)
    repeat q times:  Z = orth(A_j^H Q),  Q = orth(A_j Z)      (power iterations)
    B = Q^H A_j,  [U_B, s, V_B] = svd(B)
    C_j = Q U_B[:, :k] diag(Prox(s[:k])) V_B[:, :k]^H
and the output is L^{-1}(C).  orth() is Householder QR (numpy/LAPACK).  The
Gaussian Omega_j is drawn per call and keyed by the slice (by the canonical
member of a conjugate pair under the DFT, so the output stays real).

Pins: Thm. 4.1 optimality against perturbations, the l1 subgradient condition,
exactness when rank(L(A)^<j>) <= k or l = min(n1, n2), orthonormality of Q and
the energy identity, and the Halko-Martinsson-Tropp expected-error bound
(tests/test_oracle_tsvt.py).
"""
import numpy as np

from . import philox, prox as proxmod, transforms as tr


def _prox_vec(penalty, s, tau):
    kind, params = penalty
    return np.array([proxmod.prox_scalar(kind, float(x), tau, params) for x in s])


def gnhtsvt_exact(X, tau, penalty, transforms):
    """Deterministic GNHTSVT (full SVD of every transformed slice)."""
    LX = tr.to_slices(tr.forward(X, transforms))
    out = np.zeros_like(LX, dtype=np.complex128)
    for j in range(LX.shape[2]):
        u, s, vh = np.linalg.svd(LX[:, :, j], full_matrices=False)
        st = _prox_vec(penalty, s, tau)
        out[:, :, j] = (u * st[None, :]) @ vh
    res = tr.inverse(tr.from_slices(out, X.shape), transforms)
    return _realify(res, X)


def _realify(res, X):
    if np.iscomplexobj(X):
        return res
    scale = max(np.abs(res.real).max(initial=0.0), 1e-300)
    assert np.abs(res.imag).max(initial=0.0) <= 1e-10 * scale, "imaginary residue"
    return res.real.copy()


def objective(G, A, tau, penalty, transforms):
    """tau * ||G||_{Phi,L} + ||G - A||_F^2 / 2 (the problem solved by GNHTSVT)."""
    kind, params = penalty
    LG = tr.to_slices(tr.forward(G, transforms))
    total = 0.0
    for j in range(LG.shape[2]):
        for s in np.linalg.svd(LG[:, :, j], compute_uv=False):
            total += proxmod.phi(kind, s, params, tau)
    return tau * total / tr.rho(transforms) + 0.5 * np.linalg.norm((G - A).ravel()) ** 2


def _orth(Y):
    q, _r = np.linalg.qr(Y, mode="reduced")
    return q


def sketch_slice(Aj, Om, q):
    """Range finder with q power iterations; returns (Q, B = Q^H A_j)."""
    Q = _orth(Aj @ Om)
    for _ in range(q):
        Z = _orth(Aj.conj().T @ Q)
        Q = _orth(Aj @ Z)
    return Q, Q.conj().T @ Aj


def tsvt_slice(Aj, tau, penalty, k, q, Om, info=None):
    """The randomized estimate C_j = Q U_B[:, :k] diag(Prox(s[:k])) V_B[:, :k]^H
    of one transformed slice A_j with sketch matrix Om (n2 x l).  info, if a
    dict, receives 'sigma' (the l singular values of B), 'kept' and
    'tail_energy' ||A_j||_F^2 - ||B||_F^2."""
    Q, B = sketch_slice(Aj, Om, q)
    ub, s, vbh = np.linalg.svd(B, full_matrices=False)
    st = _prox_vec(penalty, s[:k], tau)
    if info is not None:
        info["sigma"] = s
        info["kept"] = int(np.count_nonzero(st))
        info["tail_energy"] = np.linalg.norm(Aj) ** 2 - np.linalg.norm(B) ** 2
    return (Q @ (ub[:, :k] * st[None, :])) @ vbh[:k, :]


def omegas(dims, kinds, r, p, seed, call=0, stream=0, round_to=None):
    """Omega_j for every slice: n2 x l Gaussians keyed by the canonical slice index."""
    n1, n2 = dims[0], dims[1]
    l = min(r + p, n1, n2)
    P = int(np.prod(dims[2:])) if len(dims) > 2 else 1
    out = []
    for j in range(P):
        key = tr.canonical_slice(j, dims, kinds)
        om = philox.omega(n2, l, key, call, stream, seed)
        if round_to is not None:
            om = om.astype(round_to).astype(np.float64)
        out.append(om)
    return out


def tsvt_randomized(X, tau, penalty, transforms, r, p, q, omega_list, stats=None):
    """Per-slice randomized GNHTSVT with the given sketch matrices.

    If stats is a dict it receives per-slice 'sigma' (l values of B), 'k' and
    'kept' (number of nonzero shrunk values) and 'tail_energy'
    ||A_j||_F^2 - ||B||_F^2.
    """
    n1, n2 = X.shape[:2]
    l = min(r + p, n1, n2)
    k = min(r, l)
    LX = tr.to_slices(tr.forward(X, transforms))
    P = LX.shape[2]
    out = np.zeros_like(LX, dtype=np.complex128)
    sig_all, kept_all, tail_all = [], [], []
    for j in range(P):
        Aj = LX[:, :, j]
        Om = omega_list[j]
        assert Om.shape == (n2, l)
        info = {}
        out[:, :, j] = tsvt_slice(Aj, tau, penalty, k, q, Om, info)
        s = info["sigma"]
        sig_all.append(np.pad(s, (0, l - len(s))))
        kept_all.append(info["kept"])
        tail_all.append(info["tail_energy"])
    if stats is not None:
        stats["sigma"] = np.array(sig_all)
        stats["k"] = k
        stats["kept"] = np.array(kept_all)
        stats["tail_energy"] = np.array(tail_all)
    res = tr.inverse(tr.from_slices(out, X.shape), transforms)
    return _realify(res, X)


def tsvt_randomized_widths(X, tau, penalty, transforms, widths, kepts, q, omega_list):
    """The per-slice randomized GNHTSVT with a width l_j and kept count k_j of
    its own for every slice j; Omega_j is the first l_j columns of the given
    draw (a narrower draw is the prefix of a wider one)."""
    LX = tr.to_slices(tr.forward(X, transforms))
    out = np.zeros_like(LX, dtype=np.complex128)
    for j in range(LX.shape[2]):
        l, k = int(widths[j]), int(kepts[j])
        out[:, :, j] = tsvt_slice(LX[:, :, j], tau, penalty, k, q, omega_list[j][:, :l])
    res = tr.inverse(tr.from_slices(out, X.shape), transforms)
    return _realify(res, X)
