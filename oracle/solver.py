"""Pure low-rank-prior ADMM for (robust) tensor completion, FP64.

Model (GNRHTC with the pure-L prior, i.e. the low-rank regularizer applied to L
itself instead of its gradient tensors; the special cases of the model and the
"pure L prior" variant of the discussion experiments):
    min_{L,E}  ||L||_{Phi,L} + lambda * Upsilon(P_Omega(E))
    s.t.       L + E = M           (M zero-filled off Omega)

ADMM steps per iteration t (the L-, E- and multiplier updates of Sec. V with
the gradient directions removed, so the L-subproblem is the GNHTSVT problem with
tau = 1/mu):
    L   <- D_{Phi, 1/mu}(M - E + Y/mu)
    H   <- M - L + Y/mu
    E   <- on Omega:  0 (completion) or GNHTT_{psi, lambda/mu}(P_Omega(H)) (robust; element-wise
                      "rpca", tube-wise "rpca_tube" or slice-wise "rpca_slice", Sec. IV-B)
           off Omega: H                          (the least-squares part)
    Y   <- Y + mu (M - L - E)
    mu  <- min(mu_max, vartheta * mu)
and the stopping quantity max{||dL||_inf, ||dE||_inf, ||M - L - E||_inf}.

Pins: Thm. 4.2 behaviour (the constraint residual and successive differences
decay), completion data consistency on Omega, and recovery of a low-tubal-rank
tensor (tests/test_oracle_solver.py).  The recovered values themselves are
"parity unpinned" by the paper (it prints no synthetic results).
"""
import numpy as np

from . import prox as proxmod


def admm(M, mask, model, penalty_L, penalty_E, lam, mu0, vartheta, mu_max, n_iter, tsvt_fn):
    """Run n_iter iterations.  tsvt_fn(X, tau, t) returns D_{Phi,tau}(X) for call t.

    Returns (L, E, Ymul, history) with history a list of dicts holding the
    stopping terms and mu of every iteration.
    """
    groups = {"rpca": "element", "rpca_tube": "tube", "rpca_slice": "slice"}
    if model != "completion" and model not in groups:
        raise ValueError(model)
    M = np.asarray(M, dtype=np.float64)
    mask = np.asarray(mask, dtype=bool)
    L = np.zeros_like(M)
    E = np.zeros_like(M)
    Ymul = np.zeros_like(M)
    mu = float(mu0)
    hist = []
    for t in range(n_iter):
        L_new = tsvt_fn(M - E + Ymul / mu, 1.0 / mu, t)
        H = M - L_new + Ymul / mu
        if model == "completion":
            E_obs = np.zeros_like(H)
        else:
            kind, params = penalty_E
            E_obs = proxmod.gnhtt(H, lam / mu, kind, params, groups[model], mask)
        E_new = np.where(mask, E_obs, H)
        resid = M - L_new - E_new
        Ymul = Ymul + mu * resid
        hist.append({
            "dL": float(np.abs(L_new - L).max()),
            "dE": float(np.abs(E_new - E).max()),
            "resid": float(np.abs(resid).max()),
            "resid_fro": float(np.linalg.norm(resid.ravel())),
            "mu": mu,
        })
        L, E = L_new, E_new
        mu = min(mu_max, vartheta * mu)
    return L, E, Ymul, hist


def rse(L_hat, L_true):
    """Relative error ||L_hat - L*||_F / ||L*||_F."""
    return float(np.linalg.norm((L_hat - L_true).ravel()) / np.linalg.norm(L_true.ravel()))
