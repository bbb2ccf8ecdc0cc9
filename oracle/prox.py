"""Scalar proximity operators of the penalties used by GNHTSVT and GNHTT.

Definition followed (Sec. IV-B, the proximity operator):
    Prox_{phi, mu}(v) = argmin_x  mu * phi(x) + (x - v)^2 / 2,
for a penalty phi that is proper, l.s.c., symmetric, concave and increasing on
[0, inf) with phi(0) = 0 (the Assumption on Phi).  The paper defers the closed
forms to its supplement, which is not available; this module therefore follows
the definition itself: on each interval where phi has one smooth expression the
objective's stationary point (clamped to the interval) and the interval ends are
candidates, and the candidate with the lowest objective wins (ties go to the
smaller magnitude).  Penalties and their parameters (all absolute):

  l1          phi(x) = x
  mcp(g)      phi(x) = x - x^2/(2g) for x <= g, g/2 beyond        (Zhang 2010)
  scad(a, b)  phi(x) = x                               for x <= b
                       (2 a b x - x^2 - b^2)/(2(a-1) b) for b < x <= a b
                       (a+1) b / 2                      beyond
              (Fan-Li 2001 SCAD with lambda = b, divided by b so that the
              slope at 0 is 1 like the other penalties; a > 2)
  log(e)      phi(x) = log(1 + x/e)
  capped_l1(t) phi(x) = min(x, t)
  firm(a)     firm shrinkage with thresholds (mu, a mu), a > 1 (Gao-Bruce
              1997, named among the penalties of the Assumption on Phi): the
              penalty is MCP with gamma = a mu at the threshold mu it is used
              with, so phi depends on mu (reading: the paper lists firm
              thresholding among its proximity operators; its two thresholds
              scale with the one the solver sets)

The zero threshold t0 = sup{v >= 0 : Prox(v) = 0} of every penalty is found
by bisection on prox_scalar itself (the prox is nondecreasing).

Pins: dense 1-D brute force of the defining minimization for every penalty and
parameter set, l1 = soft threshold, firm = the Gao-Bruce formula, monotonicity,
closed forms of the zero threshold where the prox has one
(tests/test_oracle_prox.py).
"""
import math

import numpy as np

PENALTIES = ("l1", "mcp", "scad", "log", "capped_l1", "firm")


def phi(kind, x, params=(), mu=None):
    """Penalty value at x >= 0 (firm needs the threshold mu it is used with)."""
    x = abs(float(x))
    if kind == "firm":
        if mu is None:
            raise ValueError("the firm penalty depends on the threshold mu")
        (a,) = params
        return phi("mcp", x, (a * mu,))
    if kind == "l1":
        return x
    if kind == "mcp":
        (g,) = params
        return x - x * x / (2.0 * g) if x <= g else g / 2.0
    if kind == "scad":
        a, b = params
        if x <= b:
            return x
        if x <= a * b:
            return (2.0 * a * b * x - x * x - b * b) / (2.0 * (a - 1.0) * b)
        return (a + 1.0) * b / 2.0
    if kind == "log":
        (e,) = params
        return math.log1p(x / e)
    if kind == "capped_l1":
        (t,) = params
        return min(x, t)
    raise ValueError(kind)


def _objective(kind, params, mu, v, x):
    return mu * phi(kind, x, params, mu) + 0.5 * (x - v) ** 2


def _candidates(kind, params, mu, v):
    """Candidate minimizers on [0, inf) for v >= 0."""
    c = [0.0, v]
    if kind == "firm":
        (a,) = params
        return _candidates("mcp", (a * mu,), mu, v)
    if kind == "l1":
        c.append(max(v - mu, 0.0))
    elif kind == "mcp":
        (g,) = params
        # on [0, g]: mu*(1 - x/g) + x - v = 0  ->  x (1 - mu/g) = v - mu
        if 1.0 - mu / g != 0.0:
            c.append(min(max((v - mu) / (1.0 - mu / g), 0.0), g))
        c += [g, max(v, g)]
    elif kind == "scad":
        a, b = params
        c.append(min(max(v - mu, 0.0), b))
        # on [b, a b]: mu*(a b - x)/((a-1) b) + x - v = 0
        den = 1.0 - mu / ((a - 1.0) * b)
        if den != 0.0:
            c.append(min(max((v - mu * a / (a - 1.0)) / den, b), a * b))
        c += [b, a * b, max(v, a * b)]
    elif kind == "log":
        (e,) = params
        # mu/(e + x) + x - v = 0  ->  x^2 + (e - v) x + (mu - v e) = 0
        disc = (v + e) ** 2 - 4.0 * mu
        if disc >= 0.0:
            for s in (1.0, -1.0):
                x = 0.5 * ((v - e) + s * math.sqrt(disc))
                if x >= 0.0:
                    c.append(x)
    elif kind == "capped_l1":
        (t,) = params
        c.append(min(max(v - mu, 0.0), t))
        c += [t, max(v, t)]
    else:
        raise ValueError(kind)
    return c


def prox_scalar(kind, v, mu, params=()):
    """Prox_{phi, mu}(v) for one real v (sign-symmetric: acts on |v|)."""
    s = -1.0 if v < 0 else 1.0
    a = abs(float(v))
    if mu <= 0.0:
        return float(v)
    best_x, best_f = None, None
    for x in sorted(set(_candidates(kind, params, mu, a))):
        f = _objective(kind, params, mu, a, x)
        if best_f is None or f < best_f - 1e-15 * max(1.0, abs(best_f)):
            best_x, best_f = x, f
    return s * best_x


def zero_threshold(kind, mu, params=()):
    """t0 = sup{v >= 0 : Prox_{phi,mu}(v) = 0}, by bisection on prox_scalar
    (doubling from mu until the prox is nonzero, then halving the bracket)."""
    if mu <= 0.0:
        return 0.0
    lo, hi = 0.0, float(mu)
    for _ in range(64):
        if prox_scalar(kind, hi, mu, params) != 0.0:
            break
        lo, hi = hi, 2.0 * hi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if not lo < mid < hi:
            break
        if prox_scalar(kind, mid, mu, params) == 0.0:
            lo = mid
        else:
            hi = mid
    return lo


def prox(kind, v, mu, params=()):
    """Element-wise Prox on an array (slow loop; oracle use only)."""
    v = np.asarray(v, dtype=np.float64)
    out = np.empty_like(v)
    flat_in, flat_out = v.reshape(-1), out.reshape(-1)
    for i in range(flat_in.size):
        flat_out[i] = prox_scalar(kind, flat_in[i], mu, params)
    return out


def prox_bruteforce(kind, v, mu, params=(), grid=20001):
    """Minimize the defining objective on a dense grid, then refine locally."""
    a = abs(float(v))
    hi = 2.0 * a + 1.0
    xs = np.linspace(0.0, hi, grid)
    fs = np.array([_objective(kind, params, mu, a, x) for x in xs])
    i = int(np.argmin(fs))
    lo_x, hi_x = xs[max(i - 1, 0)], xs[min(i + 1, grid - 1)]
    for _ in range(200):  # golden-section refinement inside the bracketing cell
        m1 = lo_x + (hi_x - lo_x) * 0.381966
        m2 = lo_x + (hi_x - lo_x) * 0.618034
        if _objective(kind, params, mu, a, m1) <= _objective(kind, params, mu, a, m2):
            hi_x = m2
        else:
            lo_x = m1
    x = 0.5 * (lo_x + hi_x)
    if _objective(kind, params, mu, a, 0.0) <= _objective(kind, params, mu, a, x):
        x = 0.0
    return (-1.0 if v < 0 else 1.0) * x


def gnhtt(A, mu, kind, params=(), group="element", mask=None):
    """GNHTT: the proximity operator of a penalty applied element-wise, tube-wise
    or slice-wise (Sec. IV-B, the three solutions of the E-subproblem):
      element  E_i = Prox(A_i)
      tube     E_{i1 i2 :...:} = A_{i1 i2 :...:} / ||A_{i1 i2 :...:}||_F * Prox(||A_{i1 i2 :...:}||_F)
      slice    E^<k> = A^<k> / ||A^<k>||_F * Prox(||A^<k>||_F)
    with Prox = Prox_{phi, mu} and a zero group mapped to zero.  With a mask
    (boolean, same shape) the groups are those of P_Omega(A): entries off the
    mask count as zero in the norms and come out zero (the reading used for the
    E-update on the observed set)."""
    A = np.asarray(A, dtype=np.float64)
    if mask is not None:
        A = np.where(mask, A, 0.0)
    if group == "element":
        return prox(kind, A, mu, params)
    n1, n2 = A.shape[:2]
    P = int(np.prod(A.shape[2:])) if A.ndim > 2 else 1
    S = A.reshape((n1, n2, P), order="F")
    out = np.zeros_like(S)
    if group == "tube":
        for i in range(n1):
            for j in range(n2):
                v = S[i, j, :]
                nrm = float(np.linalg.norm(v))
                if nrm > 0.0:
                    out[i, j, :] = v / nrm * prox_scalar(kind, nrm, mu, params)
    elif group == "slice":
        for k in range(P):
            v = S[:, :, k]
            nrm = float(np.linalg.norm(v))
            if nrm > 0.0:
                out[:, :, k] = v / nrm * prox_scalar(kind, nrm, mu, params)
    else:
        raise ValueError(group)
    return out.reshape(A.shape, order="F")
