"""Learned sketch widths: features, the rank-predicting MLP, its training step
and the width / fallback rule, in FP64 (test infrastructure, like the rest of
this package).

The paper sizes the sketch of every slice by a fixed target rank r plus
oversampling p (Alg. 1 and the randomized t-SVT of Sec. IV) and, in its
adaptive variant, grows the basis until the residual energy
||A - Q Q^T A||_F^2 = ||A||_F^2 - ||Q^T A||_F^2 falls below a tolerance
(Alg. 3, the energy identity of its stopping test).  The learned variant keeps
the fixed-width method as its fallback and judge: a small MLP predicts from the
previous iteration's sketch spectrum how many singular values of each slice
survive the shrinkage; the slice is sketched with that many columns plus p,
and redone at the fixed width when the result could be truncated:

  (i)  every kept value survived the proximity operator (kept == k_j): the
       sketch never reached below the threshold, so more values may survive;
  (ii) the residual certainly holds a value above tau: its energy
       ||A_j||^2 - ||B_j||^2 (the energy identity) exceeds (min(n1, n2) - l) tau^2,
       i.e. the mean square of its at most min(n1, n2) - l singular values is
       above tau^2, so the largest is too (values <= tau are zeroed by the L1
       and MCP shrinkages used with the solvers).
  The bound sqrt(energy) > tau, which is necessary for a missed value and
  fires whenever the residual holds many small values, would leave a
  completion iterate almost no slice at its predicted width.

The paper gives no network, features or loss for this; the reading taken here
(features from the last spectrum and energies, a 32-128-128-1 ReLU MLP, MSE on
log(1 + surviving count), Adam) is stated with each function.
"""
import math

import numpy as np

from . import prox as proxmod

N_IN, N_H = 32, 128
SHAPES = {"W1": (N_H, N_IN), "b1": (N_H,), "W2": (N_H, N_H), "b2": (N_H,), "W3": (1, N_H), "b3": (1,)}
ORDER = ["W1", "b1", "W2", "b2", "W3", "b3"]
N_PARAMS = sum(int(np.prod(SHAPES[k])) for k in ORDER)


# ---------------------------------------------------------------------------
# parameters as one flat vector (row-major blocks in ORDER)
# ---------------------------------------------------------------------------
def unflatten(theta):
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(SHAPES[k]))
        out[k] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(SHAPES[k])
        o += n
    return out


def flatten(params):
    return np.concatenate([np.asarray(params[k], dtype=np.float64).ravel() for k in ORDER])


def init_params(rng):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; rng is a numpy Generator."""
    p = {}
    for k in ORDER:
        if k.startswith("W"):
            fan_in = SHAPES[k][1]
            p[k] = rng.standard_normal(SHAPES[k]) * math.sqrt(2.0 / fan_in)
        else:
            p[k] = np.zeros(SHAPES[k])
    return flatten(p)


# ---------------------------------------------------------------------------
# network: z = W3 relu(W2 relu(W1 x + b1) + b2) + b3, a prediction of log(1 + s)
# ---------------------------------------------------------------------------
def forward(theta, X):
    """X: (n, 32).  Returns z (n,) and the activations needed by backward."""
    p = unflatten(theta)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["W3"][0] + p["b3"][0]
    return z, (X, a1, h1, a2, h2)


def loss(theta, X, y):
    """Mean squared error of z against y = log(1 + surviving count)."""
    z, _ = forward(theta, X)
    return float(np.mean((z - y) ** 2))


def backward(theta, X, y):
    """Loss and its gradient with respect to the flat parameter vector (chain
    rule through the two ReLU layers)."""
    p = unflatten(theta)
    z, (X, a1, h1, a2, h2) = forward(theta, X)
    n = X.shape[0]
    dz = 2.0 * (z - y) / n
    g = {"W3": (dz @ h2)[None, :], "b3": np.array([dz.sum()])}
    dh2 = np.outer(dz, p["W3"][0]) * (a2 > 0.0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ p["W2"]) * (a1 > 0.0)
    g["W1"] = dh1.T @ X
    g["b1"] = dh1.sum(axis=0)
    return float(np.mean((z - y) ** 2)), flatten(g)


def adam_step(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Alg. 1) with bias correction; step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------------------
# features of one slice from the previous call's statistics
# ---------------------------------------------------------------------------
def _clip(x, lo, hi):
    return min(max(x, lo), hi)


def features(sigma, kept_prev, l_prev, anorm2, tau, iteration, n1, n2):
    """32 features of a slice.  sigma: the previous call's singular values of B
    (descending, l_prev of them); kept_prev: how many survived; anorm2:
    ||A_j||_F^2 of the previous call; tau: the current threshold.
      0-15  sigma_i / sigma_1, i = 1..16 (0 past l_prev or when sigma_1 = 0)
      16    log10(||A||^2 + 1e-30) / 10
      17    tail fraction (||A||^2 - ||B||^2) / ||A||^2, clipped to [0, 1]
      18    tau / sigma_1 clipped to [0, 10] (10 when sigma_1 = 0)
      19    fraction of the l_prev values above tau
      20    kept_prev / l_prev
      21-24 log(sigma_k / sigma_{k+1}) for k = 2, 4, 8, 16, clipped to [0, 10]
            (10 when sigma_{k+1} = 0 < sigma_k; 0 when both are 0 or k >= l_prev)
      25    log10(1 / tau) / 10 (log mu; 1 when tau = 0)
      26    min(iteration, 200) / 100
      27    log(n1 / n2)
      28    log2(min(n1, n2)) / 10
      29    l_prev / 64
      30    (number of values above tau) / 64
      31    0"""
    s = np.zeros(max(l_prev, 17))
    s[:l_prev] = np.asarray(sigma[:l_prev], dtype=np.float64)
    f = np.zeros(N_IN)
    s1 = s[0]
    for i in range(16):
        f[i] = s[i] / s1 if (s1 > 0.0 and i < l_prev) else 0.0
    b2 = float(np.sum(s[:l_prev] ** 2))
    f[16] = math.log10(anorm2 + 1e-30) / 10.0
    f[17] = _clip((anorm2 - b2) / anorm2, 0.0, 1.0) if anorm2 > 0.0 else 0.0
    f[18] = _clip(tau / s1, 0.0, 10.0) if s1 > 0.0 else 10.0
    above = int(np.sum(s[:l_prev] > tau))
    f[19] = above / l_prev
    f[20] = kept_prev / l_prev
    for c, k in enumerate((2, 4, 8, 16)):
        if k >= l_prev:
            f[21 + c] = 0.0
        else:
            a, b = s[k - 1], s[k]
            if b > 0.0:
                f[21 + c] = _clip(math.log(a / b), 0.0, 10.0)
            else:
                f[21 + c] = 10.0 if a > 0.0 else 0.0
    f[25] = math.log10(1.0 / tau) / 10.0 if tau > 0.0 else 1.0
    f[26] = min(iteration, 200) / 100.0
    f[27] = math.log(n1 / n2)
    f[28] = math.log2(min(n1, n2)) / 10.0
    f[29] = l_prev / 64.0
    f[30] = above / 64.0
    return f


# ---------------------------------------------------------------------------
# width rule and fallback
# ---------------------------------------------------------------------------
def width_from_prediction(z, p, l_fix, k_fix):
    """Predicted surviving count s = exp(z) - 1; sketch width
    l = clamp(ceil(s) + p, p + 1, l_fix) and kept count k = min(k_fix, l), the
    fixed method's k = min(r, l) at the new width: the p extra columns are the
    margin of the prediction, and test (i) of the fallback fires only when all
    k values survive, i.e. when the prediction fell short by more than p."""
    s = math.expm1(z) if z < 700.0 else math.inf
    l = math.ceil(s) + p if math.isfinite(s) else l_fix
    l = int(min(max(l, p + 1), l_fix))
    return l, int(min(k_fix, l))


def needs_fallback(l, k, kept, anorm2, sigma, tau, l_fix, n_min, penalty=("l1", ())):
    """True when a slice sketched at width l < l_fix must be redone at l_fix
    (n_min = min(n1, n2)): (i) every kept value survived the shrinkage, or (ii)
    the residual energy ||A||^2 - ||B||^2 exceeds (n_min - l) t0^2 with t0 the
    penalty's zero threshold (a value above t0 survives the prox), so the
    residual certainly holds a value that would survive."""
    if l >= l_fix:
        return False
    if kept >= k:
        return True
    kind, params = penalty
    t0 = proxmod.zero_threshold(kind, tau, params)
    tail = anorm2 - float(np.sum(np.asarray(sigma[:l], dtype=np.float64) ** 2))
    return tail > (n_min - l) * t0 * t0
