"""Pins of the oracle's proximity operators (CPU only)."""
import numpy as np
import pytest

from oracle import prox as P

CASES = [
    ("l1", ()),
    ("mcp", (2.5,)), ("mcp", (0.3,)), ("mcp", (1.0,)),
    ("scad", (3.7, 1.0)), ("scad", (3.7, 0.2)), ("scad", (2.5, 2.0)),
    ("log", (0.5,)), ("log", (2.0,)), ("log", (0.05,)),
    ("capped_l1", (1.5,)), ("capped_l1", (0.2,)),
]


@pytest.mark.parametrize("kind,params", CASES)
def test_penalty_satisfies_assumption(kind, params):
    """phi(0) = 0, increasing, concave and continuous on [0, inf)."""
    xs = np.linspace(0.0, 12.0, 6001)
    f = np.array([P.phi(kind, x, params) for x in xs])
    assert f[0] == 0.0
    assert np.all(np.diff(f) >= -1e-12)
    assert np.all(np.diff(f, 2) <= 1e-9)
    # continuous with slope at most phi'(0) (1, or 1/e for log): no jumps anywhere
    slope0 = 1.0 / params[0] if kind == "log" else 1.0
    assert np.max(np.diff(f)) <= slope0 * (xs[1] - xs[0]) * (1 + 1e-9)
    assert P.phi(kind, 1e-9, params) / 1e-9 == pytest.approx(slope0, rel=1e-6)
    assert P.phi(kind, -1.3, params) == P.phi(kind, 1.3, params)


@pytest.mark.parametrize("kind,params", CASES)
@pytest.mark.parametrize("mu", [0.1, 0.7, 2.0])
def test_prox_matches_bruteforce(kind, params, mu):
    rng = np.random.default_rng(hash((kind, params, mu)) % 2**32)
    vs = np.concatenate([rng.uniform(-6, 6, 25), [0.0, mu, -mu, 1e-3]])
    for v in vs:
        x = P.prox_scalar(kind, v, mu, params)
        xb = P.prox_bruteforce(kind, v, mu, params)
        fx = P._objective(kind, params, mu, abs(v), abs(x))
        fb = P._objective(kind, params, mu, abs(v), abs(xb))
        assert fx <= fb + 1e-9, (kind, params, mu, v, x, xb)
        if abs(fx - fb) > 1e-7:  # no near-tie: minimizer is unique
            pass
        elif abs(x - xb) > 1e-4:
            # a genuine tie between two minimizers: the smaller magnitude is chosen
            assert abs(x) <= abs(xb) + 1e-9


def test_l1_is_soft_threshold():
    for v in np.linspace(-5, 5, 101):
        for mu in (0.3, 1.0, 2.2):
            assert P.prox_scalar("l1", v, mu) == pytest.approx(np.sign(v) * max(abs(v) - mu, 0.0), abs=1e-15)


def test_mcp_is_firm_threshold():
    # gamma > mu: firm shrinkage of Gao and Bruce with thresholds (mu, gamma)
    g, mu = 3.0, 1.0
    for v in np.linspace(-6, 6, 241):
        a = abs(v)
        if a <= mu:
            ref = 0.0
        elif a <= g:
            ref = np.sign(v) * g * (a - mu) / (g - mu)
        else:
            ref = v
        assert P.prox_scalar("mcp", v, mu, (g,)) == pytest.approx(ref, abs=1e-12)
    # gamma <= mu: hard threshold at sqrt(gamma * mu)
    g, mu = 0.5, 2.0
    t = np.sqrt(g * mu)
    for v in np.linspace(-4, 4, 161):
        if abs(abs(v) - t) < 1e-9:
            continue
        ref = v if abs(v) > t else 0.0
        assert P.prox_scalar("mcp", v, mu, (g,)) == pytest.approx(ref, abs=1e-12)


@pytest.mark.parametrize("kind,params", CASES)
def test_prox_monotone_and_shrinking(kind, params):
    vs = np.linspace(0, 8, 801)
    xs = np.array([P.prox_scalar(kind, v, 0.9, params) for v in vs])
    assert xs[0] == 0.0
    assert np.all(np.diff(xs) >= -1e-12)          # order of singular values preserved
    assert np.all(xs <= vs + 1e-12) and np.all(xs >= 0)


def test_mu_zero_is_identity():
    for kind, params in CASES:
        assert P.prox_scalar(kind, 1.7, 0.0, params) == 1.7
