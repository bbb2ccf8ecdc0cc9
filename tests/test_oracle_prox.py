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


def test_firm_is_gao_bruce_threshold():
    """FIRM(a) at threshold mu: 0 up to mu, a (|v| - mu)/(a - 1) up to a mu, v beyond."""
    for a in (1.5, 3.0, 10.0):
        for mu in (0.2, 1.0, 4.0):
            for v in np.linspace(-6 * a * mu, 6 * a * mu, 301):
                t = abs(v)
                if abs(t - mu) < 1e-12 or abs(t - a * mu) < 1e-12:
                    continue
                ref = 0.0 if t <= mu else (np.sign(v) * a * (t - mu) / (a - 1) if t <= a * mu else v)
                assert P.prox_scalar("firm", v, mu, (a,)) == pytest.approx(ref, abs=1e-12)


@pytest.mark.parametrize("a", [1.2, 2.5, 8.0])
@pytest.mark.parametrize("mu", [0.1, 0.7, 2.0])
def test_firm_prox_matches_bruteforce(a, mu):
    rng = np.random.default_rng(int(100 * a + 10 * mu))
    for v in np.concatenate([rng.uniform(-6, 6, 25), [0.0, mu, a * mu]]):
        x = P.prox_scalar("firm", v, mu, (a,))
        xb = P.prox_bruteforce("firm", v, mu, (a,))
        assert P._objective("firm", (a,), mu, abs(v), abs(x)) <= P._objective("firm", (a,), mu, abs(v), abs(xb)) + 1e-9


def test_firm_needs_its_threshold():
    with pytest.raises(ValueError):
        P.phi("firm", 1.0, (2.0,))
    assert P.phi("firm", 1.0, (2.0,), 1.0) == P.phi("mcp", 1.0, (2.0,))


@pytest.mark.parametrize("mu", [0.05, 0.8, 3.0])
def test_zero_threshold_closed_forms(mu):
    """Where the prox has a closed form, the bisection lands on its threshold
    (to within the oracle prox's tie tolerance: objective differences below
    1e-15 resolve to the smaller magnitude, which moves a continuous threshold
    by at most sqrt(2e-15) ~ 5e-8)."""
    t = P.zero_threshold
    tol = dict(rel=1e-9, abs=1e-7)
    assert t("l1", mu) == pytest.approx(mu, **tol)
    assert t("firm", mu, (3.0,)) == pytest.approx(mu, **tol)
    assert t("mcp", mu, (5.0 * mu,)) == pytest.approx(mu, **tol)             # firm regime, gamma > mu
    assert t("mcp", mu, (0.3 * mu,)) == pytest.approx(np.sqrt(0.3) * mu, **tol)  # hard threshold sqrt(g mu)
    for th in (0.1 * mu, mu, 4 * mu):
        assert t("capped_l1", mu, (th,)) == pytest.approx(min(mu, np.sqrt(2 * mu * th)), **tol)
    assert t("l1", 0.0) == 0.0


@pytest.mark.parametrize("kind,params", CASES + [("firm", (2.0,)), ("firm", (1.1,))])
@pytest.mark.parametrize("mu", [0.3, 1.7])
def test_zero_threshold_is_the_boundary_of_the_prox(kind, params, mu):
    """Every v below t0 maps to 0 and every v above it survives (dense grid),
    i.e. t0 is the threshold that decides which singular values survive."""
    t0 = P.zero_threshold(kind, mu, params)
    assert t0 > 0.0
    assert P.prox_scalar(kind, t0 * (1 - 1e-7), mu, params) == 0.0
    assert P.prox_scalar(kind, t0 * (1 + 1e-6), mu, params) > 0.0
    vs = np.linspace(0.0, 3.0 * t0, 601)
    surv = np.array([P.prox_scalar(kind, v, mu, params) > 0.0 for v in vs])
    first = vs[np.argmax(surv)]
    assert abs(first - t0) <= vs[1] - vs[0] + 1e-12


# ---- GNHTT (group shrinkage) -------------------------------------------------

@pytest.mark.parametrize("kind,params", [("l1", ()), ("mcp", (3.0,)), ("scad", (3.7, 1.0)), ("log", (0.5,))])
def test_gnhtt_group_minimizes_its_objective(kind, params):
    """Tube and slice GNHTT minimize mu * phi(||E_g||) + ||E_g - A_g||^2 / 2 group by
    group: no random perturbation of a group's output lowers its objective."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((3, 2, 4)) * 1.5
    mu = 0.8
    for group, axes in (("tube", lambda E: [E[i, j, :] for i in range(3) for j in range(2)]),
                        ("slice", lambda E: [E[:, :, k] for k in range(4)])):
        E = P.gnhtt(A, mu, kind, params, group)
        for eg, ag in zip(axes(E), axes(A)):
            obj = lambda x: mu * P.phi(kind, np.linalg.norm(x), params) + 0.5 * np.sum((x - ag) ** 2)
            f0 = obj(eg)
            for _ in range(300):
                d = rng.standard_normal(eg.shape) * rng.choice([1e-3, 1e-1, 1.0])
                assert obj(eg + d) >= f0 - 1e-10


def test_gnhtt_l1_tube_is_block_soft_threshold():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((4, 3, 5))
    mu = 1.1
    E = P.gnhtt(A, mu, "l1", (), "tube")
    nrm = np.linalg.norm(A, axis=2, keepdims=True)
    ref = np.maximum(0.0, 1.0 - mu / nrm) * A
    assert np.allclose(E, ref, atol=1e-14)


def test_gnhtt_groups_of_one_are_element_wise():
    """Tubes of length one (an order-2 tensor) and slices of one entry reduce to the
    element-wise proximity operator."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((5, 4))
    ref = P.prox("mcp", A, 0.7, (2.0,))
    assert np.allclose(P.gnhtt(A, 0.7, "mcp", (2.0,), "tube"), ref, atol=1e-14)
    B = rng.standard_normal((1, 1, 6))
    assert np.allclose(P.gnhtt(B, 0.7, "mcp", (2.0,), "slice"), P.prox("mcp", B, 0.7, (2.0,)), atol=1e-14)


def test_gnhtt_mask_zeroes_unobserved_entries():
    rng = np.random.default_rng(6)
    A = rng.standard_normal((4, 4, 3))
    mask = rng.random(A.shape) < 0.5
    E = P.gnhtt(A, 0.3, "l1", (), "slice", mask)
    assert np.all(E[~mask] == 0.0)
    Am = np.where(mask, A, 0.0)
    assert np.allclose(E, P.gnhtt(Am, 0.3, "l1", (), "slice"), atol=1e-15)
