"""Learned sketch widths on the GPU against the FP64 oracle (oracle/mlp.py and
the per-slice-width randomized t-SVT): the network's forward pass, gradient and
Adam step, the recorded features, the width rule and the fixed-width fallback,
and what a network trained on the method's own traces gains in the solver.

Tolerances: network outputs and gradients 1e-5 relative (FP32 against FP64);
t-SVT outputs 1e-5 relative Frobenius (FP32 path).  Integer decisions (widths,
fallbacks) are compared exactly where both sides decide in the same precision.
"""
import math

import numpy as np
import pytest

from oracle import mlp as omlp, transforms as otr, tsvt as otsvt
from workloads import synth

pytestmark = pytest.mark.gpu

MCP = ("mcp", (40.0,))


@pytest.fixture(scope="module")
def ht():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2506_09594_amd import htsvt
    return htsvt


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _theta(seed):
    g = synth.rng(seed, "mlp_init")
    th = omlp.init_params(g)
    th += 0.05 * g.standard_normal(th.shape)
    return th.astype(np.float32).astype(np.float64)


def test_mlp_forward_matches_oracle(ht):
    import torch
    th = _theta(1)
    X = np.random.default_rng(2).standard_normal((100, 32)).astype(np.float32).astype(np.float64)
    net = ht.Mlp(th)
    z = net.forward(torch.tensor(X, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    zr, _ = omlp.forward(th, X)
    assert _rel(z, zr) < 1e-5


@pytest.mark.parametrize("n", [1, 31, 300, 9000])  # one partial, ragged chunks, strided chunks
def test_mlp_gradient_matches_oracle(ht, n):
    import torch
    th = _theta(3)
    g = np.random.default_rng(n)
    X = g.standard_normal((n, 32)).astype(np.float32).astype(np.float64)
    y = g.standard_normal(n).astype(np.float32).astype(np.float64)
    net = ht.Mlp(th)
    grad, loss = net.grad(torch.tensor(X, dtype=torch.float32, device="cuda"),
                          torch.tensor(y, dtype=torch.float32, device="cuda"))
    Lr, gr = omlp.backward(th, X, y)
    assert float(loss.item()) == pytest.approx(Lr, rel=1e-5)
    grad = grad.double().cpu().numpy()
    o = 0
    for k in omlp.ORDER:  # block by block, relative to the block's norm
        m = int(np.prod(omlp.SHAPES[k]))
        assert np.linalg.norm(grad[o:o + m] - gr[o:o + m]) <= 1e-5 * np.linalg.norm(gr[o:o + m]) + 1e-12, k
        o += m


def test_mlp_adam_step_matches_oracle(ht):
    import torch
    th = _theta(4)
    g = np.random.default_rng(5)
    X = g.standard_normal((257, 32)).astype(np.float32).astype(np.float64)
    y = g.standard_normal(257).astype(np.float32).astype(np.float64)
    net = ht.Mlp(th)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    yd = torch.tensor(y, dtype=torch.float32, device="cuda")
    theta, m, v = th.copy(), np.zeros_like(th), np.zeros_like(th)
    for step in (1, 2, 3):
        _, gr = omlp.backward(theta, X, y)
        theta, m, v = omlp.adam_step(theta, m, v, gr, step, 1e-3)
        net.train_step(Xd, yd, lr=1e-3)
        got = net.theta.double().cpu().numpy()
        # each step moves a parameter by about lr * g / |g|: FP32 rounding leaves
        # the update within 1% of lr except where a gradient is at its rounding
        # level (its sign, and so its step, is then arbitrary)
        diff = np.abs(got - theta)
        assert np.mean(diff > 1e-5 * step) < 1e-3, f"step {step}"
        assert np.max(diff) <= 2.01e-3 * step, f"step {step}"


def test_mlp_training_reduces_loss_on_gpu(ht):
    import torch
    g = np.random.default_rng(7)
    X = g.standard_normal((2048, 32)).astype(np.float32)
    y = (0.5 * X[:, 0] - 0.25 * X[:, 3] + 1.0).astype(np.float32)
    net = ht.Mlp(_theta(8) * 0.5)
    Xd, yd = torch.tensor(X, device="cuda"), torch.tensor(y, device="cuda")
    l0 = float(net.train_step(Xd, yd).item())
    for _ in range(300):
        last = net.train_step(Xd, yd)
    assert float(last.item()) < 0.05 * l0


def _slice_rank_case(seed=6):
    dims, kinds = (64, 48, 4, 4), ["dct2", "dct2"]
    ranks = np.random.default_rng(seed).integers(2, 25, size=16)
    X = synth.slice_rank_tensor(dims, ranks, kinds, seed) + 1e-3 * synth.rng(seed, "noise").standard_normal(dims)
    return dims, kinds, ranks, X.astype(np.float32).astype(np.float64)


def _region(plan, ws, name, dtype):
    return plan.region(ws, name, dtype=dtype)


def test_track_mode_records_features_and_keeps_fixed_result(ht):
    import torch
    dims, kinds, ranks, X = _slice_rank_case()
    r, p, q = 20, 6, 1
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision="fp32", seed=12)
    dX = ht.to_device(X, torch.float32)
    ws = plan.alloc_workspace()
    ref = plan.gnhtsvt(dX, 2.0, MCP, call_index=0, workspace=ws).clone()
    plan.learned("track")
    plan.learned_reset(ws)
    o1 = plan.gnhtsvt(dX, 2.0, MCP, call_index=0, workspace=ws).clone()
    torch.cuda.synchronize()
    assert torch.equal(o1, ref)  # fixed widths: bit for bit the plain result
    P, lmax = plan.n_slices, plan.width
    sig1 = _region(plan, ws, "sigma", torch.float64)[: P * lmax].cpu().numpy().reshape(P, lmax)
    kept1 = _region(plan, ws, "kept", torch.int32)[:P].cpu().numpy()
    used1 = _region(plan, ws, "widths_used", torch.int32)[: 2 * P].cpu().numpy().reshape(P, 2)
    an = _region(plan, ws, "anorm", torch.float64)[: 2 * P].cpu().numpy().reshape(P, 2)
    LX = otr.to_slices(otr.forward(X, otr.build_transforms(dims, kinds)))
    assert np.allclose(an[:, 1], [np.linalg.norm(LX[:, :, j]) ** 2 for j in range(P)], rtol=1e-5)
    assert np.array_equal(an[:, 0], an[:, 1]) and np.all(used1 == [plan.width, plan.kept])
    tau2 = 1.5
    plan.gnhtsvt(dX, tau2, MCP, call_index=5, workspace=ws)
    torch.cuda.synchronize()
    feat = _region(plan, ws, "features", torch.float32)[: 32 * P].double().cpu().numpy().reshape(P, 32)
    for j in range(P):
        f = omlp.features(sig1[j], int(kept1[j]), int(used1[j, 0]), an[j, 0], tau2, 5, dims[0], dims[1])
        assert np.allclose(feat[j], f, rtol=1e-6, atol=1e-6), j
    assert plan.learned_counts(ws) == {"valid": 1, "predicted": 0, "redone": 0}


def test_predicted_widths_and_fallback_match_oracle(ht):
    """A network whose output is the constant b3 = log(1 + 7.5) asks for
    ceil(7.5) + p columns on every slice; slices of rank above 8 then keep all
    their values and are redone at the fixed width, the rest keep the narrow
    sketch.  The output equals the oracle's per-slice-width t-SVT at the widths
    the GPU used, and the decisions follow the fallback rule."""
    import torch
    dims, kinds, ranks, X = _slice_rank_case()
    r, p, q, seed, tau = 20, 6, 1, 12, 2.0
    p_th = {k: np.zeros(omlp.SHAPES[k]) for k in omlp.ORDER}
    p_th["b3"][0] = math.log(1 + 7.5)
    th = omlp.flatten(p_th).astype(np.float32)
    theta = torch.tensor(th, device="cuda")
    plan = ht.Plan(dims, kinds, r=r, p=p, q=q, precision="fp32", seed=seed)
    dX = ht.to_device(X, torch.float32)
    ws = plan.alloc_workspace()
    plan.learned("predict", theta)
    plan.learned_reset(ws)
    plan.gnhtsvt(dX, tau, MCP, call_index=0, workspace=ws)  # no history yet: fixed widths
    out = plan.gnhtsvt(dX, tau, MCP, call_index=1, workspace=ws)
    torch.cuda.synchronize()
    P = plan.n_slices
    l_fix, k_fix = plan.width, plan.kept
    wk1 = _region(plan, ws, "widths", torch.int32)[: 2 * P].cpu().numpy().reshape(P, 2)
    wk2 = _region(plan, ws, "widths_redo", torch.int32)[: 2 * P].cpu().numpy().reshape(P, 2)
    wkf = _region(plan, ws, "widths_used", torch.int32)[: 2 * P].cpu().numpy().reshape(P, 2)
    expect = omlp.width_from_prediction(float(np.float32(th[-1])), p, l_fix, k_fix)
    assert expect == (14, 14)
    assert np.all(wk1 == expect)
    redo = wk2[:, 0] > 0
    assert np.all(wkf[redo] == [l_fix, k_fix]) and np.all(wkf[~redo] == expect)
    # rank <= 7: fewer than 14 values survive and the residual is noise -> kept
    # rank >= 14: all 14 kept values survive -> redone
    assert np.all(~redo[ranks <= 7]) and np.all(redo[ranks >= 14])
    counts = plan.learned_counts(ws)
    assert counts["predicted"] == P and counts["redone"] == int(redo.sum())
    # the kept slices satisfy the rule on the statistics the GPU decided with
    sig = _region(plan, ws, "sigma", torch.float64)[: P * l_fix].cpu().numpy().reshape(P, l_fix)
    kept = _region(plan, ws, "kept", torch.int32)[:P].cpu().numpy()
    an = _region(plan, ws, "anorm", torch.float64)[: 2 * P].cpu().numpy().reshape(P, 2)
    for j in np.where(~redo)[0]:
        assert not omlp.needs_fallback(14, 14, int(kept[j]), an[j, 1], sig[j], tau, l_fix, min(dims[:2]), MCP), j
    om = otsvt.omegas(dims, kinds, r, p, seed=seed, call=1, round_to=np.float32)
    ref = otsvt.tsvt_randomized_widths(X, tau, MCP, otr.build_transforms(dims, kinds), wkf[:, 0], wkf[:, 1], q, om)
    assert _rel(ht.from_device(out, dims), ref) < 1e-5
    # forcing the fallback everywhere gives the fixed-width method bit for bit
    plain = ht.Plan(dims, kinds, r=r, p=p, q=q, precision="fp32", seed=seed)
    base = plain.gnhtsvt(dX, tau, MCP, call_index=1)
    plan.force_fallback(True)
    forced = plan.gnhtsvt(dX, tau, MCP, call_index=1, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(forced, base)
    plan.force_fallback(False)


def _completion(ht, dims, seed, r, p, sr=0.6, vartheta=1.05, ranks=(2, 20)):
    import torch
    kinds = ["dct2"] * (len(dims) - 2)
    P = int(np.prod(dims[2:]))
    rk = synth.rng(seed, "ranks").integers(ranks[0], ranks[1] + 1, size=P)
    L = synth.slice_rank_tensor(dims, rk, kinds, seed)
    mask = synth.observation_mask(dims, sr, seed)
    M = np.where(mask, L, 0.0).astype(np.float32).astype(np.float64)
    plan = ht.Plan(dims, kinds, r=r, p=p, q=2, precision="fp32", seed=seed)
    mu0 = 1.0 / synth.max_slice_norm(M, kinds)
    adm = ht.Admm(plan, "completion", phi=("mcp", (10.0,)), mu0=mu0, vartheta=vartheta, mu_max=1e10)
    return plan, adm, L, ht.to_device(M, torch.float32), ht.to_device(mask.astype(np.uint8), torch.uint8)


GAIN_CASE = dict(dims=(64, 64, 4, 4), r=30, p=8, n_iter=60)


@pytest.fixture(scope="module")
def trained_net(ht):
    """The network trained on the fixed-width solver's own traces (two seeded
    tensors of the gain case)."""
    from paper_2506_09594_amd import rankpred
    dims, r, p, n_iter = (GAIN_CASE[k] for k in ("dims", "r", "p", "n_iter"))
    X, y = [], []
    for sd in (201, 202):
        plan, adm, _, dM, dmask = _completion(ht, dims, sd, r, p)
        f, t = rankpred.collect_traces(plan, adm, dM, dmask, n_iter)
        X.append(f)
        y.append(t)
    X, y = np.concatenate(X), np.concatenate(y)
    assert X.shape == (2 * 16 * (n_iter - 1), 32) and np.all(np.isfinite(X))
    net = rankpred.init_network(3)
    hist = rankpred.train(net, X, y, epochs=60, batch=256, lr=2e-3)
    assert hist[-1] < 0.05 * hist[0]
    return net


def test_trained_network_gain_in_the_solver(ht, trained_net):
    """Trained on the fixed-width solver's own traces (two seeded tensors), the
    network lets a third tensor's completion run at a fraction of the fixed
    width with the same final recovery error; the fallback redoes few slices."""
    import torch
    from oracle import solver as osolver
    dims, r, p, n_iter = (GAIN_CASE[k] for k in ("dims", "r", "p", "n_iter"))
    net = trained_net
    res = {}
    for mode in ("fixed", "predict"):
        plan, adm, L, dM, dmask = _completion(ht, dims, 7, r, p)
        dL, dE, dY = (torch.empty(plan.N, dtype=torch.float32, device="cuda") for _ in range(3))
        ws = plan.alloc_workspace(admm=True)
        if mode == "predict":
            plan.learned("predict", net.theta)
        adm.init(dL, dE, dY, ws)
        widths = []
        for _ in range(n_iter):
            adm.iterate(dM, dmask, dL, dE, dY, 1, ws)
            if mode == "predict":
                widths.append(plan.region(ws, "widths_used", torch.int32)[: 2 * plan.n_slices].view(-1, 2)[:, 0]
                              .float().mean().item())
        torch.cuda.synchronize()
        res[mode] = (osolver.rse(ht.from_device(dL, dims), L), plan.learned_counts(ws), widths, plan.width)
    rse_fixed, rse_pred = res["fixed"][0], res["predict"][0]
    counts, widths, l_fix = res["predict"][1], res["predict"][2], res["predict"][3]
    assert rse_fixed < 1e-2  # a well-posed problem: the fixed method recovers the tensor
    assert rse_pred <= 1.05 * rse_fixed + 1e-6
    assert np.mean(widths[1:]) < 0.8 * l_fix  # the sketches shrink
    assert counts["predicted"] > 0 and counts["redone"] < 0.25 * counts["predicted"]


def test_fallback_misses_few_survivors_against_fixed_width_shadow(ht, trained_net):
    """The fixed-width method judges the predicted widths: at every iteration of
    the predicted-width completion the same input goes through a fixed-width
    plan with the same draws and threshold, and the singular values that
    survive there but not in the predicted run (missed survivors: the
    certain-miss fallback lets a slice keep a narrow sketch whose residual
    might still hold one) are counted.  Accepted bound: at most 1% of the
    fixed-width survivors over the run."""
    import torch
    dims, r, p, n_iter = (GAIN_CASE[k] for k in ("dims", "r", "p", "n_iter"))
    plan, adm, L, dM, dmask = _completion(ht, dims, 7, r, p)
    shadow = ht.Plan(dims, ["dct2"] * (len(dims) - 2), r=r, p=p, q=2, precision="fp32", seed=7)
    sws = shadow.alloc_workspace()
    dL, dE, dY = (torch.empty(plan.N, dtype=torch.float32, device="cuda") for _ in range(3))
    ws = plan.alloc_workspace(admm=True)
    plan.learned("predict", trained_net.theta)
    adm.init(dL, dE, dY, ws)
    P = plan.n_slices
    missed = total = slices_short = 0
    for t in range(n_iter):
        mu = adm.stats(ws)["mu"]
        xin = plan.region(ws, "Xin")[: plan.N].clone()  # this iteration's input (t >= 1)
        adm.iterate(dM, dmask, dL, dE, dY, 1, ws)
        if t == 0:
            continue
        kept_pred = plan.region(ws, "kept", torch.int32)[:P].cpu().numpy().astype(np.int64)
        _, _, kept_fix = shadow.gnhtsvt(xin, 1.0 / mu, ("mcp", (10.0,)), call_index=t, workspace=sws, stats=True)
        kept_fix = kept_fix.cpu().numpy().astype(np.int64)
        short = np.maximum(kept_fix - kept_pred, 0)
        missed += int(short.sum())
        total += int(kept_fix.sum())
        slices_short += int(np.count_nonzero(short))
    print(f"missed survivors {missed} of {total} ({100.0 * missed / max(total, 1):.3f}%), "
          f"slice-iterations short {slices_short} of {P * (n_iter - 1)}; {plan.learned_counts(ws)}")
    assert total > 0
    assert missed <= 0.01 * total
