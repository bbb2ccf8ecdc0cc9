"""Training driver of the width-predicting network (orchestration only: every
forward, backward and Adam step runs in the library's kernels).

Traces come from the method itself: the fixed-width solver runs in tracking
mode, one iteration per call, and after iteration t >= 1 the workspace holds
the features of every slice computed from iteration t - 1 together with the
number of its singular values that survived at iteration t.  The network is
trained to predict log(1 + surviving count) with the mean squared error.
"""
import numpy as np

from . import htsvt


def collect_traces(plan, admm, M, mask, n_iter):
    """Run n_iter solver iterations with fixed widths on (M, mask); returns
    host arrays (features n x 32 float32, targets n float32 = log(1 + kept))."""
    import torch
    dt = plan.torch_dtype
    L, E, Y = (torch.empty(plan.N, dtype=dt, device="cuda") for _ in range(3))
    ws = plan.alloc_workspace(admm=True)
    plan.learned("track")
    try:
        admm.init(L, E, Y, ws)
        P = plan.n_slices
        feats, ys = [], []
        for t in range(n_iter):
            admm.iterate(M, mask, L, E, Y, 1, ws)
            if t >= 1:
                feats.append(plan.region(ws, "features", torch.float32)[: P * 32].view(P, 32).cpu().numpy().copy())
                kept = plan.region(ws, "kept", torch.int32)[:P].cpu().numpy()
                ys.append(np.log1p(kept.astype(np.float64)).astype(np.float32))
    finally:
        plan.learned("off")
    return np.concatenate(feats), np.concatenate(ys)


def train(net, X, y, epochs=20, batch=1024, lr=1e-3, seed=0):
    """Adam on shuffled mini-batches; returns the mean loss of every epoch."""
    import torch
    g = np.random.Generator(np.random.PCG64([int(seed), 10]))
    n = X.shape[0]
    hist = []
    for _ in range(epochs):
        perm = g.permutation(n)
        Xd = torch.from_numpy(np.ascontiguousarray(X[perm])).to("cuda")
        yd = torch.from_numpy(np.ascontiguousarray(y[perm])).to("cuda")
        losses = []
        for b0 in range(0, n, batch):
            b1 = min(n, b0 + batch)
            losses.append(net.train_step(Xd[b0:b1], yd[b0:b1], lr=lr))
        hist.append(float(torch.stack(losses).mean().item()))
    return hist


def init_network(seed):
    """He-normal weights (std sqrt(2 / fan_in)) and zero biases from numpy's
    PCG64 seeded with (seed, 9)."""
    g = np.random.Generator(np.random.PCG64([int(seed), 9]))
    shapes = [(128, 32), (128,), (128, 128), (128,), (1, 128), (1,)]
    parts = []
    for s in shapes:
        if len(s) == 2:
            parts.append(g.standard_normal(s).ravel() * np.sqrt(2.0 / s[1]))
        else:
            parts.append(np.zeros(s))
    return htsvt.Mlp(np.concatenate(parts).astype(np.float32))
