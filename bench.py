#!/usr/bin/env python3
"""Throughput of the randomized high-order t-SVT on one MI355X.

Workload: a 256 x 256 x 16 x 16 FP32 tensor (256 transformed face slices of
256 x 256) of tubal rank 20 built from Gaussian t-product factors under the
orthonormal DCT on modes 3 and 4; randomized t-SVT with r = 20, p = 10, q = 2
and MCP shrinkage.  One step = one full randomized t-SVT (forward transform,
sketch, power iterations, CholeskyQR, small SVD, shrink, reconstruction,
inverse transform) on the resident input.

Prints one JSON line: frontal slices per second, the roofline of the dominant
kernel (HIP-event durations on the launch stream), and the FP64 oracle timed
on the host CPU over a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6

WORKLOAD = {
    "name": "tsvt_256x256x16x16_fp32_rank20_dct",
    "dims": (256, 256, 16, 16), "kinds": ["dct2", "dct2"], "rank": 20, "r": 20, "p": 10, "q": 2,
    "tau": 50.0, "penalty": ("mcp", (100.0,)), "precision": "fp32", "seed": 2,
}


def stage_bytes(stage, plan, es):
    """Algorithmic HBM bytes of one launch of a stage (read once, write once); the
    transformed tensor is 2 bytes per entry in the BF16-mixed path."""
    n1, n2 = plan.dims[0], plan.dims[1]
    P, l, N = plan.n_slices, plan.width, plan.N
    ea = 2 if plan.precision == "bf16" else es
    if stage == "transform_fwd":
        return N * (es + ea)
    if stage == "transform_inv":
        return 2 * N * es
    if stage in ("sketch_nn", "sketch_tn"):
        return P * (n1 * n2 * ea + (n1 + n2) * l * es)
    if stage == "recon_nt":
        return P * (n1 * n2 + (n1 + n2) * l) * es
    if stage == "recon_qk":
        return P * (2 * n1 * l + l * l) * es
    if stage == "omega":
        return P * n2 * l * es
    return None


def cpu_baseline(X, wl, budget_s=10.0):
    """The FP64 oracle on the host: whole randomized t-SVTs of the workload, repeated
    until about budget_s seconds of CPU work (each call draws its own sketch)."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import transforms as otr, tsvt as otsvt

    dims, kinds = wl["dims"], wl["kinds"]
    T = otr.build_transforms(dims, kinds)
    X64 = X.astype(np.float64)
    P = int(np.prod(dims[2:]))
    calls, t0 = 0, time.perf_counter()
    while True:
        om = otsvt.omegas(dims, kinds, wl["r"], wl["p"], seed=wl["seed"], call=calls, round_to=np.float32)
        otsvt.tsvt_randomized(X64, wl["tau"], wl["penalty"], T, wl["r"], wl["p"], wl["q"], om)
        calls += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s or calls >= 50:
            break
    threads = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    return {"value": round(calls * P / dt, 2), "unit": "slices/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{calls} full randomized t-SVTs of the workload ({P} slices each, FP64 numpy/LAPACK, "
                      f"{dt:.1f} s incl. transforms and sketch draws)"}


def counter_traffic(stage):
    """HBM bytes per launch of a sketch product from the committed rocprofv3 counter
    summary, or None if the summary is missing or the kernel sources changed since."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "sketch_256x256x16x16_fp32_hbm_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_sha256_16: ([0-9a-f]+)  \(of ([^;]+);", text)
    if not m:
        return None
    srcs = [s.strip() for s in m.group(2).split(",")]
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, s), "rb").read() for s in srcs)).hexdigest()[:16]
    if h != m.group(1):
        return None
    m = re.search(r"\(" + stage + r"\) \| \d+ \| [0-9.]+ \| [0-9.]+ \| (\d+) \|", text)
    return int(m.group(1)) if m else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--precision", choices=["fp32", "bf16"], default="fp32",
                    help="fp32 (default) or the BF16-mixed path (BF16 transformed slices and sketch products)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (known bytes) to calibrate HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the randomized t-SVT path runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2506_09594_amd import htsvt as ht
    from workloads import synth

    wl = dict(WORKLOAD)
    if args.precision != wl["precision"]:
        wl["precision"] = args.precision
        wl["name"] = wl["name"].replace("_fp32_", "_" + args.precision + "_")
    torch.cuda.set_device(0)
    X = synth.lowrank_tensor(wl["dims"], wl["rank"], wl["kinds"], seed=wl["seed"]).astype(np.float32)
    plan = ht.Plan(wl["dims"], wl["kinds"], r=wl["r"], p=wl["p"], q=wl["q"], precision=wl["precision"],
                   seed=wl["seed"])
    dX = ht.to_device(X, torch.float32)
    dOut = torch.empty_like(dX)
    ws = plan.alloc_workspace()
    for i in range(args.warmup):
        plan.gnhtsvt(dX, wl["tau"], wl["penalty"], call_index=i, out=dOut, workspace=ws)
    torch.cuda.synchronize()

    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        plan.gnhtsvt(dX, wl["tau"], wl["penalty"], call_index=args.warmup + i, out=dOut, workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)

    ms_per_step = 1e3 * dt / args.steps
    value = plan.n_slices / (dt / args.steps)
    es = 4
    stages = {k: {"ms_per_launch": (v[0] / v[1]) if v[1] else 0.0, "launches_per_step": v[1] / args.steps,
                  "ms_per_step": v[0] / args.steps} for k, v in prof.items() if v[1]}
    # dominant HBM-streaming kernel: the largest per-step total among stages with an algorithmic byte count
    hbm_stages = [k for k in stages if stage_bytes(k, plan, es) is not None]
    dom = max(hbm_stages, key=lambda k: stages[k]["ms_per_step"])
    ms = stages[dom]["ms_per_launch"]
    achieved = stage_bytes(dom, plan, es) / (ms * 1e-3) / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": counter_traffic(dom) if wl["precision"] == "fp32" else None,
            "algorithmic_bytes_per_launch": stage_bytes(dom, plan, es), "ms_per_launch": round(ms, 5)}
    if args.calib_copy:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    line = {
        "metric": "frontal slices/sec of randomized t-SVT",
        "value": round(value, 1),
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl["precision"] == "fp32" else "bf16-f32acc",
        "data": "synthetic",
        "config": {"workload": wl["name"], "dims": list(wl["dims"]), "r": wl["r"], "p": wl["p"], "q": wl["q"],
                   "transform": "dct2 on modes 3,4", "penalty": "mcp", "slices_per_step": plan.n_slices},
        "roofline": roof,
        "stages": {k: {kk: round(vv, 5) for kk, vv in v.items()} for k, v in stages.items()},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(X, wl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
