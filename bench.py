"""Benchmark of the modified ns-form operator apply on one MI355X.

A step is one pass of the whole path on the Poisson workload with k = 8, eps = 1e-6 and a
50-Gaussian seeded source: Gaussian-sum fit (host FP64), operator build (1-D blocks and screening
plan, device), adaptive projection to a redundant tree (device), the apply (neighbour closure,
FP64-MFMA contractions, assembly; device) and evaluation at 1e4 points.  The printed JSON line
reports NS-apply block-contractions per second of step time, the roofline of the contraction
kernel (FP64 MFMA) and the CPU oracle timed on a bounded sample of the same apply.  Beside it:
the precision-routed apply against the FP64 one on the same tree at tol = eps ||g|| ("mixed"),
and the batch of uneven seeded solves applied one by one, as one persistent batched launch and
as replays of a captured plan ("batch").

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-mixed] [--no-batch]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (matrix and vector)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-vs-FP64 measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-apply measurement")
    ap.add_argument("--cpu-sample-nodes", type=int, default=15000)
    ap.add_argument("--variant", type=int, default=-1, help="contraction-kernel tile variant (-1: library default)")
    ap.add_argument("--workload", choices=["c2", "c3"], default="c2",
                    help="c2: Poisson k=8 eps=1e-6 (the reported configuration); c3: Yukawa k=10 eps=1e-8")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 256 MiB elementwise copy (reference for the FETCH_SIZE/WRITE_SIZE counters)")
    return ap.parse_args()


def calibrate_copy():
    """A plain elementwise kernel that reads and writes 256 MiB each: the counters it produces scale
    FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    n = 32 * 1024 * 1024
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "elementwise copy", "bytes_read": n * 8, "bytes_written": n * 8}))


PROFILES = {"c2": ("ns_apply_kernel_poisson_k8_eps1e-6.md", "contract.hip"),
            "c3": ("ns_apply_wide_kernel_yukawa_k10_eps1e-8.md", "contract_wide.hip")}


def traffic_from_profile(workload):
    """HBM bytes of one contraction-kernel launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), provided the summary was taken on the
    current kernel source (same git blob id of the kernel's file); otherwise None."""
    import hashlib
    import re
    name, kernel_src = PROFILES[workload]
    prof = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_0706_0747_amd", "csrc", kernel_src)
    try:
        with open(prof) as fh:
            text = fh.read()
        with open(src, "rb") as fh:
            data = fh.read()
    except OSError:
        return None
    blob = hashlib.sha1(b"blob %d\0" % len(data) + data).hexdigest()
    m1 = re.search(r"kernel_source_blob: ([0-9a-f]{40})", text)
    m2 = re.search(r"traffic_bytes_per_launch: ([0-9.eE+]+)", text)
    if not m1 or not m2 or m1.group(1) != blob:
        return None
    return float(m2.group(1))


def step(M, ctx, w, pts, mode=0):
    """One pass of the whole path; returns (g, stats, depth, values, f, op).  The timed steps pass
    MWNS_TIMES_ONLY: the kernel times are recorded, the device passes of the statistics that are
    not part of the method (contraction count, ||g||) are left out."""
    f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    depth = M.mwns_tree_get_info(f)["depth"]
    tau, wt = M.mwns_fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
    op = M.mwns_op_create(ctx, w.k, tau, wt, w.eps, depth)
    g, stats = M.mwns_apply(ctx, op, f, mode)
    vals = M.mwns_tree_eval(ctx, g, pts)
    return g, stats, depth, vals, f, op


def leaf_norm(leaf, coef):
    import numpy as np
    return math.sqrt(float(np.sum(coef[leaf == 1] ** 2)))


def mixed_measurement(M, ctx, w, f, op, g64, st64, reps, ms_con64):
    """Apply-only wall time of the FP64 and the precision-routed apply on the same tree and
    operator, the latter at tol = eps ||g_F64||; the measured relative L2 error against FP64.
    ms_con64 is the FP64 contraction time of the timed steps (their average)."""
    import torch
    tol = w.eps * st64["g_norm"]
    times = {}
    for name, fn in (("fp64", lambda: M.mwns_apply(ctx, op, f, stats=False)),
                     ("mixed", lambda: M.mwns_apply_mixed(ctx, op, f, tol, stats=False))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        times[name] = 1e3 * (time.perf_counter() - t0) / reps
    gm, stm = M.mwns_apply_mixed(ctx, op, f, tol)
    _, leaf, a = M.mwns_tree_export(ctx, g64)
    _, _, b = M.mwns_tree_export(ctx, gm)
    err = leaf_norm(leaf, b - a)
    return times["fp64"] / times["mixed"], {
        "tol_rel": w.eps, "err_rel_measured": err / st64["g_norm"], "err_rel_bound": stm["err_bound"] / st64["g_norm"],
        "apply_ms_fp64": times["fp64"], "apply_ms_mixed": times["mixed"],
        "contract_ms_fp64": ms_con64, "contract_ms_mixed": stm["ms_contract"],
        "class_flop_share": {c: stm["class_flops"][i] / stm["useful_flops"]
                             for i, c in enumerate(("f64", "f32", "bf16c", "bf16"))},
        "classes": "FP64 MFMA; FP32 MFMA; BF16 MFMA on hi/lo splits (4 partial products); BF16 MFMA"}


def batch_measurement(M, ctx, reps, nmembers=64):
    """The batch of uneven solves (seeded members of mixed kernels, k and eps): total contractions
    per second for sequential single applies, one batched persistent apply, and replays of the
    captured apply plan, in FP64 and precision-routed at tol = eps ||g|| per member."""
    import torch
    members = [workloads_member(i) for i in range(nmembers)]
    kept = members
    ops, fs = [], []
    for w in kept:
        f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
        depth = M.mwns_tree_get_info(f)["depth"]
        tau, wt = M.mwns_fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
        ops.append(M.mwns_op_create(ctx, w.k, tau, wt, w.eps, depth))
        fs.append(f)
    _, st = M.mwns_apply_batch(ctx, ops, fs)
    plan = M.mwns_plan_create(ctx, ops, fs)
    tols = [w.eps * M.mwns_apply(ctx, op, f)[1]["g_norm"] for w, op, f in zip(kept, ops, fs)]
    _, stm = M.mwns_apply_batch(ctx, ops, fs, mixed=tols)
    planm = M.mwns_plan_create(ctx, ops, fs, mixed=tols)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    ms_seq = timed(lambda: [M.mwns_apply(ctx, op, f, stats=False) for op, f in zip(ops, fs)])
    ms_batch = timed(lambda: M.mwns_apply_batch(ctx, ops, fs, stats=False))
    ms_plan = timed(plan.execute)
    ms_batch_mixed = timed(lambda: M.mwns_apply_batch(ctx, ops, fs, mixed=tols, stats=False))
    ms_plan_mixed = timed(planm.execute)
    plan.close()
    planm.close()
    nodes = sum(M.mwns_tree_get_info(f)["nnodes"] for f in fs)
    c = st["contractions"]
    return {"members": len(kept), "orders": sorted({int(w.k) for w in kept}), "nodes": int(nodes),
            "contractions": int(c), "ms_sequential": ms_seq, "ms_batch": ms_batch, "ms_plan_replay": ms_plan,
            "contractions_per_s_sequential": c / (ms_seq * 1e-3), "contractions_per_s_batch": c / (ms_batch * 1e-3),
            "contractions_per_s_plan": c / (ms_plan * 1e-3),
            "mixed": {"tol": "eps ||g|| per member", "ms_batch": ms_batch_mixed, "ms_plan_replay": ms_plan_mixed,
                      "speedup_batch": ms_batch / ms_batch_mixed, "speedup_plan": ms_plan / ms_plan_mixed,
                      "class_flop_share": {cl: stm["class_flops"][i] / stm["useful_flops"]
                                           for i, cl in enumerate(("f64", "f32", "bf16c", "bf16"))}}}


def workloads_member(i):
    import workloads
    return workloads.c4_member(i)


def cpu_baseline(w, depth, nsample):
    """The oracle's modified-form apply on a seeded sample of output nodes of the same tree."""
    import numpy as np
    from oracle import apply as A
    from oracle import fit
    from oracle import tree as T
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    tr = T.redundant_tree(w.k, keys, coef)
    tau, wt = fit.fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
    op = A.Operator(w.k, tau, wt, w.eps, tr.depth)
    rng = np.random.Generator(np.random.PCG64(77))
    idx = np.sort(rng.choice(tr.keys.size, size=min(nsample, tr.keys.size), replace=False))
    cnt = _count_contractions(op.R, tr, idx)
    t0 = time.perf_counter()
    A.apply_modified(op, tr, idx)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": cnt / dt, "unit": "block-contractions/s", "cores": threads, "kind": "oracle",
            "sample": "%d of %d output nodes (seed 77), %d contractions in %.1f s; plain C, OpenMP over nodes"
                      % (idx.size, tr.keys.size, cnt, dt)}


def _count_contractions(R, tr, idx):
    """(node, l, m) triples with a non-zero coefficient for the given nodes (the apply's rule:
    c_m = [m in R_j(L)] - [internal][m in R_{j+1}(l)]), counted from the plan."""
    import numpy as np
    e = np.arange(-7, 8)
    E1, E2, E3 = np.meshgrid(e, e, e, indexing="ij")
    nlev = R.shape[0]
    total = 0
    for i in idx:
        j = int(tr.level[i])
        l = tr.l[i]
        side = 1 << j
        q = [l[0] - E1, l[1] - E2, l[2] - E3]
        inside = np.ones(E1.shape, dtype=bool)
        for d in range(3):
            inside &= (q[d] >= 0) & (q[d] < side)
        L = [(l[d] >> 1) - (np.clip(q[d], 0, None) >> 1) for d in range(3)]
        inL = (np.abs(L[0]) <= 3) & (np.abs(L[1]) <= 3) & (np.abs(L[2]) <= 3)
        Lc = [np.clip(L[d], -3, 3) + 3 for d in range(3)]
        rw = R[j][Lc[0], Lc[1], Lc[2]]
        a1 = np.where(inL, rw[..., 0], 0)
        b1 = np.where(inL, rw[..., 1], -1)
        a2 = np.zeros_like(a1)
        b2 = np.full_like(b1, -1)
        if tr.leaf[i] == 0 and j + 1 < nlev:
            inl = (np.abs(E1) <= 3) & (np.abs(E2) <= 3) & (np.abs(E3) <= 3)
            rd = R[j + 1][np.clip(E1, -3, 3) + 3, np.clip(E2, -3, 3) + 3, np.clip(E3, -3, 3) + 3]
            a2 = np.where(inl, rd[..., 0], 0)
            b2 = np.where(inl, rd[..., 1], -1)
        n1 = np.maximum(0, b1 - a1 + 1)
        n2 = np.maximum(0, b2 - a2 + 1)
        ov = np.where((n1 > 0) & (n2 > 0), np.maximum(0, np.minimum(b1, b2) - np.maximum(a1, a2) + 1), 0)
        total += int(np.sum(np.where(inside, n1 + n2 - 2 * ov, 0)))
    return total


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_0706_0747_amd as M
    import workloads
    w = workloads.c2() if args.workload == "c2" else workloads.c3()
    pts = workloads.points(10000)
    ctx = M.Context(0)
    M.mwns_ctx_set_variant(ctx, w.k, args.variant)
    for _ in range(args.warmup):
        step(M, ctx, w, pts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats_all = []
    for _ in range(args.steps):
        g, stats, depth, _, f, op = step(M, ctx, w, pts, M.MWNS_TIMES_ONLY)
        stats_all.append(stats)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    # the plan's contraction count and ||g|| (the same for every step) from one untimed apply
    g, st = M.mwns_apply(ctx, op, f)
    info = M.mwns_tree_get_info(g)
    contr = st["contractions"]
    ms_con = sum(s["ms_contract"] for s in stats_all) / len(stats_all)
    ms_clo = sum(s["ms_closure"] for s in stats_all) / len(stats_all)
    ms_asm = sum(s["ms_assemble"] for s in stats_all) / len(stats_all)
    achieved = st["useful_flops"] / (ms_con * 1e-3) / 1e12
    line = {
        "metric": "NS apply block-contractions/s + FP64-MFMA util; mixed-vs-FP64 speedup at eps",
        "value": contr / (ms_step * 1e-3),
        "unit": "block-contractions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name,
                   "kernel": "poisson 1/(4 pi r)" if w.mu == 0.0 else "yukawa exp(-mu r)/(4 pi r), mu=%.4f" % w.mu,
                   "k": w.k, "eps": w.eps,
                   "sources": int(w.a.size), "seed": w.seed, "leaves": int(info["nleaves"]),
                   "nodes": int(info["nnodes"]), "depth": int(info["depth"]), "eval_points": int(pts.shape[0])},
        "contractions_per_step": int(contr),
        "apply_contractions_per_s": contr / ((ms_clo + ms_con + ms_asm) * 1e-3),
        "apply_ms": {"closure": ms_clo, "contract": ms_con, "assemble": ms_asm},
        "mixed_vs_fp64_speedup": None,
        "mixed": None,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic_from_profile(args.workload),
                     "traffic_unit": "bytes per launch",
                     "kernel": ("ns_apply_kernel<8> (all levels of one apply)" if w.k <= 8 else
                                "ns_apply_wide_kernel<%d> (all levels of one apply)" % w.k),
                     "variant": M.mwns_ctx_get_variant(ctx, w.k),
                     "flops_per_apply": st["useful_flops"]},
    }
    if not args.no_mixed:
        line["mixed_vs_fp64_speedup"], line["mixed"] = mixed_measurement(M, ctx, w, f, op, g, st, args.steps, ms_con)
    if not args.no_batch:
        line["batch"] = batch_measurement(M, ctx, args.steps)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, info["depth"], args.cpu_sample_nodes)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
