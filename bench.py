"""Benchmark of the modified ns-form operator apply on one MI355X.

A step is one pass of the whole path on the large single apply (Poisson, k = 10, eps = 1e-10,
500 seeded Gaussians, about 9e5 leaves): Gaussian-sum fit (host FP64), operator build (1-D
blocks and screening plan, device), adaptive projection to a redundant tree (device), the FP64
apply (neighbour closure, FP64-MFMA contractions, assembly; device) and evaluation at 1e4
points.  The printed JSON line reports NS-apply block-contractions per second of step time, the
roofline of the contraction kernel (FP64 MFMA; the method's own flops over the kernel's HIP-event
time), the precision-routed apply against the FP64 one on the same tree at tol = eps ||g||
("mixed"), and the CPU oracle timed on a bounded sample with the same operator.  Beside it
("extra"): the Poisson k = 8 and bound-state Helmholtz k = 10 workloads; the batch of 64 uneven
solves (1e3 to 2e5 leaves each) applied one by one, as one persistent batched launch and as
replays of a captured plan; the 1-D cotangent operator of Sec. 2.4 ("cot1d"); Alg. 3 in two
dimensions ("ns2d").  Accuracy against
closed forms is asserted by the GPU tests.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5|c2|c3]
                    [--no-cpu-baseline] [--no-mixed] [--no-extra] [--no-batch]
"""
import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (matrix and vector)
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E
METRIC = "NS apply block-contractions/s + FP64-MFMA util; mixed-vs-FP64 speedup at eps"

# Sec. 6.1, Table 2 of the paper: the 3-D Poisson test (rho = -Laplacian of three Gaussians,
# alpha = 300) on one Pentium-4 at 2.8 GHz with 2 GB of RAM; the rate counts nodes x p^3 per second
PAPER_TABLE2 = {
    "hardware": "one Pentium-4 at 2.8 GHz, 2 GB RAM (precision and compiler not stated)",
    "workload": "3-D Poisson, rho = -Laplacian(sum of 3 Gaussians, alpha = 300), exact answer known",
    "rows": [{"eps": 1e-3, "p": 6, "E2": 5.0e-3, "Einf": 7.9e-1, "time_s": 1.2, "rate_pts_per_s": 7.2e4},
             {"eps": 1e-3, "p": 8, "E2": 1.7e-3, "Einf": 1.2e-1, "time_s": 0.51, "rate_pts_per_s": 7.3e4},
             {"eps": 1e-3, "p": 10, "E2": 4.4e-4, "Einf": 3.7e-2, "time_s": 0.68, "rate_pts_per_s": 1.1e5},
             {"eps": 1e-6, "p": 10, "E2": 4.7e-6, "Einf": 3.6e-4, "time_s": 10.3, "rate_pts_per_s": 5.7e4},
             {"eps": 1e-6, "p": 12, "E2": 8.5e-6, "Einf": 4.3e-5, "time_s": 13.5, "rate_pts_per_s": 7.5e4},
             {"eps": 1e-6, "p": 14, "E2": 6.9e-8, "Einf": 5.2e-6, "time_s": 20.0, "rate_pts_per_s": 8.0e4},
             {"eps": 1e-9, "p": 16, "E2": 2.5e-10, "Einf": 2.2e-8, "time_s": 68.1, "rate_pts_per_s": 3.5e4},
             {"eps": 1e-9, "p": 18, "E2": 7.7e-11, "Einf": 3.5e-9, "time_s": 100.3, "rate_pts_per_s": 3.4e4},
             {"eps": 1e-9, "p": 20, "E2": 1.2e-10, "Einf": 1.8e-8, "time_s": 133.4, "rate_pts_per_s": 3.5e4}],
    "note": "context only: other hardware and era; the paper prints no apply-only time, flop rate or GPU figure",
}


def progress(msg):
    """A line on stderr as each part of the run ends (the JSON line alone goes to stdout)."""
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["c5", "c2", "c3"], default="c5",
                    help="c5: Poisson k=10 eps=1e-10, 500 Gaussians (the reported configuration); "
                         "c2: Poisson k=8 eps=1e-6; c3: Yukawa k=10 eps=1e-8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-vs-FP64 measurement")
    ap.add_argument("--no-extra", action="store_true", help="skip the c2/c3 extra workloads")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-apply measurement")
    ap.add_argument("--cpu-sample-nodes", type=int, default=3000)
    ap.add_argument("--variant", type=int, default=-1, help="contraction-kernel tile variant (-1: library default)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 256 MiB elementwise copy (reference for the FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--ns2d-only", action="store_true",
                    help="only the 2-D section (--steps applies per case); prints its JSON")
    ap.add_argument("--hydrogen-only", action="store_true",
                    help="only the hydrogen section; prints its JSON")
    ap.add_argument("--hydrogen-cfg", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cot1d-only", action="store_true",
                    help="only the 1-D cotangent section (--steps applies per case); prints its JSON")
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


PROFILES = {"c5": ("ns_apply_wide_kernel_poisson_k10_eps1e-10.md", "contract_wide.hip"),
            "c2": ("ns_apply_kernel_poisson_k8_eps1e-6.md", "contract.hip"),
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


def leaf_norm(leaf, coef, chunk=1 << 16):
    import numpy as np
    idx = np.nonzero(leaf == 1)[0]
    tot = 0.0
    for i in range(0, idx.size, chunk):
        tot += float(np.sum(coef[idx[i:i + chunk]] ** 2))
    return math.sqrt(tot)


def measure(M, ctx, w, steps, warmup, pts):
    """Timed steps of the whole path on workload w; the figures of one FP64 apply."""
    import torch
    for _ in range(warmup):
        step(M, ctx, w, pts)
    torch.cuda.synchronize()
    progress("%s: %d warm-up steps done" % (w.name, warmup))
    t0 = time.perf_counter()
    stats_all = []
    for _ in range(steps):
        g, stats, depth, _, f, op = step(M, ctx, w, pts, M.MWNS_TIMES_ONLY)
        stats_all.append(stats)
        del g
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / steps
    progress("%s: %d timed steps, %.1f ms per step" % (w.name, steps, 1e3 * dt / steps))
    # the plan's contraction count and ||g|| (the same for every step) from one untimed apply
    g, st = M.mwns_apply(ctx, op, f)
    info = M.mwns_tree_get_info(g)
    avg = lambda key: sum(s[key] for s in stats_all) / len(stats_all)
    ms_con, ms_clo, ms_asm = avg("ms_contract"), avg("ms_closure"), avg("ms_assemble")
    own = st["own_flops"] / (ms_con * 1e-3) / 1e12
    executed = st["useful_flops"] / (ms_con * 1e-3) / 1e12
    kernel = ("ns_apply_kernel<%d> (all levels of one apply)" % w.k if w.k <= 8 else
              "ns_apply_wide_kernel<%d> (all levels of one apply)" % w.k)
    out = {
        "ms_per_step": ms_step, "contractions_per_step": int(st["contractions"]),
        "value": st["contractions"] / (ms_step * 1e-3),
        "config": {"workload": w.name,
                   "kernel": "poisson 1/(4 pi r)" if w.mu == 0.0 else "yukawa exp(-mu r)/(4 pi r), mu=%.4f" % w.mu,
                   "k": w.k, "eps": w.eps, "sources": int(w.a.size), "seed": w.seed,
                   "leaves": int(info["nleaves"]), "nodes": int(info["nnodes"]), "depth": int(info["depth"]),
                   "terms": int(op.M), "eval_points": int(pts.shape[0])},
        "apply_contractions_per_s": st["contractions"] / ((ms_clo + ms_con + ms_asm) * 1e-3),
        "apply_ms": {"closure": ms_clo, "contract": ms_con, "assemble": ms_asm},
        "roofline": {"bound": "mfma", "achieved": own, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": own / PEAK_FP64_TFLOPS, "traffic": None, "traffic_unit": "bytes per launch",
                     "kernel": kernel, "variant": M.mwns_ctx_get_variant(ctx, w.k),
                     "own_flops_per_apply": st["own_flops"],
                     "executed_flops_per_apply": st["useful_flops"],
                     "executed_tflops": executed,
                     "f64_mfma_flops_per_apply": st["f64_mfma_flops"],
                     "flops": "own: the factorised contraction flops 2 (2k)^4 (n1 n2 n3 + n1 n2 + n1) of every "
                              "(sibling group, term, box of displacements) job, padding excluded, without the "
                              "down-band jobs whose terms the whole band holds at every displacement of their box; "
                              "executed: with them; f64_mfma: what the matrix cores issue, tile padding included"},
    }
    return out, (g, st, f, op)


def mixed_measurement(M, ctx, w, f, op, g64, st64, reps, ms_con64):
    """Apply-only wall time of the FP64 and the precision-routed apply on the same tree and
    operator, the latter at tol = eps ||g_F64||; the measured relative L2 error against FP64."""
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
    b -= a
    err = leaf_norm(leaf, b)
    del a, b
    return times["fp64"] / times["mixed"], {
        "tol_rel": w.eps, "err_rel_measured": err / st64["g_norm"], "err_rel_bound": stm["err_bound"] / st64["g_norm"],
        "apply_ms_fp64": times["fp64"], "apply_ms_mixed": times["mixed"], "reps": reps,
        "contract_ms_fp64": ms_con64, "contract_ms_mixed": stm["ms_contract"],
        "class_flop_share": {c: stm["class_flops"][i] / stm["useful_flops"]
                             for i, c in enumerate(("f64", "f32", "bf16c", "bf16"))},
        "classes": "FP64 MFMA; FP32 MFMA; BF16 MFMA on hi/lo splits (4 partial products); BF16 MFMA"}


PAPER_TABLE1 = {"source": "Sec. 2.4.2, Table 1: the cotangent operator on a periodized Gaussian (a = 300)",
                "rows": [{"p": 5, "eps": 1e-3, "scales": [2, 3, 4], "nblocks": 8, "E2": 1.5e-4},
                         {"p": 8, "eps": 1e-6, "scales": [2, 4, 5], "nblocks": 12, "E2": 1.3e-7},
                         {"p": 11, "eps": 1e-9, "scales": [2, 4, 5], "nblocks": 14, "E2": 1.1e-10},
                         {"p": 14, "eps": 1e-12, "scales": [3, 4, 5], "nblocks": 16, "E2": 4.4e-13}]}


def cot1d_measurement(M, ctx, reps):
    """The 1-D cotangent operator (Sec. 2.4, Alg. 2) on Table 1's inputs and on a larger seeded sum
    of periodized Gaussians: tree sizes, the apply's wall time (output tree, input gathering,
    contraction, assembly; host work included) and the contraction kernel's device time.  Its
    accuracy against the closed form (Table 1's E2) is checked by the GPU tests."""
    import numpy as np
    import torch
    import workloads
    cases = [workloads.cot1d_example(r["p"], r["eps"]) for r in PAPER_TABLE1["rows"]] + [workloads.cot1d_many()]
    out = []
    for w in cases:
        f = M.mwns_cot1d_project(ctx, w.k, w.thr, w.j0, w.jmax, w.centers, w.exps, w.weights)
        keys, leaf, _ = M.mwns_cot1d_export(ctx, f)
        depth = int((keys >> np.uint64(57)).max())
        op = M.mwns_cot1d_op_create(ctx, w.k, w.eps, depth)
        g, ms_con = M.mwns_cot1d_apply(ctx, op, f)
        torch.cuda.synchronize()
        con = []
        t0 = time.perf_counter()
        for _ in range(reps):
            g, ms_con = M.mwns_cot1d_apply(ctx, op, f)
            con.append(ms_con)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        gk, gl, _ = M.mwns_cot1d_export(ctx, g)
        kms = float(np.median(con))
        # algorithmic bytes of the contraction launch: each output block's input block read once and
        # the output block written once (k doubles each)
        alg = 2.0 * gk.size * w.k * 8
        out.append({"workload": w.name, "k": w.k, "eps": w.eps, "depth": depth, "input_leaves": int(leaf.sum()),
                    "input_nodes": int(keys.size), "output_leaves": int(gl.sum()), "output_nodes": int(gk.size),
                    "bands": [int(b) for b in M.mwns_cot1d_op_bands(op)], "apply_ms": ms,
                    "contract_kernel_ms": kms,
                    "roofline": {"bound": "hbm", "achieved": alg / (kms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                                 "unit": "GB/s", "frac": alg / (kms * 1e-3) / 1e9 / PEAK_HBM_GBS, "traffic": None,
                                 "algorithmic_bytes_per_launch": alg}})
    return {"cases": out, "paper_table1": PAPER_TABLE1,
            "note": "launch- and latency-bound at these sizes (tens to thousands of blocks of k doubles): the roofline "
                    "fractions are far below 1; E2 against the closed form is asserted in tests/test_gpu_cot1d.py"}


def ns2d_measurement(M, ctx, reps):
    """Alg. 3 in two dimensions on two seeded inputs (the 2-D analogue of the k = 8 workload, and a
    larger one): the library's fit, operator, projection and apply; tree sizes, the apply's wall time
    and the contraction kernel's device time and FP64 rate (vector FMAs: 4 k^3 flops per (node, l,
    term))."""
    import numpy as np
    import torch
    import workloads
    out = []
    for w in (workloads.ns2d(), workloads.ns2d(seed=3, n=400, log10_hi=5.0)):
        f = M.mwns_project2d(ctx, w.k, w.eps, w.j0, w.jmax, w.xy, w.a, w.c)
        keys, leaf, _ = M.mwns_tree2d_export(ctx, f)
        depth = int((keys >> np.uint64(57)).max())
        tau, wt = M.mwns_fit_kernel2d(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(2.0))
        op = M.mwns_op2d_create(ctx, w.k, tau, wt, w.eps, depth)
        g, ms_con, fl = M.mwns_apply2d(ctx, op, f)
        torch.cuda.synchronize()
        con = []
        t0 = time.perf_counter()
        for _ in range(reps):
            g, ms_con, fl = M.mwns_apply2d(ctx, op, f)
            con.append(ms_con)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        kms = float(np.median(con))
        ach = fl / (kms * 1e-3) / 1e12
        out.append({"workload": w.name, "k": w.k, "eps": w.eps, "mu": w.mu, "leaves": int(leaf.sum()), "nodes": int(keys.size),
                    "depth": depth, "terms": int(tau.size), "apply_ms": ms, "contract_kernel_ms": kms,
                    "flops_per_apply": fl,
                    "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                 "frac": ach / PEAK_FP64_TFLOPS, "traffic": None}})
    return {"cases": out, "note": "accuracy against the fitted kernel in closed form and node-by-node parity with the "
                                  "d = 2 oracle are asserted in tests/test_gpu_ns2d.py"}


HYDROGEN = dict(k=10, eps=1e-6, L=16.0, jmax=15, mu0=0.8, iters=14)
HYDROGEN_SMALL = dict(k=5, eps=1e-3, L=10.0, jmax=7, mu0=0.8, iters=2)


def hydrogen_measurement(M, ctx, cfg=None):
    """Sec. 6.2's iteration in the library at the paper's requested accuracy 1e-6 (the figure of the
    iteration's convergence): |E + 1/2| after each step, rho's leaves, the device time of each apply
    and the wall time of the whole call (fit, operator, apply, discard, products, inner products)."""
    import torch
    c = dict(HYDROGEN if cfg is None else cfg)
    M.mwns_hydrogen_kalos(ctx, c["k"], c["eps"], c["L"], c["jmax"], mu0=c["mu0"], iters=1)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist, leaves, ms = M.mwns_hydrogen_kalos(ctx, c["k"], c["eps"], c["L"], c["jmax"], mu0=c["mu0"], iters=c["iters"])
    wall = time.perf_counter() - t0
    sm = dict(HYDROGEN_SMALL)
    t1 = time.perf_counter()
    M.mwns_hydrogen_kalos(ctx, sm["k"], sm["eps"], sm["L"], sm["jmax"], mu0=sm["mu0"], iters=sm["iters"])
    small = time.perf_counter() - t1
    # the dominant kernel: the contraction of the first step's apply (the largest rho), rebuilt from the
    # public entry points as the iteration builds it (projection, product, fit, operator)
    s = 2.0 * c["L"]
    a = s * s
    phi = M.mwns_project_gaussians(ctx, c["k"], c["eps"], 2, c["jmax"], [[0.5, 0.5, 0.5]], [a],
                                   [(2.0 / math.pi) ** 0.75 * (math.pi / a) ** 1.5])
    nphi = math.sqrt(s ** 3 * M.mwns_tree_dot(ctx, phi, phi))
    rho = M.mwns_tree_coulomb_product(ctx, phi, 2.0 / nphi, s, c["jmax"])
    info = M.mwns_tree_get_info(rho)
    tau, wt = M.mwns_fit_kernel(c["mu0"] * s, 1.0, c["eps"], math.sqrt(c["eps"]) * 2.0 ** -info["depth"], math.sqrt(3.0),
                                scale=s * s)
    op = M.mwns_op_create(ctx, c["k"], tau, wt, c["eps"], info["depth"])
    con = []
    for _ in range(5):
        g, st = M.mwns_apply(ctx, op, rho, M.MWNS_TIMES_ONLY)
        con.append(st["ms_contract"])
        del g
    kms = float(sorted(con)[len(con) // 2])
    ach = st["own_flops"] / (kms * 1e-3) / 1e12
    first = {"rho_leaves": int(info["nleaves"]), "rho_depth": int(info["depth"]), "terms": int(tau.size),
             "contract_kernel_ms": kms, "own_flops_per_apply": st["own_flops"],
             "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                          "frac": ach / PEAK_FP64_TFLOPS, "traffic": None}}
    return {"config": c, "mu": [m for m, _ in hist], "E": [e for _, e in hist], "E_error": [abs(e + 0.5) for _, e in hist],
            "rho_leaves": leaves, "apply_device_ms": ms, "wall_s": wall, "wall_ms_per_step": 1e3 * wall / c["iters"],
            "first_step_apply": first,
            "small": {"config": sm, "wall_s": small},
            "note": "the exact ground-state energy is -1/2; parity of mu, E and the trees with the oracle is asserted in "
                    "tests/test_gpu_hydrogen.py"}


def hydrogen_oracle_time():
    """The oracle's iteration (numpy) on the small hydrogen configuration, the whole call timed."""
    from oracle import hydrogen as H
    sm = dict(HYDROGEN_SMALL)
    t0 = time.perf_counter()
    H.kalos(sm["k"], sm["eps"], sm["L"], sm["jmax"], mu0=sm["mu0"], iters=sm["iters"])
    return {"config": sm, "wall_s": time.perf_counter() - t0, "cores": 1, "kind": "oracle (numpy, one process)"}


def ns2d_oracle_time():
    """The d = 2 oracle's apply (numpy, modified form, then assembly) on the first 2-D input: its own
    tree, fit and plan; the apply timed alone."""
    import numpy as np
    from oracle import mra
    from oracle import ns2d as N
    import workloads
    w = workloads.ns2d()
    tr = N.project2d(w.k, w.eps, w.j0, w.jmax, w.xy, w.a, w.c)
    tau, wt = N.fit_kernel2d(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -tr.depth, math.sqrt(2.0))
    F = mra.F_table(w.k, tau, tr.depth)
    H0, H1 = mra.two_scale_filters(w.k)
    R, _ = N.make_plan2d(F, H0, H1, wt, w.eps, tr.depth)
    t0 = time.perf_counter()
    N.assemble2d(tr, N.apply_modified2d(tr, F, wt, R))
    dt = time.perf_counter() - t0
    return {"workload": w.name, "nodes": int(tr.keys.size), "apply_s": dt, "cores": 1, "kind": "oracle (numpy, one process)"}


def cot1d_oracle_time(reps=1):
    """The oracle's 1-D apply (modified form on the output tree, then assembly) on the larger 1-D
    input: its own tree, blocks, bands and output tree, the apply timed alone."""
    from oracle import cot1d as C
    import workloads
    w = workloads.cot1d_many()
    tr = C.project_periodic(w.k, w.thr, w.j0, w.jmax, w.centers, w.exps, w.weights)
    R = C.cot_table(w.k, tr.depth, lmax=65)
    B = C.choose_bands(w.k, R, w.eps)
    sk = C.skeleton(tr, B)
    t0 = time.perf_counter()
    for _ in range(reps):
        C.assemble(sk, C.apply_modified(tr, R, B, sk))
    dt = (time.perf_counter() - t0) / reps
    return {"workload": w.name, "output_leaves": int(sk.leaf.sum()), "apply_s": dt, "cores": 1,
            "kind": "oracle (numpy, one process)"}


def batch_measurement(M, ctx, reps, nmembers=64):
    """The batch of uneven solves (seeded members of mixed kernels, k and eps): total contractions
    per second for sequential single applies, one batched persistent apply, and replays of the
    captured apply plan, in FP64 and precision-routed at tol = eps ||g|| per member."""
    import torch
    import workloads
    members = [workloads.c4_member(i) for i in range(nmembers)]
    ops, fs = [], []
    for w in members:
        f = M.mwns_project_gaussians(ctx, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
        depth = M.mwns_tree_get_info(f)["depth"]
        tau, wt = M.mwns_fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
        ops.append(M.mwns_op_create(ctx, w.k, tau, wt, w.eps, depth))
        fs.append(f)
    tuned = {}
    for k in sorted({int(w.k) for w in members}):   # the autotuner's pick per basis order
        i = next(i for i, w in enumerate(members) if w.k == k)
        tuned[k] = M.autotune(ctx, ops[i], fs[i])
    _, st = M.mwns_apply_batch(ctx, ops, fs)
    plan = M.mwns_plan_create(ctx, ops, fs)
    tols = [w.eps * M.mwns_apply(ctx, op, f)[1]["g_norm"] for w, op, f in zip(members, ops, fs)]
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
    leaves = [int(M.mwns_tree_get_info(f)["nleaves"]) for f in fs]
    nodes = sum(M.mwns_tree_get_info(f)["nnodes"] for f in fs)
    c = st["contractions"]
    return {"members": len(members), "orders": sorted({int(w.k) for w in members}), "nodes": int(nodes),
            "leaves_per_member": leaves, "leaves_min": min(leaves), "leaves_max": max(leaves),
            "tuned_variant_per_k": {str(k): v for k, v in tuned.items()},
            "contractions": int(c), "ms_sequential": ms_seq, "ms_batch": ms_batch, "ms_plan_replay": ms_plan,
            "contractions_per_s_sequential": c / (ms_seq * 1e-3), "contractions_per_s_batch": c / (ms_batch * 1e-3),
            "contractions_per_s_plan": c / (ms_plan * 1e-3),
            "own_tflops_batch": st["own_flops"] / (ms_batch * 1e-3) / 1e12,
            "mixed": {"tol": "eps ||g|| per member", "ms_batch": ms_batch_mixed, "ms_plan_replay": ms_plan_mixed,
                      "speedup_batch": ms_batch / ms_batch_mixed, "speedup_plan": ms_plan / ms_plan_mixed,
                      "class_flop_share": {cl: stm["class_flops"][i] / stm["useful_flops"]
                                           for i, cl in enumerate(("f64", "f32", "bf16c", "bf16"))}}}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sample_setup(w, depth, nsub):
    """The oracle's operator for workload w (its own fit at the workload's depth) and its tree of the
    first nsub source Gaussians (a tree the oracle builds in seconds; the per-node work of the apply
    depends on the order, the operator and the plan, which are the workload's)."""
    from oracle import apply as A
    from oracle import fit
    from oracle import tree as T
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz[:nsub], w.a[:nsub], w.c[:nsub])
    tr = T.redundant_tree(w.k, keys, coef)
    tau, wt = fit.fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
    op = A.Operator(w.k, tau, wt, w.eps, max(depth, tr.depth))
    return tr, op


def _oracle_rate(tr, op, nsample, seed):
    import numpy as np
    from oracle import apply as A
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = np.sort(rng.choice(tr.keys.size, size=min(nsample, tr.keys.size), replace=False))
    cnt = _count_contractions(op.R, tr, idx)
    t0 = time.perf_counter()
    A.apply_modified(op, tr, idx)
    dt = time.perf_counter() - t0
    return cnt, dt, idx.size


def cpu_baseline(w, depth, nsample, nsub=6):
    """The oracle's modified-form apply (plain C, OpenMP over output nodes) with workload w's operator
    on a seeded sample of output nodes, on all host threads and, in a child process, on one."""
    tr, op = _oracle_sample_setup(w, depth, nsub)
    progress("oracle tree and operator for the CPU baseline built")
    cnt, dt, n = _oracle_rate(tr, op, nsample, 77)
    progress("CPU baseline on all threads done (%.1f s)" % dt)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    one = None
    try:
        env = dict(os.environ, OMP_NUM_THREADS="1")
        res = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--workload",
                              w.get("key", "c5")], env=env, capture_output=True, text=True, timeout=300)
        one = json.loads(res.stdout.strip().splitlines()[-1])
    except Exception as e:     # the one-thread figure is context; report why it is missing
        one = {"error": repr(e)[:200]}
    return {"value": cnt / dt, "unit": "block-contractions/s", "cores": threads, "kind": "oracle",
            "cpu_model": _cpu_model(), "one_thread": one,
            "sample": "%d of %d output nodes (seed 77) of the oracle's tree of the first %d of the %d source Gaussians "
                      "(%d leaves), with the workload's operator (k=%d, eps=%g, %d terms, its own plan); %d "
                      "contractions in %.1f s; plain C, OpenMP over nodes"
                      % (n, tr.keys.size, nsub, w.a.size, int(tr.leaf.sum()), w.k, w.eps, op.M, cnt, dt)}


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


def _workload(name):
    import workloads
    w = getattr(workloads, name)()
    w["key"] = name
    return w


def cpu_baseline_only(args):
    """Child process of cpu_baseline: the one-thread rate (OMP_NUM_THREADS=1 set by the parent) on a
    smaller sample of the same nodes."""
    w = _workload(args.workload)
    depth = {"c5": 11, "c2": 8, "c3": 8}[args.workload]
    tr, op = _oracle_sample_setup(w, depth, 6)
    cnt, dt, n = _oracle_rate(tr, op, max(20, args.cpu_sample_nodes // 16), 77)
    print(json.dumps({"value": cnt / dt, "unit": "block-contractions/s", "cores": 1,
                      "sample": "%d output nodes, %d contractions in %.1f s" % (n, cnt, dt)}))


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.cpu_baseline_only:
        cpu_baseline_only(args)
        return
    if args.cot1d_only:
        import paper_0706_0747_amd as M
        print(json.dumps(cot1d_measurement(M, M.Context(0), args.steps)))
        return
    if args.hydrogen_only:
        import paper_0706_0747_amd as M
        cfg = json.loads(args.hydrogen_cfg) if args.hydrogen_cfg else None
        print(json.dumps(hydrogen_measurement(M, M.Context(0), cfg)))
        return
    if args.ns2d_only:
        import paper_0706_0747_amd as M
        print(json.dumps(ns2d_measurement(M, M.Context(0), args.steps)))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import paper_0706_0747_amd as M
    import workloads
    w = _workload(args.workload)
    pts = workloads.points(10000)
    ctx = M.Context(0)
    M.mwns_ctx_set_variant(ctx, w.k, args.variant)
    head, (g, st, f, op) = measure(M, ctx, w, args.steps, args.warmup, pts)
    head["roofline"]["traffic"] = traffic_from_profile(args.workload)
    line = {
        "metric": METRIC,
        "value": head.pop("value"),
        "unit": "block-contractions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": head.pop("config"),
        "roofline": head.pop("roofline"),
    }
    line.update(head)
    line["mixed_vs_fp64_speedup"], line["mixed"] = None, None
    if not args.no_mixed:
        reps = min(args.steps, 3) if w.k > 8 else args.steps
        line["mixed_vs_fp64_speedup"], line["mixed"] = mixed_measurement(
            M, ctx, w, f, op, g, st, reps, line["apply_ms"]["contract"])
        progress("mixed-vs-FP64 measurement done")
    del g
    ctx.release_cache()
    line["paper_table2"] = PAPER_TABLE2
    if not args.no_extra:
        line["extra"] = {}
        for name in ("c2", "c3"):
            if name == args.workload:
                continue
            wx = _workload(name)
            M.mwns_ctx_set_variant(ctx, wx.k, -1)
            ex, (gx, stx, fx, opx) = measure(M, ctx, wx, max(args.steps, 5), 2, pts)
            ex["roofline"]["traffic"] = traffic_from_profile(name)
            if not args.no_mixed:
                ex["mixed_vs_fp64_speedup"], ex["mixed"] = mixed_measurement(
                    M, ctx, wx, fx, opx, gx, stx, max(args.steps, 5), ex["apply_ms"]["contract"])
            line["extra"][name] = ex
            progress("extra workload %s done" % name)
            del gx
        ctx.release_cache()
    if not args.no_batch:
        line["batch"] = batch_measurement(M, ctx, min(args.steps, 5))
        progress("batch done")
    line["cot1d"] = cot1d_measurement(M, ctx, 5)
    progress("1-D cotangent operator done")
    line["ns2d"] = ns2d_measurement(M, ctx, 5)
    progress("2-D apply done")
    line["hydrogen"] = hydrogen_measurement(M, ctx)
    progress("hydrogen iteration done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, line["config"]["depth"], args.cpu_sample_nodes)
        line["cpu_baseline"]["cot1d"] = cot1d_oracle_time()
        progress("1-D oracle timed")
        line["cpu_baseline"]["ns2d"] = ns2d_oracle_time()
        progress("2-D oracle timed")
        line["cpu_baseline"]["hydrogen"] = hydrogen_oracle_time()
        progress("hydrogen oracle timed")
    print(json.dumps(line))


if __name__ == "__main__":
    main()
