"""Calibrates the batch members' Gaussian counts (writes c4_sizes.json beside this file).

For member i, the count n of leading Gaussians of c4_draw(i)'s pool is searched so that the
oracle's adaptive projection (Alg. 1) gives a tree whose leaf count is within 25% of the member's
target, or as close as the search gets in a few trees; the counts it found are recorded with the
leaf counts.  Only the oracle builds trees here.

    python workloads/calibrate_c4.py [first last]
    python workloads/calibrate_c4.py --estimate [first last]

The oracle's projection of the largest members (k = 10, 1e5-2e5 leaves, a few hundred Gaussians)
takes about half an hour per tree; --estimate records for every member not yet searched the count
extrapolated from the searched members of the same order (log n linear in log leaves, least
squares over those with at least 2e4 leaves), marked "estimated" with no leaf count; a later plain
run searches those members and replaces the estimates.
"""
import json
import math
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import workloads                       # noqa: E402
from oracle import tree as T           # noqa: E402


def leaves(d, n):
    keys, _ = T.project_gaussians(d.k, d.eps, d.j0, d.jmax, d.xyz[:n], d.a[:n], d.c[:n])
    return int(keys.size)


def calibrate(i, done, tries=6, tol=math.log(1.25)):
    """Searches n for member i; `done` holds the members calibrated so far (the nearest one of the
    same order gives the first guess)."""
    d = workloads.c4_draw(i)
    seen = {}
    same = [r for r in done.values() if r["k"] == d.k]
    if same:
        ref = min(same, key=lambda r: abs(math.log(r["target"] / d.target)))
        n = int(round(ref["n"] * (d.target / ref["leaves"]) ** 1.25))
    else:
        n = int(round(d.target / 300.0))
    n = max(1, min(workloads.C4_POOL, n))
    p = 0.8                                  # leaves ~ n^p, refined from the last two trees
    prev = None
    for _ in range(tries):
        if n in seen:
            break
        seen[n] = leaves(d, n)
        err = math.log(seen[n] / d.target)
        if abs(err) < tol:
            break
        if prev is not None and prev[0] != n and seen[n] != prev[1]:
            p = min(2.0, max(0.1, math.log(seen[n] / prev[1]) / math.log(n / prev[0])))
        prev = (n, seen[n])
        n = max(1, min(workloads.C4_POOL, int(round(n * math.exp(-err / p)))))
    best = min(seen, key=lambda m: abs(math.log(seen[m] / d.target)))
    return {"n": best, "leaves": seen[best], "target": d.target, "u": d.u, "k": d.k, "eps": d.eps}


def estimate(i, done):
    d = workloads.c4_draw(i)
    pts = [(math.log(r["leaves"]), math.log(r["n"])) for r in done.values()
           if r["k"] == d.k and not r.get("estimated") and r["leaves"] >= 2e4]
    x = [p[0] for p in pts]
    y = [p[1] for p in pts]
    mx, my = sum(x) / len(x), sum(y) / len(y)
    beta = sum((a - mx) * (b - my) for a, b in zip(x, y)) / sum((a - mx) ** 2 for a in x)
    n = int(round(math.exp(my + beta * (math.log(d.target) - mx))))
    return {"n": max(1, min(workloads.C4_POOL, n)), "leaves": None, "target": d.target, "u": d.u, "k": d.k,
            "eps": d.eps, "estimated": True}


def main():
    args = [a for a in sys.argv[1:] if a != "--estimate"]
    est = "--estimate" in sys.argv[1:]
    first, last = (int(args[0]), int(args[1])) if len(args) > 1 else (0, 63)
    out = {"pool": workloads.C4_POOL, "leaf_range": list(workloads.C4_LEAVES), "members": {}}
    if os.path.exists(workloads.C4_SIZES):
        with open(workloads.C4_SIZES) as fh:
            out = json.load(fh)
    if est:
        for i in range(first, last + 1):
            if str(i) not in out["members"]:
                out["members"][str(i)] = estimate(i, out["members"])
                print("member %2d estimated n %d" % (i, out["members"][str(i)]["n"]), flush=True)
        with open(workloads.C4_SIZES, "w") as fh:
            json.dump(out, fh, indent=1, sort_keys=True)
        return
    # cheap members first, so that an interrupted run keeps the most members
    order = sorted(range(first, last + 1), key=lambda i: workloads.c4_draw(i).target)
    for i in order:
        if str(i) in out["members"] and not out["members"][str(i)].get("estimated"):
            continue
        t0 = time.time()
        done = {kk: r for kk, r in out["members"].items() if not r.get("estimated")}
        res = calibrate(i, done)
        with open(workloads.C4_SIZES) as fh:      # the file may have gained entries meanwhile
            out = json.load(fh)
        out["members"][str(i)] = res
        r = out["members"][str(i)]
        print("member %2d k=%2d target %8.0f -> n %4d leaves %7d (%.0f s)"
              % (i, r["k"], r["target"], r["n"], r["leaves"], time.time() - t0), flush=True)
        with open(workloads.C4_SIZES + ".tmp", "w") as fh:
            json.dump(out, fh, indent=1, sort_keys=True)
        os.replace(workloads.C4_SIZES + ".tmp", workloads.C4_SIZES)


if __name__ == "__main__":
    main()
