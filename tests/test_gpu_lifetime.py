"""Handle lifetimes: trees, operators and plans keep their context alive, so they may be
destroyed after the context handle (as Python's garbage collector may do at interpreter exit or
when a traceback holds them)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import gc, math, sys
sys.path.insert(0, %r)
import torch
import paper_0706_0747_amd as M
import workloads
w = workloads.small_adaptive(8, k=6, eps=1e-4, jmax=5)
c = M.Context(0)
f = M.mwns_project_gaussians(c, w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
depth = M.mwns_tree_get_info(f)["depth"]
tau, wt = M.mwns_fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -depth, math.sqrt(3))
op = M.mwns_op_create(c, w.k, tau, wt, w.eps, depth)
g, _ = M.mwns_apply(c, op, f)
gm, _ = M.mwns_apply_mixed(c, op, f, 1e-6)
plan = M.mwns_plan_create(c, [op], [f])
plan.execute()
torch.cuda.synchronize()
out = plan.output(0)
c.close()                      # the handle goes first; the objects below still hold the context
del out
for o in (plan, gm, g, op, f):
    o.close()
gc.collect()
print("clean", flush=True)
"""


def test_objects_destroyed_after_their_context():
    res = subprocess.run([sys.executable, "-c", SCRIPT % ROOT], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    assert "clean" in res.stdout
    assert "corrupted" not in res.stderr and "double free" not in res.stderr
