"""Host code and the oracle's C core built with AddressSanitizer and UndefinedBehaviorSanitizer and
run on the CPU (no device call): every out-of-bounds access, use after free, signed overflow or
misaligned load in them aborts the run.  The drivers live in tests/sanitize/."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
# sanitizers on the host side only: device code is not instrumented
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), res.stdout[-4000:], res.stderr[-4000:])
    return res


def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    csrc = os.path.join(ROOT, "paper_0706_0747_amd", "csrc")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + HOST_SAN
    objs = []
    for src in (os.path.join(csrc, "fit.hip"), os.path.join(csrc, "host_common.hip"), os.path.join(SAN, "host_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([hipcc] + flags + ["-c", src, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "host_driver")
    _run([hipcc, "--offload-arch=gfx950"] + HOST_SAN + objs + ["-o", exe])
    res = _run([exe], env=ENV)
    assert "host driver: ok" in res.stdout


def test_oracle_core_under_sanitizers(tmp_path):
    import math
    from oracle import apply as A
    from oracle import fit, mra
    from oracle import tree as T
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    _run([gcc, "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "ns_core.c"), os.path.join(SAN, "oracle_driver.c"),
          "-lm", "-o", exe])
    w = workloads.small_adaptive(11, k=4, eps=1e-3, jmax=4)
    keys, coef = T.project_gaussians(w.k, w.eps, w.j0, w.jmax, w.xyz, w.a, w.c)
    tr = T.redundant_tree(w.k, keys, coef)
    tau, wt = fit.fit_kernel(w.mu, w.alpha, w.eps, math.sqrt(w.eps) * 2.0 ** -tr.depth, math.sqrt(3))
    op = A.Operator(w.k, tau, wt, w.eps, tr.depth)
    out_idx = np.arange(tr.keys.size, dtype=np.int64)
    boxes = T.children_keys(tr.keys[(tr.level == 1)][:2])
    a = np.ascontiguousarray(w.a, dtype=np.float64)
    cf = np.asarray(w.c) * (a / np.pi) ** 1.5
    gx, gw = mra.gauss_legendre01(w.k)
    thr = w.eps * T.source_norm(w.xyz, w.a, w.c)
    inp = str(tmp_path / "case.bin")
    with open(inp, "wb") as fh:
        np.array([w.k, op.F.shape[0], op.R.shape[0], op.M], dtype=np.int32).tofile(fh)
        np.array([tr.keys.size, out_idx.size, boxes.size, a.size, 2], dtype=np.int64).tofile(fh)
        for arr, dt in ((tr.keys, np.uint64), (tr.leaf, np.uint8), (tr.coef, np.float64), (op.w, np.float64),
                        (op.F, np.float64), (op.R, np.int32), (op.H0, np.float64), (op.H1, np.float64),
                        (out_idx, np.int64), (boxes, np.uint64), (w.xyz, np.float64), (a, np.float64),
                        (cf, np.float64), (np.array([thr]), np.float64), (gx, np.float64), (gw, np.float64)):
            np.ascontiguousarray(arr, dtype=dt).tofile(fh)
    outp = str(tmp_path / "out.bin")
    _run([exe, inp, outp], env=ENV)
    k3 = w.k ** 3
    raw = open(outp, "rb").read()
    n = out_idx.size * k3
    g1 = np.frombuffer(raw, np.float64, n, 0).reshape(-1, w.k, w.k, w.k)
    g2 = np.frombuffer(raw, np.float64, n, 8 * n).reshape(-1, w.k, w.k, w.k)
    s = np.frombuffer(raw, np.float64, boxes.size * k3, 16 * n).reshape(-1, w.k, w.k, w.k)
    ref1, ref2 = A.apply_modified(op, tr), A.apply_difference(op, tr)
    assert np.abs(g1 - ref1).max() <= 1e-14 * np.abs(ref1).max()
    assert np.abs(g2 - ref2).max() <= 1e-14 * np.abs(ref2).max()
    sref, _, _ = T.project_boxes(w.k, w.eps, 19, w.xyz, w.a, w.c, boxes)
    assert np.abs(s - sref).max() <= 1e-14 * np.abs(sref).max()
