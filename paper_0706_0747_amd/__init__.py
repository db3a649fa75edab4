"""MI355X-native modified non-standard-form operator apply (Beylkin, Cheruvu, Perez).

Thin Python binding of the C ABI in include/mwns.h.  The functions carry the C names and only
marshal arguments (numpy arrays for host data); every step runs in libmwns.so.  PyTorch supplies
the HIP stream and, through the allocator callbacks, the device memory.

    ctx = Context()                                         # mwns_ctx_create on torch's stream
    tau, w = mwns_fit_kernel(mu, alpha, eps, delta, R)      # (1) fit
    op = mwns_op_create(ctx, k, tau, w, eps, max_level)     # (2) operator
    f = mwns_project_gaussians(ctx, k, eps, j0, jmax, xyz, a, c)   # (3) project
    g, stats = mwns_apply(ctx, op, f)                       # (4) apply (FP64)
    g, stats = mwns_apply_mixed(ctx, op, f, tol)            #     or precision-routed, ||g - g_F64|| <= tol
    vals = mwns_tree_eval(ctx, g, pts)                      # (5) evaluate
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import (MWNS_CLASS_BF16, MWNS_CLASS_BF16C, MWNS_CLASS_F32, MWNS_F64, MWNS_NO_ASSEMBLY, MWNS_TIMES_ONLY, MwnsError, check,
                   lib)

__all__ = ["mwns_abi_version", "Context", "Operator", "Tree", "MwnsError", "MWNS_F64", "MWNS_NO_ASSEMBLY", "MWNS_TIMES_ONLY", "MWNS_CLASS_F32",
           "MWNS_CLASS_BF16C", "MWNS_CLASS_BF16", "mwns_apply_mixed", "default_classes", "mwns_tree_detail_norms", "mwns_tree_prune",
           "mwns_tree_discard", "Op1", "Tree1", "mwns_cot1d_op_create", "mwns_cot1d_op_bands", "mwns_cot1d_op_set_bands",
           "mwns_cot1d_op_blocks", "mwns_cot1d_project", "mwns_cot1d_from_leaves", "mwns_cot1d_apply", "mwns_cot1d_export",
           "mwns_cot1d_eval", "Op2", "Tree2", "mwns_fit_kernel2d", "mwns_op2d_create", "mwns_op2d_plan_export",
           "mwns_op2d_plan_import", "mwns_project2d", "mwns_tree2d_from_leaves", "mwns_apply2d", "mwns_tree2d_export",
           "mwns_tree_coulomb_product", "mwns_tree_dot", "mwns_hydrogen_kalos",
           "mwns_tree2d_eval",
           "mwns_apply_batch", "Plan", "mwns_plan_create", "mwns_tree_set_leaves",
           "mwns_tune_apply", "autotune", "mwns_ctx_create", "mwns_num_variants", "mwns_num_variants_for", "mwns_variant_shape", "mwns_ctx_set_variant",
           "mwns_ctx_get_variant",
           "mwns_fit_kernel", "mwns_op_create", "mwns_op_plan_export", "mwns_op_plan_import",
           "mwns_op_tables_export", "mwns_project_gaussians", "mwns_tree_from_leaves", "mwns_tree_export",
           "mwns_tree_get_info", "mwns_apply", "mwns_tree_eval", "LIB_PATH"]

LIB_PATH = _lib.LIB_PATH


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Context:
    """mwns_ctx on torch's current HIP stream with torch's caching allocator (use_torch=True), or
    on the null stream with hipMalloc (use_torch=False)."""

    def __init__(self, device=0, use_torch=True, byte_budget=0):
        self._keep = []
        self.device = device
        stream = None
        alloc = _lib.ALLOC_FN()
        free = _lib.FREE_FN()
        if use_torch:
            import torch
            torch.cuda.set_device(device)
            s = torch.cuda.current_stream(device)
            stream = s.cuda_stream

            def _alloc(nbytes, user):
                return torch.cuda.caching_allocator_alloc(int(nbytes), device, s)

            def _free(ptr, user):
                try:
                    torch.cuda.caching_allocator_delete(ptr)
                except (AttributeError, TypeError):
                    pass            # interpreter shutdown: torch is already gone

            alloc = _lib.ALLOC_FN(_alloc)
            free = _lib.FREE_FN(_free)
            self._keep = [alloc, free, s]
        h = ctypes.c_void_p()
        check(lib.mwns_ctx_create(device, stream, alloc, free, None, byte_budget, ctypes.byref(h)), "mwns_ctx_create")
        self.h = h

    def synchronize(self):
        check(lib.mwns_ctx_synchronize(self.h), "mwns_ctx_synchronize")

    def bytes_in_use(self):
        return lib.mwns_ctx_bytes_in_use(self.h)

    def bytes_cached(self):
        return lib.mwns_ctx_bytes_cached(self.h)

    def release_cache(self):
        check(lib.mwns_ctx_release_cache(self.h), "mwns_ctx_release_cache")

    def close(self, _destroy=lib.mwns_ctx_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Operator:
    def __init__(self, ctx, h, k, M, max_level):
        self.ctx, self.h, self.k, self.M, self.max_level = ctx, h, k, M, max_level

    @property
    def threshold(self):
        return lib.mwns_op_threshold(self.h)

    def close(self, _destroy=lib.mwns_op_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Tree:
    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h

    def close(self, _destroy=lib.mwns_tree_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class BorrowedTree:
    """A tree handle owned by something else (a plan's output): never destroyed from here."""

    def __init__(self, ctx, h, owner):
        self.ctx, self.h, self._owner = ctx, h, owner

    def close(self):
        pass


class Plan:
    """mwns_plan: a batched apply captured once as a hipGraph and replayed by execute()."""

    def __init__(self, ctx, h, n, keep):
        self.ctx, self.h, self.n, self._keep = ctx, h, n, keep

    def execute(self):
        check(lib.mwns_plan_execute(self.h), "mwns_plan_execute")

    def output(self, i):
        g = ctypes.c_void_p()
        check(lib.mwns_plan_output(self.h, i, ctypes.byref(g)), "mwns_plan_output")
        return BorrowedTree(self.ctx, g, self)

    def stats(self):
        st = _lib.ApplyStats()
        check(lib.mwns_plan_stats(self.h, ctypes.byref(st)), "mwns_plan_stats")
        return _stats_dict(st)

    def close(self, _destroy=lib.mwns_plan_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def _handles(objs):
    arr = (ctypes.c_void_p * len(objs))()
    for i, o in enumerate(objs):
        arr[i] = o.h.value if isinstance(o.h, ctypes.c_void_p) else o.h
    return arr


def default_classes(k):
    """Every reduced class the kernels have for order k: FP32 and both BF16 classes for k <= 8,
    FP32 alone above (the whole-brick kernel of k = 9, 10 has no BF16 class)."""
    return MWNS_CLASS_F32 | MWNS_CLASS_BF16C | MWNS_CLASS_BF16 if k <= 8 else MWNS_CLASS_F32


def _mixed_array(mixed, fs):
    if mixed is None:
        return None
    n = len(fs)
    if isinstance(mixed, (int, float)):
        mixed = [mixed] * n
    arr = (_lib.MixedOpts * n)()
    for i, m in enumerate(mixed):
        tol, classes = (m, None) if isinstance(m, (int, float)) else m
        if classes is None:
            classes = default_classes(mwns_tree_get_info(fs[i])["k"])
        arr[i] = _lib.MixedOpts(float(tol), int(classes))
    return arr


def mwns_apply_batch(ctx, ops, fs, mixed=None, flags=0, stats=True):
    """Batched apply of the pairs (ops[i], fs[i]) in one persistent launch per basis order.
    mixed: None (FP64), a tol for every tree, or a list of tol or (tol, classes) per tree (classes
    None: default_classes of the tree's k).  Returns (list of Trees, aggregated stats or None)."""
    n = len(ops)
    if len(fs) != n:
        raise ValueError("ops and fs differ in length")
    gs = (ctypes.c_void_p * n)()
    st = _lib.ApplyStats()
    mx = _mixed_array(mixed, fs)
    check(lib.mwns_apply_batch(ctx.h, n, _handles(ops), _handles(fs), mx, flags, gs,
                               ctypes.byref(st) if stats else None), "mwns_apply_batch")
    return [Tree(ctx, ctypes.c_void_p(gs[i])) for i in range(n)], (_stats_dict(st) if stats else None)


def mwns_plan_create(ctx, ops, fs, mixed=None, flags=0):
    n = len(ops)
    if len(fs) != n:
        raise ValueError("ops and fs differ in length")
    h = ctypes.c_void_p()
    mx = _mixed_array(mixed, fs)
    check(lib.mwns_plan_create(ctx.h, n, _handles(ops), _handles(fs), mx, flags, ctypes.byref(h)), "mwns_plan_create")
    return Plan(ctx, h, n, (list(ops), list(fs)))


def mwns_tree_set_leaves(ctx, tree, coeffs):
    """Replace the leaf coefficients (canonical leaf order, [nleaves, k, k, k]) in place."""
    info = mwns_tree_get_info(tree)
    k = info["k"]
    coeffs = _f64(coeffs, (info["nleaves"], k, k, k))
    check(lib.mwns_tree_set_leaves(ctx.h, tree.h, coeffs.ctypes.data), "mwns_tree_set_leaves")


def mwns_tune_apply(ctx, op, f, reps=3):
    """Times every tile variant on this apply, selects the fastest for f's k; returns (best, ms[])."""
    best = ctypes.c_int(0)
    t = np.zeros(mwns_num_variants_for(mwns_tree_get_info(f)["k"]))
    check(lib.mwns_tune_apply(ctx.h, op.h, f.h, reps, ctypes.byref(best), t.ctypes.data), "mwns_tune_apply")
    return best.value, t


def autotune(ctx, op, f, cache_path=None, reps=3):
    """Tile variant for f's k: read from the JSON cache at cache_path (keyed by device and k) when
    present, else measured with mwns_tune_apply and written there.  The choice is set on ctx."""
    import json
    import os
    import torch
    k = mwns_tree_get_info(f)["k"]
    key = "%s/k%d" % (torch.cuda.get_device_name(ctx_device(ctx)), k)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    if key in cache and 0 <= int(cache[key]) < mwns_num_variants_for(k):
        mwns_ctx_set_variant(ctx, k, int(cache[key]))
        return int(cache[key])
    best, _ = mwns_tune_apply(ctx, op, f, reps)
    if cache_path:
        cache[key] = best
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return best


def ctx_device(ctx):
    return ctx.device


def mwns_ctx_create(device=0, use_torch=True, byte_budget=0):
    return Context(device, use_torch, byte_budget)


def mwns_abi_version():
    """The version of the C interface and of the array layouts it exports."""
    return int(lib.mwns_abi_version())


def mwns_num_variants():
    return lib.mwns_num_variants()


def mwns_num_variants_for(k):
    return lib.mwns_num_variants_for(k)


def mwns_variant_shape(v):
    """(waves per workgroup, prefetch depth, waves per SIMD, FP64 terms per pass) of variant v."""
    out = [ctypes.c_int() for _ in range(4)]
    check(lib.mwns_variant_shape(v, *[ctypes.byref(o) for o in out]), "mwns_variant_shape")
    return tuple(o.value for o in out)


def mwns_ctx_set_variant(ctx, k, variant):
    check(lib.mwns_ctx_set_variant(ctx.h, k, variant), "mwns_ctx_set_variant")


def mwns_ctx_get_variant(ctx, k):
    v = ctypes.c_int(0)
    check(lib.mwns_ctx_get_variant(ctx.h, k, ctypes.byref(v)), "mwns_ctx_get_variant")
    return v.value


def mwns_fit_kernel(mu, alpha, eps, delta, R, scale=1.0, cap=4096):
    """(tau, w) of the Gaussian-sum fit (host FP64 in the library)."""
    M = ctypes.c_int(0)
    tau = np.zeros(cap)
    w = np.zeros(cap)
    check(lib.mwns_fit_kernel(mu, alpha, scale, eps, delta, R, cap, ctypes.byref(M), tau.ctypes.data, w.ctypes.data),
          "mwns_fit_kernel")
    return tau[:M.value].copy(), w[:M.value].copy()


def mwns_op_create(ctx, k, tau, w, eps, max_level, group_regions=1, allow_band_overflow=0):
    tau, w = _f64(tau), _f64(w)
    opts = _lib.OpOpts(int(group_regions), int(allow_band_overflow))
    h = ctypes.c_void_p()
    check(lib.mwns_op_create(ctx.h, k, tau.size, tau.ctypes.data, w.ctypes.data, eps, max_level, ctypes.byref(opts),
                             ctypes.byref(h)), "mwns_op_create")
    return Operator(ctx, h, k, tau.size, max_level)


def mwns_op_plan_export(op):
    n = ctypes.c_size_t(0)
    check(lib.mwns_op_plan_export(op.h, None, ctypes.byref(n)), "mwns_op_plan_export")
    plan = np.zeros(n.value, dtype=np.int32)
    check(lib.mwns_op_plan_export(op.h, plan.ctypes.data, ctypes.byref(n)), "mwns_op_plan_export")
    return plan.reshape(op.max_level + 1, 7, 7, 7, 2)


def mwns_op_plan_import(op, plan):
    plan = np.ascontiguousarray(plan, dtype=np.int32).ravel()
    check(lib.mwns_op_plan_import(op.h, plan.ctypes.data, plan.size), "mwns_op_plan_import")


def mwns_op_tables_export(ctx, op):
    n = ctypes.c_size_t(0)
    check(lib.mwns_op_tables_export(ctx.h, op.h, None, ctypes.byref(n)), "mwns_op_tables_export")
    F = np.zeros(n.value)
    check(lib.mwns_op_tables_export(ctx.h, op.h, F.ctypes.data, ctypes.byref(n)), "mwns_op_tables_export")
    return F.reshape(op.max_level + 1, op.M, 15, op.k, op.k)


def mwns_project_gaussians(ctx, k, eps, j0, jmax, xyz, a, c):
    xyz = _f64(xyz, (-1, 3))
    a, c = _f64(a), _f64(c)
    h = ctypes.c_void_p()
    check(lib.mwns_project_gaussians(ctx.h, k, eps, j0, jmax, a.size, xyz.ctypes.data, a.ctypes.data, c.ctypes.data,
                                     ctypes.byref(h)), "mwns_project_gaussians")
    return Tree(ctx, h)


def mwns_tree_from_leaves(ctx, k, keys, coeffs):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    coeffs = _f64(coeffs, (keys.size, k, k, k))
    h = ctypes.c_void_p()
    check(lib.mwns_tree_from_leaves(ctx.h, k, keys.size, keys.ctypes.data, coeffs.ctypes.data, ctypes.byref(h)),
          "mwns_tree_from_leaves")
    return Tree(ctx, h)


def mwns_tree_get_info(tree):
    info = _lib.TreeInfo()
    check(lib.mwns_tree_get_info(tree.h, ctypes.byref(info)), "mwns_tree_get_info")
    return {f: getattr(info, f) for f, _ in _lib.TreeInfo._fields_}


def mwns_tree_export(ctx, tree, coeffs=True):
    """(keys, is_leaf, coeffs[N, k, k, k]) in canonical order."""
    n = ctypes.c_int64(0)
    check(lib.mwns_tree_export(ctx.h, tree.h, ctypes.byref(n), None, None, None), "mwns_tree_export")
    k = mwns_tree_get_info(tree)["k"]
    keys = np.zeros(n.value, dtype=np.uint64)
    leaf = np.zeros(n.value, dtype=np.uint8)
    coef = np.zeros((n.value, k, k, k)) if coeffs else None
    check(lib.mwns_tree_export(ctx.h, tree.h, ctypes.byref(n), keys.ctypes.data, leaf.ctypes.data,
                               coef.ctypes.data if coeffs else None), "mwns_tree_export")
    return keys, leaf, coef


def mwns_apply(ctx, op, f, mode=MWNS_F64, stats=True):
    """g = T f; returns (g, stats dict or None)."""
    h = ctypes.c_void_p()
    st = _lib.ApplyStats()
    check(lib.mwns_apply(ctx.h, op.h, f.h, mode, ctypes.byref(h), ctypes.byref(st) if stats else None), "mwns_apply")
    return Tree(ctx, h), (_stats_dict(st) if stats else None)


def _stats_dict(st):
    out = {}
    for fld, _ in _lib.ApplyStats._fields_:
        v = getattr(st, fld)
        out[fld] = list(v) if fld == "class_flops" else v
    return out


def mwns_apply_mixed(ctx, op, f, tol, classes=None, flags=0, stats=True):
    """g = T f with contractions routed to FP64 / FP32 / BF16 so that ||g - g_F64||_2 <= tol
    (classes None: default_classes of f's k); returns (g, stats dict or None)."""
    if classes is None:
        classes = default_classes(mwns_tree_get_info(f)["k"])
    h = ctypes.c_void_p()
    st = _lib.ApplyStats()
    opts = _lib.MixedOpts(float(tol), int(classes))
    check(lib.mwns_apply_mixed(ctx.h, op.h, f.h, ctypes.byref(opts), flags, ctypes.byref(h),
                               ctypes.byref(st) if stats else None), "mwns_apply_mixed")
    return Tree(ctx, h), (_stats_dict(st) if stats else None)


def mwns_tree_eval(ctx, tree, pts):
    pts = _f64(pts, (-1, 3))
    out = np.zeros(pts.shape[0])
    check(lib.mwns_tree_eval(ctx.h, tree.h, pts.shape[0], pts.ctypes.data, out.ctypes.data), "mwns_tree_eval")
    return out


def mwns_tree_eval_noalloc(ctx, tree, npts, xyz_dev, out_dev):
    """Values of tree at npts points on the device: xyz_dev and out_dev are device addresses (ints,
    e.g. torch tensors' data_ptr()) of npts x 3 and npts doubles; nothing is allocated, copied or
    waited for (the values are ready when the context's stream passes the call)."""
    check(lib.mwns_tree_eval_noalloc(ctx.h, tree.h, int(npts), ctypes.c_void_p(int(xyz_dev)), ctypes.c_void_p(int(out_dev))),
          "mwns_tree_eval_noalloc")


def mwns_tree_detail_norms(ctx, tree):
    """Squared detail norm of every node in canonical order (0 at leaves)."""
    out = np.zeros(mwns_tree_get_info(tree)["nnodes"])
    check(lib.mwns_tree_detail_norms(ctx.h, tree.h, out.ctypes.data), "mwns_tree_detail_norms")
    return out


def mwns_tree_prune(ctx, tree, eta):
    """l2 pruning within eta (absolute); returns (pruned Tree, removed squared norm)."""
    h = ctypes.c_void_p()
    removed = ctypes.c_double()
    check(lib.mwns_tree_prune(ctx.h, tree.h, float(eta), ctypes.byref(h), ctypes.byref(removed)), "mwns_tree_prune")
    return Tree(ctx, h), removed.value


def mwns_tree_discard(ctx, tree, eps):
    """Alg. 3 Step 4: pruning within eps ||tree||_2; returns (pruned Tree, removed squared norm)."""
    h = ctypes.c_void_p()
    removed = ctypes.c_double()
    check(lib.mwns_tree_discard(ctx.h, tree.h, float(eps), ctypes.byref(h), ctypes.byref(removed)), "mwns_tree_discard")
    return Tree(ctx, h), removed.value


# ---- the 1-D cotangent operator (Sec. 2.4, Alg. 2) ---------------------------------------------


class Op1:
    def __init__(self, ctx, h, k, max_level):
        self.ctx, self.h, self.k, self.max_level = ctx, h, k, max_level

    def close(self, _destroy=lib.mwns_cot1d_op_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Tree1:
    def __init__(self, ctx, h, k):
        self.ctx, self.h, self.k = ctx, h, k

    def close(self, _destroy=lib.mwns_tree1_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def mwns_cot1d_op_create(ctx, k, eps, max_level):
    h = ctypes.c_void_p()
    check(lib.mwns_cot1d_op_create(ctx.h, int(k), float(eps), int(max_level), ctypes.byref(h)), "mwns_cot1d_op_create")
    return Op1(ctx, h, int(k), int(max_level))


def mwns_cot1d_op_bands(op):
    n = ctypes.c_int(0)
    check(lib.mwns_cot1d_op_bands(op.h, None, ctypes.byref(n)), "mwns_cot1d_op_bands")
    out = np.zeros(n.value, dtype=np.int32)
    check(lib.mwns_cot1d_op_bands(op.h, out.ctypes.data, ctypes.byref(n)), "mwns_cot1d_op_bands")
    return out


def mwns_cot1d_op_set_bands(op, bands):
    b = np.ascontiguousarray(bands, dtype=np.int32)
    check(lib.mwns_cot1d_op_set_bands(op.h, b.ctypes.data, int(b.size)), "mwns_cot1d_op_set_bands")


def mwns_cot1d_op_blocks(ctx, op):
    """R[max_level + 1][131][k][k] for l = -65..65."""
    n = ctypes.c_size_t(0)
    check(lib.mwns_cot1d_op_blocks(ctx.h, op.h, None, ctypes.byref(n)), "mwns_cot1d_op_blocks")
    out = np.zeros(n.value)
    check(lib.mwns_cot1d_op_blocks(ctx.h, op.h, out.ctypes.data, ctypes.byref(n)), "mwns_cot1d_op_blocks")
    return out.reshape(op.max_level + 1, 131, op.k, op.k)


def mwns_cot1d_project(ctx, k, thr, j0, jmax, centers, exps, weights):
    c = np.ascontiguousarray(centers, dtype=np.float64)
    a = np.ascontiguousarray(exps, dtype=np.float64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    h = ctypes.c_void_p()
    check(lib.mwns_cot1d_project(ctx.h, int(k), float(thr), int(j0), int(jmax), int(c.size), c.ctypes.data,
                                 a.ctypes.data, w.ctypes.data, ctypes.byref(h)), "mwns_cot1d_project")
    return Tree1(ctx, h, int(k))


def mwns_cot1d_from_leaves(ctx, k, keys, coeffs):
    kk = np.ascontiguousarray(keys, dtype=np.uint64)
    cc = np.ascontiguousarray(coeffs, dtype=np.float64)
    h = ctypes.c_void_p()
    check(lib.mwns_cot1d_from_leaves(ctx.h, int(k), int(kk.size), kk.ctypes.data, cc.ctypes.data, ctypes.byref(h)),
          "mwns_cot1d_from_leaves")
    return Tree1(ctx, h, int(k))


def mwns_cot1d_apply(ctx, op, f):
    """(g, device ms of the contraction kernel)."""
    h = ctypes.c_void_p()
    ms = ctypes.c_double()
    check(lib.mwns_cot1d_apply(ctx.h, op.h, f.h, ctypes.byref(h), ctypes.byref(ms)), "mwns_cot1d_apply")
    return Tree1(ctx, h, f.k), ms.value


def mwns_cot1d_export(ctx, t):
    """(keys, is_leaf, coeffs[N, k]) in key order."""
    n = ctypes.c_int64(0)
    check(lib.mwns_cot1d_export(ctx.h, t.h, ctypes.byref(n), None, None, None), "mwns_cot1d_export")
    keys = np.zeros(n.value, dtype=np.uint64)
    leaf = np.zeros(n.value, dtype=np.uint8)
    coef = np.zeros((n.value, t.k))
    check(lib.mwns_cot1d_export(ctx.h, t.h, ctypes.byref(n), keys.ctypes.data, leaf.ctypes.data, coef.ctypes.data),
          "mwns_cot1d_export")
    return keys, leaf, coef


def mwns_cot1d_eval(ctx, t, x):
    xx = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(xx.size)
    check(lib.mwns_cot1d_eval(ctx.h, t.h, int(xx.size), xx.ctypes.data, out.ctypes.data), "mwns_cot1d_eval")
    return out


# ---- Alg. 3 in two dimensions ------------------------------------------------------------------


class Op2:
    def __init__(self, ctx, h, k, M, max_level):
        self.ctx, self.h, self.k, self.M, self.max_level = ctx, h, k, M, max_level

    def close(self, _destroy=lib.mwns_op2d_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Tree2:
    def __init__(self, ctx, h, k):
        self.ctx, self.h, self.k = ctx, h, k

    def close(self, _destroy=lib.mwns_tree2d_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def mwns_fit_kernel2d(mu, alpha, eps, delta, R):
    n = ctypes.c_int(0)
    check(lib.mwns_fit_kernel2d(float(mu), float(alpha), float(eps), float(delta), float(R), 0, ctypes.byref(n), None,
                                None), "mwns_fit_kernel2d")
    tau = np.zeros(n.value)
    w = np.zeros(n.value)
    check(lib.mwns_fit_kernel2d(float(mu), float(alpha), float(eps), float(delta), float(R), n.value, ctypes.byref(n),
                                tau.ctypes.data, w.ctypes.data), "mwns_fit_kernel2d")
    return tau, w


def mwns_op2d_create(ctx, k, tau, w, eps, max_level, allow_band_overflow=False):
    t = np.ascontiguousarray(tau, dtype=np.float64)
    ww = np.ascontiguousarray(w, dtype=np.float64)
    h = ctypes.c_void_p()
    check(lib.mwns_op2d_create(ctx.h, int(k), int(t.size), t.ctypes.data, ww.ctypes.data, float(eps), int(max_level),
                               int(bool(allow_band_overflow)), ctypes.byref(h)), "mwns_op2d_create")
    return Op2(ctx, h, int(k), int(t.size), int(max_level))


def mwns_op2d_plan_export(op):
    n = ctypes.c_size_t(0)
    check(lib.mwns_op2d_plan_export(op.h, None, ctypes.byref(n)), "mwns_op2d_plan_export")
    out = np.zeros(n.value, dtype=np.int32)
    check(lib.mwns_op2d_plan_export(op.h, out.ctypes.data, ctypes.byref(n)), "mwns_op2d_plan_export")
    return out.reshape(op.max_level + 1, 7, 7, 2)


def mwns_op2d_plan_import(op, plan):
    p = np.ascontiguousarray(plan, dtype=np.int32)
    check(lib.mwns_op2d_plan_import(op.h, p.ctypes.data, int(p.size)), "mwns_op2d_plan_import")


def mwns_project2d(ctx, k, eps, j0, jmax, xy, a, c):
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    h = ctypes.c_void_p()
    check(lib.mwns_project2d(ctx.h, int(k), float(eps), int(j0), int(jmax), int(a.size), xy.ctypes.data, a.ctypes.data,
                             c.ctypes.data, ctypes.byref(h)), "mwns_project2d")
    return Tree2(ctx, h, int(k))


def mwns_tree2d_from_leaves(ctx, k, keys, coeffs):
    kk = np.ascontiguousarray(keys, dtype=np.uint64)
    cc = np.ascontiguousarray(coeffs, dtype=np.float64)
    h = ctypes.c_void_p()
    check(lib.mwns_tree2d_from_leaves(ctx.h, int(k), int(kk.size), kk.ctypes.data, cc.ctypes.data, ctypes.byref(h)),
          "mwns_tree2d_from_leaves")
    return Tree2(ctx, h, int(k))


def mwns_apply2d(ctx, op, f):
    """(g, device ms of the contraction kernel, flops)."""
    h = ctypes.c_void_p()
    ms = ctypes.c_double()
    fl = ctypes.c_double()
    check(lib.mwns_apply2d(ctx.h, op.h, f.h, ctypes.byref(h), ctypes.byref(ms), ctypes.byref(fl)), "mwns_apply2d")
    return Tree2(ctx, h, f.k), ms.value, fl.value


def mwns_tree2d_export(ctx, t):
    n = ctypes.c_int64(0)
    check(lib.mwns_tree2d_export(ctx.h, t.h, ctypes.byref(n), None, None, None), "mwns_tree2d_export")
    keys = np.zeros(n.value, dtype=np.uint64)
    leaf = np.zeros(n.value, dtype=np.uint8)
    coef = np.zeros((n.value, t.k, t.k))
    check(lib.mwns_tree2d_export(ctx.h, t.h, ctypes.byref(n), keys.ctypes.data, leaf.ctypes.data, coef.ctypes.data),
          "mwns_tree2d_export")
    return keys, leaf, coef


def mwns_tree2d_eval(ctx, t, pts):
    p = np.ascontiguousarray(pts, dtype=np.float64)
    out = np.zeros(p.shape[0])
    check(lib.mwns_tree2d_eval(ctx.h, t.h, int(p.shape[0]), p.ctypes.data, out.ctypes.data), "mwns_tree2d_eval")
    return out


# ---- the hydrogen ground state (Sec. 6.2) --------------------------------------------------------


def mwns_tree_coulomb_product(ctx, f, c, s, jmax):
    """rho = c / (s |x - 1/2|) * f on f's tree refined once and, at the centre, down to jmax."""
    h = ctypes.c_void_p()
    check(lib.mwns_tree_coulomb_product(ctx.h, f.h, float(c), float(s), int(jmax), ctypes.byref(h)),
          "mwns_tree_coulomb_product")
    return Tree(ctx, h)


def mwns_tree_dot(ctx, u, v):
    """<u, v> over the unit cube from u's leaves and v's blocks of the same boxes."""
    out = ctypes.c_double()
    check(lib.mwns_tree_dot(ctx.h, u.h, v.h, ctypes.byref(out)), "mwns_tree_dot")
    return out.value


def mwns_hydrogen_kalos(ctx, k, eps, L, jmax, mu0=1.0, iters=6, Z=1.0, j0=2):
    """The iteration of Sec. 6.2: ([(mu, E) per step], rho's leaves per step, device ms of each apply)."""
    mu = np.zeros(iters)
    E = np.zeros(iters)
    nl = np.zeros(iters, dtype=np.int64)
    ms = np.zeros(iters)
    check(lib.mwns_hydrogen_kalos(ctx.h, int(k), float(eps), float(L), int(jmax), float(mu0), float(Z), int(j0),
                                  int(iters), mu.ctypes.data, E.ctypes.data, nl.ctypes.data, ms.ctypes.data),
          "mwns_hydrogen_kalos")
    return list(zip(mu.tolist(), E.tolist())), nl.tolist(), ms.tolist()
