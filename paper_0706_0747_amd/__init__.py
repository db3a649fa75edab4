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
from ._lib import (MWNS_CLASS_BF16, MWNS_CLASS_BF16C, MWNS_CLASS_F32, MWNS_F64, MWNS_NO_ASSEMBLY, MwnsError, check,
                   lib)

__all__ = ["Context", "Operator", "Tree", "MwnsError", "MWNS_F64", "MWNS_NO_ASSEMBLY", "MWNS_CLASS_F32",
           "MWNS_CLASS_BF16C", "MWNS_CLASS_BF16", "mwns_apply_mixed", "mwns_ctx_create", "mwns_num_variants", "mwns_ctx_set_variant",
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
                torch.cuda.caching_allocator_delete(ptr)

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


def mwns_ctx_create(device=0, use_torch=True, byte_budget=0):
    return Context(device, use_torch, byte_budget)


def mwns_num_variants():
    return lib.mwns_num_variants()


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


def mwns_op_create(ctx, k, tau, w, eps, max_level, group_regions=1):
    tau, w = _f64(tau), _f64(w)
    opts = _lib.OpOpts(int(group_regions))
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


def mwns_apply_mixed(ctx, op, f, tol, classes=MWNS_CLASS_F32 | MWNS_CLASS_BF16C | MWNS_CLASS_BF16, flags=0, stats=True):
    """g = T f with contractions routed to FP64 / FP32 / BF16 so that ||g - g_F64||_2 <= tol;
    returns (g, stats dict or None)."""
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
