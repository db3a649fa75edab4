"""ctypes binding of libmwns.so: the C-ABI entry points under their C names, argument marshalling
only.  Every computation happens in the library's HIP kernels (or, for the fit, its host FP64
code); nothing here falls back to Python or the CPU.  Importing fails loudly when the shared
library has not been built."""
import ctypes
import os

try:
    # The binding runs libmwns on the HIP runtime that PyTorch-ROCm loads (its streams and memory
    # are torch's): import torch first so that the library binds to that runtime.
    import torch  # noqa: F401
except ImportError:
    pass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmwns.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libmwns.so is not built (run `python paper_0706_0747_amd/build.py`); "
                      "there is no fallback for the MI355X kernels")

lib = ctypes.CDLL(LIB_PATH)

c_int, c_i64, c_dbl, c_size, c_vp = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
P = ctypes.POINTER

MWNS_OK, MWNS_EINVAL, MWNS_ENOMEM, MWNS_EDEVICE, MWNS_ERANGE, MWNS_ESTATE = range(6)
MWNS_F64 = 0
MWNS_NO_ASSEMBLY = 1 << 8
MWNS_TIMES_ONLY = 1 << 9
MWNS_CLASS_F32, MWNS_CLASS_BF16C, MWNS_CLASS_BF16 = 1, 2, 4
STATUS_NAMES = {0: "MWNS_OK", 1: "MWNS_EINVAL", 2: "MWNS_ENOMEM", 3: "MWNS_EDEVICE", 4: "MWNS_ERANGE", 5: "MWNS_ESTATE"}

ALLOC_FN = ctypes.CFUNCTYPE(c_vp, c_size, c_vp)
FREE_FN = ctypes.CFUNCTYPE(None, c_vp, c_vp)


class OpOpts(ctypes.Structure):
    _fields_ = [("group_regions", c_int), ("allow_band_overflow", c_int)]


class TreeInfo(ctypes.Structure):
    _fields_ = [("k", c_int), ("depth", c_int), ("nnodes", c_i64), ("nleaves", c_i64),
                ("threshold", c_dbl), ("min_margin", c_dbl)]


class ApplyStats(ctypes.Structure):
    _fields_ = [("contractions", c_i64), ("brick_jobs", c_i64), ("ghost_bricks", c_i64), ("useful_flops", c_dbl),
                ("ms_closure", c_dbl), ("ms_contract", c_dbl), ("ms_assemble", c_dbl), ("err_bound", c_dbl),
                ("g_norm", c_dbl), ("class_flops", c_dbl * 4), ("own_flops", c_dbl), ("f64_mfma_flops", c_dbl)]


class MixedOpts(ctypes.Structure):
    _fields_ = [("tol", c_dbl), ("classes", c_int)]


SIGNATURES = {
    "mwns_ctx_create": (c_int, [c_int, c_vp, ALLOC_FN, FREE_FN, c_vp, c_size, P(c_vp)]),
    "mwns_ctx_destroy": (None, [c_vp]),
    "mwns_ctx_synchronize": (c_int, [c_vp]),
    "mwns_ctx_bytes_in_use": (c_size, [c_vp]),
    "mwns_ctx_bytes_cached": (c_size, [c_vp]),
    "mwns_ctx_release_cache": (c_int, [c_vp]),
    "mwns_last_error": (ctypes.c_char_p, []),
    "mwns_abi_version": (c_int, []),
    "mwns_num_variants": (c_int, []),
    "mwns_num_variants_for": (c_int, [c_int]),
    "mwns_variant_shape": (c_int, [c_int, P(c_int), P(c_int), P(c_int), P(c_int)]),
    "mwns_ctx_set_variant": (c_int, [c_vp, c_int, c_int]),
    "mwns_ctx_get_variant": (c_int, [c_vp, c_int, P(c_int)]),
    "mwns_fit_kernel": (c_int, [c_dbl, c_dbl, c_dbl, c_dbl, c_dbl, c_dbl, c_int, P(c_int), c_vp, c_vp]),
    "mwns_op_create": (c_int, [c_vp, c_int, c_int, c_vp, c_vp, c_dbl, c_int, P(OpOpts), P(c_vp)]),
    "mwns_op_plan_export": (c_int, [c_vp, c_vp, P(c_size)]),
    "mwns_op_plan_import": (c_int, [c_vp, c_vp, c_size]),
    "mwns_op_tables_export": (c_int, [c_vp, c_vp, c_vp, P(c_size)]),
    "mwns_op_threshold": (c_dbl, [c_vp]),
    "mwns_op_destroy": (None, [c_vp]),
    "mwns_project_gaussians": (c_int, [c_vp, c_int, c_dbl, c_int, c_int, c_int, c_vp, c_vp, c_vp, P(c_vp)]),
    "mwns_tree_from_leaves": (c_int, [c_vp, c_int, c_i64, c_vp, c_vp, P(c_vp)]),
    "mwns_tree_get_info": (c_int, [c_vp, P(TreeInfo)]),
    "mwns_tree_export": (c_int, [c_vp, c_vp, P(c_i64), c_vp, c_vp, c_vp]),
    "mwns_tree_destroy": (None, [c_vp]),
    "mwns_apply": (c_int, [c_vp, c_vp, c_vp, c_int, P(c_vp), P(ApplyStats)]),
    "mwns_apply_mixed": (c_int, [c_vp, c_vp, c_vp, P(MixedOpts), c_int, P(c_vp), P(ApplyStats)]),
    "mwns_apply_batch": (c_int, [c_vp, c_int, c_vp, c_vp, c_vp, c_int, c_vp, P(ApplyStats)]),
    "mwns_plan_create": (c_int, [c_vp, c_int, c_vp, c_vp, c_vp, c_int, P(c_vp)]),
    "mwns_plan_execute": (c_int, [c_vp]),
    "mwns_plan_output": (c_int, [c_vp, c_int, P(c_vp)]),
    "mwns_plan_stats": (c_int, [c_vp, P(ApplyStats)]),
    "mwns_plan_destroy": (None, [c_vp]),
    "mwns_tree_set_leaves": (c_int, [c_vp, c_vp, c_vp]),
    "mwns_tune_apply": (c_int, [c_vp, c_vp, c_vp, c_int, P(c_int), c_vp]),
    "mwns_tree_eval": (c_int, [c_vp, c_vp, c_i64, c_vp, c_vp]),
    "mwns_tree_eval_noalloc": (c_int, [c_vp, c_vp, c_i64, c_vp, c_vp]),
    "mwns_tree_detail_norms": (c_int, [c_vp, c_vp, c_vp]),
    "mwns_tree_prune": (c_int, [c_vp, c_vp, ctypes.c_double, P(c_vp), P(ctypes.c_double)]),
    "mwns_tree_discard": (c_int, [c_vp, c_vp, ctypes.c_double, P(c_vp), P(ctypes.c_double)]),
    "mwns_cot1d_op_create": (c_int, [c_vp, c_int, c_dbl, c_int, P(c_vp)]),
    "mwns_cot1d_op_bands": (c_int, [c_vp, c_vp, P(c_int)]),
    "mwns_cot1d_op_set_bands": (c_int, [c_vp, c_vp, c_int]),
    "mwns_cot1d_op_blocks": (c_int, [c_vp, c_vp, c_vp, P(c_size)]),
    "mwns_cot1d_op_destroy": (None, [c_vp]),
    "mwns_cot1d_project": (c_int, [c_vp, c_int, c_dbl, c_int, c_int, c_int, c_vp, c_vp, c_vp, P(c_vp)]),
    "mwns_cot1d_from_leaves": (c_int, [c_vp, c_int, c_i64, c_vp, c_vp, P(c_vp)]),
    "mwns_cot1d_apply": (c_int, [c_vp, c_vp, c_vp, P(c_vp), P(c_dbl)]),
    "mwns_cot1d_export": (c_int, [c_vp, c_vp, P(c_i64), c_vp, c_vp, c_vp]),
    "mwns_cot1d_eval": (c_int, [c_vp, c_vp, c_i64, c_vp, c_vp]),
    "mwns_tree1_destroy": (None, [c_vp]),
    "mwns_fit_kernel2d": (c_int, [c_dbl, c_dbl, c_dbl, c_dbl, c_dbl, c_int, P(c_int), c_vp, c_vp]),
    "mwns_op2d_create": (c_int, [c_vp, c_int, c_int, c_vp, c_vp, c_dbl, c_int, c_int, P(c_vp)]),
    "mwns_op2d_plan_export": (c_int, [c_vp, c_vp, P(c_size)]),
    "mwns_op2d_plan_import": (c_int, [c_vp, c_vp, c_size]),
    "mwns_op2d_destroy": (None, [c_vp]),
    "mwns_project2d": (c_int, [c_vp, c_int, c_dbl, c_int, c_int, c_int, c_vp, c_vp, c_vp, P(c_vp)]),
    "mwns_tree2d_from_leaves": (c_int, [c_vp, c_int, c_i64, c_vp, c_vp, P(c_vp)]),
    "mwns_apply2d": (c_int, [c_vp, c_vp, c_vp, P(c_vp), P(c_dbl), P(c_dbl)]),
    "mwns_tree2d_export": (c_int, [c_vp, c_vp, P(c_i64), c_vp, c_vp, c_vp]),
    "mwns_tree2d_eval": (c_int, [c_vp, c_vp, c_i64, c_vp, c_vp]),
    "mwns_tree2d_destroy": (None, [c_vp]),
    "mwns_tree_coulomb_product": (c_int, [c_vp, c_vp, c_dbl, c_dbl, c_int, P(c_vp)]),
    "mwns_tree_dot": (c_int, [c_vp, c_vp, c_vp, P(c_dbl)]),
    "mwns_hydrogen_kalos": (c_int, [c_vp, c_int, c_dbl, c_dbl, c_int, c_dbl, c_dbl, c_int, c_int, c_vp, c_vp, c_vp,
                                    c_vp]),
}

for _name, (_res, _args) in SIGNATURES.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class MwnsError(RuntimeError):
    def __init__(self, status, where):
        msg = lib.mwns_last_error().decode(errors="replace")
        super().__init__("%s returned %s: %s" % (where, STATUS_NAMES.get(status, status), msg))
        self.status = status


def check(status, where):
    if status != MWNS_OK:
        raise MwnsError(status, where)
