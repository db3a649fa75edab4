"""Loader of the oracle's plain-C core (test infrastructure only).

``build()`` compiles ``ns_core.c`` with gcc into ``oracle/_ns_core.so``; ``lib()`` loads it,
compiling first when the shared object is missing or older than its source.
"""
import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ns_core.c")
_SO = os.path.join(_HERE, "_ns_core.so")
_lib = None


def build():
    """Compile the oracle core (plain C, OpenMP over independent output nodes)."""
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _SO)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.orc_project_level.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, i64, P, ctypes.c_int,
                                        P, P, P, ctypes.c_double, P, P, P, P, P]
        L.orc_project_level.restype = ctypes.c_int
        for name in ("orc_apply_modified", "orc_apply_difference"):
            fn = getattr(L, name)
            fn.argtypes = [ctypes.c_int, i64, P, P, P, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, P,
                           P, P, i64, P, P]
            fn.restype = ctypes.c_int
        _lib = L
    return _lib
