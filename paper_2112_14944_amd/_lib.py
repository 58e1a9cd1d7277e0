"""ctypes loader for libpprviz.so (the gfx950 HIP library) and the C types of
include/pprviz.h.  No arithmetic happens here."""
from __future__ import annotations

import ctypes as C
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpprviz.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "pprviz.h")

PPR_OK = 0
PPR_EINVAL = -1
PPR_ENOCONV = -2
PPR_EWORKSPACE = -3
PPR_EHIP = -4
PPR_ENONFINITE = -5
PPR_EUNSUPPORTED = -6

vp = C.c_void_p
i32 = C.c_int32
i64 = C.c_int64
f32 = C.c_float
f64 = C.c_double
sz = C.c_size_t


class ppr_csr(C.Structure):
    _fields_ = [("n", i32), ("nnz", i64), ("row_ptr", vp), ("col_idx", vp), ("weight", vp)]


class ppr_batch(C.Structure):
    _fields_ = [("n_graphs", i32), ("n_nodes", i64), ("nnz", i64), ("max_n", i32), ("pool_size", i64), ("node_off", vp),
                ("row_ptr", vp), ("col_idx", vp), ("mat_off", vp)]


_SIGS = {
    "pprviz_version": (C.c_char_p, []),
    "pprviz_status_string": (C.c_char_p, [C.c_int]),
    "pprviz_pushes_for_tolerance": (C.c_int, [f32, f64, i32, C.POINTER(i32), C.POINTER(i32)]),
    "ppr_matrix_workspace": (sz, [C.POINTER(ppr_csr), i32, i32]),
    "ppr_matrix": (C.c_int, [C.POINTER(ppr_csr), vp, i32, vp, i32, f32, f64, i32, vp, vp,
                             C.POINTER(f64), C.POINTER(i32), vp, sz, vp]),
    "ppr_matrix_noalloc_max_scratch": (sz, []),
    "ppr_matrix_noalloc": (C.c_int, [C.POINTER(ppr_csr), vp, i32, vp, i32, f32, f64, i32, vp, vp,
                                     C.POINTER(f64), C.POINTER(i32), vp]),
    "gfp_workspace": (sz, [C.POINTER(ppr_csr), i32, i32]),
    "gfp_level_dppr": (C.c_int, [C.POINTER(ppr_csr), vp, vp, i32, i64, f32, f64, i32, vp, vp, vp,
                                 C.POINTER(i32), vp, sz, vp]),
    "gbp_level_dppr": (C.c_int, [C.POINTER(ppr_csr), vp, vp, i32, i64, vp, i32, vp, f32, i32, vp, vp, vp,
                                 C.POINTER(i32), vp, sz, vp]),
    "tau_push_level_dppr": (C.c_int, [C.POINTER(ppr_csr), vp, vp, i32, i64, f32, f64, f64, f64, i32, vp,
                                      C.POINTER(i32), C.POINTER(i32), vp, sz, vp]),
    "pdist": (C.c_int, [vp, i32, i64, vp, vp]),
    "pdist_backward": (C.c_int, [vp, vp, i32, i64, vp, vp]),
    "layout_workspace": (sz, [i32]),
    "stress_eval": (C.c_int, [vp, i32, vp, vp, vp, sz, vp]),
    "layout_step": (C.c_int, [vp, i32, vp, vp, vp, vp, sz, vp]),
    "stress_backward": (C.c_int, [vp, i32, vp, f32, vp, vp, vp]),
    "layout_metrics_workspace": (sz, [i32]),
    "layout_metrics": (C.c_int, [vp, i32, C.POINTER(ppr_csr), C.POINTER(f64), C.POINTER(f64), vp, sz, vp]),
    "layout_exact_workspace": (sz, [i32]),
    "layout_step_exact": (C.c_int, [vp, i32, vp, vp, f64, i32, C.POINTER(i32), vp, sz, vp]),
    "ppr_backward_workspace": (sz, [C.POINTER(ppr_csr), C.c_int]),
    "ppr_matrix_backward": (C.c_int, [C.POINTER(ppr_csr), f32, i32, vp, vp, vp, vp, sz, vp]),
    "pprviz_batch_max_n": (i32, []),
    "pprviz_batch_workspace": (sz, [C.POINTER(ppr_batch)]),
    "pprviz_batch": (C.c_int, [C.POINTER(ppr_batch), f32, f64, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]),
    "pprviz_batch_profile": (C.c_int, [C.POINTER(ppr_batch), f32, f64, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp,
                                       C.POINTER(f64)]),
    "pprviz_batch_step_exact": (C.c_int, [C.POINTER(ppr_batch), vp, vp, vp, f64, i32, vp, vp, vp]),
    "pprviz_batch_plan_create": (C.c_int, [C.POINTER(ppr_batch), f32, f64, i32, i32, vp, vp, vp, vp, vp, vp, sz,
                                           vp, C.POINTER(vp)]),
    "pprviz_batch_plan_launch": (C.c_int, [vp, vp]),
    "pprviz_batch_plan_destroy": (None, [vp]),
}

_lib = None


def header_functions():
    """Names of the functions include/pprviz.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*\(", text)
    skip = {"if", "defined", "sizeof"}
    decl = []
    for m in re.finditer(r"^[A-Za-z_][^;{}#]*?\b([A-Za-z_][A-Za-z0-9_]*)\s*\([^;{}]*\)\s*;", text, flags=re.M | re.S):
        name = m.group(1)
        if name not in skip:
            decl.append(name)
    del names
    return sorted(set(decl))


def lib():
    """Load libpprviz.so; raises if it has not been built.  There is no
    fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2112_14944_amd.build` "
                           "(or __graft_entry__.build()); there is no non-HIP fallback")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class PprvizError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        msg = lib().pprviz_status_string(status).decode()
        super().__init__(f"{fn} failed: {msg} (status {status})")


def check(fn, status, allow=(PPR_OK,)):
    if status not in allow:
        raise PprvizError(fn, status)
    return status
