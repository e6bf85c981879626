"""ctypes declarations of the C ABI in include/pcm.h (libpcm.so, built in-tree for gfx950).

There is no fallback: if the shared library is missing, importing the package fails.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcm.so")

PCM_OK, PCM_E_ARG, PCM_E_ALLOC, PCM_E_HIP, PCM_E_NOCONV, PCM_E_NOTPD, PCM_E_UNSUPPORTED, PCM_E_STATE = range(8)
STATUS_NAMES = {0: "PCM_OK", 1: "PCM_E_ARG", 2: "PCM_E_ALLOC", 3: "PCM_E_HIP", 4: "PCM_E_NOCONV",
                5: "PCM_E_NOTPD", 6: "PCM_E_UNSUPPORTED", 7: "PCM_E_STATE"}
PCM_FP64, PCM_MIXED, PCM_DYNAMIC = 0, 1, 2
PCM_PRECOND_NONE, PCM_PRECOND_JACOBI, PCM_PRECOND_RBJ, PCM_PRECOND_OCTREE = 0, 1, 2, 3
PCM_THRESH_FIXED, PCM_THRESH_TWO_DELTA, PCM_THRESH_DYNAMIC = 0, 1, 2

EXPORTED = ["pcm_default_params", "pcm_default_solve_opts", "pcm_create", "pcm_destroy", "pcm_last_error",
            "pcm_build_surface", "pcm_update_geometry", "pcm_esp", "pcm_esp_deriv", "pcm_fock", "pcm_fock_grad", "pcm_solve", "pcm_energy", "pcm_grad",
            "pcm_matvec_share", "pcm_matvec_share_noalloc", "pcm_dynamic_threshold", "pcm_default_threshold_policy", "pcm_cg_threshold", "pcm_rbj_partition",
            "pcm_octree_partition", "pcm_surface_get", "pcm_mol_sizes", "pcm_pair_list",
            "pcm_mol_destroy", "pcm_batch_create", "pcm_batch_destroy", "pcm_esp_batched", "pcm_fock_batched",
            "pcm_solve_batched", "pcm_grad_batched",
            "pcm_graph_capture", "pcm_graph_launch", "pcm_graph_info", "pcm_graph_destroy",
            "pcm_profile_enable", "pcm_profile_collect", "pcm_profile_entry"]


class pcm_params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("k_factor", ctypes.c_double), ("zeta0", ctypes.c_double),
                ("switch_thresh", ctypes.c_double), ("schwarz_thresh", ctypes.c_double),
                ("diag_const", ctypes.c_double), ("precision", ctypes.c_int), ("autotune", ctypes.c_int),
                ("dp_thresh", ctypes.c_double)]


class pcm_basis(ctypes.Structure):
    _fields_ = [("n_shells", ctypes.c_int), ("shell_atom", ctypes.c_void_p), ("shell_l", ctypes.c_void_p),
                ("shell_nprim", ctypes.c_void_p), ("shell_off", ctypes.c_void_p), ("prim_exp", ctypes.c_void_p),
                ("prim_coef", ctypes.c_void_p)]


class pcm_solve_opts(ctypes.Structure):
    _fields_ = [("precond", ctypes.c_int), ("block", ctypes.c_int), ("seed", ctypes.c_ulonglong),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("warm_start", ctypes.c_int),
                ("precision", ctypes.c_int), ("inner_rtol", ctypes.c_double)]


class pcm_threshold_policy(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("delta", ctypes.c_double), ("scale", ctypes.c_double),
                ("switch_at", ctypes.c_double), ("switched", ctypes.c_int)]


class pcm_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("refinements", ctypes.c_int), ("resid", ctypes.c_double),
                ("energy", ctypes.c_double), ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double)]


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1505_07851_amd.build` "
                          "(the C-PCM path has no CPU fallback)")
    L = ctypes.CDLL(path)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "pcm_default_params": (None, [P(pcm_params)]),
        "pcm_default_solve_opts": (None, [P(pcm_solve_opts)]),
        "pcm_create": (i, [P(pcm_params), vp, P(vp)]),
        "pcm_destroy": (None, [vp]),
        "pcm_last_error": (ctypes.c_char_p, [vp]),
        "pcm_build_surface": (i, [vp, i, vp, vp, vp, i, vp, vp, P(pcm_basis), P(vp), P(i)]),
        "pcm_update_geometry": (i, [vp, vp, vp, vp]),
        "pcm_esp": (i, [vp, vp, vp, vp, vp]),
        "pcm_fock": (i, [vp, vp, vp, vp]),
        "pcm_esp_deriv": (i, [vp, vp, vp, vp, vp, vp]),
        "pcm_fock_grad": (i, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "pcm_solve": (i, [vp, vp, vp, P(pcm_solve_opts), vp, P(pcm_solve_info)]),
        "pcm_energy": (i, [vp, vp, vp, vp, vp, P(d)]),
        "pcm_grad": (i, [vp, vp, vp, vp, vp, vp]),
        "pcm_matvec_share": (i, [vp, vp, vp, vp, i, i]),
        "pcm_matvec_share_noalloc": (i, [vp, vp, vp, vp, i, i]),
        "pcm_dynamic_threshold": (d, [d]),
        "pcm_default_threshold_policy": (None, [P(pcm_threshold_policy), i]),
        "pcm_cg_threshold": (d, [P(pcm_threshold_policy), d]),
        "pcm_rbj_partition": (i, [i, vp, vp, i, ctypes.c_ulonglong, vp, vp]),
        "pcm_octree_partition": (i, [i, vp, i, vp, vp]),
        "pcm_surface_get": (i, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "pcm_mol_sizes": (i, [vp, P(i), P(i), P(i), vp, vp, vp, vp]),
        "pcm_pair_list": (i, [vp, vp, i, vp, vp, vp, vp, vp]),
        "pcm_mol_destroy": (None, [vp]),
        "pcm_batch_create": (i, [vp, P(vp), i, P(vp)]),
        "pcm_batch_destroy": (None, [vp]),
        "pcm_esp_batched": (i, [vp, vp, P(vp), P(vp), P(vp)]),
        "pcm_fock_batched": (i, [vp, vp, P(vp), P(vp)]),
        "pcm_solve_batched": (i, [vp, vp, P(vp), P(pcm_solve_opts), P(vp), P(pcm_solve_info)]),
        "pcm_grad_batched": (i, [vp, vp, P(vp), P(vp), P(vp), P(vp)]),
        "pcm_graph_capture": (i, [vp, vp, P(vp), P(vp), P(vp), P(vp), P(vp), vp, P(pcm_solve_opts), P(vp)]),
        "pcm_graph_launch": (i, [vp, vp]),
        "pcm_graph_info": (i, [vp, vp, P(pcm_solve_info), P(ctypes.c_longlong)]),
        "pcm_graph_destroy": (None, [vp]),
        "pcm_profile_enable": (i, [vp, i]),
        "pcm_profile_collect": (i, [vp]),
        "pcm_profile_entry": (i, [vp, i, ctypes.c_char_p, i, P(d), P(ctypes.c_longlong), P(d)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB
