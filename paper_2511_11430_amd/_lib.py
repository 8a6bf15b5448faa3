"""ctypes loader for libvpm.so (built by paper_2511_11430_amd/build.py).

There is no fallback: if the library is missing or fails to load, importing the binding
raises, so nothing can silently run elsewhere.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvpm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "vpm.h")

c_i32, c_i64, c_dbl, c_sz, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
c_i64p = ctypes.POINTER(ctypes.c_int64)


class VpmOptions(ctypes.Structure):
    _fields_ = [("scheme", c_i32), ("sigma_rule", c_i32), ("self_", c_i32), ("accumulate", c_i32),
                ("variant", c_i32), ("gradient", c_i32), ("reserved", c_i32 * 2)]


# name -> (restype, argtypes), matching include/vpm.h
SIGNATURES = {
    "vpm_eval_velocity_stretching": (c_i32, [c_i32, c_i32, c_i64p, c_i64p, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp,
                                             c_vp, c_i64, c_vp, c_vp, c_vp, c_i64, ctypes.POINTER(VpmOptions),
                                             c_vp, c_sz, c_vp]),
    "vpm_workspace_size": (c_sz, [c_i32, c_i32, c_i64p, c_i64p, ctypes.POINTER(VpmOptions)]),
    "vpm_eval_velocity_gradient": (c_i32, [c_i32, c_i32, c_i64p, c_i64p, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp,
                                           c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_i64, ctypes.POINTER(VpmOptions),
                                           c_vp, c_sz, c_vp]),
    "vpm_sgs_vreman": (c_i32, [c_i32, c_i64, c_vp, c_vp, c_i64, c_dbl, c_vp, c_vp]),
    "vpm_eval_diffusion": (c_i32, [c_i32, c_i32, c_i64p, c_vp, c_vp, c_vp, c_vp, c_vp, c_i64, c_dbl, c_vp, c_i64,
                                   c_i32, c_vp, c_sz, c_vp]),
    "vpm_diffusion_workspace_size": (c_sz, [c_i32, c_i32, c_i64p]),
    "vpm_aic_assemble": (c_i32, [c_i64, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_i64, c_dbl, c_i32, c_vp, c_i64,
                                 c_vp]),
    "vpm_lu_factor": (c_i32, [c_i64, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "vpm_lu_solve": (c_i32, [c_i64, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "vpm_wake_shed": (c_i32, [c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "vpm_wake_convert": (c_i32, [c_i32, c_i64, c_vp, c_vp, c_i64, c_vp, c_vp, c_i32, c_i32, c_dbl, c_i64, c_vp, c_vp,
                                 c_vp, c_i64, c_vp, c_vp, c_sz, c_vp]),
    "vpm_wake_convert_workspace_size": (c_sz, [c_i64]),
    "vpm_aic_update": (c_i32, [c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp, c_i64, c_i64, c_vp, c_vp, c_vp, c_vp, c_i64,
                               c_vp, c_dbl, c_i32, c_vp]),
    "vpm_neumann_rhs": (c_i32, [c_i32, c_i64, c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp]),
    "vpm_rk3_advect": (c_i32, [c_i32, c_i32, c_i64, c_dbl, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp]),
    "vpm_eval_segments": (c_i32, [c_i32, c_i64, c_vp, c_vp, c_vp, c_i64, c_dbl, c_i32, c_i64, c_vp, c_i64,
                                  c_vp, c_i64, c_i32, c_vp]),
    "vpm_eval_segments_gradient": (c_i32, [c_i32, c_i64, c_vp, c_vp, c_vp, c_i64, c_dbl, c_i32, c_i64, c_vp, c_vp,
                                           c_i64, c_i32, c_vp, c_vp, c_vp, c_i64, c_i32, c_vp]),
    "vpm_segments_backward": (c_i32, [c_i32, c_i64, c_vp, c_vp, c_vp, c_i64, c_dbl, c_i32, c_i64, c_vp, c_vp, c_i64,
                                      c_i32, c_vp, c_vp, c_i64, c_vp, c_vp, c_i64, c_vp]),
    "vpm_fmm_eval": (c_i32, [c_i32, c_i64, c_vp, c_vp, c_vp, c_i64, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_i64, c_vp,
                             c_sz, c_vp]),
    "vpm_fmm_workspace_size": (c_sz, [c_i32, c_i64, c_i32, c_i32]),
    "vpm_backward": (c_i32, [c_i32, c_i32, c_i64p, c_i64p, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_i64,
                             c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(VpmOptions), c_vp, c_sz, c_vp]),
    "vpm_rk3_stage": (c_i32, [c_i32, c_i32, c_i32, c_i64, c_dbl, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i64,
                              c_vp, c_vp, c_vp]),
    "vpm_rk3_stage_backward": (c_i32, [c_i32, c_i32, c_i32, c_i64, c_dbl, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                       c_i64, c_vp]),
    "vpm_convert": (c_i32, [c_i32, c_i32, c_i64, c_vp, c_i64, c_vp, c_i64, c_i32, c_vp]),
    "vpm_diagnostics": (c_i32, [c_i32, c_i64, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_sz, c_vp]),
    "vpm_diagnostics_workspace_size": (c_sz, []),
    "vpm_backward_workspace_size": (c_sz, [c_i32, c_i32, c_i64p, c_i64p]),
    "vpm_check_inputs": (c_i32, [c_i32, c_i64, c_vp, c_vp, c_vp, c_i64, c_vp, c_sz, c_vp]),
    "vpm_check_inputs_workspace_size": (c_sz, []),
    "vpm_fma_chain": (c_i32, [c_i64, c_i32, c_i32, c_vp, c_i64p, c_vp]),
    "vpm_eval_velocity_stretching_noalloc": (c_i32, [c_i32, c_i32, c_i64p, c_i64p, c_vp, c_vp, c_vp, c_i64, c_vp,
                                                     c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_i64,
                                                     ctypes.POINTER(VpmOptions), c_vp]),
    "vpm_noalloc_scratch_bytes": (c_sz, []),
    "vpm_autotune": (c_i32, [c_i32, c_i32, c_i64p, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_sz, c_i32,
                             ctypes.POINTER(c_i32), ctypes.POINTER(ctypes.c_float), c_vp]),
    "vpm_validate_inputs": (c_i32, [c_i32, c_i64, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_sz, c_vp]),
    "vpm_axial_loss": (c_i32, [c_i32, c_i64, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp]),
    "vpm_variant_count": (c_i32, []),
    "vpm_variant_info": (c_i32, [c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]),
    "vpm_set_plan": (c_i32, [c_i32, c_i32, c_i64, c_i64, c_i32]),
    "vpm_get_plan": (c_i32, [c_i32, c_i32, c_i64]),
    "vpm_status_string": (ctypes.c_char_p, [c_i32]),
    "vpm_version": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libvpm.so and declare its signatures; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libvpm.so not found at {LIB_PATH}; build it with "
                              "`python paper_2511_11430_amd/build.py` (or __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        # kernel-shape plans from a matching tuning cache, if any
        from . import tune
        tune.apply_cache()
    return _lib
