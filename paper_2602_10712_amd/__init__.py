"""MI355X-native ray-grid solar radiation pressure (SRP).

The compute path is libsrp.so (hand-written HIP kernels for gfx950 behind the C ABI declared in
include/srp.h); the Python modules only marshal arguments to it.  The first use of any binding
loads the library and raises ImportError if it has not been built
(`python -m paper_2602_10712_amd`) -- there is no CPU fallback.
"""
import importlib

_BINDING_NAMES = {"SRPError", "Scene", "TraceParams", "lib_path", "srp_frames", "srp_scene_create",
                  "srp_scene_destroy", "srp_scene_get_vertices", "srp_scene_set_vertices", "srp_scene_set_phong", "srp_scene_info", "srp_scene_set_design",
                  "srp_sync", "srp_trace", "srp_trace_noalloc", "srp_trace_records", "ray_mask_bits", "srp_scene_ray_stats", "ray_stats",
                  "srp_trace_adjoint", "srp_path_record_bytes", "srp_trace_recorded", "srp_trace_adjoint_recorded", "PathRecord", "srp_batch_trace", "srp_autotune_tiles_per_wave", "srp_surface_estimate", "srp_surface_designs", "srp_scene_build_gpu", "Surrogate", "srp_mlp_create", "srp_mlp_num_params", "srp_mlp_forward", "srp_mlp_ensemble",
                  "srp_mlp_backward", "srp_mlp_adam_step", "srp_mlp_zero_grad", "srp_mlp_mse", "srp_mlp_get_params",
                  "srp_mlp_set_params", "srp_mlp_destroy", "srp_orbit_rk4", "srp_orbit_rk4_adjoint",
                  "AttitudeParams", "srp_attitude_rk4"}


_AUTOGRAD_NAMES = {"SRPForce", "srp_force"}
_ORBIT_NAMES = {"DesignProblem", "SurrogateDesignProblem"}


def __getattr__(name):
    if name in _BINDING_NAMES:
        return getattr(importlib.import_module("._binding", __name__), name)
    if name in _AUTOGRAD_NAMES:
        return getattr(importlib.import_module(".autograd", __name__), name)
    if name in _ORBIT_NAMES:
        return getattr(importlib.import_module(".orbit", __name__), name)
    raise AttributeError(name)


__all__ = sorted(_BINDING_NAMES | _AUTOGRAD_NAMES | _ORBIT_NAMES)
