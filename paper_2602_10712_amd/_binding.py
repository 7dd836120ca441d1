"""ctypes binding of libsrp (include/srp.h): argument marshalling only.

Functions keep the C names and take torch tensors for device arrays (their data_ptr() is passed)
and numpy arrays for host arrays.  `stream` defaults to torch's current stream on the scene's
device.  Every non-zero status raises SRPError with srp_last_error().
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libsrp.so")

if not os.path.exists(_LIB):
    raise ImportError(f"{_LIB} is not built; run `python -m paper_2602_10712_amd.build` (hipcc, gfx950)")

_lib = ctypes.CDLL(_LIB)

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64


class srp_hinge(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("axis", ctypes.c_double * 3)]


class TraceParams(ctypes.Structure):
    """srp_trace_params.  ray_mask: a device tensor of 32-bit words (see ray_mask_bits) or None; the
    object keeps a reference to it, so it stays alive as long as these parameters."""
    _fields_ = [("nu", I32), ("nv", I32), ("bounces", I32), ("jitter", I32), ("flux", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("dir_index_base", I64), ("design_index", I32), ("frame_mode", I32),
                ("tiles_per_wave", I32), ("sampling", I32), ("edge_samples", I32), ("ray_mask", P)]

    def __init__(self, nu=256, nv=256, bounces=1, jitter=1, flux=1361.0, seed=0, dir_index_base=0, design_index=0,
                 frame_mode=0, tiles_per_wave=0, sampling=0, ray_mask=None, edge_samples=0):
        super().__init__(int(nu), int(nv), int(bounces), int(bool(jitter)), float(flux), int(seed),
                         int(dir_index_base), int(design_index), int(frame_mode), int(tiles_per_wave), int(sampling),
                         int(edge_samples), _dptr(ray_mask))
        self._mask_ref = ray_mask


def ray_mask_bits(left_out, device="cuda"):
    """Packs a bool array [D][nu * nv] (True = primary pixel left out) into the uint32 bitmap
    [D][ceil(nu * nv / 32)] that srp_trace_params.ray_mask takes (bit p & 31 of word p >> 5), as a
    device tensor (int32 storage of the same bits)."""
    import torch
    m = np.asarray(left_out, dtype=bool)
    m = m.reshape(m.shape[0], -1)
    words = (m.shape[1] + 31) // 32
    pad = np.zeros((m.shape[0], words * 32), dtype=bool)
    pad[:, :m.shape[1]] = m
    w = np.packbits(pad.reshape(m.shape[0], words, 4, 8), axis=-1, bitorder="little").astype(np.uint32)
    packed = (w[..., 0, 0] | (w[..., 1, 0] << 8) | (w[..., 2, 0] << 16) | (w[..., 3, 0] << 24)).view(np.int32)
    return torch.from_numpy(np.ascontiguousarray(packed)).to(device)


_sigs = {
    "srp_scene_create": [P, I64, P, I64, P, P, I32, P, ctypes.POINTER(P)],
    "srp_scene_set_design": [P, P, P, P, P, P],
    "srp_scene_get_vertices": [P, P, I64],
    "srp_scene_set_vertices": [P, P, I64, I32, P],
    "srp_scene_set_phong": [P, P, P],
    "srp_scene_info": [P, P, P, P],
    "srp_frames": [P, P, I64, I32, I32, P, P],
    "srp_trace": [P, P, I64, ctypes.POINTER(TraceParams), P, P, P, P],
    "srp_trace_noalloc": [P, P, I64, ctypes.POINTER(TraceParams), P, P, P, P],
    "srp_trace_records": [P, P, I64, ctypes.POINTER(TraceParams), P, P, I64, P, P, P, P],
    "srp_scene_ray_stats": [P, P, I64, ctypes.POINTER(TraceParams), P, I64, P],
    "srp_trace_adjoint": [P, P, I64, ctypes.POINTER(TraceParams), P, P, P, P, P, P, P],
    "srp_path_record_bytes": [P, I64, ctypes.POINTER(TraceParams), ctypes.POINTER(I64)],
    "srp_trace_recorded": [P, P, I64, ctypes.POINTER(TraceParams), P, P, P, P, I64, P],
    "srp_trace_adjoint_recorded": [P, P, I64, ctypes.POINTER(TraceParams), P, P, P, P, I64, P, P, P, P],
    "srp_batch_trace": [P, I32, P, I64, ctypes.POINTER(TraceParams), P, P, P],
    "srp_autotune_tiles_per_wave": [P, I32, P, I64, ctypes.POINTER(TraceParams), ctypes.POINTER(I32), P, P],
    "srp_surface_estimate": [P, I32, P, I64, I64, ctypes.POINTER(TraceParams), I32, P, P, P, P, P, P],
    "srp_surface_designs": [P, P, I32, P, P, I64, I32, ctypes.POINTER(TraceParams), P, P, P, P, P, P],
    "srp_scene_build_gpu": [P, ctypes.POINTER(I32), ctypes.POINTER(I32), P],
    "srp_scene_destroy": [P],
    "srp_mlp_create": [I32, I32, I32, I32, ctypes.c_uint64, ctypes.POINTER(P)],
    "srp_mlp_num_params": [P, ctypes.POINTER(I64)],
    "srp_mlp_forward": [P, P, I64, P, I32, P],
    "srp_mlp_ensemble": [P, P, P, I64, ctypes.c_float, ctypes.c_float, P, P, P, P, P],
    "srp_mlp_backward": [P, P, I64, P, P],
    "srp_mlp_adam_step": [P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, P],
    "srp_mlp_zero_grad": [P, P],
    "srp_mlp_mse": [P, P, P, I64, P, P, P],
    "srp_mlp_get_params": [P, P, P, P, P, ctypes.POINTER(I64), I64],
    "srp_mlp_set_params": [P, P, P, P, I64, I64],
    "srp_mlp_destroy": [P],
    "srp_orbit_rk4": [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, I64, P, P, P, P],
    "srp_orbit_rk4_adjoint": [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, I64, P, P, P, I64, P, P],
    "srp_sync": [P],
}
for _name, _args in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = I32
_lib.srp_last_error.argtypes = []
_lib.srp_last_error.restype = ctypes.c_char_p


class AttitudeParams(ctypes.Structure):
    """srp_attitude_params (see srp.h)."""
    _fields_ = [("mu", ctypes.c_double), ("mass", ctypes.c_double), ("inertia", ctypes.c_double * 9),
                ("sun", ctypes.c_double * 3), ("force_scale", ctypes.c_double), ("torque_scale", ctypes.c_double),
                ("earth_radius", ctypes.c_double), ("dt", ctypes.c_double), ("n_steps", I64),
                ("steps_per_design", I64)]

    def __init__(self, mu, mass, inertia, sun, force_scale, torque_scale, dt, n_steps, earth_radius=0.0,
                 steps_per_design=0):
        super().__init__()
        self.steps_per_design = int(steps_per_design)
        self.mu, self.mass = float(mu), float(mass)
        self.inertia[:] = [float(x) for x in np.asarray(inertia, dtype=np.float64).reshape(9)]
        self.sun[:] = [float(x) for x in np.asarray(sun, dtype=np.float64).reshape(3)]
        self.force_scale, self.torque_scale = float(force_scale), float(torque_scale)
        self.earth_radius, self.dt, self.n_steps = float(earth_radius), float(dt), int(n_steps)


_lib.srp_attitude_rk4.argtypes = [P, ctypes.POINTER(AttitudeParams), P, P, I64, P, P, P]
_lib.srp_attitude_rk4.restype = I32


class SRPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libsrp status {status}: {msg}")
        self.status = status


def lib_path() -> str:
    return _LIB


def _check(st: int) -> None:
    if st != 0:
        raise SRPError(st, _lib.srp_last_error().decode())


def _dptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device (cuda) tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _hptr(a):
    return None if a is None else a.ctypes.data


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _dtype_check(t, dtype, name):
    if t is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")


# ------------------------------------------------------------------------------------------------
# C functions, same names
# ------------------------------------------------------------------------------------------------
def srp_scene_create(verts, tris, vert_hinge=None, hinge_origin=None, hinge_axis=None, com=None):
    v = np.ascontiguousarray(verts, dtype=np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    vh = None if vert_hinge is None else np.ascontiguousarray(vert_hinge, dtype=np.int32)
    n_h = 0 if hinge_origin is None else len(hinge_origin)
    harr = None
    if n_h:
        harr = (srp_hinge * n_h)()
        for k in range(n_h):
            harr[k].origin[:] = [float(x) for x in hinge_origin[k]]
            harr[k].axis[:] = [float(x) for x in hinge_axis[k]]
    c = None if com is None else np.ascontiguousarray(com, dtype=np.float64)
    out = P()
    _check(_lib.srp_scene_create(_hptr(v), len(v), _hptr(t), len(t), _hptr(vh),
                                 ctypes.cast(harr, P) if harr is not None else None, n_h, _hptr(c),
                                 ctypes.byref(out)))
    return out


def srp_scene_set_design(scene, hinge_angles, rho_s, rho_d, p_spec=None, stream=None):
    import torch
    _dtype_check(rho_s, torch.float32, "rho_s")
    _dtype_check(rho_d, torch.float32, "rho_d")
    _dtype_check(p_spec, torch.float32, "p_spec")
    ang = None if hinge_angles is None else np.ascontiguousarray(hinge_angles, dtype=np.float64)
    _check(_lib.srp_scene_set_design(scene, _hptr(ang), _dptr(rho_s), _dptr(rho_d), _dptr(p_spec), _stream(stream)))


def srp_scene_set_vertices(scene, verts, mode=0, stream=None):
    v = np.ascontiguousarray(verts, dtype=np.float64).reshape(-1, 3)
    _check(_lib.srp_scene_set_vertices(scene, _hptr(v), v.shape[0], int(mode), _stream(stream)))


def srp_scene_set_phong(scene, exponents=None, stream=None):
    import torch
    _dtype_check(exponents, torch.float32, "exponents")
    _check(_lib.srp_scene_set_phong(scene, _dptr(exponents), _stream(stream)))


def srp_scene_get_vertices(scene, n_verts):
    out = np.zeros((n_verts, 3))
    _check(_lib.srp_scene_get_vertices(scene, _hptr(out), n_verts))
    return out


def srp_scene_info(scene):
    a, b, c = I32(), I32(), I32()
    _check(_lib.srp_scene_info(scene, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return {"n_nodes": a.value, "depth": b.value, "n_tris": c.value}


def srp_frames(scene, sun_dirs, nu, nv, frames, stream=None):
    import torch
    _dtype_check(sun_dirs, torch.float64, "sun_dirs")
    _dtype_check(frames, torch.float64, "frames")
    _check(_lib.srp_frames(scene, _dptr(sun_dirs), sun_dirs.shape[0], nu, nv, _dptr(frames), _stream(stream)))


def srp_trace(scene, sun_dirs, params: TraceParams, force, torque=None, frames=None, stream=None):
    import torch
    _dtype_check(sun_dirs, torch.float64, "sun_dirs")
    _dtype_check(force, torch.float64, "force")
    _dtype_check(torque, torch.float64, "torque")
    _dtype_check(frames, torch.float64, "frames")
    _check(_lib.srp_trace(scene, _dptr(sun_dirs), sun_dirs.shape[0], ctypes.byref(params), _dptr(frames),
                          _dptr(force), _dptr(torque), _stream(stream)))


def srp_trace_noalloc(scene, sun_dirs, params: TraceParams, force, torque=None, frames=None, stream=None):
    import torch
    _dtype_check(sun_dirs, torch.float64, "sun_dirs")
    _dtype_check(force, torch.float64, "force")
    _dtype_check(torque, torch.float64, "torque")
    _dtype_check(frames, torch.float64, "frames")
    _check(_lib.srp_trace_noalloc(scene, _dptr(sun_dirs), sun_dirs.shape[0], ctypes.byref(params), _dptr(frames),
                                  _dptr(force), _dptr(torque), _stream(stream)))


def srp_trace_records(scene, sun_dirs, params: TraceParams, hit_prim, ray_force=None, pix=None, frames=None,
                      stream=None, hit_point=None):
    import torch
    _dtype_check(sun_dirs, torch.float64, "sun_dirs")
    _dtype_check(hit_prim, torch.int32, "hit_prim")
    _dtype_check(ray_force, torch.float32, "ray_force")
    _dtype_check(hit_point, torch.float32, "hit_point")
    _dtype_check(pix, torch.int64, "pix")
    n_pix = 0 if pix is None else pix.shape[0]
    _check(_lib.srp_trace_records(scene, _dptr(sun_dirs), sun_dirs.shape[0], ctypes.byref(params), _dptr(frames),
                                  _dptr(pix), n_pix, _dptr(hit_prim), _dptr(ray_force), _dptr(hit_point),
                                  _stream(stream)))


def srp_trace_adjoint(scene, sun_dirs, params: TraceParams, g_force, g_torque=None, g_rho_s=None, g_rho_d=None,
                      g_hinge=None, frames=None, stream=None):
    """Adds dL/d rho_s, dL/d rho_d (float32 [n_tris]) and dL/d hinge (float64 [n_hinges]) for
    L = sum_j g_force[j] . F_j + g_torque[j] . tau_j (see srp.h)."""
    import torch
    _dtype_check(sun_dirs, torch.float64, "sun_dirs")
    _dtype_check(g_force, torch.float64, "g_force")
    _dtype_check(g_torque, torch.float64, "g_torque")
    _dtype_check(g_rho_s, torch.float32, "g_rho_s")
    _dtype_check(g_rho_d, torch.float32, "g_rho_d")
    _dtype_check(g_hinge, torch.float64, "g_hinge")
    _dtype_check(frames, torch.float64, "frames")
    _check(_lib.srp_trace_adjoint(scene, _dptr(sun_dirs), sun_dirs.shape[0], ctypes.byref(params), _dptr(frames),
                                  _dptr(g_force), _dptr(g_torque), _dptr(g_rho_s), _dptr(g_rho_d), _dptr(g_hinge),
                                  _stream(stream)))


def srp_path_record_bytes(scene, D, params: TraceParams):
    """Bytes of the path record srp_trace_recorded writes for D directions."""
    n = I64(0)
    _check(_lib.srp_path_record_bytes(scene, D, ctypes.byref(params), ctypes.byref(n)))
    return n.value


def srp_trace_recorded(scene, sun_dirs, params: TraceParams, force, torque, paths, frames=None, stream=None):
    """srp_trace that also writes every traced path's facets into `paths` (device int32 tensor of
    at least srp_path_record_bytes bytes)."""
    import torch
    _dtype_check(sun_dirs, torch.float64, "sun_dirs")
    _dtype_check(force, torch.float64, "force")
    _dtype_check(torque, torch.float64, "torque")
    _dtype_check(frames, torch.float64, "frames")
    _dtype_check(paths, torch.int32, "paths")
    _check(_lib.srp_trace_recorded(scene, _dptr(sun_dirs), sun_dirs.shape[0], ctypes.byref(params), _dptr(frames),
                                   _dptr(force), _dptr(torque), _dptr(paths), paths.numel() * 4, _stream(stream)))


def srp_trace_adjoint_recorded(scene, sun_dirs, params: TraceParams, g_force, paths, g_torque=None, g_rho_s=None,
                               g_rho_d=None, g_hinge=None, frames=None, stream=None):
    """srp_trace_adjoint taking the facets of every path from the record of the last
    srp_trace_recorded with the same scene state and arguments (see srp.h)."""
    import torch
    _dtype_check(sun_dirs, torch.float64, "sun_dirs")
    _dtype_check(g_force, torch.float64, "g_force")
    _dtype_check(g_torque, torch.float64, "g_torque")
    _dtype_check(g_rho_s, torch.float32, "g_rho_s")
    _dtype_check(g_rho_d, torch.float32, "g_rho_d")
    _dtype_check(g_hinge, torch.float64, "g_hinge")
    _dtype_check(frames, torch.float64, "frames")
    _dtype_check(paths, torch.int32, "paths")
    _check(_lib.srp_trace_adjoint_recorded(scene, _dptr(sun_dirs), sun_dirs.shape[0], ctypes.byref(params),
                                           _dptr(frames), _dptr(g_force), _dptr(g_torque), _dptr(paths),
                                           paths.numel() * 4, _dptr(g_rho_s), _dptr(g_rho_d), _dptr(g_hinge),
                                           _stream(stream)))


def srp_batch_trace(scenes, sun_dirs, params: TraceParams, force, torque=None, stream=None):
    """scenes: sequence of scene handles (or Scene objects); force/torque device double [S][D][3]."""
    import torch
    _dtype_check(sun_dirs, torch.float64, "sun_dirs")
    _dtype_check(force, torch.float64, "force")
    _dtype_check(torque, torch.float64, "torque")
    hs = [s.handle if isinstance(s, Scene) else s for s in scenes]
    arr = (P * len(hs))(*[h.value if isinstance(h, P) else h for h in hs])
    _check(_lib.srp_batch_trace(ctypes.cast(arr, P), len(hs), _dptr(sun_dirs), sun_dirs.shape[0], ctypes.byref(params),
                                _dptr(force), _dptr(torque), _stream(stream)))


def srp_scene_build_gpu(scene, stream=None):
    """Rebuilds the scene's BVH on the GPU (see srp.h); returns (nodes, depth) of the new tree."""
    nn, dd = I32(0), I32(0)
    _check(_lib.srp_scene_build_gpu(scene.handle if isinstance(scene, Scene) else scene, ctypes.byref(nn),
                                    ctypes.byref(dd), _stream(stream)))
    return int(nn.value), int(dd.value)


def srp_surface_estimate(scenes, sun_dirs, n_samples, params: TraceParams, force, torque=None, brute_force=False,
                         rec_facet=None, rec_hits=None, rec_lit=None, stream=None):
    """Surface-sampling estimate (see srp.h): force/torque device double [S][D][3]; records int32."""
    import torch
    _dtype_check(sun_dirs, torch.float64, "sun_dirs")
    _dtype_check(force, torch.float64, "force")
    _dtype_check(torque, torch.float64, "torque")
    for name, t in (("rec_facet", rec_facet), ("rec_hits", rec_hits), ("rec_lit", rec_lit)):
        _dtype_check(t, torch.int32, name)
    hs = [s.handle if isinstance(s, Scene) else s for s in scenes]
    arr = (P * len(hs))(*[h.value if isinstance(h, P) else h for h in hs])
    _check(_lib.srp_surface_estimate(ctypes.cast(arr, P), len(hs), _dptr(sun_dirs), sun_dirs.shape[0], int(n_samples),
                                     ctypes.byref(params), int(bool(brute_force)), _dptr(force), _dptr(torque),
                                     _dptr(rec_facet), _dptr(rec_hits), _dptr(rec_lit), _stream(stream)))


def srp_surface_designs(scene, facet_group, n_groups, sun_dirs, designs, samples, params: TraceParams, force,
                        torque=None, rec_facet=None, rec_hits=None, rec_lit=None, stream=None):
    """Multi-world surface sampling (see srp.h): facet_group host int32 [n_tris]; sun_dirs device
    double [N][3]; designs device float [N][n_hinges + 3 n_groups]; force/torque device double [N][3]."""
    import torch
    _dtype_check(sun_dirs, torch.float64, "sun_dirs")
    _dtype_check(designs, torch.float32, "designs")
    _dtype_check(force, torch.float64, "force")
    _dtype_check(torque, torch.float64, "torque")
    for name, t in (("rec_facet", rec_facet), ("rec_hits", rec_hits), ("rec_lit", rec_lit)):
        _dtype_check(t, torch.int32, name)
    g = np.ascontiguousarray(facet_group, dtype=np.int32)
    h = scene.handle if isinstance(scene, Scene) else scene
    _check(_lib.srp_surface_designs(h, _hptr(g), int(n_groups), _dptr(sun_dirs), _dptr(designs), sun_dirs.shape[0],
                                    int(samples), ctypes.byref(params), _dptr(force), _dptr(torque), _dptr(rec_facet),
                                    _dptr(rec_hits), _dptr(rec_lit), _stream(stream)))


def srp_autotune_tiles_per_wave(scenes, sun_dirs, params: TraceParams, stream=None):
    """Fastest tiles_per_wave (8..16) for this workload, and every candidate's time in ms (see srp.h).
    One scene tunes srp_trace, several tune srp_batch_trace."""
    import torch
    _dtype_check(sun_dirs, torch.float64, "sun_dirs")
    hs = [s.handle if isinstance(s, Scene) else s for s in scenes]
    arr = (P * len(hs))(*[h.value if isinstance(h, P) else h for h in hs])
    best = I32(0)
    ms = np.zeros(9)
    _check(_lib.srp_autotune_tiles_per_wave(ctypes.cast(arr, P), len(hs), _dptr(sun_dirs), sun_dirs.shape[0],
                                            ctypes.byref(params), ctypes.byref(best), _hptr(ms), _stream(stream)))
    return int(best.value), dict(zip(range(8, 17), ms.tolist()))


def srp_scene_ray_stats(scene, sun_dirs, params: TraceParams, pixel_stride=1, frames=None):
    """Host arrays in, dict out: rays, segments, nodes, tris, hits (see srp.h)."""
    sd = np.ascontiguousarray(sun_dirs, dtype=np.float64).reshape(-1, 3)
    fr = None if frames is None else np.ascontiguousarray(frames, dtype=np.float64).reshape(-1, 12)
    out = np.zeros(6)
    _check(_lib.srp_scene_ray_stats(scene, _hptr(sd), len(sd), ctypes.byref(params), _hptr(fr), int(pixel_stride),
                                    _hptr(out)))
    return dict(zip(("rays", "segments", "nodes", "tris", "hits", "hit_rays"), out.tolist()))


# bytes a single ray must touch (bandwidth model): one 64-byte node record per node fetched,
# 36 bytes (v0, e1, e2 as float) per triangle tested, 20 bytes (normal + rho_s, rho_d) per hit
NODE_BYTES, TRI_BYTES, HIT_BYTES = 64.0, 36.0, 20.0


def ray_stats(scene, sun_dirs, params: TraceParams, n_dirs=16, pixel_stride=97):
    """Per-ray averages of srp_scene_ray_stats over n_dirs directions spread over sun_dirs."""
    sd = np.asarray(sun_dirs, dtype=np.float64).reshape(-1, 3)
    idx = np.linspace(0, len(sd) - 1, min(n_dirs, len(sd))).astype(int)
    tot = {"rays": 0.0, "segments": 0.0, "nodes": 0.0, "tris": 0.0, "hits": 0.0, "hit_rays": 0.0}
    for j in idx:
        p = TraceParams(params.nu, params.nv, params.bounces, params.jitter, params.flux, params.seed,
                        params.dir_index_base + int(j), params.design_index, 0)
        st = srp_scene_ray_stats(scene.handle if isinstance(scene, Scene) else scene, sd[j:j + 1], p, pixel_stride)
        for k in tot:
            tot[k] += st[k]
    r, s = max(tot["rays"], 1.0), max(tot["segments"], 1.0)
    return {"rays": tot["rays"], "segments_per_ray": tot["segments"] / r, "nodes_per_segment": tot["nodes"] / s,
            "tris_per_segment": tot["tris"] / s, "hits_per_ray": tot["hits"] / r, "hit_ray_fraction": tot["hit_rays"] / r,
            "bytes_per_ray": (NODE_BYTES * tot["nodes"] + TRI_BYTES * tot["tris"] + HIT_BYTES * tot["hits"]) / r}


def srp_scene_destroy(scene):
    _check(_lib.srp_scene_destroy(scene))


def srp_sync(stream=None):
    _check(_lib.srp_sync(_stream(stream)))


# ------------------------------------------------------------------------------------------------
# convenience object over the same calls
# ------------------------------------------------------------------------------------------------
class PathRecord:
    """What trace_recorded hands to adjoint_recorded: the device directions and frames of the call
    (the adjoint must pass the same arrays) and the path record itself."""

    def __init__(self, sun_dirs, frames, paths):
        self.sun_dirs = sun_dirs
        self.frames = frames
        self.paths = paths


class Scene:
    """A mesh on the GPU: srp_scene_create + srp_scene_set_design + traces."""

    def __init__(self, verts, tris, vert_hinge=None, hinge_origin=None, hinge_axis=None, com=None):
        self.n_verts = int(np.asarray(verts).reshape(-1, 3).shape[0])
        self.n_tris = int(np.asarray(tris).reshape(-1, 3).shape[0])
        self.n_hinges = 0 if hinge_origin is None else len(hinge_origin)
        self.handle = srp_scene_create(verts, tris, vert_hinge, hinge_origin, hinge_axis, com)

    @classmethod
    def from_mesh(cls, mesh):
        return cls(mesh.verts, mesh.tris, mesh.vert_hinge, mesh.hinge_origin if mesh.n_hinges else None,
                   mesh.hinge_axis if mesh.n_hinges else None, mesh.com)

    def set_design(self, rho_s, rho_d, hinge_angles=None, p_spec=None, stream=None):
        import torch
        dev = torch.device("cuda")
        as_dev = lambda x: None if x is None else torch.as_tensor(x, dtype=torch.float32, device=dev).contiguous()
        srp_scene_set_design(self.handle, hinge_angles, as_dev(rho_s), as_dev(rho_d), as_dev(p_spec), stream)

    def vertices(self):
        return srp_scene_get_vertices(self.handle, self.n_verts)

    def set_phong(self, exponents=None, stream=None):
        """Per-facet Phong exponents for the surface-sampling estimator (srp_scene_set_phong);
        None restores ideal mirrors."""
        import torch
        ex = None if exponents is None else torch.as_tensor(
            np.broadcast_to(np.asarray(exponents, dtype=np.float32), (self.n_tris,)).copy(), device="cuda")
        srp_scene_set_phong(self.handle, ex, stream)

    def set_vertices(self, verts, rebuild=False, stream=None):
        """New rest-pose vertices (srp_scene_set_vertices): the tree refitted on the device, or
        rebuilt on the host when `rebuild`."""
        srp_scene_set_vertices(self.handle, verts, 1 if rebuild else 0, stream)

    def info(self):
        return srp_scene_info(self.handle)

    def build_gpu(self, stream=None):
        """Rebuilds the BVH on the GPU (srp_scene_build_gpu); returns (nodes, depth)."""
        return srp_scene_build_gpu(self.handle, stream)

    def trace(self, sun_dirs, params: TraceParams, frames=None, stream=None):
        import torch
        sd = torch.as_tensor(sun_dirs, dtype=torch.float64, device="cuda").contiguous()
        D = sd.shape[0]
        F = torch.empty((D, 3), dtype=torch.float64, device="cuda")
        T = torch.empty((D, 3), dtype=torch.float64, device="cuda")
        fr = None if frames is None else torch.as_tensor(frames, dtype=torch.float64, device="cuda").contiguous()
        srp_trace(self.handle, sd, params, F, T, fr, stream)
        return F, T

    def adjoint(self, sun_dirs, params: TraceParams, g_force, g_torque=None, frames=None, stream=None):
        """Returns (dL/d rho_s, dL/d rho_d, dL/d hinge) as new device tensors."""
        import torch
        dev = torch.device("cuda")
        sd = torch.as_tensor(sun_dirs, dtype=torch.float64, device=dev).contiguous()
        gF = torch.as_tensor(g_force, dtype=torch.float64, device=dev).contiguous()
        gT = None if g_torque is None else torch.as_tensor(g_torque, dtype=torch.float64, device=dev).contiguous()
        fr = None if frames is None else torch.as_tensor(frames, dtype=torch.float64, device=dev).contiguous()
        grs = torch.zeros(self.n_tris, dtype=torch.float32, device=dev)
        grd = torch.zeros(self.n_tris, dtype=torch.float32, device=dev)
        gh = torch.zeros(max(self.n_hinges, 1), dtype=torch.float64, device=dev)
        srp_trace_adjoint(self.handle, sd, params, gF, gT, grs, grd, gh if self.n_hinges else None, fr, stream)
        return grs, grd, gh[:self.n_hinges]

    def trace_recorded(self, sun_dirs, params: TraceParams, frames=None, stream=None):
        """trace() that also keeps every path's facets for adjoint_recorded; returns (F, T, record).
        The record holds the device arrays the adjoint must see again (directions, frames, paths)."""
        import torch
        sd = torch.as_tensor(sun_dirs, dtype=torch.float64, device="cuda").contiguous()
        D = sd.shape[0]
        F = torch.empty((D, 3), dtype=torch.float64, device="cuda")
        T = torch.empty((D, 3), dtype=torch.float64, device="cuda")
        fr = None if frames is None else torch.as_tensor(frames, dtype=torch.float64, device="cuda").contiguous()
        nb = srp_path_record_bytes(self.handle, D, params)
        paths = torch.empty(max(nb // 4, 1), dtype=torch.int32, device="cuda")
        srp_trace_recorded(self.handle, sd, params, F, T, paths, fr, stream)
        return F, T, PathRecord(sd, fr, paths)

    def adjoint_recorded(self, record, params: TraceParams, g_force, g_torque=None, stream=None):
        """adjoint() for the paths of `record` (from trace_recorded with the same params and no design
        change since); returns (dL/d rho_s, dL/d rho_d, dL/d hinge) as new device tensors."""
        import torch
        dev = torch.device("cuda")
        gF = torch.as_tensor(g_force, dtype=torch.float64, device=dev).contiguous()
        gT = None if g_torque is None else torch.as_tensor(g_torque, dtype=torch.float64, device=dev).contiguous()
        grs = torch.zeros(self.n_tris, dtype=torch.float32, device=dev)
        grd = torch.zeros(self.n_tris, dtype=torch.float32, device=dev)
        gh = torch.zeros(max(self.n_hinges, 1), dtype=torch.float64, device=dev)
        srp_trace_adjoint_recorded(self.handle, record.sun_dirs, params, gF, record.paths, gT, grs, grd,
                                   gh if self.n_hinges else None, record.frames, stream)
        return grs, grd, gh[:self.n_hinges]

    def records(self, sun_dirs, params: TraceParams, pix=None, frames=None, stream=None, points=False):
        """(hit_prim, ray_force) or, with points, (hit_prim, ray_force, hit_point) as device tensors."""
        import torch
        sd = torch.as_tensor(sun_dirs, dtype=torch.float64, device="cuda").contiguous()
        D = sd.shape[0]
        n_pix = params.nu * params.nv if pix is None else len(pix)
        hp = torch.empty((D, n_pix, params.bounces), dtype=torch.int32, device="cuda")
        rf = torch.empty((D, n_pix, 3), dtype=torch.float32, device="cuda")
        hx = torch.empty((D, n_pix, params.bounces, 3), dtype=torch.float32, device="cuda") if points else None
        px = None if pix is None else torch.as_tensor(np.asarray(pix), dtype=torch.int64, device="cuda").contiguous()
        fr = None if frames is None else torch.as_tensor(frames, dtype=torch.float64, device="cuda").contiguous()
        srp_trace_records(self.handle, sd, params, hp, rf, px, fr, stream, hit_point=hx)
        return (hp, rf, hx) if points else (hp, rf)

    def close(self):
        if getattr(self, "handle", None):
            srp_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------------
# surrogate MLP
# ------------------------------------------------------------------------------------------------
def srp_mlp_create(n_in=11, width=256, depth=4, n_out=3, seed=0):
    out = P()
    _check(_lib.srp_mlp_create(n_in, width, depth, n_out, int(seed), ctypes.byref(out)))
    return out


def srp_mlp_num_params(mlp):
    n = I64()
    _check(_lib.srp_mlp_num_params(mlp, ctypes.byref(n)))
    return n.value


def srp_mlp_forward(mlp, x, y, keep_activations=False, stream=None):
    import torch
    _dtype_check(x, torch.float32, "x")
    _dtype_check(y, torch.float32, "y")
    _check(_lib.srp_mlp_forward(mlp, _dptr(x), x.shape[0], _dptr(y), int(bool(keep_activations)), _stream(stream)))


def srp_mlp_ensemble(mlp_a, mlp_b, x, threshold, out_scale, y, fail_idx, n_fail, disagree=None, stream=None):
    import torch
    _dtype_check(x, torch.float32, "x")
    _dtype_check(y, torch.float32, "y")
    _dtype_check(disagree, torch.float32, "disagree")
    _dtype_check(fail_idx, torch.int32, "fail_idx")
    _dtype_check(n_fail, torch.int32, "n_fail")
    _check(_lib.srp_mlp_ensemble(mlp_a, mlp_b, _dptr(x), x.shape[0], float(threshold), float(out_scale), _dptr(y),
                                 _dptr(disagree), _dptr(fail_idx), _dptr(n_fail), _stream(stream)))


def srp_mlp_backward(mlp, g_y, g_x=None, stream=None):
    import torch
    _dtype_check(g_y, torch.float32, "g_y")
    _dtype_check(g_x, torch.float32, "g_x")
    _check(_lib.srp_mlp_backward(mlp, _dptr(g_y), g_y.shape[0], _dptr(g_x), _stream(stream)))


def srp_mlp_adam_step(mlp, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(_lib.srp_mlp_adam_step(mlp, float(lr), float(beta1), float(beta2), float(eps), _stream(stream)))


def srp_mlp_zero_grad(mlp, stream=None):
    _check(_lib.srp_mlp_zero_grad(mlp, _stream(stream)))


def srp_mlp_mse(mlp, y, target, g_y, loss, stream=None):
    import torch
    _dtype_check(y, torch.float32, "y")
    _dtype_check(target, torch.float32, "target")
    _dtype_check(g_y, torch.float32, "g_y")
    _dtype_check(loss, torch.float64, "loss")
    _check(_lib.srp_mlp_mse(mlp, _dptr(y), _dptr(target), y.shape[0], _dptr(g_y), _dptr(loss), _stream(stream)))


def srp_mlp_get_params(mlp):
    n = srp_mlp_num_params(mlp)
    p, g, m, v = (np.zeros(n, dtype=np.float32) for _ in range(4))
    step = I64()
    _check(_lib.srp_mlp_get_params(mlp, _hptr(p), _hptr(g), _hptr(m), _hptr(v), ctypes.byref(step), n))
    return {"params": p, "grads": g, "adam_m": m, "adam_v": v, "step": step.value}


def srp_mlp_set_params(mlp, params, adam_m=None, adam_v=None, step=0):
    n = srp_mlp_num_params(mlp)
    arr = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
    p, m, v = arr(params), arr(adam_m), arr(adam_v)
    for a in (p, m, v):
        if a is not None and a.size != n:
            raise ValueError(f"expected {n} values")
    _check(_lib.srp_mlp_set_params(mlp, _hptr(p), _hptr(m), _hptr(v), int(step), n))


def srp_mlp_destroy(mlp):
    _check(_lib.srp_mlp_destroy(mlp))


class Surrogate:
    """The force surrogate on the GPU: srp_mlp_* calls with torch tensors."""

    def __init__(self, n_in=11, width=256, depth=4, n_out=3, seed=0):
        self.n_in, self.width, self.depth, self.n_out = n_in, width, depth, n_out
        self.handle = srp_mlp_create(n_in, width, depth, n_out, seed)
        self.n_params = srp_mlp_num_params(self.handle)

    def forward(self, x, keep_activations=False, stream=None):
        import torch
        x = torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous()
        y = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device="cuda")
        srp_mlp_forward(self.handle, x, y, keep_activations, stream)
        return y

    def train_step(self, x, target, lr, betas=(0.9, 0.999), eps=1e-8, stream=None):
        """One forward + MSE + backward + Adam step; returns the loss as a device double tensor."""
        import torch
        y = self.forward(x, keep_activations=True, stream=stream)
        g_y = torch.empty_like(y)
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
        srp_mlp_mse(self.handle, y, target, g_y, loss, stream)
        srp_mlp_backward(self.handle, g_y, None, stream)
        srp_mlp_adam_step(self.handle, lr, betas[0], betas[1], eps, stream)
        return loss

    def get_params(self):
        return srp_mlp_get_params(self.handle)

    def set_params(self, params, adam_m=None, adam_v=None, step=0):
        srp_mlp_set_params(self.handle, params, adam_m, adam_v, step)

    def close(self):
        if getattr(self, "handle", None):
            srp_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------------
# orbit integration (host FP64)
# ------------------------------------------------------------------------------------------------
def srp_orbit_rk4(z0, mu, mass, dt, n_steps, F_body, R, keep_states=False):
    z0 = np.ascontiguousarray(z0, dtype=np.float64)
    F = np.ascontiguousarray(F_body, dtype=np.float64).reshape(2 * n_steps + 1, 3)
    Rm = np.ascontiguousarray(R, dtype=np.float64).reshape(2 * n_steps + 1, 9)
    zs = np.zeros((n_steps + 1, 6)) if keep_states else None
    zf = np.zeros(6)
    _check(_lib.srp_orbit_rk4(_hptr(z0), float(mu), float(mass), float(dt), int(n_steps), _hptr(F), _hptr(Rm),
                              _hptr(zs), _hptr(zf)))
    return (zf, zs) if keep_states else zf


def srp_orbit_rk4_adjoint(z0, mu, mass, dt, n_steps, F_body, R, g_final, ckpt_every=60):
    z0 = np.ascontiguousarray(z0, dtype=np.float64)
    F = np.ascontiguousarray(F_body, dtype=np.float64).reshape(2 * n_steps + 1, 3)
    Rm = np.ascontiguousarray(R, dtype=np.float64).reshape(2 * n_steps + 1, 9)
    g = np.ascontiguousarray(g_final, dtype=np.float64)
    gF = np.zeros((2 * n_steps + 1, 3))
    gz = np.zeros(6)
    _check(_lib.srp_orbit_rk4_adjoint(_hptr(z0), float(mu), float(mass), float(dt), int(n_steps), _hptr(F), _hptr(Rm),
                                      _hptr(g), int(ckpt_every), _hptr(gF), _hptr(gz)))
    return gF, gz


def srp_attitude_rk4(model, params: AttitudeParams, z0, design, z_final, z_all=None, stream=None):
    """13-D orbit-and-attitude RK4 with the network as force-and-torque model (see srp.h): z0 and
    z_final device double [B][13], design device float [B][n_in - 3] (or None), z_all device double
    [n_steps + 1][B][13] or None."""
    import torch
    _dtype_check(z0, torch.float64, "z0")
    _dtype_check(z_final, torch.float64, "z_final")
    _dtype_check(z_all, torch.float64, "z_all")
    _dtype_check(design, torch.float32, "design")
    if not isinstance(model, Surrogate):
        raise TypeError("model must be a Surrogate (its shape sizes the design rows)")
    B = z0.shape[0]
    nd = model.n_in - 3
    if tuple(z0.shape) != (B, 13) or tuple(z_final.shape) != (B, 13):
        raise ValueError("z0 and z_final must be [B][13]")
    if params.steps_per_design > 0 and nd > 0:
        n_seg = max(1, -(-params.n_steps // params.steps_per_design))
        if design is None or tuple(design.shape) != (n_seg, B, nd):
            raise ValueError(f"design must be [{n_seg}][B][{nd}] for this schedule")
    elif nd > 0 and (design is None or tuple(design.shape) != (B, nd)):
        raise ValueError(f"design must be [B][{nd}]")
    if z_all is not None and tuple(z_all.shape) != (params.n_steps + 1, B, 13):
        raise ValueError("z_all must be [n_steps + 1][B][13]")
    for t in (z0, design, z_final, z_all):
        if t is not None and not t.is_contiguous():
            raise ValueError("tensors must be contiguous")
    h = model.handle
    _check(_lib.srp_attitude_rk4(h, ctypes.byref(params), _dptr(z0), _dptr(design), z0.shape[0], _dptr(z_final),
                                 _dptr(z_all), _stream(stream)))
