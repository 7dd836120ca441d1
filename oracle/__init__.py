"""Oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, double-precision CPU reference of everything the GPU path computes.  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may import this package;
the product library never does, and this package never imports the product.

Parts:
  srp_oracle.c   brute-force FP64 ray-grid SRP tracer (Philox draws, grid frames, bounce loop,
                 force/torque sums, per-ray records and degeneracy flags) -- loaded here via ctypes
  design.py      hinge rotation of panel vertices (design apply), FP64
  (further modules add the adjoint, the MLP surrogate and the orbit integrator)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None



def default_threads():
    """Worker threads for the oracle: the process's CPU affinity, capped at 16 (one GPU's host share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))

def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain C, -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "srp_oracle.c")
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
               "-o", tmp, src, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.oracle_philox4x32_10.argtypes = [P, P, P]
        L.oracle_philox4x32_10.restype = None
        L.oracle_basis.argtypes = [P, P, P]
        L.oracle_basis.restype = None
        L.oracle_frames.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P]
        L.oracle_frames.restype = ctypes.c_int
        L.oracle_default_pspec.argtypes = [ctypes.c_float, ctypes.c_float]
        L.oracle_default_pspec.restype = ctypes.c_float
        L.oracle_trace.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, P, P, P, P, ctypes.c_int64, P,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                   ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, P, ctypes.c_int64,
                                   P, P, P, P, P, P, P, ctypes.c_int32]
        L.oracle_trace.restype = ctypes.c_int
        L.oracle_degen_thresholds.argtypes = [P]
        L.oracle_degen_thresholds.restype = None
        L.oracle_trace_adjoint_rho.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, P, P, P, P, ctypes.c_int64, P,
                                               ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.c_double, ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, P,
                                               ctypes.c_int64, P, P, P, P, ctypes.c_int32, P, ctypes.c_int32]
        L.oracle_trace_adjoint_rho.restype = ctypes.c_int
        L.oracle_trace_frozen.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int64, P, P, P, P, P, ctypes.c_int64, P,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                          ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, P, ctypes.c_int64, P,
                                          ctypes.c_int32, P, P]
        L.oracle_edge_term.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, P, P, ctypes.c_int32, P, P, P, P, P,
                                       ctypes.c_int64, P, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                                       ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32, P, ctypes.c_int64, P, P,
                                       ctypes.c_int32]
        L.oracle_edge_term.restype = ctypes.c_int
        L.oracle_trace_frozen.restype = ctypes.c_int
        L.oracle_surface_estimate.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int64,
                                              ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                                              ctypes.c_int64, ctypes.c_uint32, P, P, P, P, P, P, P, ctypes.c_int32,
                                              ctypes.c_int32]
        L.oracle_surface_estimate.restype = ctypes.c_int
        L.oracle_surface_designs.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, P, P, ctypes.c_int32, P,
                                             ctypes.c_int32, P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                             ctypes.c_double, ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32,
                                             ctypes.c_int32, P, P, P, P, P, P, P, ctypes.c_int32]
        L.oracle_surface_designs.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 block: 4 x uint32 counter, 2 x uint32 key -> 4 x uint32."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def basis(n) -> tuple[np.ndarray, np.ndarray]:
    n = np.ascontiguousarray(n, dtype=np.float64)
    b1 = np.zeros(3)
    b2 = np.zeros(3)
    lib().oracle_basis(_ptr(n), _ptr(b1), _ptr(b2))
    return b1, b2


def frames(verts, sun_dirs, nu: int, nv: int) -> np.ndarray:
    """Grid frames [D][12] = u[3], v[3], o0[3], du, dv, 0 for each sun direction."""
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    sun = np.ascontiguousarray(sun_dirs, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((len(sun), 12))
    st = lib().oracle_frames(_ptr(verts), len(verts), _ptr(sun), len(sun), nu, nv, _ptr(out))
    if st != 0:
        raise ValueError(f"oracle_frames failed ({st})")
    return out


def default_pspec(rho_s, rho_d) -> np.ndarray:
    rs = np.asarray(rho_s, dtype=np.float32).ravel()
    rd = np.asarray(rho_d, dtype=np.float32).ravel()
    f = lib().oracle_default_pspec
    return np.array([f(float(a), float(b)) for a, b in zip(rs, rd)], dtype=np.float32)


def degen_thresholds() -> dict:
    """Constants of the degenerate-segment classification (see srp_oracle.c): lat, the position
    uncertainty across a primary ray in units of the scene size L (it grows by 1/cos(theta) at each
    interaction); depth, the base uncertainty of an origin's distance from a plane, in units of L;
    graze, the cosine below which a hit counts as grazing."""
    out = np.zeros(3)
    lib().oracle_degen_thresholds(_ptr(out))
    return dict(zip(("lat", "depth", "graze"), out.tolist()))


def degeneracy_uncertainty(L, cosines) -> np.ndarray:
    """Uncertainty across the ray (m) of the segments of one path whose earlier interactions had
    the given incidence cosines: u_1 = lat L, u_(b+1) = u_b / max(cos_b, graze) + lat L."""
    th = degen_thresholds()
    u = [th["lat"] * L]
    for c in cosines:
        u.append(u[-1] / max(c, th["graze"]) + th["lat"] * L)
    return np.array(u)


class TraceResult:
    def __init__(self, force, torque, hit_prim=None, degen=None, ray_force=None, ray_torque=None, hit_x=None):
        self.force = force
        self.torque = torque
        self.hit_prim = hit_prim
        self.degen = degen
        self.ray_force = ray_force
        self.ray_torque = ray_torque
        self.hit_x = hit_x

    def path_degenerate(self) -> np.ndarray:
        """[D][n_pix] bool: the path has a degenerate segment (records only)."""
        return self.degen.astype(bool).any(axis=2)


def trace(verts, tris, rho_s, rho_d, sun_dirs, *, nu: int, nv: int, bounces: int, jitter: bool = True,
          flux: float = 1361.0, seed: int = 0, dir_index_base: int = 0, design_index: int = 0,
          p_spec=None, com=None, frames_in=None, pix=None, records: bool = False, threads: int | None = None
          ) -> TraceResult:
    """FP64 brute-force ray-grid SRP estimate; see srp_oracle.c for the definition."""
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    rs = np.ascontiguousarray(rho_s, dtype=np.float32)
    rd = np.ascontiguousarray(rho_d, dtype=np.float32)
    ps = None if p_spec is None else np.ascontiguousarray(p_spec, dtype=np.float32)
    c = None if com is None else np.ascontiguousarray(com, dtype=np.float64)
    sun = np.ascontiguousarray(sun_dirs, dtype=np.float64).reshape(-1, 3)
    D = len(sun)
    fr = None if frames_in is None else np.ascontiguousarray(frames_in, dtype=np.float64).reshape(D, 12)
    px = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
    n_pix = nu * nv if px is None else len(px)
    force = np.zeros((D, 3))
    torque = np.zeros((D, 3))
    hp = dg = rf = rt = hx = None
    if records:
        hp = np.zeros((D, n_pix, bounces), dtype=np.int32)
        dg = np.zeros((D, n_pix, bounces), dtype=np.uint8)
        rf = np.zeros((D, n_pix, 3))
        rt = np.zeros((D, n_pix, 3))
        hx = np.zeros((D, n_pix, bounces, 3))
    if threads is None:
        threads = default_threads()
    st = lib().oracle_trace(_ptr(verts), len(verts), _ptr(tris), len(tris), _ptr(rs), _ptr(rd), _ptr(ps), _ptr(c),
                            _ptr(sun), D, _ptr(fr), nu, nv, bounces, int(bool(jitter)), float(flux), int(seed),
                            int(dir_index_base), int(design_index), _ptr(px), n_pix, _ptr(force), _ptr(torque),
                            _ptr(hp), _ptr(dg), _ptr(rf), _ptr(rt), _ptr(hx), int(threads))
    if st != 0:
        raise ValueError(f"oracle_trace failed ({st})")
    return TraceResult(force, torque, hp, dg, rf, rt, hx)


def trace_adjoint_rho(verts, tris, rho_s, rho_d, sun_dirs, g_force, g_torque=None, *, nu: int, nv: int, bounces: int,
                      jitter: bool = True, flux: float = 1361.0, seed: int = 0, dir_index_base: int = 0,
                      design_index: int = 0, p_spec=None, com=None, frames_in=None, pix=None,
                      threads: int | None = None, drop_degenerate: bool = False):
    """FP64 dL/d rho_s, dL/d rho_d [n_tris] of L = sum_j g_force[j] . F_j + g_torque[j] . tau_j for the
    estimator with frozen counters and specular-sampling probabilities (see srp_oracle.c).
    With drop_degenerate, paths with a degenerate segment are left out and a third value is
    returned: the [D][n_pix] bool mask of those paths."""
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    rs = np.ascontiguousarray(rho_s, dtype=np.float32)
    rd = np.ascontiguousarray(rho_d, dtype=np.float32)
    ps = None if p_spec is None else np.ascontiguousarray(p_spec, dtype=np.float32)
    c = None if com is None else np.ascontiguousarray(com, dtype=np.float64)
    sun = np.ascontiguousarray(sun_dirs, dtype=np.float64).reshape(-1, 3)
    D = len(sun)
    fr = None if frames_in is None else np.ascontiguousarray(frames_in, dtype=np.float64).reshape(D, 12)
    px = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
    n_pix = nu * nv if px is None else len(px)
    gF = np.ascontiguousarray(g_force, dtype=np.float64).reshape(D, 3)
    gT = None if g_torque is None else np.ascontiguousarray(g_torque, dtype=np.float64).reshape(D, 3)
    g_rs = np.zeros(len(tris))
    g_rd = np.zeros(len(tris))
    mask = np.zeros((D, n_pix), dtype=np.uint8) if drop_degenerate else None
    if threads is None:
        threads = default_threads()
    st = lib().oracle_trace_adjoint_rho(_ptr(verts), len(verts), _ptr(tris), len(tris), _ptr(rs), _ptr(rd), _ptr(ps),
                                        _ptr(c), _ptr(sun), D, _ptr(fr), nu, nv, bounces, int(bool(jitter)),
                                        float(flux), int(seed), int(dir_index_base), int(design_index), _ptr(px),
                                        n_pix, _ptr(gF), _ptr(gT), _ptr(g_rs), _ptr(g_rd), int(bool(drop_degenerate)),
                                        _ptr(mask), int(threads))
    if st != 0:
        raise ValueError(f"oracle_trace_adjoint_rho failed ({st})")
    if drop_degenerate:
        return g_rs, g_rd, mask.astype(bool)
    return g_rs, g_rd


def trace_frozen(verts, verts0, tris, rho_s, rho_d, sun_dirs, ref_hits, frames_in, *, nu: int, nv: int, bounces: int,
                 jitter: bool = True, flux: float = 1361.0, seed: int = 0, dir_index_base: int = 0,
                 design_index: int = 0, p_spec=None, com=None, pix=None, footprint: bool = True):
    """Frozen-visibility estimate (F, tau) at vertices `verts` with the facet sequences `ref_hits`
    [D][n_pix][bounces] recorded at the reference vertices `verts0` (see srp_oracle.c); footprint
    scales each path by its primary facet's projected-area ratio."""
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    verts0 = np.ascontiguousarray(verts0, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    rs = np.ascontiguousarray(rho_s, dtype=np.float32)
    rd = np.ascontiguousarray(rho_d, dtype=np.float32)
    ps = None if p_spec is None else np.ascontiguousarray(p_spec, dtype=np.float32)
    c = None if com is None else np.ascontiguousarray(com, dtype=np.float64)
    sun = np.ascontiguousarray(sun_dirs, dtype=np.float64).reshape(-1, 3)
    D = len(sun)
    fr = np.ascontiguousarray(frames_in, dtype=np.float64).reshape(D, 12)
    px = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
    n_pix = nu * nv if px is None else len(px)
    hits = np.ascontiguousarray(ref_hits, dtype=np.int32).reshape(D, n_pix, bounces)
    F = np.zeros((D, 3))
    T = np.zeros((D, 3))
    st = lib().oracle_trace_frozen(_ptr(verts), _ptr(verts0), len(verts), _ptr(tris), len(tris), _ptr(rs), _ptr(rd),
                                   _ptr(ps), _ptr(c), _ptr(sun), D, _ptr(fr), nu, nv, bounces, int(bool(jitter)),
                                   float(flux), int(seed), int(dir_index_base), int(design_index), _ptr(px), n_pix,
                                   _ptr(hits), int(bool(footprint)), _ptr(F), _ptr(T))
    if st != 0:
        raise ValueError(f"oracle_trace_frozen failed ({st})")
    return F, T


def edge_term(verts, tris, vert_hinge, hinge_origin, hinge_axis, rho_s, rho_d, sun_dirs, frames_in, *, bounces: int,
              samples: int, flux: float = 1361.0, seed: int = 0, dir_index_base: int = 0, design_index: int = 0,
              p_spec=None, com=None, threads: int | None = None, drop_smooth: bool = True):
    """Visibility-edge part of d(F, tau)/d(hinge angle) by edge sampling (see srp_oracle.c):
    [D][H][6] (force, torque per radian) and the number of moving edges.  drop_smooth leaves out
    the edges across which the integrand is continuous (oracle/edges.py)."""
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    vh = np.ascontiguousarray(vert_hinge, dtype=np.int32)
    ho = np.ascontiguousarray(hinge_origin, dtype=np.float64).reshape(-1, 3)
    ha = np.ascontiguousarray(hinge_axis, dtype=np.float64).reshape(-1, 3)
    ha = np.ascontiguousarray(ha / np.linalg.norm(ha, axis=1)[:, None]) if len(ha) else ha
    rs = np.ascontiguousarray(rho_s, dtype=np.float32)
    rd = np.ascontiguousarray(rho_d, dtype=np.float32)
    ps = None if p_spec is None else np.ascontiguousarray(p_spec, dtype=np.float32)
    c = None if com is None else np.ascontiguousarray(com, dtype=np.float64)
    sun = np.ascontiguousarray(sun_dirs, dtype=np.float64).reshape(-1, 3)
    D = len(sun)
    fr = np.ascontiguousarray(frames_in, dtype=np.float64).reshape(D, 12)
    out = np.zeros((D, len(ho), 6))
    ne = ctypes.c_int64(0)
    if threads is None:
        threads = default_threads()
    keep = None
    if drop_smooth:
        from .edges import smooth_edge_mask
        keep = np.ascontiguousarray(~smooth_edge_mask(verts, tris, vh, rs, rd, ps), dtype=np.uint8)
    st = lib().oracle_edge_term(_ptr(verts), len(verts), _ptr(tris), len(tris), _ptr(vh), _ptr(ho), _ptr(ha), len(ho),
                                _ptr(rs), _ptr(rd), _ptr(ps), _ptr(c), _ptr(sun), D, _ptr(fr), int(bounces), float(flux),
                                int(seed), int(dir_index_base), int(design_index), int(samples), _ptr(keep),
                                0 if keep is None else len(keep), _ptr(out), ctypes.byref(ne), int(threads))
    if st != 0:
        raise ValueError(f"oracle_edge_term failed ({st})")
    return out, int(ne.value)


class SurfaceResult:
    def __init__(self, force, torque, facet=None, hits=None, lit=None, degen=None, sample_force=None):
        self.force = force
        self.torque = torque
        self.facet = facet
        self.hits = hits
        self.lit = lit
        self.degen = degen
        self.sample_force = sample_force


def surface_estimate(verts, tris, rho_s, rho_d, sun_dirs, *, n_samples: int, bounces: int, flux: float = 1361.0,
                     seed: int = 0, dir_index_base: int = 0, design_index: int = 0, p_spec=None, com=None,
                     records: bool = False, threads: int | None = None, sampling: int = 0,
                     phong=None) -> SurfaceResult:
    """FP64 surface-sampling estimate (area-sampled points, path-traced gathering with next-event
    estimation toward the Sun); see srp_oracle.c for the definition.  force/torque: sample means.
    sampling: bit 0 stratified surface, bit 1 uniform hemisphere directions (plain MC).
    phong: per-facet Phong exponents (>= 1, inf = ideal mirror), None = all mirrors."""
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    rs = np.ascontiguousarray(rho_s, dtype=np.float32)
    rd = np.ascontiguousarray(rho_d, dtype=np.float32)
    ps = None if p_spec is None else np.ascontiguousarray(p_spec, dtype=np.float32)
    ph = None if phong is None else np.ascontiguousarray(np.broadcast_to(phong, (len(tris),)), dtype=np.float32)
    c = None if com is None else np.ascontiguousarray(com, dtype=np.float64)
    sun = np.ascontiguousarray(sun_dirs, dtype=np.float64).reshape(-1, 3)
    D = len(sun)
    force = np.zeros((D, 3))
    torque = np.zeros((D, 3))
    fa = hi = li = dg = sf = None
    if records:
        fa = np.zeros((D, n_samples), dtype=np.int32)
        hi = np.zeros((D, n_samples, max(bounces - 1, 1)), dtype=np.int32)
        li = np.zeros((D, n_samples), dtype=np.int32)
        dg = np.zeros((D, n_samples), dtype=np.uint8)
        sf = np.zeros((D, n_samples, 3))
    if threads is None:
        threads = default_threads()
    st = lib().oracle_surface_estimate(_ptr(verts), len(verts), _ptr(tris), len(tris), _ptr(rs), _ptr(rd), _ptr(ps),
                                       _ptr(ph), _ptr(c), _ptr(sun), D, int(n_samples), int(bounces), float(flux), int(seed),
                                       int(dir_index_base), int(design_index), _ptr(force), _ptr(torque), _ptr(fa),
                                       _ptr(hi), _ptr(li), _ptr(dg), _ptr(sf), int(sampling), int(threads))
    if st != 0:
        raise ValueError(f"oracle_surface_estimate failed ({st})")
    if records and bounces == 1:
        hi = hi[:, :, :0]
    return SurfaceResult(force, torque, fa, hi, li, dg, sf)


def surface_designs(verts, tris, vert_hinge, hinge_origin, hinge_axis, group, n_groups, designs, sun, *,
                    samples: int, bounces: int, flux: float = 1361.0, seed: int = 0, dir_index_base: int = 0,
                    design_index: int = 0, sampling: int = 0, com=None, records: bool = False,
                    threads: int | None = None) -> SurfaceResult:
    """FP64 multi-world surface sampling: pair i (sun[i], designs[i]) applies its hinge angles to the
    rest pose and its group materials (rho_s, rho_d, Phong exponent per group) and averages
    `samples` samples with direction index dir_index_base + i (see srp_oracle.c).  force/torque:
    [N][3] per pair; records [N][samples]."""
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    vh = None if vert_hinge is None else np.ascontiguousarray(vert_hinge, dtype=np.int32)
    ho = np.ascontiguousarray(hinge_origin, dtype=np.float64).reshape(-1, 3)
    ha = np.ascontiguousarray(hinge_axis, dtype=np.float64).reshape(-1, 3)
    ha = np.ascontiguousarray(ha / np.linalg.norm(ha, axis=1)[:, None]) if len(ha) else ha
    grp = np.ascontiguousarray(group, dtype=np.int32)
    dsg = np.ascontiguousarray(designs, dtype=np.float64).reshape(len(np.atleast_2d(designs)), -1)
    sn = np.ascontiguousarray(sun, dtype=np.float64).reshape(-1, 3)
    N = len(sn)
    assert dsg.shape == (N, len(ho) + 3 * int(n_groups))
    c = None if com is None else np.ascontiguousarray(com, dtype=np.float64)
    force = np.zeros((N, 3))
    torque = np.zeros((N, 3))
    fa = hi = li = dg = None
    if records:
        fa = np.zeros((N, samples), dtype=np.int32)
        hi = np.zeros((N, samples, max(bounces - 1, 1)), dtype=np.int32)
        li = np.zeros((N, samples), dtype=np.int32)
        dg = np.zeros((N, samples), dtype=np.uint8)
    if threads is None:
        threads = default_threads()
    st = lib().oracle_surface_designs(_ptr(verts), len(verts), _ptr(tris), len(tris), _ptr(vh), _ptr(ho), _ptr(ha),
                                      len(ho), _ptr(grp), int(n_groups), _ptr(dsg), _ptr(sn), N, int(samples),
                                      int(bounces), float(flux), int(seed), int(dir_index_base), int(design_index),
                                      int(sampling), _ptr(c), _ptr(force), _ptr(torque), _ptr(fa), _ptr(hi), _ptr(li),
                                      _ptr(dg), int(threads))
    if st != 0:
        raise ValueError(f"oracle_surface_designs failed ({st})")
    if records and bounces == 1:
        hi = hi[:, :, :0]
    return SurfaceResult(force, torque, fa, hi, li, dg, None)

