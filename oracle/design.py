"""Oracle: design application -- TEST INFRASTRUCTURE ONLY.

The design vector moves the hinged panels (Sec. 3.1 / Sec. 3.2: the spacecraft is a map from
design parameters to a triangle mesh).  Panel k's vertices rotate by the angle theta_k about the
hinge line (origin_k, unit axis_k), right-hand rule (Rodrigues' rotation formula).
"""
from __future__ import annotations

import numpy as np


def rotate_about(points, origin, axis, angle):
    p = np.asarray(points, dtype=np.float64) - origin
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    c, s = np.cos(angle), np.sin(angle)
    return origin + p * c + np.cross(a, p) * s + np.outer(p @ a, a) * (1.0 - c)


def apply_hinges(verts, vert_hinge, hinge_origin, hinge_axis, angles) -> np.ndarray:
    out = np.array(verts, dtype=np.float64, copy=True)
    vh = np.asarray(vert_hinge)
    for k, ang in enumerate(np.asarray(angles, dtype=np.float64).ravel()):
        m = vh == k
        if m.any():
            out[m] = rotate_about(out[m], np.asarray(hinge_origin[k], dtype=np.float64), hinge_axis[k], ang)
    return out
