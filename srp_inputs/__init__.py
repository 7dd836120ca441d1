"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and by the oracle.

This module holds no arithmetic of the radiation-pressure method itself: it only builds the
things the method is applied to -- triangle meshes of spacecraft-like bodies (with hinge groups
and material groups), per-facet reflectance draws and sets of sun directions.  Both the GPU path
and the oracle consume these, so they trace exactly the same inputs.

Workload shapes follow the paper's evaluation: box-wing buses with flat panels (the classic
box-wing decomposition named in Sec. 2) and ~20k-triangle satellites with unbalanced, partly
degenerate tessellation (Sec. 4.2, Tab. "Speed": high-resolution meshes of 2.2k-25k triangles
"with unbalanced and degenerate meshing").  The real meshes are not available; the generators
below stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BUS, PANEL, PAYLOAD = 0, 1, 2


@dataclass
class Mesh:
    """Triangle mesh in the body frame (metres).

    verts      [V][3] float64
    tris       [T][3] int32, counter-clockwise seen from outside (outward normal (v1-v0)x(v2-v0))
    vert_hinge [V] int32, -1 for rigid vertices, k for vertices carried by hinge k
    hinge_origin, hinge_axis [H][3] float64 (axis unit length)
    group      [T] int32 material group: BUS, PANEL or PAYLOAD
    com        [3] float64 centre of mass
    """

    verts: np.ndarray
    tris: np.ndarray
    vert_hinge: np.ndarray
    hinge_origin: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    hinge_axis: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    group: np.ndarray | None = None
    com: np.ndarray = field(default_factory=lambda: np.zeros(3))

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_hinges(self) -> int:
        return int(self.hinge_origin.shape[0])


class _Builder:
    def __init__(self):
        self.v: list[np.ndarray] = []
        self.t: list[np.ndarray] = []
        self.h: list[np.ndarray] = []
        self.g: list[np.ndarray] = []
        self.nv = 0

    def add(self, verts, tris, hinge=-1, group=BUS):
        verts = np.asarray(verts, dtype=np.float64).reshape(-1, 3)
        tris = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
        self.v.append(verts)
        self.t.append(tris + self.nv)
        self.h.append(np.full(len(verts), hinge, dtype=np.int32))
        self.g.append(np.full(len(tris), group, dtype=np.int32))
        self.nv += len(verts)

    def mesh(self, hinge_origin=None, hinge_axis=None, com=None) -> Mesh:
        ho = np.zeros((0, 3)) if hinge_origin is None else np.asarray(hinge_origin, dtype=np.float64).reshape(-1, 3)
        ha = np.zeros((0, 3)) if hinge_axis is None else np.asarray(hinge_axis, dtype=np.float64).reshape(-1, 3)
        return Mesh(
            verts=np.ascontiguousarray(np.concatenate(self.v)),
            tris=np.ascontiguousarray(np.concatenate(self.t).astype(np.int32)),
            vert_hinge=np.ascontiguousarray(np.concatenate(self.h)),
            hinge_origin=ho,
            hinge_axis=ha,
            group=np.ascontiguousarray(np.concatenate(self.g)),
            com=np.zeros(3) if com is None else np.asarray(com, dtype=np.float64),
        )


def quad_grid(origin, eu, ev, nu: int, nv: int):
    """Parallelogram origin + s*eu + t*ev, s,t in [0,1], split into nu x nv quads (2 tris each).
    The triangles face eu x ev."""
    origin, eu, ev = (np.asarray(a, dtype=np.float64) for a in (origin, eu, ev))
    s = np.linspace(0.0, 1.0, nu + 1)
    t = np.linspace(0.0, 1.0, nv + 1)
    S, Tt = np.meshgrid(s, t, indexing="ij")
    verts = origin + S[..., None] * eu + Tt[..., None] * ev
    verts = verts.reshape(-1, 3)
    idx = np.arange((nu + 1) * (nv + 1)).reshape(nu + 1, nv + 1)
    a = idx[:-1, :-1].ravel()
    b = idx[1:, :-1].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[:-1, 1:].ravel()
    tris = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    return verts, tris


def box_faces(lo, hi, n: int = 1):
    """Six outward-facing faces of an axis-aligned box, each n x n quads."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    sx, sy, sz = hi - lo
    X, Y, Z = np.eye(3)
    faces = [
        ((hi[0], lo[1], lo[2]), Y * sy, Z * sz),  # +x
        ((lo[0], lo[1], lo[2]), Z * sz, Y * sy),  # -x
        ((lo[0], hi[1], lo[2]), Z * sz, X * sx),  # +y
        ((lo[0], lo[1], lo[2]), X * sx, Z * sz),  # -y
        ((lo[0], lo[1], hi[2]), X * sx, Y * sy),  # +z
        ((lo[0], lo[1], lo[2]), Y * sy, X * sx),  # -z
    ]
    out = []
    for o, eu, ev in faces:
        out.append(quad_grid(o, eu, ev, n, n))
    return out


def two_sided(verts, tris):
    """Return (verts, tris) of the same surface with the opposite winding (back layer)."""
    return verts.copy(), tris[:, [0, 2, 1]].copy()


def cylinder(center, radius, z0, z1, sides: int, caps: bool = True):
    """Cylinder along +z with outward-facing side and (optionally) caps; fan-triangulated caps
    without a centre vertex (sides-2 triangles each)."""
    cx, cy = center
    phi = 2.0 * np.pi * np.arange(sides) / sides
    ring = np.stack([cx + radius * np.cos(phi), cy + radius * np.sin(phi)], 1)
    bottom = np.concatenate([ring, np.full((sides, 1), z0)], 1)
    top = np.concatenate([ring, np.full((sides, 1), z1)], 1)
    verts = np.concatenate([bottom, top])
    k = np.arange(sides)
    k1 = (k + 1) % sides
    b0, b1, t0, t1 = k, k1, sides + k, sides + k1
    tris = [np.stack([b0, b1, t1], 1), np.stack([b0, t1, t0], 1)]
    if caps:
        m = np.arange(1, sides - 1)
        tris.append(np.stack([np.full_like(m, sides), sides + m, sides + m + 1], 1))  # top, +z
        tris.append(np.stack([np.zeros_like(m), m + 1, m], 1))  # bottom, -z
    return verts, np.concatenate(tris)


def transform(verts, R, t):
    return np.asarray(verts) @ np.asarray(R, dtype=np.float64).T + np.asarray(t, dtype=np.float64)


def paraboloid_dish(radius: float, depth: float, radii: np.ndarray, sectors: int):
    """Concave side of a paraboloid dish opening toward +z: z = depth*(r/radius)^2.
    `radii` are the ring radii (ascending, > 0); a centre fan joins the first ring."""
    phi = 2.0 * np.pi * np.arange(sectors) / sectors
    rings = []
    for r in radii:
        z = depth * (r / radius) ** 2
        rings.append(np.stack([r * np.cos(phi), r * np.sin(phi), np.full(sectors, z)], 1))
    verts = np.concatenate([np.zeros((1, 3))] + rings)
    k = np.arange(sectors)
    k1 = (k + 1) % sectors
    tris = [np.stack([np.zeros(sectors, dtype=np.int64), 1 + k, 1 + k1], 1)]
    for j in range(len(radii) - 1):
        a = 1 + j * sectors + k
        a1 = 1 + j * sectors + k1
        b = 1 + (j + 1) * sectors + k
        b1 = 1 + (j + 1) * sectors + k1
        tris.append(np.stack([a, b, b1], 1))
        tris.append(np.stack([a, b1, a1], 1))
    return verts, np.concatenate(tris)


# ---------------------------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------------------------
def box_wing() -> Mesh:
    """1 m cube bus (12 tris) + two 5 x 1.5 m two-sided flat panels in the z = 0 plane
    (x in [-0.75, 0.75], y in +-[1, 6]; 2 tris per side each): 20 tris."""
    B = _Builder()
    for v, t in box_faces((-0.5, -0.5, -0.5), (0.5, 0.5, 0.5), 1):
        B.add(v, t, group=BUS)
    for k, (y0, y1) in enumerate([(1.0, 6.0), (-6.0, -1.0)]):
        v, t = quad_grid((-0.75, y0, 0.0), (1.5, 0, 0), (0, y1 - y0, 0), 1, 1)  # faces +z
        B.add(v, t, hinge=k, group=PANEL)
        vb, tb = two_sided(v, t)
        B.add(vb, tb, hinge=k, group=PANEL)
    return B.mesh(hinge_origin=[(0, 1.0, 0), (0, -1.0, 0)], hinge_axis=[(0, 1, 0), (0, 1, 0)])


def meo_satellite(bus_n: int = 20, cyl_sides: int = 64, panel_n: int = 16, dish_rings: int = 24,
                  dish_sectors: int = 48, strut_sides: int = 16, n_antennas: int = 12) -> Mesh:
    """Procedural MEO-style satellite, ~20.6k triangles at the default tessellation:
    bus 2.5 x 2 x 2 m (faces bus_n x bus_n quads), an array of closed cylindrical antennas on +z,
    two hinged wings of 4 segments 1.8 x 1.6 m each (two-sided, panel_n x panel_n quads), a
    two-sided parabolic dish (diameter 1.2 m, depth 0.2 m) on -x whose outer 5 rings are radially
    thin slivers (aspect > 20), and 2 open struts holding it."""
    B = _Builder()
    for v, t in box_faces((-1.25, -1.0, -1.0), (1.25, 1.0, 1.0), bus_n):
        B.add(v, t, group=BUS)
    xs = [-0.9, -0.3, 0.3, 0.9]
    ys = [-0.6, 0.0, 0.6]
    pos = [(x, y) for y in ys for x in xs][:n_antennas]
    for (x, y) in pos:
        v, t = cylinder((x, y), 0.1, 1.0, 1.6, cyl_sides, caps=True)
        B.add(v, t, group=PAYLOAD)
    gap = 0.02
    for k, sgn in enumerate([1.0, -1.0]):
        for seg in range(4):
            y0 = 1.2 + gap + seg * 1.8
            ya, yb = (y0, y0 + 1.8 - gap) if sgn > 0 else (-(y0 + 1.8 - gap), -y0)
            v, t = quad_grid((-0.8, ya, 0.0), (1.6, 0, 0), (0, yb - ya, 0), panel_n, panel_n)
            B.add(v, t, hinge=k, group=PANEL)
            vb, tb = two_sided(v, t)
            B.add(vb, tb, hinge=k, group=PANEL)
    n_thin = 5
    n_reg = dish_rings - n_thin
    radii = np.concatenate([0.59 * np.arange(1, n_reg + 1) / n_reg, 0.59 + 0.002 * np.arange(1, n_thin + 1)])
    v, t = paraboloid_dish(0.6, 0.2, radii, dish_sectors)
    # local (x, y, z) -> body (x_v - z, y, x): the dish opens toward -x with its vertex at x = -1.7
    R = np.array([[0.0, 0.0, -1.0], [0.0, 1.0, 0.0], [1.0, 0.0, 0.0]])
    v = transform(v, R, (-1.7, 0.0, 0.0))
    B.add(v, t, group=PAYLOAD)
    vb, tb = two_sided(v, t)
    B.add(vb, tb, group=PAYLOAD)
    # struts along -x from the bus face to the dish
    Rs = np.array([[0.0, 0.0, -1.0], [0.0, 1.0, 0.0], [1.0, 0.0, 0.0]])
    for y in (0.3, -0.3):
        v, t = cylinder((0.0, y), 0.03, 0.0, 0.47, strut_sides, caps=False)
        v = transform(v, Rs, (-1.25, 0.0, 0.0))
        B.add(v, t, group=PAYLOAD)
    return B.mesh(hinge_origin=[(0, 1.2, 0), (0, -1.2, 0)], hinge_axis=[(0, 1, 0), (0, 1, 0)])


def meo_variant(target_tris: int) -> Mesh:
    """MEO-style satellite with its tessellation scaled so that it has roughly target_tris."""
    s = np.sqrt(max(target_tris, 500) / 20592.0)
    return meo_satellite(bus_n=max(2, int(round(20 * s))), cyl_sides=max(8, int(round(64 * s))),
                         panel_n=max(2, int(round(16 * s))), dish_rings=max(8, int(round(24 * s))),
                         dish_sectors=max(8, int(round(48 * s))), strut_sides=max(6, int(round(16 * s))))


def icosphere(level: int = 2, radius: float = 1.0) -> Mesh:
    """Icosahedron subdivided `level` times, vertices pushed to the sphere; outward winding."""
    p = (1.0 + 5 ** 0.5) / 2.0
    v = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0), (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
         (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(x, dtype=np.float64) / np.linalg.norm(x) for x in v]
    faces = list(f)
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.array(verts) * radius
    T = np.array(faces, dtype=np.int32)
    # orient outward
    n = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    flip = np.einsum("ij,ij->i", n, V[T].mean(1)) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    B = _Builder()
    B.add(V, T)
    return B.mesh()


def plate(width: float, height: float, center=(0.0, 0.0, 0.0), tilt_deg: float = 0.0, nu: int = 1, nv: int = 1) -> Mesh:
    """One-sided width x height plate facing +z, tilted by tilt_deg about the x axis
    (its normal turns toward -y), centred at `center`."""
    v, t = quad_grid((-width / 2, -height / 2, 0.0), (width, 0, 0), (0, height, 0), nu, nv)
    a = np.deg2rad(tilt_deg)
    R = np.array([[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]])
    v = transform(v, R, center)
    B = _Builder()
    B.add(v, t)
    return B.mesh()


def dihedral(length: float, height: float) -> Mesh:
    """Two one-sided length x height plates meeting at 90 degrees along the z axis: one in the
    x = 0 plane facing +x (y in [0, length]), one in the y = 0 plane facing +y (x in [0, length])."""
    B = _Builder()
    v, t = quad_grid((0, 0, 0), (0, length, 0), (0, 0, height), 1, 1)  # faces y x z = +x
    B.add(v, t)
    v, t = quad_grid((0, 0, 0), (0, 0, height), (length, 0, 0), 1, 1)  # faces z x x = +y
    B.add(v, t)
    return B.mesh()


def fibonacci_dirs(n: int) -> np.ndarray:
    """Spherical Fibonacci point set: z_k = 1 - (2k+1)/n, phi_k = k*pi*(3 - sqrt 5)."""
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = k * np.pi * (3.0 - np.sqrt(5.0))
    return np.ascontiguousarray(np.stack([r * np.cos(phi), r * np.sin(phi), z], 1))


def random_dirs(n: int, seed: int) -> np.ndarray:
    """Uniform directions on the sphere (normalised Gaussian vectors)."""
    g = np.random.default_rng(seed).standard_normal((n, 3))
    return np.ascontiguousarray(g / np.linalg.norm(g, axis=1, keepdims=True))


def materials(n_tris: int, seed: int, lo: float = 0.0, hi: float = 0.5):
    """Per-facet (rho_s, rho_d) ~ U(lo, hi) as float32; absorbed fraction 1 - rho_s - rho_d."""
    rng = np.random.default_rng(seed)
    rs = rng.uniform(lo, hi, n_tris).astype(np.float32)
    rd = rng.uniform(lo, hi, n_tris).astype(np.float32)
    return rs, rd


# Design vector of the procedural satellites (8 parameters):
# [hinge_1, hinge_2 (rad), rho_s_bus, rho_d_bus, rho_s_panel, rho_d_panel, rho_s_payload, rho_d_payload]
DESIGN_LO = np.array([-np.pi / 6, -np.pi / 6, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
DESIGN_HI = np.array([np.pi / 6, np.pi / 6, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5])


def design_materials(mesh: Mesh, theta) -> tuple[np.ndarray, np.ndarray]:
    """Broadcast the group reflectances of a design vector to per-facet float32 arrays."""
    theta = np.asarray(theta, dtype=np.float64)
    rs = theta[2 + 2 * mesh.group].astype(np.float32)
    rd = theta[3 + 2 * mesh.group].astype(np.float32)
    return rs, rd


def random_designs(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return DESIGN_LO + (DESIGN_HI - DESIGN_LO) * rng.uniform(size=(n, 8))


# ---------------------------------------------------------------------------------------------
# orbit scenario (inputs of the orbit integration: initial state, attitude at the stage times,
# body-frame sun directions); a circular MEO orbit with a nadir-pointing attitude law
# ---------------------------------------------------------------------------------------------
MU_EARTH = 3.986004418e14  # m^3/s^2


@dataclass
class OrbitScenario:
    z0: np.ndarray          # [6] inertial position (m) and velocity (m/s)
    mu: float
    mass: float             # kg
    dt: float               # s
    n_steps: int
    R: np.ndarray           # [2 n + 1][3][3] body -> inertial rotation at the stage times t = k dt / 2
    sun_body: np.ndarray    # [2 n + 1][3] unit sun direction in the body frame at the stage times
    sun_inertial: np.ndarray


def meo_orbit(n_steps: int = 1440, dt: float = 60.0, radius: float = 26_560_000.0, incl_deg: float = 55.0,
              beta_deg: float = 30.0, mass: float = 1000.0) -> OrbitScenario:
    """Circular orbit (right ascension of the ascending node 0) starting at the ascending node; the
    attitude follows the nominal circular orbit (body +z to nadir, +y against the orbit normal,
    +x = y x z along track), so it is a function of time only; the Sun is fixed in inertial space at
    elevation beta above the orbit plane (beta = 30 deg > 13.9 deg: no eclipse at this radius)."""
    i = np.deg2rad(incl_deg)
    n_mean = np.sqrt(MU_EARTH / radius ** 3)
    z0 = np.array([radius, 0.0, 0.0, 0.0, radius * n_mean * np.cos(i), radius * n_mean * np.sin(i)])
    h_hat = np.array([0.0, -np.sin(i), np.cos(i)])
    beta = np.deg2rad(beta_deg)
    sun = np.cos(beta) * np.array([1.0, 0.0, 0.0]) + np.sin(beta) * h_hat
    t = np.arange(2 * n_steps + 1) * (dt / 2.0)
    u = n_mean * t
    r_hat = np.stack([np.cos(u), np.sin(u) * np.cos(i), np.sin(u) * np.sin(i)], 1)
    z_b = -r_hat
    y_b = np.broadcast_to(-h_hat, z_b.shape)
    x_b = np.cross(y_b, z_b)
    R = np.ascontiguousarray(np.stack([x_b, y_b, z_b], 2))  # columns = body axes in inertial coordinates
    sun_body = np.ascontiguousarray(np.einsum("kij,i->kj", R, sun))
    return OrbitScenario(z0=z0, mu=MU_EARTH, mass=mass, dt=dt, n_steps=n_steps, R=R, sun_body=sun_body,
                         sun_inertial=sun)


# body-frame inertia tensor of a 1000 kg bus with deployed arrays (kg m^2), slightly off-principal
ATTITUDE_INERTIA = np.array([[900.0, 12.0, -5.0], [12.0, 1300.0, 8.0], [-5.0, 8.0, 1600.0]])


def attitude_states(B: int, seed: int, radius: float = 2.656e7, spread: float = 0.05, sun_plane=None) -> np.ndarray:
    """B seeded 13-D states (r, v, q, w): near-circular orbits of radius radius (1 +- spread) in
    random planes (planes holding `sun_plane` when given, so that low orbits cross the shadow),
    random unit attitude quaternions and body rates uniform in +-0.02 rad/s."""
    rng = np.random.default_rng(seed)
    z = np.zeros((B, 13))
    n = rng.normal(size=(B, 3))
    if sun_plane is not None:
        n = np.cross(np.asarray(sun_plane, dtype=np.float64), n)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    u = np.cross(n, rng.normal(size=(B, 3)))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    r = radius * (1 + spread * rng.uniform(-1, 1, size=(B, 1)))
    z[:, :3] = r * u
    z[:, 3:6] = np.sqrt(MU_EARTH / r) * np.cross(n, u)
    q = rng.normal(size=(B, 4))
    z[:, 6:10] = q / np.linalg.norm(q, axis=1, keepdims=True)
    z[:, 10:13] = rng.uniform(-0.02, 0.02, size=(B, 3))
    return z
