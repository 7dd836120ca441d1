"""Pins of the oracle's multi-world surface sampling (oracle_surface_designs, CPU only).

Pair i of a call is its own world: the hinge angles of its design applied to the rest pose and the
materials of its groups.  Each pair must equal the pinned single-design estimator
(oracle.surface_estimate) run on the mesh that the pinned design step (oracle.design.apply_hinges)
gives for that design, with the per-facet materials of its groups and the pair's direction index:
same samples, so the same records and the same force up to the last bits of the two FP64 rotations.
Invalid designs and groups are refused.
"""
import numpy as np
import pytest

import oracle
import srp_inputs as si
from oracle.design import apply_hinges


def _designs(n, n_groups, seed):
    rng = np.random.default_rng(seed)
    ang = rng.uniform(-0.5, 0.5, (n, 2))
    mats = []
    for g in range(n_groups):
        rs = rng.uniform(0.0, 0.5, n)
        rd = rng.uniform(0.0, 0.5, n)
        m = np.where(rng.uniform(size=n) < 0.3, np.inf, rng.uniform(1.0, 80.0, n))
        mats.append(np.stack([rs, rd, m], 1))
    return np.concatenate([ang] + mats, 1)


@pytest.mark.parametrize("sampling", [0, 3])
def test_each_pair_is_its_own_world(sampling):
    m = si.meo_satellite(bus_n=4, cyl_sides=12, panel_n=3, dish_rings=6, dish_sectors=12, strut_sides=6)
    G = 3
    group = np.asarray(m.group, dtype=np.int32)
    N, K = 5, 200
    dsg = _designs(N, G, 11 + sampling)
    sun = si.random_dirs(N, seed=12)
    res = oracle.surface_designs(m.verts, m.tris, m.vert_hinge, m.hinge_origin, m.hinge_axis, group, G, dsg, sun,
                                 samples=K, bounces=3, seed=13, dir_index_base=100, design_index=7, sampling=sampling,
                                 com=m.com, records=True)
    for i in range(N):
        V = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, dsg[i, :2])
        mat = dsg[i, 2:].reshape(G, 3)[group]
        one = oracle.surface_estimate(V, m.tris, mat[:, 0].astype(np.float32), mat[:, 1].astype(np.float32),
                                      sun[i:i + 1], n_samples=K, bounces=3, seed=13, dir_index_base=100 + i,
                                      design_index=7, sampling=sampling, com=m.com, records=True,
                                      phong=mat[:, 2].astype(np.float32))
        assert np.array_equal(res.facet[i], one.facet[0])
        assert np.array_equal(res.lit[i], one.lit[0])
        assert np.array_equal(res.hits[i], one.hits[0])
        assert np.allclose(res.force[i], one.force[0], rtol=1e-12, atol=1e-22)
        assert np.allclose(res.torque[i], one.torque[0], rtol=1e-12, atol=1e-22)


def test_invalid_designs_refused():
    m = si.box_wing()
    group = np.asarray(m.group, dtype=np.int32)
    dsg = _designs(2, 3, 1)
    sun = si.random_dirs(2, seed=2)
    kw = dict(samples=4, bounces=2)
    args = (m.verts, m.tris, m.vert_hinge, m.hinge_origin, m.hinge_axis)
    bad = dsg.copy()
    bad[1, 2] = 0.7
    bad[1, 3] = 0.5  # rho_s + rho_d > 1
    with pytest.raises(ValueError):
        oracle.surface_designs(*args, group, 3, bad, sun, **kw)
    bad = dsg.copy()
    bad[0, 4] = 0.5  # Phong exponent below 1
    with pytest.raises(ValueError):
        oracle.surface_designs(*args, group, 3, bad, sun, **kw)
    with pytest.raises(ValueError):
        oracle.surface_designs(*args, np.full_like(group, 3), 3, dsg, sun, **kw)
