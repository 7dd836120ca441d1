"""Host checks of the BVH builder and refit (g++ build of the library's builder, no GPU), with
AddressSanitizer + UBSan: every triangle in exactly one leaf, every leaf box contains its
triangles, child boxes nest in their parents, children after parents (pre-order), leaves <= 7,
depth below the traversal stack; the same after refitting to hinge-rotated vertices."""
import os
import subprocess

import numpy as np
import pytest

import srp_inputs as si
from oracle.design import apply_hinges

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("bvh") / "bvh_check")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-o", exe, os.path.join(HERE, "native", "bvh_check.cpp"),
           os.path.join(ROOT, "paper_2602_10712_amd", "csrc", "bvh_build.cpp")]
    try:
        subprocess.run(cmd, check=True, capture_output=True)
    except (OSError, subprocess.CalledProcessError) as e:
        pytest.skip(f"host build unavailable: {e}")
    return exe


def run(exe, V, T, pad, V2=None):
    lines = [f"{len(V)} {len(T)} {pad!r} {0 if V2 is None else 1}"]
    lines.append(" ".join(repr(float(x)) for x in np.asarray(V).ravel()))
    lines.append(" ".join(str(int(x)) for x in np.asarray(T).ravel()))
    if V2 is not None:
        lines.append(" ".join(repr(float(x)) for x in np.asarray(V2).ravel()))
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True)
    assert r.returncode == 0, (r.stdout, r.stderr[-2000:])
    rows = [list(map(int, l.split())) for l in r.stdout.strip().splitlines()]
    for nodes, depth, max_leaf, once, contain, nested in rows:
        assert once and contain and nested
        assert max_leaf <= 7 and depth < 62
    return rows


def test_meo_satellite_and_refit(checker):
    m = si.meo_satellite()
    V2 = apply_hinges(m.verts, m.vert_hinge, m.hinge_origin, m.hinge_axis, [0.5, -0.4])
    rows = run(checker, m.verts, m.tris, 1e-6 * 17.0, V2)
    assert rows[0][0] < m.n_tris  # binary tree with leaves of several triangles


@pytest.mark.parametrize("case", ["plate", "box_wing", "coincident", "soup"])
def test_small_and_degenerate_inputs(checker, case):
    rng = np.random.default_rng(3)
    if case == "plate":
        m = si.plate(1.0, 1.0)
        V, T = m.verts, m.tris
    elif case == "box_wing":
        m = si.box_wing()
        V, T = m.verts, m.tris
    elif case == "coincident":
        # 300 copies of the same triangle: all centroids equal -> object-median splits only
        V = np.tile(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float), (300, 1))
        T = np.arange(900).reshape(300, 3)
    else:
        V = rng.normal(0, 1, (3000, 3))
        T = rng.integers(0, 3000, (1000, 3))
    run(checker, V, T, 1e-6)
