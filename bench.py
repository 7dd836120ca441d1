"""Benchmark of the ray-grid SRP hot path on one MI355X.

One step = one forward trace of the procedural MEO-style satellite (20,592 triangles, binned-SAH
BVH) for 1024 spherical-Fibonacci sun directions x 1024 x 1024 parallel rays, up to 3 surface
interactions per path, FP64 force and torque per direction.  Inputs (mesh, BVH, materials, sun
directions) are resident in HBM before the timed region; the BVH build is timed separately.

Prints ONE JSON line:
  value            forward Mrays/s (primary grid rays, whole paths, per second)
  fwd_adjoint      forward + adjoint replay Mrays/s at 512 x 512 rays per direction
  surrogate        fused MLP surrogate evals/s on 1M queries, with its MFMA roofline fraction
  batched          one launch over 256 design variants (2k-50k tris) x 256 dirs x 512^2 rays
  orbit            one design-gradient iteration through a day of RK4 orbit (2881 directions, 512^2)
  surface          the paper's surface-sampling estimator: samples/s with the BVH and by brute force;
                   the GPU BVH build and what its tree costs the walks
  attitude         13-D orbit-and-attitude RK4 (FP64) with the network answering force and torque at
                   every stage: trajectory-steps/s for 65,536 trajectories x 2,880 steps of 15 s
  rates            grid rays, traced segments and surface interactions per second
  roofline         dominant kernel (k_trace): algorithmic VALU lane-ops per launch / mean launch time
                   against the ALU peak (the scene is cache-resident); HBM-equivalent bytes beside it
  cpu_baseline     the FP64 oracle on a bounded sample of the same workload, host cores
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SRP Mrays/s (20k tri, 3 bounce) fwd & fwd+adjoint; surrogate force evals/s"
HBM_PEAK_GBS = 8000.0
# Vector-ALU issue rates of gfx950 in lanes per SIMD-cycle, by instruction class (measured by
# paper_2602_10712_amd/valu_rates): FP32 FMA/MUL/ADD and integer add 32 (the 157.3 TFLOP/s FP32
# vector peak: 256 CUs x 4 SIMDs x 32 lanes x 2 flop x 2.4 GHz), min/max/compare/select 16,
# transcendentals (reciprocal, exp) 8.
LANES_FAST, LANES_HALF, LANES_TRANS = 32.0, 16.0, 8.0
SIMDS, CLOCK_GHZ = 1024, 2.4
FP32_LANE_PEAK_TOPS = SIMDS * LANES_FAST * CLOCK_GHZ / 1e3  # 78.6 T lane-ops/s, every op an FMA
# Algorithmic lane-ops of the walk by class.  Child-box slab test: 6 FMA (two slab distances per
# axis) + 11 min/max/compare (order each axis's pair, combine the three axes with the ray's
# interval, test entry <= exit).  Moller-Trumbore triangle test: 29 FMA/MUL/ADD (two cross
# products, three dot products, the edge offset, the barycentric sum, t = num / det), 7
# compare/select, 1 reciprocal.
BOX_FAST, BOX_HALF = 6, 11
TRI_FAST, TRI_HALF, TRI_TRANS = 29, 7, 1
ADJ_ATOMIC_BYTES = 16.0  # at most two FP64 gradient updates per hit


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = ["srp_path.h", "srp_traverse.h", "srp_internal.h", "trace_kernels.hip"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2602_10712_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_record(name):
    """The JSON record of a committed counter summary under profiles/, or None when it is missing or
    the trace kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        text = open(path).read()
        blob = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(blob)
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec


def measured_traffic():
    """HBM bytes per k_trace launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's counters)."""
    rec = profile_record("k_trace_meo20k_traffic.md")
    return None if rec is None else rec.get("hbm_bytes_per_launch")


def measured_l2_hit_rate():
    """L2 hit rate of k_trace on the benchmark workload (TCC_HIT / (TCC_HIT + TCC_MISS))."""
    rec = profile_record("k_trace_meo20k_counters.md")
    return None if rec is None else rec.get("l2_hit_rate")


def measured_l2_slot_frac():
    """Share of the L2 request slots (8 XCDs x 16 channels x 1 per cycle) k_trace uses."""
    rec = profile_record("k_trace_meo20k_counters.md")
    return None if rec is None else rec.get("l2_slot_frac")


def measured_valu_issue():
    """Issue time the instruction mix k_trace actually issued needs at the class rates (counters),
    as a fraction of the launch's cycles: [low, high], since the counters do not separate the fast
    moves and bitwise operations from the half-rate min/max/compare/select."""
    rec = profile_record("k_trace_meo20k_counters.md")
    return None if rec is None else rec.get("valu_issue_frac")


def walk_lane_ops(st, passes=1.0):
    """Algorithmic lane-ops per ray of the BVH walk, by class, from the host single-ray traversal
    statistics (child-box tests two per node visited, triangle tests per segment)."""
    seg = st["segments_per_ray"] * passes
    boxes = 2.0 * st["nodes_per_segment"] * seg
    tris = st["tris_per_segment"] * seg
    fast = BOX_FAST * boxes + TRI_FAST * tris
    half = BOX_HALF * boxes + TRI_HALF * tris
    trans = TRI_TRANS * tris
    return fast, half, trans


def alu_roofline(st, rays, seconds, passes=1.0, extra_tris_per_ray=0.0):
    """ALU roofline of the walk: algorithmic lane-ops / time against the class-weighted peak (the
    rate the SIMDs reach on exactly this mix of FMA-class, half-rate and transcendental lane-ops).
    extra_tris_per_ray: triangle tests beyond the walks (the recorded adjoint's)."""
    fast, half, trans = walk_lane_ops(st, passes)
    fast += TRI_FAST * extra_tris_per_ray
    half += TRI_HALF * extra_tris_per_ray
    trans += TRI_TRANS * extra_tris_per_ray
    ops = fast + half + trans
    cycles_per_ray = fast / LANES_FAST + half / LANES_HALF + trans / LANES_TRANS  # SIMD-cycles
    peak = ops / cycles_per_ray * SIMDS * CLOCK_GHZ / 1e3
    achieved = ops * rays / seconds / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 2), "unit": "T lane-ops/s",
            "frac": round(achieved / peak, 4), "lane_ops_per_ray": round(ops, 1),
            "lane_ops_by_class": {"fma_class": round(fast, 1), "half_rate": round(half, 1), "transcendental": round(trans, 2)},
            "peak_if_all_fma": {"peak": round(FP32_LANE_PEAK_TOPS, 1), "frac": round(achieved / FP32_LANE_PEAK_TOPS, 4),
                                "note": "every lane-op at the FP32 FMA rate (157.3 TFLOP/s with an FMA as one lane-op)"}}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dirs", type=int, default=1024)
    ap.add_argument("--grid", type=int, default=1024)
    ap.add_argument("--bounces", type=int, default=3)
    ap.add_argument("--adjoint-grid", type=int, default=512)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-orbit", action="store_true")
    ap.add_argument("--no-surface", action="store_true")
    ap.add_argument("--no-surrogate-training", action="store_true")
    ap.add_argument("--no-attitude", action="store_true")
    ap.add_argument("--attitude-batch", type=int, default=65536)
    ap.add_argument("--attitude-steps", type=int, default=2880)
    ap.add_argument("--batch-designs", type=int, default=256)
    ap.add_argument("--batch-dirs", type=int, default=256)
    ap.add_argument("--batch-grid", type=int, default=512)
    ap.add_argument("--surrogate-batch", type=int, default=1 << 20)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates the HBM traffic counters)")
    ap.add_argument("--cpu-sample-dirs", type=int, default=64)
    ap.add_argument("--cpu-sample-grid", type=int, default=256)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): this build has no multi-GPU path "
              "(directions and designs would shard across ranks with one all-gather of the results)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration:
        torch.cuda.set_device(0)
        n = 1 << 28  # 2^28 float32 = 1 GiB read + 1 GiB written per copy
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch": 4 * n, "launches": 3}), flush=True)
        return

    import paper_2602_10712_amd as p
    import srp_inputs as si

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    mesh = si.meo_satellite()
    rs, rd = si.materials(mesh.n_tris, 1)
    sun = si.fibonacci_dirs(args.dirs)
    angles = [0.0, 0.0]

    t0 = time.perf_counter()
    sc = p.Scene.from_mesh(mesh)
    sc.set_design(rs, rd, hinge_angles=angles)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = sc.info()
    log(f"scene: {mesh.n_tris} tris, {info['n_nodes']} BVH nodes, depth {info['depth']}, build+upload {build_s:.3f} s")

    sun_d = torch.as_tensor(sun, dtype=torch.float64, device=dev).contiguous()
    D = sun_d.shape[0]
    F = torch.empty((D, 3), dtype=torch.float64, device=dev)
    T = torch.empty((D, 3), dtype=torch.float64, device=dev)
    params = p.TraceParams(nu=args.grid, nv=args.grid, bounces=args.bounces, jitter=1, seed=2)
    stream = torch.cuda.current_stream()

    def step():
        p.srp_trace(sc.handle, sun_d, params, F, T, stream=stream.cuda_stream)

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    per_step = []
    t_wall = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        e_a = torch.cuda.Event(enable_timing=True)
        e_b = torch.cuda.Event(enable_timing=True)
        e_a.record(stream)
        step()
        e_b.record(stream)
        per_step.append((e_a, e_b))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    total_ms = ev0.elapsed_time(ev1)
    step_ms = [a.elapsed_time(b) for a, b in per_step]
    for i, ms in enumerate(step_ms):
        log(f"step {i + 1}/{args.steps}: {ms:.2f} ms")
    ms_per_step = total_ms / args.steps
    rays = float(D) * args.grid * args.grid
    mrays = rays / (ms_per_step * 1e-3) / 1e6
    log(f"forward: {ms_per_step:.2f} ms/step, {mrays:.1f} Mrays/s (wall {wall:.2f} s)")
    # rates beside the grid-ray rate (filled from the traversal statistics below): most grid rays
    # miss the scene, so the surface interactions and traced segments per second are printed too
    rates = {"grid_rays_per_s": round(rays / (ms_per_step * 1e-3), 1)}

    # ---- forward + adjoint (differentiable workload: 512^2 rays per direction) --------------------
    fwd_adj = None
    if not args.no_adjoint:
        g = args.adjoint_grid
        pa = p.TraceParams(nu=g, nv=g, bounces=args.bounces, jitter=1, seed=2)
        gen = torch.Generator(device="cpu").manual_seed(3)
        gF = torch.randn((D, 3), generator=gen, dtype=torch.float64).to(dev)
        gT = torch.randn((D, 3), generator=gen, dtype=torch.float64).to(dev)
        g_rs = torch.zeros(mesh.n_tris, dtype=torch.float32, device=dev)
        g_rd = torch.zeros(mesh.n_tris, dtype=torch.float32, device=dev)
        g_h = torch.zeros(2, dtype=torch.float64, device=dev)

        # the forward records every path's facets, and the adjoint reads them back instead of
        # walking the BVH again (same gradients as the walking replay, srp_trace_adjoint)
        paths = torch.empty(p.srp_path_record_bytes(sc.handle, D, pa) // 4, dtype=torch.int32, device=dev)

        def step_adj():
            p.srp_trace_recorded(sc.handle, sun_d, pa, F, T, paths, stream=stream.cuda_stream)
            p.srp_trace_adjoint_recorded(sc.handle, sun_d, pa, gF, paths, gT, g_rs, g_rd, g_h,
                                         stream=stream.cuda_stream)

        def step_replay():
            p.srp_trace(sc.handle, sun_d, pa, F, T, stream=stream.cuda_stream)
            p.srp_trace_adjoint(sc.handle, sun_d, pa, gF, gT, g_rs, g_rd, g_h, stream=stream.cuda_stream)

        for i in range(args.warmup):
            step_adj()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(args.steps):
            step_adj()
        e1.record(stream)
        torch.cuda.synchronize()
        ms_adj = e0.elapsed_time(e1) / args.steps
        rays_a = float(D) * g * g
        fwd_adj = {"value": round(rays_a / (ms_adj * 1e-3) / 1e6, 2), "unit": "Mrays/s", "ms_per_step": round(ms_adj, 3),
                   "workload": f"{D} dirs x {g}x{g} rays, {args.bounces} bounces: forward trace recording each "
                               "path's facets + adjoint over the record (d/d rho_s, rho_d per facet, d/d 2 hinge "
                               "angles)", "record_bytes": int(paths.numel() * 4)}
        try:
            from paper_2602_10712_amd import ray_stats
            sa = ray_stats(sc, sun, pa, n_dirs=16, pixel_stride=97)
            # the forward pass and the replay each touch the path's nodes, triangles and hit records;
            # the replay adds at most two FP64 gradient atomics per hit (one for the sampled event
            # at a reflection, one each for rho_s and rho_d at the final interaction)
            # ALU roofline, as for the forward: the forward and the replay each run the walk's
            # algorithmic lane-ops; the HBM-equivalent figure (the forward's bytes twice plus at most
            # two FP64 gradient atomics per hit) stays beside it, labelled
            # recorded paths: one walk per ray (the adjoint re-tests only the recorded triangle of
            # each segment: counted), 4 B of record written and read per segment
            bpr = sa["bytes_per_ray"] + ADJ_ATOMIC_BYTES * sa["hits_per_ray"] + 8.0 * sa["segments_per_ray"]
            ach = bpr * rays_a / (ms_adj * 1e-3) / 1e9
            fwd_adj["roofline"] = alu_roofline(sa, rays_a, ms_adj * 1e-3, passes=1.0,
                                               extra_tris_per_ray=sa["hits_per_ray"])
            fwd_adj["roofline"].update({"hits_per_ray": round(sa["hits_per_ray"], 4),
                                        "hbm_equivalent": {"achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                                           "frac": round(ach / HBM_PEAK_GBS, 4),
                                                           "bytes_per_ray": round(bpr, 1),
                                                           "note": "not a bound: the scene is L2-resident"}})
        except Exception as e:
            log(f"adjoint roofline stats unavailable: {e!r}")
        log(f"forward+adjoint: {ms_adj:.2f} ms/step, {fwd_adj['value']:.1f} Mrays/s")

        # the two halves alone, and the adjoint with the visibility-edge part of the hinge gradient
        # (edge sampling: 16 points per moving edge and direction, two side paths each)
        def timed(fn):
            fn()
            torch.cuda.synchronize()
            e0.record(stream)
            for i in range(args.steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / args.steps

        pe = p.TraceParams(nu=g, nv=g, bounces=args.bounces, jitter=1, seed=2, edge_samples=16)
        ms_f = timed(lambda: p.srp_trace(sc.handle, sun_d, pa, F, T, stream=stream.cuda_stream))
        ms_fr = timed(lambda: p.srp_trace_recorded(sc.handle, sun_d, pa, F, T, paths, stream=stream.cuda_stream))
        ms_br = timed(lambda: p.srp_trace_adjoint_recorded(sc.handle, sun_d, pa, gF, paths, gT, g_rs, g_rd, g_h,
                                                           stream=stream.cuda_stream))
        ms_e = timed(lambda: p.srp_trace_adjoint_recorded(sc.handle, sun_d, pe, gF, paths, gT, g_rs, g_rd, g_h,
                                                          stream=stream.cuda_stream))
        ms_b = timed(lambda: p.srp_trace_adjoint(sc.handle, sun_d, pa, gF, gT, g_rs, g_rd, g_h,
                                                 stream=stream.cuda_stream))
        ms_rp = timed(step_replay)
        fwd_adj["forward_ms"] = round(ms_f, 3)
        fwd_adj["recorded_forward_ms"] = round(ms_fr, 3)
        fwd_adj["adjoint_ms"] = round(ms_br, 3)
        fwd_adj["adjoint_over_forward"] = round(ms_br / ms_f, 3)
        fwd_adj["replay"] = {"note": "srp_trace + srp_trace_adjoint: the adjoint walks the BVH again",
                             "ms_per_step": round(ms_rp, 3), "value": round(rays_a / (ms_rp * 1e-3) / 1e6, 2),
                             "adjoint_ms": round(ms_b, 3), "adjoint_over_forward": round(ms_b / ms_f, 3)}
        # the design problem's materials (one per part): the flat panels' interior edges carry no
        # jump and are skipped
        sc.set_design(*si.design_materials(mesh, [0.0, 0.0, 0.2, 0.3, 0.1, 0.4, 0.25, 0.15]), hinge_angles=angles)
        ms_bg = timed(lambda: p.srp_trace_adjoint(sc.handle, sun_d, pa, gF, gT, g_rs, g_rd, g_h,
                                                  stream=stream.cuda_stream))
        ms_eg = timed(lambda: p.srp_trace_adjoint(sc.handle, sun_d, pe, gF, gT, g_rs, g_rd, g_h,
                                                  stream=stream.cuda_stream))
        sc.set_design(rs, rd, hinge_angles=angles)
        fwd_adj["edge_term"] = {"edge_samples": 16, "adjoint_ms_with_edges": round(ms_e, 3),
                                "edge_ms": round(ms_e - ms_br, 3),
                                "group_materials": {"edge_ms": round(ms_eg - ms_bg, 3),
                                                    "note": "one material per part: the interior edges of the flat "
                                                            "panels carry no jump and are skipped"}}
        log(f"forward {ms_f:.2f} ms (recording {ms_fr:.2f} ms), adjoint over the record {ms_br:.2f} ms "
            f"({ms_br / ms_f:.2f}x), walking replay {ms_b:.2f} ms ({ms_b / ms_f:.2f}x); forward+adjoint with the "
            f"replay {ms_rp:.2f} ms; adjoint with edge terms {ms_e:.2f} ms; edge terms with one material per "
            f"part {ms_eg - ms_bg:.2f} ms")
        del paths

    # ---- design gradient through the orbit: 1 day of 60 s RK4 steps, 2881 stage-time sun directions ----
    orbit = None
    if not args.no_orbit:
        sc_o = si.meo_orbit(n_steps=1440, dt=60.0)
        po = p.TraceParams(nu=args.adjoint_grid, nv=args.adjoint_grid, bounces=args.bounces, jitter=1, seed=5)
        prob = p.DesignProblem(mesh, sc_o, po, si.DESIGN_LO, si.DESIGN_HI)
        theta_t = np.array([0.3, -0.2, 0.35, 0.1, 0.2, 0.3, 0.05, 0.4])
        prob.r_target = prob.final_state(theta_t)[0][:3]
        theta = np.array([0.0, 0.0, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25])
        # each iteration moves the hinges, as an optimiser step does (BVH refit and upload included)
        step_h = np.array([1e-3, -1e-3, 0, 0, 0, 0, 0, 0])
        for i in range(max(args.warmup, 1)):
            prob.loss_and_grad(theta - step_h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            prob.loss_and_grad(theta + i * step_h)
        torch.cuda.synchronize()
        ms_o = (time.perf_counter() - t0) * 1e3 / args.steps
        n_st = prob.n_stage
        orbit = {"ms_per_iteration": round(ms_o, 2), "stage_directions": n_st,
                 "rays_per_pass": n_st * args.adjoint_grid ** 2,
                 "workload": f"one design-gradient iteration: trace {n_st} stage-time sun directions x "
                             f"{args.adjoint_grid}x{args.adjoint_grid} rays, RK4 over 1440 x 60 s steps, discrete "
                             "adjoint with 24 checkpoints, ray adjoint, group sums (host wall clock)"}
        log(f"orbit: {ms_o:.1f} ms per design-gradient iteration ({n_st} directions)")
        # the same iteration with the two-network surrogate answering the force at every stage time
        # (the proxy inside the ODE): ensemble inference, RK4, orbit adjoint, the networks' input
        # gradients.  Networks of the benchmark's shape; the time does not depend on their weights.
        nets = [p.Surrogate(11, 256, 4, 3, seed=7 + s) for s in range(2)]
        sp = p.SurrogateDesignProblem(mesh, sc_o, nets, 1361.0 * 20.0 / 299792458.0, si.DESIGN_LO, si.DESIGN_HI,
                                      r_target=prob.r_target)
        for i in range(max(args.warmup, 1)):
            sp.loss_and_grad(theta - step_h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            sp.loss_and_grad(theta + i * step_h)
        torch.cuda.synchronize()
        ms_so = (time.perf_counter() - t0) * 1e3 / args.steps
        orbit["surrogate_ms_per_iteration"] = round(ms_so, 2)
        orbit["surrogate_speedup"] = round(ms_o / ms_so, 1)
        log(f"orbit with the surrogate: {ms_so:.2f} ms per iteration ({ms_o / ms_so:.0f}x)")
        for net_o in nets:
            net_o.close()
        prob.close()

    # ---- surrogate inference: fused BF16-MFMA MLP 11 -> 4 x 256 (SiLU) -> 3 on 1M queries ---------
    surrogate = None
    if not args.no_surrogate:
        net = p.Surrogate(11, 256, 4, 3, seed=0)
        nq = args.surrogate_batch
        gen = torch.Generator(device="cpu").manual_seed(5)
        xq = (torch.rand((nq, 11), generator=gen) * 2 - 1).to(dev)
        xq[:, :3] = torch.nn.functional.normalize(xq[:, :3], dim=1)
        yq = torch.empty((nq, 3), dtype=torch.float32, device=dev)
        for i in range(max(args.warmup, 1)):
            p.srp_mlp_forward(net.handle, xq, yq, False, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(args.steps):
            p.srp_mlp_forward(net.handle, xq, yq, False, stream=stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_s = e0.elapsed_time(e1) / args.steps
        flop = 2.0 * (11 * 256 + 3 * 256 * 256 + 256 * 3) * nq
        tf = flop / (ms_s * 1e-3) / 1e12
        surrogate = {"value": round(nq / (ms_s * 1e-3), 1), "unit": "evals/s", "ms_per_batch": round(ms_s, 4),
                     "batch": nq, "roofline": {"bound": "mfma", "achieved": round(tf, 1), "peak": 2500.0,
                                               "unit": "TFLOP/s", "frac": round(tf / 2500.0, 4)}}
        log(f"surrogate: {ms_s:.3f} ms per {nq} queries, {nq / ms_s / 1e6:.3f} G evals/s, {tf:.1f} TFLOP/s")
        # the ensemble as the pipeline calls it: both networks, their mean, the disagreement and
        # domain test and the compaction of the failing queries (srp_mlp_ensemble), one call
        net_b = p.Surrogate(11, 256, 4, 3, seed=1)
        y_e = torch.empty((nq, 3), dtype=torch.float32, device=dev)
        idx_e = torch.empty(nq, dtype=torch.int32, device=dev)
        cnt_e = torch.empty(1, dtype=torch.int32, device=dev)

        def ens():
            p.srp_mlp_ensemble(net.handle, net_b.handle, xq, 0.05, 1.0, y_e, idx_e, cnt_e, stream=stream.cuda_stream)

        for i in range(max(args.warmup, 1)):
            ens()
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(args.steps):
            ens()
        e1.record(stream)
        torch.cuda.synchronize()
        ms_e = e0.elapsed_time(e1) / args.steps
        surrogate["ensemble"] = {"value": round(nq / (ms_e * 1e-3), 1), "unit": "evals/s", "ms_per_batch": round(ms_e, 4),
                                 "note": "two networks + disagreement/domain test + compaction of failing queries"}
        log(f"ensemble: {ms_e:.3f} ms per {nq} queries, {nq / ms_e / 1e6:.3f} G evals/s")
        net_b.close()
        # training throughput: one Adam step = forward with kept activations, MSE gradient, backward
        # and the update, on batches of 4096 synthetic samples (the training recipe's batch)
        if not args.no_surrogate_training:
            bt = 4096
            xt = (torch.rand((bt, 11), generator=gen) * 2 - 1).to(dev)
            yt = torch.randn((bt, 3), generator=gen).to(dev)
            for i in range(20):
                net.train_step(xt, yt, 1e-4, stream=stream.cuda_stream)
            torch.cuda.synchronize()
            n_tr = 200
            e0.record(stream)
            for i in range(n_tr):
                net.train_step(xt, yt, 1e-4, stream=stream.cuda_stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms_t = e0.elapsed_time(e1) / n_tr
            tf_t = 3 * 400384 * bt / (ms_t * 1e-3) / 1e12
            surrogate["training"] = {"samples_per_s": round(bt / (ms_t * 1e-3), 1), "ms_per_step": round(ms_t, 4),
                                     "batch": bt, "tflops": round(tf_t, 2), "frac_of_bf16_peak": round(tf_t / 2500.0, 4)}
            log(f"surrogate training: {ms_t:.3f} ms per Adam step of {bt} samples, {bt / ms_t / 1e3:.2f} M samples/s")
        net.close()

    # ---- 13-D orbit and attitude: RK4 in FP64 with the network answering force and torque ---------
    attitude = None
    if not args.no_attitude:
        B_a, n_a, dt_a = args.attitude_batch, args.attitude_steps, 15.0
        net_a = p.Surrogate(11, 256, 4, 6, seed=1)
        z0_a = torch.as_tensor(si.attitude_states(B_a, 21), dtype=torch.float64, device=dev).contiguous()
        gen_a = np.random.default_rng(22)
        des_a = torch.as_tensor(gen_a.uniform(-1, 1, (B_a, 8)), dtype=torch.float32, device=dev).contiguous()
        zf_a = torch.empty_like(z0_a)

        def att_params(n):
            return p.AttitudeParams(si.MU_EARTH, 1000.0, si.ATTITUDE_INERTIA, (0.3, -0.5, 0.81), 5e-5, 2e-5, dt_a, n,
                                    earth_radius=6378137.0)

        p.srp_attitude_rk4(net_a, att_params(8), z0_a, des_a, zf_a, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        ea0 = torch.cuda.Event(enable_timing=True)
        ea1 = torch.cuda.Event(enable_timing=True)
        ea0.record(stream)
        p.srp_attitude_rk4(net_a, att_params(n_a), z0_a, des_a, zf_a, stream=stream.cuda_stream)
        ea1.record(stream)
        torch.cuda.synchronize()
        ms_a = ea0.elapsed_time(ea1)
        # the network call at this batch on its own (same inputs shape), for the split of a stage
        xa = torch.zeros((B_a, 11), dtype=torch.float32, device=dev)
        xa[:, :3] = torch.nn.functional.normalize(torch.randn((B_a, 3), device=dev), dim=1)
        ya = torch.empty((B_a, 6), dtype=torch.float32, device=dev)
        p.srp_mlp_forward(net_a.handle, xa, ya, False, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        # launched from Python one by one the calls cannot keep up with the GPU, so the 200 calls are
        # captured once into a HIP graph (inference allocates and clears nothing) and replayed
        n_m = 200
        ms_m = None
        try:
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                cap = torch.cuda.current_stream()
                for i in range(n_m):
                    p.srp_mlp_forward(net_a.handle, xa, ya, False, stream=cap.cuda_stream)
            graph.replay()
            torch.cuda.synchronize()
            ea0.record(stream)
            graph.replay()
            ea1.record(stream)
            torch.cuda.synchronize()
            ms_m = ea0.elapsed_time(ea1) / n_m
            del graph
        except RuntimeError as e:
            log(f"attitude: graph timing of the network call unavailable: {e!r}")
        stages = 4 * n_a
        flop_q = 2.0 * (11 * 256 + 3 * 256 * 256 + 256 * 6)
        tf_m = flop_q * B_a / (ms_m * 1e-3) / 1e12 if ms_m else None
        attitude = {
            "value": round(B_a * n_a / (ms_a * 1e-3), 1), "unit": "trajectory-steps/s", "ms": round(ms_a, 2),
            "network_evals_per_s": round(stages * B_a / (ms_a * 1e-3), 1),
            "ms_per_stage": round(ms_a / stages, 5), "network_ms_per_call": round(ms_m, 5) if ms_m else None,
            "network_roofline": {"bound": "mfma", "achieved": round(tf_m, 1), "peak": 2500.0, "unit": "TFLOP/s",
                                 "frac": round(tf_m / 2500.0, 4)} if tf_m else None,
            "workload": f"{B_a} trajectories x {n_a} RK4 steps of {dt_a:.0f} s (12 h), 13-D FP64 state, network "
                        "11 -> 4 x 256 -> 6 (force, torque) at every stage, cylinder eclipse"}
        log(f"attitude: {ms_a:.1f} ms for {B_a} x {n_a} steps, {attitude['value'] / 1e6:.1f} M trajectory-steps/s, "
            f"{ms_a / stages * 1e3:.1f} us per stage (network {ms_m * 1e3 if ms_m else float('nan'):.1f} us)")
        net_a.close()

    # ---- batched designs: 256 MEO-style variants, 256 directions each, one launch ---------------
    batched = None
    if not args.no_batch:
        from concurrent.futures import ThreadPoolExecutor
        S_n = args.batch_designs
        rng = np.random.default_rng(6)
        sizes = np.exp(rng.uniform(np.log(2000.0), np.log(50000.0), S_n)).astype(int)
        dsg = si.random_designs(S_n, seed=6)

        def make(k):
            m = si.meo_variant(int(sizes[k]))
            sck = p.Scene.from_mesh(m)
            rsk, rdk = si.materials(m.n_tris, 100 + k)
            sck.set_design(rsk, rdk, hinge_angles=dsg[k][:2])
            return sck, m.n_tris

        t0 = time.perf_counter()
        with ThreadPoolExecutor(16) as ex:
            built = list(ex.map(make, range(S_n)))
        torch.cuda.synchronize()
        build_b = time.perf_counter() - t0
        scenes = [b[0] for b in built]
        tris_b = np.array([b[1] for b in built])
        sun_b = torch.as_tensor(si.fibonacci_dirs(args.batch_dirs), dtype=torch.float64, device=dev).contiguous()
        pb = p.TraceParams(nu=args.batch_grid, nv=args.batch_grid, bounces=args.bounces, jitter=1, seed=2)
        # launch shape from the autotuner, on every 8th direction (untimed, like the BVH builds)
        t0 = time.perf_counter()
        tpw, tune_ms = p.srp_autotune_tiles_per_wave(scenes, sun_b[::8].contiguous(), pb,
                                                     stream=stream.cuda_stream)
        tune_s = time.perf_counter() - t0
        pb.tiles_per_wave = tpw
        log(f"batched: autotuned tiles_per_wave = {tpw} in {tune_s:.1f} s "
            f"({', '.join(f'{k}: {v:.1f}' for k, v in tune_ms.items())} ms)")
        Fb = torch.empty((S_n, args.batch_dirs, 3), dtype=torch.float64, device=dev)
        Tb = torch.empty_like(Fb)
        for i in range(max(args.warmup, 1)):
            p.srp_batch_trace(scenes, sun_b, pb, Fb, Tb, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        nb = max(1, min(args.steps, 3))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(nb):
            p.srp_batch_trace(scenes, sun_b, pb, Fb, Tb, stream=stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_b = e0.elapsed_time(e1) / nb
        rays_b = float(S_n) * args.batch_dirs * args.batch_grid ** 2
        batched = {"value": round(rays_b / (ms_b * 1e-3) / 1e6, 1), "unit": "Mrays/s", "ms_per_launch": round(ms_b, 2),
                   "launches": nb, "scene_build_s": round(build_b, 2), "tiles_per_wave": tpw,
                   "autotune_s": round(tune_s, 2),
                   "workload": f"{S_n} MEO-style variants ({int(tris_b.min())}-{int(tris_b.max())} tris, "
                               f"{int(tris_b.sum())} total), {args.batch_dirs} Fibonacci dirs x "
                               f"{args.batch_grid}x{args.batch_grid} rays, {args.bounces} bounces, one launch"}
        log(f"batched: {ms_b:.1f} ms per launch, {batched['value']:.0f} Mrays/s (scene build {build_b:.1f} s)")
        for sck in scenes:
            sck.close()

    # ---- the paper's own estimator: surface sampling, BVH walk vs brute force -------------------
    surface = None
    if not args.no_surface:
        def surf_time(scenes_s, D_s, N_s, brute):
            sun_s = torch.as_tensor(si.fibonacci_dirs(D_s), dtype=torch.float64, device=dev).contiguous()
            Fs = torch.empty((len(scenes_s), D_s, 3), dtype=torch.float64, device=dev)
            ps_ = p.TraceParams(bounces=args.bounces, seed=3)
            p.srp_surface_estimate(scenes_s, sun_s, N_s, ps_, Fs, brute_force=brute, stream=stream.cuda_stream)
            torch.cuda.synchronize()
            reps = 3
            e0.record(stream)
            for _ in range(reps):
                p.srp_surface_estimate(scenes_s, sun_s, N_s, ps_, Fs, brute_force=brute, stream=stream.cuda_stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms_ = e0.elapsed_time(e1) / reps
            return {"samples_per_s": round(len(scenes_s) * D_s * N_s / (ms_ * 1e-3), 1), "ms": round(ms_, 3),
                    "designs": len(scenes_s), "dirs": D_s, "samples": N_s}
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        bw = si.box_wing()
        rbs, rbd = si.materials(bw.n_tris, 1)
        sbw = p.Scene.from_mesh(bw)
        sbw.set_design(rbs, rbd)
        surface = {
            "workload": f"{args.bounces} bounces; samples per second of the whole estimate (facet by area, point, "
                        "gathering with next-event estimation, outgoing event)",
            "meo_bvh": surf_time([sc], 64, 65536, False),
            "meo_brute_force": surf_time([sc], 64, 4096, True),
            "box_wing_bvh": surf_time([sbw], 64, 65536, False),
            "box_wing_brute_force": surf_time([sbw], 64, 65536, True),
        }
        # samples per design above which building a BVH (host SAH build, timed here on one thread)
        # and walking it beats testing every triangle, for the 20.6k-triangle satellite
        t0 = time.perf_counter()
        for _ in range(3):
            tmp = p.Scene.from_mesh(mesh)
            tmp.close()
        build_one = (time.perf_counter() - t0) / 3
        r_b = surface["meo_bvh"]["samples_per_s"]
        r_f = surface["meo_brute_force"]["samples_per_s"]
        surface["meo_bvh_build_s"] = round(build_one, 4)
        surface["meo_crossover_samples_per_design"] = round(build_one / (1.0 / r_f - 1.0 / r_b))
        log(f"surface estimator: MEO BVH {r_b / 1e9:.2f} G samples/s, brute force {r_f / 1e6:.2f} M samples/s, "
            f"box-wing BVH {surface['box_wing_bvh']['samples_per_s'] / 1e9:.2f} / brute "
            f"{surface['box_wing_brute_force']['samples_per_s'] / 1e9:.2f} G samples/s; crossover "
            f"{surface['meo_crossover_samples_per_design']} samples per design")
        sbw.close()

        # the same tree rebuilt on the GPU (linear BVH): the build's cost, what the tree costs the
        # ray-grid trace and the surface walk, and the crossover when each design gets a GPU build
        sg = p.Scene.from_mesh(mesh)
        sg.set_design(rs, rd, hinge_angles=angles)
        p.srp_scene_build_gpu(sg, stream=stream.cuda_stream)  # first call: workspace, code objects
        tb = []
        for _ in range(7):
            t0 = time.perf_counter()
            nn_g, dep_g = p.srp_scene_build_gpu(sg, stream=stream.cuda_stream)
            tb.append(time.perf_counter() - t0)
        gpu_build = float(np.median(tb))
        sun_t = sun_d[::8].contiguous()
        Ft = torch.empty((sun_t.shape[0], 3), dtype=torch.float64, device=dev)

        def trace_ms(scene):
            p.srp_trace(scene.handle, sun_t, params, Ft, stream=stream.cuda_stream)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(3):
                p.srp_trace(scene.handle, sun_t, params, Ft, stream=stream.cuda_stream)
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / 3

        rays_t = float(sun_t.shape[0]) * args.grid * args.grid
        ms_sah, ms_lbvh = trace_ms(sc), trace_ms(sg)
        s_lbvh = surf_time([sg], 64, 65536, False)
        r_bg = s_lbvh["samples_per_s"]
        surface["meo_gpu_build"] = {
            "build_s": round(gpu_build, 5), "nodes": nn_g, "depth": dep_g,
            "sah_nodes": info["n_nodes"], "sah_depth": info["depth"],
            "trace_mrays_s_sah": round(rays_t / (ms_sah * 1e-3) / 1e6, 1),
            "trace_mrays_s_lbvh": round(rays_t / (ms_lbvh * 1e-3) / 1e6, 1),
            "surface_bvh_samples_per_s": r_bg,
            "crossover_samples_per_design": round(gpu_build / (1.0 / r_f - 1.0 / r_bg)),
            "workload": f"{sun_t.shape[0]} dirs x {args.grid}x{args.grid} rays for the trace rates; build_s is the "
                        "whole synchronous call (kernels, read-back of the host copies), median of 7"}
        log(f"GPU BVH build: {gpu_build * 1e3:.2f} ms ({nn_g} nodes, depth {dep_g}); trace SAH "
            f"{surface['meo_gpu_build']['trace_mrays_s_sah']:.0f} vs LBVH "
            f"{surface['meo_gpu_build']['trace_mrays_s_lbvh']:.0f} Mrays/s; surface LBVH {r_bg / 1e9:.2f} G samples/s;"
            f" crossover {surface['meo_gpu_build']['crossover_samples_per_design']} samples per design")
        sg.close()

        # the paper's convergence study (MSE against a high-sample reference for plain MC, BRDF
        # importance sampling, stratified surface sampling and both): 32 independent seeds of N
        # samples for 16 directions, reference 2^22 samples per direction with both options; once
        # with ideal mirrors and once with every facet a Phong lobe (m = 20), where importance
        # sampling of the lobe matters
        def variance_study(scene, what):
            sun_v = torch.as_tensor(si.fibonacci_dirs(16), dtype=torch.float64, device=dev).contiguous()
            Fv = torch.empty((1, 16, 3), dtype=torch.float64, device=dev)
            p.srp_surface_estimate([scene], sun_v, 1 << 22, p.TraceParams(bounces=args.bounces, seed=999, sampling=1),
                                   Fv, stream=stream.cuda_stream)
            ref_v = Fv.clone()
            mse = {}
            for n_v in (1024, 16384):
                for mode, name in ((2, "plain"), (0, "brdf_is"), (3, "stratified"), (1, "both")):
                    acc = torch.zeros((), dtype=torch.float64, device=dev)
                    for k in range(32):
                        p.srp_surface_estimate([scene], sun_v, n_v, p.TraceParams(bounces=args.bounces, seed=1000 + k,
                                                                                  sampling=mode), Fv,
                                               stream=stream.cuda_stream)
                        acc += ((Fv - ref_v) ** 2).sum(-1).mean()
                    mse[f"{name}_{n_v}"] = (acc / 32).item()
            scale = (ref_v ** 2).sum(-1).mean().item()
            out = {"mse_N2": {k: float(f"{v:.4e}") for k, v in mse.items()},
                   "rel_rms": {k: round((v / scale) ** 0.5, 5) for k, v in mse.items()},
                   "plain_over_both": {n: round(mse[f"plain_{n}"] / mse[f"both_{n}"], 2) for n in (1024, 16384)},
                   "workload": f"satellite ({what}), 16 Fibonacci dirs, 32 seeds per option and sample count, "
                               "reference 2^22 samples (stratified + importance sampled)"}
            log(f"surface variance study, {what} (relative RMS): " +
                ", ".join(f"{k} {v:.4f}" for k, v in out["rel_rms"].items()))
            return out

        surface["variance"] = variance_study(sc, "ideal mirrors")
        sp = p.Scene.from_mesh(mesh)
        sp.set_design(rs, rd, hinge_angles=angles)
        sp.set_phong(np.full(mesh.n_tris, 20.0, np.float32))
        surface["variance_phong"] = variance_study(sp, "every facet a Phong lobe, m = 20")
        sp.close()

        # multi-world sampling (the paper's setting: every pair of sun direction and design its own
        # world, brute force): 16384 random designs x 16 samples on the satellite, 3 bounces
        n_pw, k_pw = 16384, 16
        grp = np.asarray(mesh.group, dtype=np.int32)
        rng_pw = np.random.default_rng(17)
        dsg_pw = np.concatenate([rng_pw.uniform(-0.5, 0.5, (n_pw, 2))] + [
            np.stack([rng_pw.uniform(0, 0.5, n_pw), rng_pw.uniform(0, 0.5, n_pw), rng_pw.uniform(1, 60, n_pw)], 1)
            for _ in range(3)], 1).astype(np.float32)
        d_pw = torch.as_tensor(dsg_pw, device=dev).contiguous()
        s_pw = torch.as_tensor(si.random_dirs(n_pw, seed=18), dtype=torch.float64, device=dev).contiguous()
        F_pw = torch.empty((n_pw, 3), dtype=torch.float64, device=dev)
        rest = p.Scene.from_mesh(mesh)
        prm_pw = p.TraceParams(bounces=args.bounces, seed=19)
        p.srp_surface_designs(rest, grp, 3, s_pw, d_pw, k_pw, prm_pw, F_pw, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            p.srp_surface_designs(rest, grp, 3, s_pw, d_pw, k_pw, prm_pw, F_pw, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        ms_pw = (time.perf_counter() - t0) * 1e3 / 3
        surface["multi_world"] = {"samples_per_s": round(n_pw * k_pw / (ms_pw * 1e-3), 1), "ms": round(ms_pw, 3),
                                  "pairs": n_pw, "samples_per_pair": k_pw,
                                  "workload": "satellite, 16384 (sun direction, design) pairs with random hinge angles, "
                                              "group reflectances and Phong exponents, 16 samples each, brute force "
                                              "(host wall clock of the call, which checks the designs first)"}
        log(f"multi-world sampling: {ms_pw:.2f} ms for {n_pw} x {k_pw} samples, "
            f"{n_pw * k_pw / ms_pw / 1e3:.2f} M samples/s")
        rest.close()

    # ---- roofline of the dominant kernel --------------------------------------------------------
    # k_trace walks a scene that stays in every XCD's L2 (99.9 % hits, counters under profiles/), so
    # what binds it is vector-ALU issue, not HBM: the roofline is the ALU one.  Algorithmic lane-ops
    # of the walk a ray needs (two child-box slab tests per node visited, triangle tests, counts from
    # the host's single-ray traversal of the same BVH) against the peak of that op mix (FMA-class
    # lane-ops at 32 lanes per SIMD-cycle, min/max/compare at 16, reciprocals at 8; 1024 SIMDs at
    # 2.4 GHz); the all-FMA peak (78.6 T) is kept beside it.  issue_frac is the counters' issued
    # instruction mix at the same class rates, as a share of the launch's cycles (a range); the HBM-equivalent
    # figure (algorithmic bytes against 8 TB/s) is kept beside it, labelled, and exceeds 1 because
    # the scene is cached.
    roofline = None
    try:
        from paper_2602_10712_amd import ray_stats
        st = ray_stats(sc, sun, params, n_dirs=16, pixel_stride=97)
        launch_s = np.median(step_ms) * 1e-3  # one launch = all D x grid^2 rays (frames + reduce < 1 %)
        bytes_per_ray = st["bytes_per_ray"]
        hbm_eq = bytes_per_ray * rays / launch_s / 1e9
        roofline = alu_roofline(st, rays, launch_s)
        roofline.update({"traffic": measured_traffic(), "issue_frac": measured_valu_issue(),
                         "l2_hit_rate": measured_l2_hit_rate(), "l2_slot_frac": measured_l2_slot_frac(),
                         "segments_per_ray": round(st["segments_per_ray"], 4),
                         "hits_per_ray": round(st["hits_per_ray"], 4),
                         "nodes_per_segment": round(st["nodes_per_segment"], 2),
                         "tris_per_segment": round(st["tris_per_segment"], 2),
                         "hbm_equivalent": {"note": "algorithmic bytes / launch time against the HBM peak; the "
                                                    "scene is L2-resident, so this is not a bound and may exceed 1",
                                            "achieved": round(hbm_eq, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                            "frac": round(hbm_eq / HBM_PEAK_GBS, 4),
                                            "bytes_per_ray": round(bytes_per_ray, 1)}})
        rates["segments_per_s"] = round(st["segments_per_ray"] * rays / launch_s, 1)
        rates["hits_per_s"] = round(st["hits_per_ray"] * rays / launch_s, 1)
    except Exception as e:  # the stats entry point is optional for the timing itself
        log(f"roofline stats unavailable: {e!r}")

    # ---- CPU baseline: the oracle on a bounded sample --------------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        n_s, g_s = args.cpu_sample_dirs, args.cpu_sample_grid
        idx = np.linspace(0, D - 1, n_s).astype(int)
        # the host share of one GPU is 16 cores whatever the machine reports
        cores = max(1, min(16, len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "16"))))
        from oracle.design import apply_hinges
        V = apply_hinges(mesh.verts, mesh.vert_hinge, mesh.hinge_origin, mesh.hinge_axis, angles)
        t0 = time.perf_counter()
        for k, j in enumerate(idx):
            oracle.trace(V, mesh.tris, rs, rd, sun[j:j + 1], nu=g_s, nv=g_s, bounces=args.bounces, seed=2,
                         dir_index_base=int(j), threads=cores)
        cpu_s = time.perf_counter() - t0
        cpu_mrays = n_s * g_s * g_s / cpu_s / 1e6
        cpu = {"value": round(cpu_mrays, 5), "unit": "Mrays/s", "cores": cores, "kind": "oracle",
               "host_cpu_count": os.cpu_count(),
               "cores_note": "threads used: the host share of one GPU (16 on this pool), not every core the "
                             "machine reports",
               "sample": f"{n_s} of the {D} directions x {g_s}x{g_s} rays, {args.bounces} bounces, FP64 brute force, "
                         f"{cpu_s:.1f} s"}
        log(f"cpu baseline: {cpu_mrays:.4f} Mrays/s on {cores} threads ({cpu_s:.1f} s)")
        if attitude is not None:
            # the 13-D integration of the oracle (numpy FP64, BF16-emulating network) on 2 trajectories
            from oracle import attitude as oatt
            from oracle import mlp as omlp
            net_c = p.Surrogate(11, 256, 4, 6, seed=1)
            layers = omlp.unpack(p.srp_mlp_get_params(net_c.handle)["params"].astype(np.float64), 11, 256, 4, 6)
            net_c.close()
            n_c = 240
            zc = si.attitude_states(2, 21)
            dc = np.random.default_rng(22).uniform(-1, 1, (2, 8)).astype(np.float32).astype(np.float64)
            sun_c = np.array([0.3, -0.5, 0.81]) / np.linalg.norm([0.3, -0.5, 0.81])
            t0 = time.perf_counter()
            oatt.rk4(zc, dc, oatt.mlp_model(layers, 5e-5, 2e-5), mu=si.MU_EARTH, mass=1000.0,
                     inertia=si.ATTITUDE_INERTIA, sun=sun_c, dt=15.0, n_steps=n_c, earth_radius=6378137.0)
            att_s = time.perf_counter() - t0
            cpu["attitude"] = {"value": round(2 * n_c / att_s, 2), "unit": "trajectory-steps/s", "cores": 1,
                               "sample": f"2 trajectories x {n_c} steps, {att_s:.1f} s"}

    out = {
        "metric": METRIC, "value": round(mrays, 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"MEO-style satellite {mesh.n_tris} tris, {D} Fibonacci sun dirs x "
                               f"{args.grid}x{args.grid} rays, {args.bounces} bounces, forward",
                   "tris": mesh.n_tris, "dirs": D, "grid": args.grid, "bounces": args.bounces,
                   "bvh_nodes": info["n_nodes"], "bvh_build_s": round(build_s, 4)},
        "rates": rates, "roofline": roofline, "cpu_baseline": cpu, "fwd_adjoint": fwd_adj,
        "surrogate": surrogate, "batched": batched, "orbit": orbit, "surface": surface, "attitude": attitude,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
