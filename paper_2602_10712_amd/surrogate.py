"""Force surrogate pipeline (paper Sec. 3.3 and Alg. 1, proxy learning).

The tracer generates samples (sun direction, design) -> body-frame force over random designs; the
MLP (libsrp srp_mlp_*) is trained on them with Adam and then answers force queries at a fraction of
the tracer's cost.  The tracer stays the reference for the surrogate's error and its fallback: a query
is sent back to the tracer when it lies outside the training box of the design space or when two
independently trained networks disagree by more than a threshold calibrated on held-out data.

Inputs: x = [s_x, s_y, s_z, design scaled to [-1, 1] (8)]; outputs: F / F_ref with
F_ref = Phi * A_ref / c (and, for networks that also answer torque, tau / (F_ref L_ref)).  All compute runs in libsrp; this module only sequences the calls.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding as B

C_LIGHT = 299792458.0


def input_features(sun, theta, lo, hi):
    sun = np.asarray(sun, dtype=np.float64).reshape(-1, 3)
    th = np.asarray(theta, dtype=np.float64).reshape(-1, 8)
    scaled = 2.0 * (th - lo) / (hi - lo) - 1.0
    return np.concatenate([sun, scaled], 1).astype(np.float32)


def generate_samples(mesh, designs, sun_per_design, params: B.TraceParams, flux=1361.0, torque=False):
    """Traces every design for its own sun directions: designs [N_d][8], sun_per_design
    [N_d][K][3] -> forces [N_d][K][3] (N, FP64, body frame), and with torque=True also the torques
    about the centre of mass [N_d][K][3] (N m)."""
    scene = B.Scene.from_mesh(mesh)
    group = np.asarray(mesh.group)
    out = np.zeros((len(designs), sun_per_design.shape[1], 3))
    out_t = np.zeros_like(out) if torque else None
    for d, th in enumerate(designs):
        rs = th[2 + 2 * group].astype(np.float32)
        rd = th[3 + 2 * group].astype(np.float32)
        scene.set_design(rs, rd, hinge_angles=th[:2])
        p = B.TraceParams(params.nu, params.nv, params.bounces, params.jitter, flux, params.seed,
                          0, d, params.frame_mode, params.tiles_per_wave)
        F, T = scene.trace(sun_per_design[d], p)
        out[d] = F.cpu().numpy()
        if torque:
            out_t[d] = T.cpu().numpy()
    scene.close()
    return (out, out_t) if torque else out


def train(net: B.Surrogate, x, y, steps, batch=4096, lr=1e-3, lr_final=1e-5, seed=0, log_every=0):
    """Adam on minibatches drawn with replacement; cosine-decayed learning rate.
    Returns the list of minibatch losses."""
    xd = torch.as_tensor(x, dtype=torch.float32, device="cuda")
    yd = torch.as_tensor(y, dtype=torch.float32, device="cuda")
    n = xd.shape[0]
    g = torch.Generator(device="cuda").manual_seed(seed)
    losses = []
    for s in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), device="cuda", generator=g)
        a = 0.5 * (1 + np.cos(np.pi * s / max(steps - 1, 1)))
        loss = net.train_step(xd[idx].contiguous(), yd[idx].contiguous(), lr=lr_final + (lr - lr_final) * a)
        if log_every and (s % log_every == 0 or s == steps - 1):
            losses.append((s, float(loss.item())))
    return losses


def rel_rms(pred, ref):
    pred = np.asarray(pred, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(((pred - ref) ** 2).sum(-1).mean() / (ref ** 2).sum(-1).mean()))


class SurrogateForce:
    """Two-member ensemble with the library's confidence test (srp_mlp_ensemble: mean, disagreement,
    domain check, compaction of failing queries); failing queries are answered by the tracer."""

    def __init__(self, nets, lo, hi, f_ref, threshold):
        assert len(nets) == 2
        self.nets = nets
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.f_ref = f_ref
        self.threshold = threshold

    def evaluate(self, x, out_scale=None, threshold=None, stream=None):
        """srp_mlp_ensemble on inputs x [N][11] (host or device): device tensors (y [N][n_out] scaled by
        out_scale (default f_ref), disagreement [N], failing query indices [N] int32, their count [1])."""
        xd = torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous()
        n = xd.shape[0]
        y = torch.empty((n, self.nets[0].n_out), dtype=torch.float32, device="cuda")
        dis = torch.empty(n, dtype=torch.float32, device="cuda")
        idx = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        cnt = torch.empty(1, dtype=torch.int32, device="cuda")
        B.srp_mlp_ensemble(self.nets[0].handle, self.nets[1].handle, xd,
                           self.threshold if threshold is None else threshold,
                           self.f_ref if out_scale is None else out_scale, y, idx, cnt, disagree=dis, stream=stream)
        return y, dis, idx, cnt

    def predict(self, x):
        """Ensemble mean (network units) and disagreement, no test applied."""
        y, dis, _, _ = self.evaluate(x, out_scale=1.0, threshold=np.inf)
        return y, dis

    @staticmethod
    def calibrate(disagree, err, target, max_coverage=1.0):
        """Disagreement threshold for held-out queries: the largest one whose accepted queries keep the
        relative RMS error <= target (err: per-query squared error divided by the mean squared
        reference), lowered if needed so that at most max_coverage of the queries are accepted."""
        order = np.argsort(disagree)
        cum = np.cumsum(err[order]) / np.arange(1, len(err) + 1)
        ok = np.nonzero(np.sqrt(cum) <= target)[0]
        thr = float(disagree[order][ok[-1]]) if len(ok) else 0.0
        if max_coverage < 1.0:
            thr = min(thr, float(np.quantile(disagree, max_coverage)))
        return thr

    def forces(self, mesh, sun, theta, params: B.TraceParams):
        """Forces [N][3] (N, device FP32 tensor): the ensemble where it passes the confidence test, the
        tracer elsewhere; also the host bool mask of the queries the tracer answered."""
        sun = np.asarray(sun, dtype=np.float64).reshape(-1, 3)
        th = np.asarray(theta, dtype=np.float64).reshape(-1, 8)
        x = input_features(sun, th, self.lo, self.hi)
        F, _, idx, cnt = self.evaluate(x)
        n_fail = int(cnt.item())
        fall = np.zeros(len(x), dtype=bool)
        if n_fail:
            sel_all = idx[:n_fail].cpu().numpy().astype(np.int64)
            fall[sel_all] = True
            # group the failing queries by design and trace each design once
            designs, inv = np.unique(th[sel_all], axis=0, return_inverse=True)
            scene = B.Scene.from_mesh(mesh)
            group = np.asarray(mesh.group)
            for k, dsg in enumerate(designs):
                sel = sel_all[inv.ravel() == k]
                scene.set_design(dsg[2 + 2 * group].astype(np.float32), dsg[3 + 2 * group].astype(np.float32),
                                 hinge_angles=dsg[:2])
                Ft, _ = scene.trace(sun[sel], params)
                F.index_copy_(0, torch.as_tensor(sel, device="cuda"), Ft.to(torch.float32))
            scene.close()
        return F, fall
