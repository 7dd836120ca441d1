"""Design optimisation through the orbit (paper Sec. 3.4 and Alg. 1, design loop).

One evaluation of the design vector
    theta = [hinge_1, hinge_2, rho_s_bus, rho_d_bus, rho_s_panel, rho_d_panel, rho_s_payload, rho_d_payload]
applies the design (hinge rotation + group reflectances), traces the body-frame force for the
body-frame sun direction at every RK4 stage time in ONE batched srp_trace (the attitude depends on
time only), integrates the orbit (srp_orbit_rk4) and scores L = |r_N - r_target|^2.  Its gradient
chains the discrete RK4 adjoint (srp_orbit_rk4_adjoint, checkpointed) into the ray adjoint
(seeds = dL/dF at each stage time), then sums facet gradients per design group.  The forward
records every path's facets (srp_trace_recorded) and the ray adjoint reads them back
(srp_trace_adjoint_recorded) instead of walking the BVH again; record_paths=False uses the walking
replay (srp_trace_adjoint), with the same gradients.
All compute runs in libsrp; this module only sequences the calls.  Bounded parameters are clipped
after every optimiser step (Sec. 3.4.3).
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding as B

GROUP_NAMES = ("hinge_1", "hinge_2", "rho_s_bus", "rho_d_bus", "rho_s_panel", "rho_d_panel", "rho_s_payload",
               "rho_d_payload")


class DesignProblem:
    def __init__(self, mesh, scenario, params: B.TraceParams, lo, hi, r_target=None, ckpt_every=60,
                 record_paths=True):
        self.mesh = mesh
        self.sc = scenario
        self.params = params
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.scene = B.Scene.from_mesh(mesh)
        self.sun = torch.as_tensor(scenario.sun_body, dtype=torch.float64, device="cuda").contiguous()
        self.group = np.asarray(mesh.group)
        self.r_target = None if r_target is None else np.asarray(r_target, dtype=np.float64)
        self.ckpt_every = ckpt_every
        self.n_stage = 2 * scenario.n_steps + 1
        assert self.sun.shape[0] == self.n_stage
        self.record_paths = record_paths and params.bounces <= 3  # records hold 3 interactions
        self._record = None  # path record of the last forward (record_paths)

    def materials(self, theta):
        rs = theta[2 + 2 * self.group].astype(np.float32)
        rd = theta[3 + 2 * self.group].astype(np.float32)
        return rs, rd

    def forces(self, theta):
        """Body-frame force at every stage time [2n+1][3] (host FP64)."""
        rs, rd = self.materials(theta)
        self.scene.set_design(rs, rd, hinge_angles=theta[:2])
        if self.record_paths:
            self._record = None  # release the previous record before the new one is allocated
            F, _, self._record = self.scene.trace_recorded(self.sun, self.params)
        else:
            F, _ = self.scene.trace(self.sun, self.params)
        return F.cpu().numpy()

    def final_state(self, theta):
        F = self.forces(theta)
        return B.srp_orbit_rk4(self.sc.z0, self.sc.mu, self.sc.mass, self.sc.dt, self.sc.n_steps, F, self.sc.R), F

    def loss(self, theta):
        z, _ = self.final_state(theta)
        d = z[:3] - self.r_target
        return float(d @ d)

    def design_grad(self, theta, F, g_final):
        """d(g_final . z_N)/d theta for the forces F of design theta: the RK4 adjoint (checkpointed)
        chained into the ray adjoint and summed per group."""
        gF, _ = B.srp_orbit_rk4_adjoint(self.sc.z0, self.sc.mu, self.sc.mass, self.sc.dt, self.sc.n_steps, F,
                                        self.sc.R, g_final, self.ckpt_every)
        if self.record_paths and self._record is not None:
            g_rs, g_rd, g_h = self.scene.adjoint_recorded(self._record, self.params, gF)
        else:
            g_rs, g_rd, g_h = self.scene.adjoint(self.sun, self.params, gF)
        g_rs = g_rs.cpu().numpy().astype(np.float64)
        g_rd = g_rd.cpu().numpy().astype(np.float64)
        grad = np.zeros(8)
        grad[:2] = g_h.cpu().numpy()[:2]
        for k in range(3):
            m = self.group == k
            grad[2 + 2 * k] = g_rs[m].sum()
            grad[3 + 2 * k] = g_rd[m].sum()
        return grad

    def loss_and_grad(self, theta):
        theta = np.asarray(theta, dtype=np.float64)
        z, F = self.final_state(theta)
        d = z[:3] - self.r_target
        return float(d @ d), self.design_grad(theta, F, np.concatenate([2.0 * d, np.zeros(3)]))

    def miss_and_jacobian(self, theta):
        """The final-position miss r = r_N - r_target [3] and its Jacobian dr/d theta [3][8]: one
        forward pass and one adjoint pass per position component."""
        theta = np.asarray(theta, dtype=np.float64)
        z, F = self.final_state(theta)
        J = np.stack([self.design_grad(theta, F, np.eye(6)[i]) for i in range(3)])
        return z[:3] - self.r_target, J

    def clip(self, theta):
        th = np.clip(theta, self.lo, self.hi)
        for k in range(3):  # rho_s + rho_d <= 1 per group
            s = th[2 + 2 * k] + th[3 + 2 * k]
            if s > 1.0:
                th[2 + 2 * k] /= s
                th[3 + 2 * k] /= s
        return th

    def optimise(self, theta0, iters=30, lr=None, betas=(0.9, 0.999), eps=1e-12, free=None, callback=None):
        """Adam on theta with per-parameter step sizes lr (default: 2 % of each parameter's range)
        decayed by a cosine schedule to 5 % of it, clipping after every step.  Returns (theta,
        history of losses)."""
        theta = self.clip(np.asarray(theta0, dtype=np.float64))
        lr = 0.02 * (self.hi - self.lo) if lr is None else np.asarray(lr, dtype=np.float64)
        mask = np.ones(8) if free is None else np.asarray(free, dtype=np.float64)
        m = np.zeros(8)
        v = np.zeros(8)
        hist = []
        for t in range(1, iters + 1):
            L, g = self.loss_and_grad(theta)
            g = g * mask
            hist.append(L)
            m = betas[0] * m + (1 - betas[0]) * g
            v = betas[1] * v + (1 - betas[1]) * g * g
            decay = 0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * (t - 1) / max(iters - 1, 1)))
            step = decay * lr * (m / (1 - betas[0] ** t)) / (np.sqrt(v / (1 - betas[1] ** t)) + eps)
            theta = self.clip(theta - step)
            if callback:
                callback(t, L, theta)
        hist.append(self.loss(theta))
        return theta, hist

    def optimise_lm(self, theta0, iters=10, max_step=0.15, lam=1e-3, free=None, callback=None):
        """Levenberg-Marquardt on the three components of the final-position miss.  In parameters
        scaled to their ranges the step is the damped minimum-norm solution
        ds = -Js^T (Js Js^T + lam tr(Js Js^T)/3 I)^-1 r (three residuals, up to eight parameters),
        capped at max_step of each range and clipped to the bounds.  A step that lowers the loss is
        taken and the damping divided by 3; otherwise the damping is multiplied by 10.  Returns
        (theta, history of losses of the accepted points)."""
        theta = self.clip(np.asarray(theta0, dtype=np.float64))
        mask = np.ones(8) if free is None else np.asarray(free, dtype=np.float64)
        scale = (self.hi - self.lo) * mask
        r, J = self.miss_and_jacobian(theta)
        L = float(r @ r)
        hist = [L]
        for t in range(1, iters + 1):
            Js = J * scale
            A = Js @ Js.T
            ds = -Js.T @ np.linalg.solve(A + lam * np.trace(A) / 3.0 * np.eye(3), r)
            big = np.abs(ds).max()
            if big > max_step:
                ds *= max_step / big
            th_new = self.clip(theta + ds * scale)
            r_new, J_new = self.miss_and_jacobian(th_new)
            L_new = float(r_new @ r_new)
            if L_new < L:
                theta, r, J, L = th_new, r_new, J_new, L_new
                lam = max(lam / 3.0, 1e-9)
                hist.append(L)
            else:
                lam *= 10.0
            if callback:
                callback(t, L, theta)
        return theta, hist

    def close(self):
        self._record = None
        self.scene.close()


class SurrogateDesignProblem(DesignProblem):
    """The same design problem with the force at every stage time answered by the surrogate ensemble
    instead of the tracer -- the paper's Alg. 1, where the proxy sits inside the ODE.  The force is
    the ensemble mean scaled by f_ref (srp_mlp_ensemble, fused inference); its design gradient is
    the networks' input gradient (srp_mlp_backward with g_x) chained with the orbit adjoint and the
    input scaling 2 / (hi - lo).  The networks' weight-gradient buffers are cleared afterwards."""

    def __init__(self, mesh, scenario, nets, f_ref, lo, hi, r_target=None, ckpt_every=60):
        self.mesh = mesh
        self.sc = scenario
        self.nets = nets
        self.f_ref = float(f_ref)
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.sun_np = np.asarray(scenario.sun_body, dtype=np.float64)
        self.group = np.asarray(mesh.group)
        self.r_target = None if r_target is None else np.asarray(r_target, dtype=np.float64)
        self.ckpt_every = ckpt_every
        self.n_stage = 2 * scenario.n_steps + 1
        assert self.sun_np.shape[0] == self.n_stage
        n = self.n_stage
        self._y = torch.empty((n, 3), dtype=torch.float32, device="cuda")
        self._dis = torch.empty(n, dtype=torch.float32, device="cuda")
        self._idx = torch.empty(n, dtype=torch.int32, device="cuda")
        self._cnt = torch.empty(1, dtype=torch.int32, device="cuda")

    def inputs(self, theta):
        th = np.broadcast_to(np.asarray(theta, dtype=np.float64), (self.n_stage, 8))
        scaled = 2.0 * (th - self.lo) / (self.hi - self.lo) - 1.0
        x = np.concatenate([self.sun_np, scaled], 1).astype(np.float32)
        return torch.as_tensor(x, device="cuda").contiguous()

    def forces(self, theta):
        x = self.inputs(theta)
        B.srp_mlp_ensemble(self.nets[0].handle, self.nets[1].handle, x, np.inf, self.f_ref, self._y, self._idx,
                           self._cnt)
        return self._y.cpu().numpy().astype(np.float64)

    def design_grad(self, theta, F, g_final):
        x = self.inputs(theta)
        gF, _ = B.srp_orbit_rk4_adjoint(self.sc.z0, self.sc.mu, self.sc.mass, self.sc.dt, self.sc.n_steps, F,
                                        self.sc.R, g_final, self.ckpt_every)
        # F = f_ref (y_a + y_b) / 2: each network receives dL/dy = f_ref / 2 dL/dF
        g_y = torch.as_tensor((0.5 * self.f_ref * gF).astype(np.float32), device="cuda").contiguous()
        g_x = np.zeros((self.n_stage, x.shape[1]))
        for net in self.nets:
            net.forward(x, keep_activations=True)
            gx = torch.empty_like(x)
            B.srp_mlp_backward(net.handle, g_y, gx)
            B.srp_mlp_zero_grad(net.handle)
            g_x += gx.cpu().numpy().astype(np.float64)
        return g_x[:, 3:].sum(0) * 2.0 / (self.hi - self.lo)

    def close(self):
        pass
