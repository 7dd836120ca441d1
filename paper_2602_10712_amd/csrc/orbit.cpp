// Orbit integration with solar radiation pressure and its discrete adjoint (host, FP64).
//
// Paper Sec. 3.4.1 (Eq. ODE): the translational state moves by dr/dt = v and
// dv/dt = m^-1 T^T F(w_body, theta) + o(z), with F the body-frame radiation-pressure force, T the
// attitude (body <- inertial) and o the other accelerations; the integrator is the classic
// fourth-order Runge-Kutta scheme in double precision, and the design is optimised through the
// adjoint of the integration (Sec. 3.4.3).  Here o is point-mass gravity -mu r / |r|^3, the
// attitude is a function of time only (so the body-frame sun direction at every stage time is
// known before integrating and the forces of all stage times come from one batched trace), and
// the adjoint is the exact discrete adjoint of the RK4 steps with checkpoints: the reverse sweep
// recomputes each segment of `ckpt_every` steps from its stored state.
//
// Stage times of step n (step length h): t_n (k1), t_n + h/2 (k2, k3), t_n + h (k4); the force
// table holds one body-frame force per distinct stage time, index 2n, 2n + 1, 2n + 2.
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/srp.h"
#include "scene.h"

namespace {

struct OrbitCtx {
    double mu, inv_mass, h;
    const double* F;  // [2 n + 1][3] body frame
    const double* R;  // [2 n + 1][9] body -> inertial, row-major
};

// f(z) = (v, -mu r / |r|^3 + R_k F_k / m)
void deriv(const OrbitCtx& c, const double z[6], int64_t k, double out[6])
{
    const double* r = z;
    const double rr = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const double g = -c.mu / (rr * rr * rr);
    const double* R = c.R + 9 * k;
    const double* F = c.F + 3 * k;
    for (int a = 0; a < 3; ++a) {
        out[a] = z[3 + a];
        out[3 + a] = g * r[a] + c.inv_mass * (R[3 * a] * F[0] + R[3 * a + 1] * F[1] + R[3 * a + 2] * F[2]);
    }
}

void step(const OrbitCtx& c, const double z[6], int64_t n, double out[6])
{
    double k1[6], k2[6], k3[6], k4[6], y[6];
    deriv(c, z, 2 * n, k1);
    for (int a = 0; a < 6; ++a) y[a] = z[a] + 0.5 * c.h * k1[a];
    deriv(c, y, 2 * n + 1, k2);
    for (int a = 0; a < 6; ++a) y[a] = z[a] + 0.5 * c.h * k2[a];
    deriv(c, y, 2 * n + 1, k3);
    for (int a = 0; a < 6; ++a) y[a] = z[a] + c.h * k3[a];
    deriv(c, y, 2 * n + 2, k4);
    for (int a = 0; a < 6; ++a) out[a] = z[a] + c.h / 6.0 * (k1[a] + 2.0 * k2[a] + 2.0 * k3[a] + k4[a]);
}

// lam_out = J(y)^T a for f's Jacobian at state y: J^T a = (G(r) a_v, a_r), G = d(gravity)/dr
// (symmetric); also adds R_k^T a_v / m to the force adjoint of stage k.
void deriv_adjoint(const OrbitCtx& c, const double y[6], int64_t k, const double a[6], double lam_out[6], double* gF)
{
    const double* r = y;
    const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double rr = std::sqrt(r2);
    const double i3 = 1.0 / (rr * r2), i5 = i3 / r2;
    const double* av = a + 3;
    const double rav = r[0] * av[0] + r[1] * av[1] + r[2] * av[2];
    for (int q = 0; q < 3; ++q) {
        lam_out[q] = -c.mu * (av[q] * i3 - 3.0 * r[q] * rav * i5);
        lam_out[3 + q] = a[q];
    }
    const double* R = c.R + 9 * k;
    for (int q = 0; q < 3; ++q)
        gF[3 * k + q] += c.inv_mass * (R[q] * av[0] + R[3 + q] * av[1] + R[6 + q] * av[2]);
}

// reverse of one RK4 step from state z (step n): lam (dL/dz_{n+1}) -> dL/dz_n, accumulating gF
void step_adjoint(const OrbitCtx& c, const double z[6], int64_t n, double lam[6], double* gF)
{
    const double h = c.h;
    double k1[6], k2[6], k3[6], y2[6], y3[6], y4[6];
    deriv(c, z, 2 * n, k1);
    for (int a = 0; a < 6; ++a) y2[a] = z[a] + 0.5 * h * k1[a];
    deriv(c, y2, 2 * n + 1, k2);
    for (int a = 0; a < 6; ++a) y3[a] = z[a] + 0.5 * h * k2[a];
    deriv(c, y3, 2 * n + 1, k3);
    for (int a = 0; a < 6; ++a) y4[a] = z[a] + h * k3[a];
    double a1[6], a2[6], a3[6], a4[6], t[6], lz[6];
    for (int q = 0; q < 6; ++q) {
        a1[q] = h / 6.0 * lam[q];
        a2[q] = h / 3.0 * lam[q];
        a3[q] = h / 3.0 * lam[q];
        a4[q] = h / 6.0 * lam[q];
        lz[q] = lam[q];
    }
    deriv_adjoint(c, y4, 2 * n + 2, a4, t, gF);
    for (int q = 0; q < 6; ++q) {
        lz[q] += t[q];
        a3[q] += h * t[q];
    }
    deriv_adjoint(c, y3, 2 * n + 1, a3, t, gF);
    for (int q = 0; q < 6; ++q) {
        lz[q] += t[q];
        a2[q] += 0.5 * h * t[q];
    }
    deriv_adjoint(c, y2, 2 * n + 1, a2, t, gF);
    for (int q = 0; q < 6; ++q) {
        lz[q] += t[q];
        a1[q] += 0.5 * h * t[q];
    }
    deriv_adjoint(c, z, 2 * n, a1, t, gF);
    for (int q = 0; q < 6; ++q) lam[q] = lz[q] + t[q];
}

srp_status check(const double* z0, double mu, double mass, double dt, int64_t n_steps, const double* F,
                 const double* R)
{
    if (!z0 || !F || !R) return srp_fail(SRP_EINVAL, "z0, forces and rotations are required");
    if (!(mu > 0) || !(mass > 0) || !(dt > 0) || n_steps < 0) return srp_fail(SRP_EINVAL, "bad orbit parameters");
    if (n_steps > (int64_t(1) << 30)) return srp_fail(SRP_EINVAL, "too many steps");
    const double r2 = z0[0] * z0[0] + z0[1] * z0[1] + z0[2] * z0[2];
    if (!(r2 > 0) || !std::isfinite(r2)) return srp_fail(SRP_EINVAL, "initial position must be finite and non-zero");
    return SRP_OK;
}

}  // namespace

extern "C" {

srp_status srp_orbit_rk4(const double* z0, double mu, double mass, double dt, int64_t n_steps, const double* F_body,
                         const double* R_body_to_inertial, double* z_all, double* z_final)
{
    srp_status st = check(z0, mu, mass, dt, n_steps, F_body, R_body_to_inertial);
    if (st != SRP_OK) return st;
    if (!z_final) return srp_fail(SRP_EINVAL, "z_final is required");
    const OrbitCtx c{mu, 1.0 / mass, dt, F_body, R_body_to_inertial};
    double z[6], zn[6];
    std::memcpy(z, z0, sizeof(z));
    if (z_all) std::memcpy(z_all, z, sizeof(z));
    for (int64_t n = 0; n < n_steps; ++n) {
        step(c, z, n, zn);
        std::memcpy(z, zn, sizeof(z));
        if (z_all) std::memcpy(z_all + 6 * (n + 1), z, sizeof(z));
    }
    std::memcpy(z_final, z, sizeof(z));
    return SRP_OK;
}

srp_status srp_orbit_rk4_adjoint(const double* z0, double mu, double mass, double dt, int64_t n_steps,
                                 const double* F_body, const double* R_body_to_inertial, const double* g_final,
                                 int64_t ckpt_every, double* g_F, double* g_z0)
{
    srp_status st = check(z0, mu, mass, dt, n_steps, F_body, R_body_to_inertial);
    if (st != SRP_OK) return st;
    if (!g_final || !g_F) return srp_fail(SRP_EINVAL, "g_final and g_F are required");
    if (ckpt_every < 1) return srp_fail(SRP_EINVAL, "ckpt_every must be >= 1");
    const OrbitCtx c{mu, 1.0 / mass, dt, F_body, R_body_to_inertial};
    std::memset(g_F, 0, sizeof(double) * 3 * (2 * n_steps + 1));
    // forward sweep: keep one state per segment
    const int64_t n_seg = (n_steps + ckpt_every - 1) / ckpt_every;
    std::vector<double> ckpt(6 * (n_seg + 1));
    double z[6], zn[6];
    std::memcpy(z, z0, sizeof(z));
    for (int64_t n = 0; n < n_steps; ++n) {
        if (n % ckpt_every == 0) std::memcpy(&ckpt[6 * (n / ckpt_every)], z, sizeof(z));
        step(c, z, n, zn);
        std::memcpy(z, zn, sizeof(z));
    }
    // reverse sweep: recompute each segment's states from its checkpoint
    double lam[6];
    std::memcpy(lam, g_final, sizeof(lam));
    std::vector<double> seg(6 * (ckpt_every + 1));
    for (int64_t s = n_seg - 1; s >= 0; --s) {
        const int64_t n0 = s * ckpt_every;
        const int64_t n1 = std::min<int64_t>(n0 + ckpt_every, n_steps);
        std::memcpy(&seg[0], &ckpt[6 * s], sizeof(double) * 6);
        for (int64_t n = n0; n < n1 - 1; ++n) step(c, &seg[6 * (n - n0)], n, &seg[6 * (n - n0 + 1)]);
        for (int64_t n = n1 - 1; n >= n0; --n) step_adjoint(c, &seg[6 * (n - n0)], n, lam, g_F);
    }
    if (g_z0) std::memcpy(g_z0, lam, sizeof(lam));
    return SRP_OK;
}

}  // extern "C"
