// libsrp: 13-D orbit-and-attitude integration with the network as force-and-torque model
// (paper Sec. 3.4.1, Eq. ODE, and the proxy of Sec. 3.3 inside it).  Host side: argument checks,
// the inverse inertia tensor, the workspace carve-up and the launch sequence
//   init, then per step and stage: network inference on the stage inputs, stage kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/srp.h"
#include "attitude_internal.h"
#include "mlp_internal.h"
#include "scene.h"

namespace {

#define ATT_HIP(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return srp_fail(SRP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// inverse of a symmetric positive-definite 3x3 (adjugate / determinant); false when it is not
bool spd_inverse(const double I[9], double out[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < i; ++j) {
            const double s = std::fabs(I[3 * i + j]) + std::fabs(I[3 * j + i]);
            if (!std::isfinite(I[3 * i + j]) || std::fabs(I[3 * i + j] - I[3 * j + i]) > 1e-12 * (s + 1e-300))
                return false;
        }
    // leading principal minors
    const double m1 = I[0], m2 = I[0] * I[4] - I[1] * I[3];
    const double c00 = I[4] * I[8] - I[5] * I[7], c01 = I[5] * I[6] - I[3] * I[8], c02 = I[3] * I[7] - I[4] * I[6];
    const double det = I[0] * c00 + I[1] * c01 + I[2] * c02;
    if (!(m1 > 0) || !(m2 > 0) || !(det > 0) || !std::isfinite(det)) return false;
    const double adj[9] = {c00, I[2] * I[7] - I[1] * I[8], I[1] * I[5] - I[2] * I[4],
                           c01, I[0] * I[8] - I[2] * I[6], I[2] * I[3] - I[0] * I[5],
                           c02, I[1] * I[6] - I[0] * I[7], I[0] * I[4] - I[1] * I[3]};
    for (int k = 0; k < 9; ++k) out[k] = adj[k] / det;
    return true;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

extern "C" {

srp_status srp_attitude_rk4(srp_mlp model, const srp_attitude_params* p, const double* z0, const float* design,
                            int64_t B, double* z_final, double* z_all, void* stream_)
{
    if (!model || !p) return srp_fail(SRP_EINVAL, "model and params are required");
    int n_in = 0, n_out = 0, device = 0;
    srp::mlp_shape(model, &n_in, &n_out, &device);
    if (n_in < 3 || n_out < 6) return srp_fail(SRP_EINVAL, "the network needs n_in >= 3 and n_out >= 6");
    if (B < 0 || B > (int64_t(1) << 30)) return srp_fail(SRP_EINVAL, "B must be in [0, 2^30]");
    if (!(p->mu > 0) || !(p->mass > 0) || !(p->dt > 0) || !std::isfinite(p->dt) || p->n_steps < 0 ||
        !(p->earth_radius >= 0) || !std::isfinite(p->force_scale) || !std::isfinite(p->torque_scale))
        return srp_fail(SRP_EINVAL, "bad integration parameters");
    if (p->n_steps > (int64_t(1) << 40)) return srp_fail(SRP_EINVAL, "too many steps");
    if (p->steps_per_design < 0) return srp_fail(SRP_EINVAL, "steps_per_design must be >= 0");
    const double sn = std::sqrt(p->sun[0] * p->sun[0] + p->sun[1] * p->sun[1] + p->sun[2] * p->sun[2]);
    if (!(sn > 0) || !std::isfinite(sn)) return srp_fail(SRP_EINVAL, "sun direction must be finite and nonzero");
    srp::AttArgs a{};
    if (!spd_inverse(p->inertia, a.Iinv)) return srp_fail(SRP_EINVAL, "inertia must be symmetric positive definite");
    if (B == 0) return SRP_OK;
    if (!z0 || !z_final) return srp_fail(SRP_EINVAL, "z0 and z_final are required");
    if (n_in > 3 && !design) return srp_fail(SRP_EINVAL, "design rows are required when n_in > 3");
    int cur = -1;
    ATT_HIP(hipGetDevice(&cur));
    if (cur != device) ATT_HIP(hipSetDevice(device));
    hipStream_t stream = static_cast<hipStream_t>(stream_);

    a.B = B;
    a.n_in = n_in;
    a.n_out = n_out;
    a.mu = p->mu;
    a.inv_mass = 1.0 / p->mass;
    for (int k = 0; k < 9; ++k) a.I[k] = p->inertia[k];
    for (int k = 0; k < 3; ++k) a.sun[k] = p->sun[k] / sn;
    a.force_scale = p->force_scale;
    a.torque_scale = p->torque_scale;
    a.re2 = p->earth_radius * p->earth_radius;
    a.h = p->dt;
    a.z_all = z_all;
    a.z_final = z_final;
    a.design = design;
    a.steps_per_design = n_in > 3 ? p->steps_per_design : 0;
    a.n_segments = a.steps_per_design > 0
                       ? std::max<int64_t>(1, (p->n_steps + a.steps_per_design - 1) / a.steps_per_design)
                       : 1;
    // workspace: Z, Y, A [13][B] double, X [B][n_in] float, O [B][n_out] float
    const size_t nb = static_cast<size_t>(B);
    const size_t s_state = align256(13 * nb * sizeof(double));
    const size_t s_x = align256(nb * n_in * sizeof(float));
    const size_t s_o = align256(nb * n_out * sizeof(float));
    void* ws = nullptr;
    ATT_HIP(srp::mlp_aux(model, 3 * s_state + s_x + s_o, &ws));
    char* w = static_cast<char*>(ws);
    a.Z = reinterpret_cast<double*>(w);
    a.Y = reinterpret_cast<double*>(w + s_state);
    a.A = reinterpret_cast<double*>(w + 2 * s_state);
    a.X = reinterpret_cast<float*>(w + 3 * s_state);
    float* O = reinterpret_cast<float*>(w + 3 * s_state + s_x);
    a.O = O;

    ATT_HIP(srp::launch_att_init(a, z0, design, stream));
    if (p->n_steps == 0) {
        ATT_HIP(srp::launch_att_copy_out(a, stream));
        return SRP_OK;
    }
    for (int64_t n = 0; n < p->n_steps; ++n) {
        for (int stage = 1; stage <= 4; ++stage) {
            const srp_status st = srp_mlp_forward(model, a.X, B, O, 0, stream);
            if (st != SRP_OK) return st;
            ATT_HIP(srp::launch_att_stage(a, stage, n, stage == 4 && n == p->n_steps - 1, stream));
        }
    }
    return SRP_OK;
}

}  // extern "C"
