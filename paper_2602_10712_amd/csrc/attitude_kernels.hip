// 13-D orbit-and-attitude integration on the GPU (paper Sec. 3.4.1, Eq. ODE; RK4 in FP64): the
// stage kernels between the network calls that supply force and torque.
//
// One lane per trajectory, state in FP64 structure-of-arrays (coalesced loads of each component).
// Per stage the kernel takes the stage state Y and the network's answer for it, forms the
// derivative k, adds it to the stage sum with the RK4 weights (in the order k1 + 2 k2 + 2 k3 +
// k4), and writes the next stage's state and network input (the Sun direction in the body frame
// at that state); the fourth stage completes the step.
#include "attitude_internal.h"

namespace srp {
namespace {

constexpr int kAttThreads = 256;

// R(q / |q|), body -> inertial, row-major
__device__ __forceinline__ void rot(const double q[4], double R[9])
{
    const double inv = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double q0 = q[0] * inv, q1 = q[1] * inv, q2 = q[2] * inv, q3 = q[3] * inv;
    R[0] = 1.0 - 2.0 * (q2 * q2 + q3 * q3);
    R[1] = 2.0 * (q1 * q2 - q0 * q3);
    R[2] = 2.0 * (q1 * q3 + q0 * q2);
    R[3] = 2.0 * (q1 * q2 + q0 * q3);
    R[4] = 1.0 - 2.0 * (q1 * q1 + q3 * q3);
    R[5] = 2.0 * (q2 * q3 - q0 * q1);
    R[6] = 2.0 * (q1 * q3 - q0 * q2);
    R[7] = 2.0 * (q2 * q3 + q0 * q1);
    R[8] = 1.0 - 2.0 * (q1 * q1 + q2 * q2);
}

// network input of a state: float(R(q)^T sun)
__device__ __forceinline__ void write_input(const AttArgs& a, const double y[13], int64_t b)
{
    double R[9];
    rot(y + 6, R);
    float* x = a.X + b * a.n_in;
    for (int i = 0; i < 3; ++i)
        x[i] = static_cast<float>(R[i] * a.sun[0] + R[3 + i] * a.sun[1] + R[6 + i] * a.sun[2]);
}

// cylinder eclipse factor
__device__ __forceinline__ double lit(const AttArgs& a, const double r[3])
{
    if (a.re2 <= 0.0) return 1.0;
    const double along = r[0] * a.sun[0] + r[1] * a.sun[1] + r[2] * a.sun[2];
    const double p0 = r[0] - along * a.sun[0], p1 = r[1] - along * a.sun[1], p2 = r[2] - along * a.sun[2];
    return (along < 0.0 && p0 * p0 + p1 * p1 + p2 * p2 < a.re2) ? 0.0 : 1.0;
}

// k = f(y) with the network output o (force and torque in units of the scales)
__device__ __forceinline__ void deriv(const AttArgs& a, const double y[13], const float* o, double k[13])
{
    const double* r = y;
    const double* v = y + 3;
    const double* q = y + 6;
    const double* w = y + 10;
    double R[9];
    rot(q, R);
    const double nu = lit(a, r);
    const double F[3] = {a.force_scale * o[0], a.force_scale * o[1], a.force_scale * o[2]};
    const double tau[3] = {a.torque_scale * o[3], a.torque_scale * o[4], a.torque_scale * o[5]};
    const double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const double g = -a.mu / (rr * rr * rr);
    for (int i = 0; i < 3; ++i) {
        k[i] = v[i];
        const double RF = R[3 * i] * F[0] + R[3 * i + 1] * F[1] + R[3 * i + 2] * F[2];
        k[3 + i] = g * r[i] + nu * RF * a.inv_mass;
    }
    // 1/2 q (x) (0, w)
    k[6] = 0.5 * (-q[1] * w[0] - q[2] * w[1] - q[3] * w[2]);
    k[7] = 0.5 * (q[0] * w[0] + q[2] * w[2] - q[3] * w[1]);
    k[8] = 0.5 * (q[0] * w[1] + q[3] * w[0] - q[1] * w[2]);
    k[9] = 0.5 * (q[0] * w[2] + q[1] * w[1] - q[2] * w[0]);
    // I^-1 (nu tau - w x I w)
    double Iw[3], m[3];
    for (int i = 0; i < 3; ++i) Iw[i] = a.I[3 * i] * w[0] + a.I[3 * i + 1] * w[1] + a.I[3 * i + 2] * w[2];
    m[0] = nu * tau[0] - (w[1] * Iw[2] - w[2] * Iw[1]);
    m[1] = nu * tau[1] - (w[2] * Iw[0] - w[0] * Iw[2]);
    m[2] = nu * tau[2] - (w[0] * Iw[1] - w[1] * Iw[0]);
    for (int i = 0; i < 3; ++i) k[10 + i] = a.Iinv[3 * i] * m[0] + a.Iinv[3 * i + 1] * m[1] + a.Iinv[3 * i + 2] * m[2];
}

__global__ void k_att_init(AttArgs a, const double* __restrict__ z0, const float* __restrict__ design)
{
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    double y[13];
    for (int c = 0; c < 13; ++c) {
        y[c] = z0[13 * b + c];
        a.Z[c * a.B + b] = y[c];
        a.Y[c * a.B + b] = y[c];
        if (a.z_all) a.z_all[13 * b + c] = y[c];
    }
    const int nd = a.n_in - 3;
    for (int j = 0; j < nd; ++j) a.X[b * a.n_in + 3 + j] = design[b * nd + j];
    write_input(a, y, b);
}

__global__ void k_att_stage(AttArgs a, int stage, int64_t step, int last)
{
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    const int64_t B = a.B;
    double y[13], k[13];
    for (int c = 0; c < 13; ++c) y[c] = a.Y[c * B + b];
    deriv(a, y, a.O + b * a.n_out, k);
    if (stage < 4) {
        const double c_next = stage == 3 ? a.h : 0.5 * a.h;
        for (int c = 0; c < 13; ++c) {
            const double acc = stage == 1 ? k[c] : a.A[c * B + b] + 2.0 * k[c];
            a.A[c * B + b] = acc;
            y[c] = a.Z[c * B + b] + c_next * k[c];
            a.Y[c * B + b] = y[c];
        }
    } else {
        const double w = a.h / 6.0;
        double* out = a.z_all ? a.z_all + ((step + 1) * B + b) * 13 : nullptr;
        for (int c = 0; c < 13; ++c) {
            const double acc = a.A[c * B + b] + k[c];
            y[c] = a.Z[c * B + b] + w * acc;
            a.Z[c * B + b] = y[c];
            a.Y[c * B + b] = y[c];
            if (out) out[c] = y[c];
            if (last) a.z_final[13 * b + c] = y[c];
        }
        // a design schedule: the next step's row (its stages all use it)
        if (a.steps_per_design > 0 && !last) {
            const int64_t seg = min((step + 1) / a.steps_per_design, a.n_segments - 1);
            const int nd = a.n_in - 3;
            const float* row = a.design + (seg * B + b) * nd;
            for (int j = 0; j < nd; ++j) a.X[b * a.n_in + 3 + j] = row[j];
        }
    }
    write_input(a, y, b);
}

__global__ void k_att_copy_out(AttArgs a)
{
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    for (int c = 0; c < 13; ++c) a.z_final[13 * b + c] = a.Z[c * a.B + b];
}

unsigned blocks(int64_t B) { return static_cast<unsigned>((B + kAttThreads - 1) / kAttThreads); }

}  // namespace

hipError_t launch_att_init(const AttArgs& a, const double* z0, const float* design, hipStream_t stream)
{
    hipLaunchKernelGGL(k_att_init, dim3(blocks(a.B)), dim3(kAttThreads), 0, stream, a, z0, design);
    return hipGetLastError();
}

hipError_t launch_att_stage(const AttArgs& a, int stage, int64_t step, bool last, hipStream_t stream)
{
    hipLaunchKernelGGL(k_att_stage, dim3(blocks(a.B)), dim3(kAttThreads), 0, stream, a, stage, step, last ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_att_copy_out(const AttArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_att_copy_out, dim3(blocks(a.B)), dim3(kAttThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace srp
