// Internal interface of the 13-D orbit-and-attitude integrator (device part).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srp {

// One batch of trajectories.  Workspace arrays are structure-of-arrays over the trajectories
// ([13][B] doubles): Z the state at the start of the step, Y the state of the current stage, A the
// running stage sum k1 + 2 k2 + 2 k3 + k4; X [B][n_in] float the network input, O [B][n_out]
// float its output.
struct AttArgs {
    int64_t B;
    int32_t n_in, n_out;
    double mu, inv_mass;
    double I[9], Iinv[9];
    double sun[3];
    double force_scale, torque_scale;
    double re2;  // earth radius squared; 0: no eclipse
    double h;
    double* Z;
    double* Y;
    double* A;
    float* X;
    const float* O;
    double* z_all;    // [n_steps + 1][B][13] or null
    double* z_final;  // [B][13]
    const float* design;       // [n_segments][B][n_in - 3] (one segment: constant design)
    int64_t steps_per_design;  // 0: constant
    int64_t n_segments;
};

// k_att_init: Z = Y = z0, network input of stage 1 (design columns written once), z_all[0].
hipError_t launch_att_init(const AttArgs& a, const double* z0, const float* design, hipStream_t stream);
// Stage `stage` (1..4) of step `step`: k from Y and the network output, the stage sum, and the
// next stage's state and network input; stage 4 completes the step (z_all[step + 1], and z_final
// when `last`).
hipError_t launch_att_stage(const AttArgs& a, int stage, int64_t step, bool last, hipStream_t stream);
// z_final = Z (for n_steps = 0).
hipError_t launch_att_copy_out(const AttArgs& a, hipStream_t stream);

}  // namespace srp
