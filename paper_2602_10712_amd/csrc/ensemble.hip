// Confidence test of the two-network surrogate ensemble (paper Sec. 3.3: the proxy answers force
// queries in place of the simulator; here the simulator stays as the fallback and the judge of the
// proxy's error).
//
// k_ensemble  per query: mean of the two networks' outputs (scaled to physical units), their
//             disagreement ||y_a - y_b||, and the failure flag -- outside the training domain (the
//             sun input not a unit vector, or a scaled design input outside [-1, 1]) or
//             disagreement above the threshold.
// The failing queries are then compacted in ascending order (rocPRIM flagged select), so the
// caller can hand exactly those to the tracer.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <rocprim/device/device_select.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "mlp_internal.h"

namespace srp {
namespace {

constexpr float kUnitTol = 1e-5f;    // | ||sun|| - 1 | allowed for a float unit vector
constexpr float kBoxTol = 1e-6f;     // scaled design inputs: |x| <= 1 + this

__global__ void k_ensemble(const float* __restrict__ x, int n_in, const float* __restrict__ ya,
                           const float* __restrict__ yb, int n_out, int64_t N, float threshold, float scale,
                           float* __restrict__ y, float* __restrict__ dis, uint8_t* __restrict__ flag)
{
    const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const float* xq = x + q * n_in;
    const float sx = xq[0], sy = xq[1], sz = xq[2];
    bool out = !(fabsf(sqrtf(sx * sx + sy * sy + sz * sz) - 1.0f) <= kUnitTol);
    for (int i = 3; i < n_in; ++i) out |= !(fabsf(xq[i]) <= 1.0f + kBoxTol);
    float d2 = 0.0f;
    for (int c = 0; c < n_out; ++c) {
        const float a = ya[q * n_out + c], b = yb[q * n_out + c];
        y[q * n_out + c] = scale * (0.5f * (a + b));
        d2 += (a - b) * (a - b);
    }
    const float d = sqrtf(d2);
    if (dis) dis[q] = d;
    flag[q] = (out || !(d <= threshold)) ? 1 : 0;
}

}  // namespace

size_t ensemble_select_bytes(int64_t N)
{
    size_t bytes = 0;
    (void)rocprim::select(nullptr, bytes, rocprim::counting_iterator<int32_t>(0), static_cast<const uint8_t*>(nullptr),
                          static_cast<int32_t*>(nullptr), static_cast<int32_t*>(nullptr), static_cast<size_t>(N));
    return bytes;
}

hipError_t launch_ensemble(const float* x, int n_in, const float* ya, const float* yb, int n_out, int64_t N,
                           float threshold, float scale, float* y, float* dis, uint8_t* flag, void* tmp,
                           size_t tmp_bytes, int32_t* fail_idx, int32_t* n_fail, hipStream_t stream)
{
    if (N <= 0) return hipSuccess;
    const unsigned blocks = static_cast<unsigned>((N + 255) / 256);
    hipLaunchKernelGGL(k_ensemble, dim3(blocks), dim3(256), 0, stream, x, n_in, ya, yb, n_out, N, threshold, scale, y,
                       dis, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return rocprim::select(tmp, tmp_bytes, rocprim::counting_iterator<int32_t>(0), flag, fail_idx, n_fail,
                           static_cast<size_t>(N), stream);
}

}  // namespace srp
