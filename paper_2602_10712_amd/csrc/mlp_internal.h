// Internal interfaces of the surrogate-MLP part of libsrp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct srp_mlp_s;

namespace srp {

enum GemmEpilogue : int32_t {
    kEpiStore = 0,       // C = acc (+ bias[n])
    kEpiHidden = 1,      // z = acc + bias[n]; C = z (if C); Cb = bf16(SiLU(z))
    kEpiBackprop = 2,    // g = acc * SiLU'(Z[m][n]); C = g (if C); Cb = bf16(g)
    kEpiAccumulate = 3,  // C += acc
};

// C[M][N] = op(A)[M][K] . op(B)[K][N]; op(A)[m][k] = A[m*lda + k] (or A[k*lda + m] transposed),
// op(B)[k][n] = B[k*ldb + n] (or B[n*ldb + k] transposed); A, B are BF16 (uint16 bit patterns).
struct GemmArgs {
    const uint16_t* A;
    const uint16_t* B;
    int32_t M, N, K;
    int32_t lda, ldb;
    int32_t epi;
    const float* bias;
    float* C;
    int32_t ldc;
    uint16_t* Cb;
    int32_t ldcb;
    const float* Z;
    int32_t ldz;
};

hipError_t launch_gemm(const GemmArgs& g, bool trans_a, bool trans_b, hipStream_t stream);

// Split-batch weight gradient of one layer (see k_wgrad): G [K][ldg] and A [K][lda] BF16, Gf the
// FP32 gradient [K][ldgf] for the bias partials (null: none); part [splits][M][N], bpart
// [splits][M]; kc rows per split.
struct WgradArgs {
    const uint16_t* G;
    const uint16_t* A;
    const float* Gf;
    int32_t M, N, K, kc;
    int32_t ldg, lda, ldgf;
    float* part;
    float* bpart;
};
hipError_t launch_wgrad(const WgradArgs& g, int splits, hipStream_t stream);

constexpr int kMaxLayers = 17;
// Fixed-order sum of the split partials of every layer into the gradient buffer.
struct ReduceArgs {
    int32_t layers;
    int64_t total;                 // sum over layers of fout * fin + fout
    int64_t first[kMaxLayers];     // running start of each layer in that enumeration
    int32_t fin[kMaxLayers], fout[kMaxLayers], splits[kMaxLayers];
    int64_t w_off[kMaxLayers], b_off[kMaxLayers], part_off[kMaxLayers], bpart_off[kMaxLayers];
    const float* part;
    const float* bpart;
    float* grad;
};
hipError_t launch_wgrad_reduce(const ReduceArgs& r, hipStream_t stream);

// Adam step on all P parameters, gradient cleared, BF16 row-major packs rewritten.
struct AdamPackArgs {
    float* p;
    float* g;
    float* m;
    float* v;
    int64_t P;
    float lr, b1, b2, eps, c1, c2;
    int32_t layers;
    int64_t w_off[kMaxLayers], wb_off[kMaxLayers];
    int32_t fin[kMaxLayers], fout[kMaxLayers], fin_pad[kMaxLayers];
    uint16_t* wb;
};
hipError_t launch_adam_pack(const AdamPackArgs& a, hipStream_t stream);
hipError_t launch_to_bf16(const float* in, int64_t rows, int cols, int ld_in, uint16_t* out, int ld_out,
                          hipStream_t stream);
hipError_t launch_pack(const float* W, int out, int in, uint16_t* Wb, int out_pad, int in_pad, hipStream_t stream);
hipError_t launch_mse(const float* y, const float* t, int64_t count, float* gy, double* partial, double* loss,
                      hipStream_t stream);

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t stream);

// Fused inference (all layers in one kernel, weights staged in LDS, activations in registers).
bool mlp_fused_supported(int n_in, int width, int depth, int n_out);
int64_t mlp_fused_layer_elems(int layer, int depth);
hipError_t launch_pack_mfma(const float* W, int out, int in, int layer, int depth, uint16_t* dst, hipStream_t stream);
hipError_t launch_mlp_infer(const float* x, int32_t N, const uint16_t* wf, const int64_t* wf_off_dev,
                            const float* params, const int64_t* b_off_dev, int n_in, int depth, int n_out, float* y,
                            hipStream_t stream);

// Ensemble confidence test (ensemble.hip): mean, disagreement and failure flags of two networks'
// outputs, then the failing query indices compacted in ascending order.
size_t ensemble_select_bytes(int64_t N);
hipError_t launch_ensemble(const float* x, int n_in, const float* ya, const float* yb, int n_out, int64_t N,
                           float threshold, float scale, float* y, float* dis, uint8_t* flag, void* tmp,
                           size_t tmp_bytes, int32_t* fail_idx, int32_t* n_fail, hipStream_t stream);

// The network as a model inside other integrators: its shape and a workspace it owns (grown on
// demand, freed with the network; calls using one network must be ordered).
void mlp_shape(const srp_mlp_s* m, int* n_in, int* n_out, int* device);
hipError_t mlp_aux(srp_mlp_s* m, size_t bytes, void** out);

}  // namespace srp
