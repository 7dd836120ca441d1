// libsrp host side of the force-surrogate MLP: C ABI (include/srp.h), parameter storage (FP32
// masters, Adam moments, BF16 packed copies), workspaces and the layer-by-layer orchestration of
// the kernels in mlp_kernels.hip and mlp_infer.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/srp.h"
#include "mlp_internal.h"
#include "scene.h"
#include "srp_path.h"

namespace {

#define MLP_HIP(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return srp_fail(SRP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

int round8(int x) { return (x + 7) / 8 * 8; }

template <class T>
hipError_t grow(T*& ptr, size_t& cap, size_t n)
{
    if (n <= cap && ptr) return hipSuccess;
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    cap = 0;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&ptr), std::max<size_t>(n, 1) * sizeof(T));
    if (e == hipSuccess) cap = std::max<size_t>(n, 1);
    return e;
}

}  // namespace

struct srp_mlp_s {
    int device = 0;
    int n_in = 0, width = 0, depth = 0, n_out = 0;
    int64_t P = 0;
    int64_t step = 0;
    // per layer l = 0..depth (depth = output layer)
    std::vector<int> fin, fout, fin_pad, fout_pad;
    std::vector<int64_t> w_off, b_off, wb_off;
    float* d_p = nullptr;   // FP32 masters [P]
    float* d_g = nullptr;   // gradients [P] (accumulated by backward, cleared by the Adam step)
    float* d_m = nullptr;
    float* d_v = nullptr;
    uint16_t* d_wb = nullptr;  // BF16 weights, layer l: [fout_pad][fin_pad]
    int64_t wb_total = 0;
    bool fused = false;        // the fused inference kernel serves this shape
    uint16_t* d_wf = nullptr;  // BF16 weights in A-operand pieces for the fused kernel
    std::vector<int64_t> wf_off;
    int64_t* d_wf_off = nullptr;  // device copies of wf_off and b_off
    int64_t* d_b_off = nullptr;
    // workspaces
    size_t cap_xb = 0, cap_Z = 0, cap_A = 0, cap_G = 0, cap_Gb = 0, cap_lp = 0;
    uint16_t* d_xb = nullptr;
    float* d_Z = nullptr;
    uint16_t* d_A = nullptr;
    float* d_G = nullptr;
    uint16_t* d_Gb = nullptr;  // two halves, ping-pong
    double* d_lpart = nullptr;
    int64_t cached_N = -1;
    // workspace of callers that use the network as a model (attitude integration)
    char* d_aux = nullptr;
    size_t cap_aux = 0;
    // ensemble workspace (this network as member a): both outputs, flags, compaction scratch
    char* d_ens = nullptr;
    size_t cap_ens = 0;
    // split-batch weight-gradient partials [splits][fout][fin] and bias partials per layer
    float* d_wpart = nullptr;
    size_t cap_wpart = 0;
    float* d_bpart = nullptr;
    size_t cap_bpart = 0;
    bool wf_stale = false;  // the fused kernel's weight pieces lag the masters (refreshed before use)
};

namespace {

srp_status bind(const srp_mlp_s* m)
{
    int cur = -1;
    MLP_HIP(hipGetDevice(&cur));
    if (cur != m->device) MLP_HIP(hipSetDevice(m->device));
    return SRP_OK;
}

// The fused inference kernel's weight pieces, rebuilt from the masters when they changed.
srp_status refresh_fused(srp_mlp_s* m, hipStream_t stream)
{
    if (!m->fused || !m->wf_stale) return SRP_OK;
    for (int l = 0; l <= m->depth; ++l)
        MLP_HIP(srp::launch_pack_mfma(m->d_p + m->w_off[l], m->fout[l], m->fin[l], l, m->depth, m->d_wf + m->wf_off[l],
                                      stream));
    m->wf_stale = false;
    return SRP_OK;
}

srp_status repack(srp_mlp_s* m, hipStream_t stream)
{
    for (int l = 0; l <= m->depth; ++l)
        MLP_HIP(srp::launch_pack(m->d_p + m->w_off[l], m->fout[l], m->fin[l], m->d_wb + m->wb_off[l], m->fout_pad[l],
                                 m->fin_pad[l], stream));
    m->wf_stale = true;
    return refresh_fused(m, stream);
}

// Batch splits of a layer's weight gradient: enough workgroups to fill the chip (about 256 tiles x
// splits), at least 32 rows per split.  Returns the split count; *kc receives rows per split.
int wgrad_splits(int fout, int fin, int64_t K, int* kc)
{
    const int tiles = ((fout + 63) / 64) * ((fin + 63) / 64);
    const int64_t want = std::max<int64_t>(1, 256 / tiles);
    int64_t c = (K + want - 1) / want;
    c = std::max<int64_t>(32, (c + 31) / 32 * 32);
    *kc = static_cast<int>(c);
    return static_cast<int>((K + c - 1) / c);
}

srp_status ensure_ws(srp_mlp_s* m, int64_t N, bool training)
{
    const int64_t wmax = std::max(m->width, round8(m->n_out));
    MLP_HIP(grow(m->d_xb, m->cap_xb, static_cast<size_t>(N * m->fin_pad[0])));
    const int64_t layers_kept = training ? m->depth : 1;
    MLP_HIP(grow(m->d_A, m->cap_A, static_cast<size_t>(layers_kept * N * m->width)));
    if (training) {
        MLP_HIP(grow(m->d_Z, m->cap_Z, static_cast<size_t>(m->depth * N * m->width)));
        MLP_HIP(grow(m->d_G, m->cap_G, static_cast<size_t>(N * wmax)));
        MLP_HIP(grow(m->d_Gb, m->cap_Gb, static_cast<size_t>(2 * N * wmax)));
    } else if (m->depth > 1) {
        // inference without cache: two activation buffers (ping-pong)
        MLP_HIP(grow(m->d_A, m->cap_A, static_cast<size_t>(2 * N * m->width)));
    }
    return SRP_OK;
}

}  // namespace

extern "C" {

srp_status srp_mlp_create(int32_t n_in, int32_t width, int32_t depth, int32_t n_out, uint64_t seed, srp_mlp* out)
{
    if (!out) return srp_fail(SRP_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_in < 1 || n_in > 64 || n_out < 1 || n_out > 64 || depth < 1 || depth > 16 || width < 8 || width > 4096 ||
        width % 8 != 0)
        return srp_fail(SRP_EINVAL, "need 1 <= n_in, n_out <= 64, 1 <= depth <= 16, width a multiple of 8 in [8, 4096]");
    srp_mlp_s* m = new (std::nothrow) srp_mlp_s();
    if (!m) return srp_fail(SRP_ENOMEM, "host allocation failed");
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return srp_fail(SRP_EDEVICE, "hipGetDevice failed");
    }
    m->n_in = n_in;
    m->width = width;
    m->depth = depth;
    m->n_out = n_out;
    int64_t off = 0, woff = 0;
    for (int l = 0; l <= depth; ++l) {
        const int fi = l == 0 ? n_in : width, fo = l == depth ? n_out : width;
        m->fin.push_back(fi);
        m->fout.push_back(fo);
        m->fin_pad.push_back(round8(fi));
        m->fout_pad.push_back(round8(fo));
        m->w_off.push_back(off);
        off += static_cast<int64_t>(fi) * fo;
        m->b_off.push_back(off);
        off += fo;
        m->wb_off.push_back(woff);
        woff += static_cast<int64_t>(round8(fi)) * round8(fo);
    }
    m->P = off;
    m->wb_total = woff;
    m->fused = srp::mlp_fused_supported(n_in, width, depth, n_out);
    int64_t foff = 0;
    for (int l = 0; l <= depth; ++l) {
        m->wf_off.push_back(foff);
        if (m->fused) foff += srp::mlp_fused_layer_elems(l, depth);
    }
    // seeded initial weights and biases: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from Philox draws
    std::vector<float> h(m->P);
    for (int l = 0; l <= depth; ++l) {
        const float bound = 1.0f / std::sqrt(static_cast<float>(m->fin[l]));
        const int64_t n = static_cast<int64_t>(m->fin[l]) * m->fout[l] + m->fout[l];
        for (int64_t i = 0; i < n; ++i) {
            uint32_t c0 = static_cast<uint32_t>(i), c1 = static_cast<uint32_t>(l), c2 = 0x4D4C50u, c3 = 0u;
            srp::philox4x32_10(c0, c1, c2, c3, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
            h[m->w_off[l] + i] = (2.0f * srp::unit24(c0) - 1.0f) * bound;
        }
    }
    hipError_t e = hipMalloc(&m->d_p, sizeof(float) * m->P);
    if (e == hipSuccess) e = hipMalloc(&m->d_g, sizeof(float) * m->P);
    if (e == hipSuccess) e = hipMalloc(&m->d_m, sizeof(float) * m->P);
    if (e == hipSuccess) e = hipMalloc(&m->d_v, sizeof(float) * m->P);
    if (e == hipSuccess) e = hipMalloc(&m->d_wb, sizeof(uint16_t) * m->wb_total);
    if (e == hipSuccess && m->fused) e = hipMalloc(&m->d_wf, sizeof(uint16_t) * std::max<int64_t>(foff, 1));
    if (e == hipSuccess) e = hipMalloc(&m->d_wf_off, sizeof(int64_t) * (depth + 1));
    if (e == hipSuccess) e = hipMalloc(&m->d_b_off, sizeof(int64_t) * (depth + 1));
    if (e == hipSuccess)
        e = hipMemcpy(m->d_wf_off, m->wf_off.data(), sizeof(int64_t) * (depth + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(m->d_b_off, m->b_off.data(), sizeof(int64_t) * (depth + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d_p, h.data(), sizeof(float) * m->P, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->d_g, 0, sizeof(float) * m->P);
    if (e == hipSuccess) e = hipMemset(m->d_m, 0, sizeof(float) * m->P);
    if (e == hipSuccess) e = hipMemset(m->d_v, 0, sizeof(float) * m->P);
    if (e != hipSuccess) {
        srp_mlp_destroy(m);
        return srp_fail(SRP_EDEVICE, std::string("MLP buffers: ") + hipGetErrorString(e));
    }
    srp_status st = repack(m, nullptr);
    if (st == SRP_OK && hipDeviceSynchronize() != hipSuccess) st = srp_fail(SRP_EDEVICE, "MLP init failed");
    if (st != SRP_OK) {
        srp_mlp_destroy(m);
        return st;
    }
    *out = m;
    return SRP_OK;
}

srp_status srp_mlp_num_params(srp_mlp m, int64_t* n)
{
    if (!m || !n) return srp_fail(SRP_EINVAL, "NULL argument");
    *n = m->P;
    return SRP_OK;
}

srp_status srp_mlp_forward(srp_mlp m, const float* x, int64_t N, float* y, int32_t keep_activations, void* stream_)
{
    if (!m) return srp_fail(SRP_EINVAL, "mlp is NULL");
    if (N < 0) return srp_fail(SRP_EINVAL, "N must be >= 0");
    if (N == 0) return SRP_OK;
    if (!x || !y) return srp_fail(SRP_EINVAL, "x and y are required");
    if (N > (int64_t(1) << 30)) return srp_fail(SRP_EINVAL, "N exceeds 2^30");
    srp_status st = bind(m);
    if (st != SRP_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const bool training = keep_activations != 0;
    if (!training && m->fused) {
        st = refresh_fused(m, stream);
        if (st != SRP_OK) return st;
        MLP_HIP(srp::launch_mlp_infer(x, static_cast<int32_t>(N), m->d_wf, m->d_wf_off, m->d_p, m->d_b_off, m->n_in,
                                      m->depth, m->n_out, y, stream));
        m->cached_N = -1;
        return SRP_OK;
    }
    st = ensure_ws(m, N, training);
    if (st != SRP_OK) return st;
    const int N32 = static_cast<int>(N);
    MLP_HIP(srp::launch_to_bf16(x, N, m->n_in, m->n_in, m->d_xb, m->fin_pad[0], stream));
    const uint16_t* prev = m->d_xb;
    int prev_ld = m->fin_pad[0];
    for (int l = 0; l < m->depth; ++l) {
        uint16_t* act = training ? m->d_A + static_cast<int64_t>(l) * N * m->width
                                 : m->d_A + static_cast<int64_t>(l & 1) * N * m->width;
        srp::GemmArgs g{};
        g.A = prev;
        g.lda = prev_ld;
        g.B = m->d_wb + m->wb_off[l];
        g.ldb = m->fin_pad[l];
        g.M = N32;
        g.N = m->width;
        g.K = m->fin_pad[l];
        g.epi = srp::kEpiHidden;
        g.bias = m->d_p + m->b_off[l];
        g.C = training ? m->d_Z + static_cast<int64_t>(l) * N * m->width : nullptr;
        g.ldc = m->width;
        g.Cb = act;
        g.ldcb = m->width;
        MLP_HIP(srp::launch_gemm(g, false, true, stream));
        prev = act;
        prev_ld = m->width;
    }
    srp::GemmArgs g{};
    g.A = prev;
    g.lda = prev_ld;
    g.B = m->d_wb + m->wb_off[m->depth];
    g.ldb = m->fin_pad[m->depth];
    g.M = N32;
    g.N = m->n_out;
    g.K = m->width;
    g.epi = srp::kEpiStore;
    g.bias = m->d_p + m->b_off[m->depth];
    g.C = y;
    g.ldc = m->n_out;
    MLP_HIP(srp::launch_gemm(g, false, true, stream));
    m->cached_N = training ? N : -1;
    return SRP_OK;
}

srp_status srp_mlp_ensemble(srp_mlp a, srp_mlp b, const float* x, int64_t N, float threshold, float out_scale,
                            float* y, float* disagree, int32_t* fail_idx, int32_t* n_fail, void* stream_)
{
    if (!a || !b) return srp_fail(SRP_EINVAL, "both networks are required");
    if (a->n_in != b->n_in || a->n_out != b->n_out || a->device != b->device)
        return srp_fail(SRP_EINVAL, "the two networks must have the same inputs, outputs and device");
    if (a->n_in < 3) return srp_fail(SRP_EINVAL, "the inputs must start with the sun unit vector (n_in >= 3)");
    if (N < 0 || N > (int64_t(1) << 30)) return srp_fail(SRP_EINVAL, "N must be in 0..2^30");
    if (!n_fail) return srp_fail(SRP_EINVAL, "n_fail is required");
    if (N > 0 && (!x || !y || !fail_idx)) return srp_fail(SRP_EINVAL, "x, y and fail_idx are required");
    srp_status st = bind(a);
    if (st != SRP_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if (N == 0) {
        MLP_HIP(hipMemsetAsync(n_fail, 0, sizeof(int32_t), stream));
        return SRP_OK;
    }
    const size_t out_bytes = (static_cast<size_t>(N) * a->n_out * sizeof(float) + 255) / 256 * 256;
    const size_t flag_bytes = (static_cast<size_t>(N) + 255) / 256 * 256;
    const size_t tmp_bytes = srp::ensemble_select_bytes(N);
    MLP_HIP(grow(a->d_ens, a->cap_ens, 2 * out_bytes + flag_bytes + tmp_bytes));
    float* ya = reinterpret_cast<float*>(a->d_ens);
    float* yb = reinterpret_cast<float*>(a->d_ens + out_bytes);
    uint8_t* flag = reinterpret_cast<uint8_t*>(a->d_ens + 2 * out_bytes);
    void* tmp = a->d_ens + 2 * out_bytes + flag_bytes;
    st = srp_mlp_forward(a, x, N, ya, 0, stream_);
    if (st != SRP_OK) return st;
    st = srp_mlp_forward(b, x, N, yb, 0, stream_);
    if (st != SRP_OK) return st;
    MLP_HIP(srp::launch_ensemble(x, a->n_in, ya, yb, a->n_out, N, threshold, out_scale, y, disagree, flag, tmp,
                                 tmp_bytes, fail_idx, n_fail, stream));
    return SRP_OK;
}

srp_status srp_mlp_backward(srp_mlp m, const float* g_y, int64_t N, float* g_x, void* stream_)
{
    if (!m || !g_y) return srp_fail(SRP_EINVAL, "mlp and g_y are required");
    if (N != m->cached_N) return srp_fail(SRP_EINVAL, "backward needs a forward with keep_activations on the same N");
    srp_status st = bind(m);
    if (st != SRP_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const int N32 = static_cast<int>(N);
    const int64_t wmax = std::max(m->width, round8(m->n_out));
    uint16_t* gb[2] = {m->d_Gb, m->d_Gb + N * wmax};
    int cur = 0;
    // split-batch partials of every layer's weight and bias gradients, summed at the end
    srp::ReduceArgs red{};
    red.layers = m->depth + 1;
    int64_t part_total = 0, bpart_total = 0, total = 0;
    int kc[srp::kMaxLayers];
    for (int l = 0; l <= m->depth; ++l) {
        const int S = wgrad_splits(m->fout[l], m->fin[l], N, &kc[l]);
        red.first[l] = total;
        red.fin[l] = m->fin[l];
        red.fout[l] = m->fout[l];
        red.splits[l] = S;
        red.w_off[l] = m->w_off[l];
        red.b_off[l] = m->b_off[l];
        red.part_off[l] = part_total;
        red.bpart_off[l] = bpart_total;
        part_total += static_cast<int64_t>(S) * m->fout[l] * m->fin[l];
        bpart_total += static_cast<int64_t>(S) * m->fout[l];
        total += static_cast<int64_t>(m->fout[l]) * m->fin[l] + m->fout[l];
    }
    red.total = total;
    MLP_HIP(grow(m->d_wpart, m->cap_wpart, static_cast<size_t>(part_total)));
    MLP_HIP(grow(m->d_bpart, m->cap_bpart, static_cast<size_t>(bpart_total)));
    red.part = m->d_wpart;
    red.bpart = m->d_bpart;
    red.grad = m->d_g;
    // output layer: dL/dz = g_y (FP32) and its BF16 copy
    MLP_HIP(srp::launch_to_bf16(g_y, N, m->n_out, m->n_out, gb[cur], m->fout_pad[m->depth], stream));
    for (int l = m->depth; l >= 0; --l) {
        const uint16_t* in = l == 0 ? m->d_xb : m->d_A + static_cast<int64_t>(l - 1) * N * m->width;
        const int in_ld = l == 0 ? m->fin_pad[0] : m->width;
        const int g_ld = m->fout_pad[l];
        // weight gradient dW_l[o][i] = sum_n dL/dz[n][o] a_{l-1}[n][i] and bias gradient sum_n dL/dz[n][o]
        srp::WgradArgs w{};
        w.G = gb[cur];
        w.ldg = g_ld;
        w.A = in;
        w.lda = in_ld;
        w.Gf = l == m->depth ? g_y : m->d_G;
        w.ldgf = l == m->depth ? m->n_out : m->width;
        w.M = m->fout[l];
        w.N = m->fin[l];
        w.K = N32;
        w.kc = kc[l];
        w.part = m->d_wpart + red.part_off[l];
        w.bpart = m->d_bpart + red.bpart_off[l];
        MLP_HIP(srp::launch_wgrad(w, red.splits[l], stream));
        if (l == 0 && !g_x) break;
        // input gradient of the layer: dL/da_{l-1} = dL/dz_l . W_l, times SiLU'(z_{l-1}) below layer 0
        srp::GemmArgs d{};
        d.A = gb[cur];
        d.lda = g_ld;
        d.B = m->d_wb + m->wb_off[l];
        d.ldb = m->fin_pad[l];
        d.M = N32;
        d.K = g_ld;
        if (l > 0) {
            d.N = m->width;
            d.epi = srp::kEpiBackprop;
            d.Z = m->d_Z + static_cast<int64_t>(l - 1) * N * m->width;
            d.ldz = m->width;
            d.C = m->d_G;
            d.ldc = m->width;
            d.Cb = gb[cur ^ 1];
            d.ldcb = m->width;
            MLP_HIP(srp::launch_gemm(d, false, false, stream));
            cur ^= 1;
        } else {
            d.N = m->n_in;
            d.epi = srp::kEpiStore;
            d.C = g_x;
            d.ldc = m->n_in;
            MLP_HIP(srp::launch_gemm(d, false, false, stream));
        }
    }
    MLP_HIP(srp::launch_wgrad_reduce(red, stream));
    return SRP_OK;
}

srp_status srp_mlp_adam_step(srp_mlp m, float lr, float b1, float b2, float eps, void* stream_)
{
    if (!m) return srp_fail(SRP_EINVAL, "mlp is NULL");
    if (!(lr >= 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
        return srp_fail(SRP_EINVAL, "bad Adam hyper-parameters");
    srp_status st = bind(m);
    if (st != SRP_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    m->step += 1;
    srp::AdamPackArgs a{};
    a.p = m->d_p;
    a.g = m->d_g;
    a.m = m->d_m;
    a.v = m->d_v;
    a.P = m->P;
    a.lr = lr;
    a.b1 = b1;
    a.b2 = b2;
    a.eps = eps;
    a.c1 = static_cast<float>(1.0 - std::pow(static_cast<double>(b1), static_cast<double>(m->step)));
    a.c2 = static_cast<float>(1.0 - std::pow(static_cast<double>(b2), static_cast<double>(m->step)));
    a.layers = m->depth + 1;
    for (int l = 0; l <= m->depth; ++l) {
        a.w_off[l] = m->w_off[l];
        a.wb_off[l] = m->wb_off[l];
        a.fin[l] = m->fin[l];
        a.fout[l] = m->fout[l];
        a.fin_pad[l] = m->fin_pad[l];
    }
    a.wb = m->d_wb;
    MLP_HIP(srp::launch_adam_pack(a, stream));
    m->wf_stale = true;
    return SRP_OK;
}

srp_status srp_mlp_zero_grad(srp_mlp m, void* stream)
{
    if (!m) return srp_fail(SRP_EINVAL, "mlp is NULL");
    srp_status st = bind(m);
    if (st != SRP_OK) return st;
    MLP_HIP(srp::launch_fill_f32(m->d_g, m->P, 0.0f, static_cast<hipStream_t>(stream)));
    return SRP_OK;
}

srp_status srp_mlp_get_params(srp_mlp m, float* params, float* grads, float* adam_m, float* adam_v, int64_t* step,
                              int64_t n)
{
    if (!m) return srp_fail(SRP_EINVAL, "mlp is NULL");
    if (n != m->P) return srp_fail(SRP_EINVAL, "n must equal the parameter count");
    srp_status st = bind(m);
    if (st != SRP_OK) return st;
    MLP_HIP(hipDeviceSynchronize());
    if (params) MLP_HIP(hipMemcpy(params, m->d_p, sizeof(float) * n, hipMemcpyDeviceToHost));
    if (grads) MLP_HIP(hipMemcpy(grads, m->d_g, sizeof(float) * n, hipMemcpyDeviceToHost));
    if (adam_m) MLP_HIP(hipMemcpy(adam_m, m->d_m, sizeof(float) * n, hipMemcpyDeviceToHost));
    if (adam_v) MLP_HIP(hipMemcpy(adam_v, m->d_v, sizeof(float) * n, hipMemcpyDeviceToHost));
    if (step) *step = m->step;
    return SRP_OK;
}

srp_status srp_mlp_set_params(srp_mlp m, const float* params, const float* adam_m, const float* adam_v, int64_t step,
                              int64_t n)
{
    if (!m) return srp_fail(SRP_EINVAL, "mlp is NULL");
    if (n != m->P) return srp_fail(SRP_EINVAL, "n must equal the parameter count");
    if (step < 0) return srp_fail(SRP_EINVAL, "step must be >= 0");
    srp_status st = bind(m);
    if (st != SRP_OK) return st;
    MLP_HIP(hipDeviceSynchronize());
    if (params) MLP_HIP(hipMemcpy(m->d_p, params, sizeof(float) * n, hipMemcpyHostToDevice));
    if (adam_m) MLP_HIP(hipMemcpy(m->d_m, adam_m, sizeof(float) * n, hipMemcpyHostToDevice));
    if (adam_v) MLP_HIP(hipMemcpy(m->d_v, adam_v, sizeof(float) * n, hipMemcpyHostToDevice));
    m->step = step;
    MLP_HIP(hipMemset(m->d_g, 0, sizeof(float) * n));
    st = repack(m, nullptr);
    if (st != SRP_OK) return st;
    MLP_HIP(hipDeviceSynchronize());
    return SRP_OK;
}

srp_status srp_mlp_mse(srp_mlp m, const float* y, const float* target, int64_t N, float* g_y, double* loss,
                       void* stream_)
{
    if (!m) return srp_fail(SRP_EINVAL, "mlp is NULL");
    if (N < 0 || (N > 0 && (!y || !target || !g_y || !loss))) return srp_fail(SRP_EINVAL, "bad argument");
    if (N == 0) return SRP_OK;
    srp_status st = bind(m);
    if (st != SRP_OK) return st;
    const int64_t count = N * m->n_out;
    MLP_HIP(grow(m->d_lpart, m->cap_lp, static_cast<size_t>((count + 255) / 256)));
    MLP_HIP(srp::launch_mse(y, target, count, g_y, m->d_lpart, loss, static_cast<hipStream_t>(stream_)));
    return SRP_OK;
}

}  // extern "C"

namespace srp {

void mlp_shape(const srp_mlp_s* m, int* n_in, int* n_out, int* device)
{
    *n_in = m->n_in;
    *n_out = m->n_out;
    *device = m->device;
}

hipError_t mlp_aux(srp_mlp_s* m, size_t bytes, void** out)
{
    hipError_t e = grow(m->d_aux, m->cap_aux, bytes);
    *out = m->d_aux;
    return e;
}

}  // namespace srp

extern "C" {

srp_status srp_mlp_destroy(srp_mlp m)
{
    if (!m) return SRP_OK;
    (void)hipSetDevice(m->device);
    for (void* p : {static_cast<void*>(m->d_p), static_cast<void*>(m->d_g), static_cast<void*>(m->d_m),
                    static_cast<void*>(m->d_v), static_cast<void*>(m->d_wb), static_cast<void*>(m->d_xb),
                    static_cast<void*>(m->d_Z), static_cast<void*>(m->d_A), static_cast<void*>(m->d_G),
                    static_cast<void*>(m->d_Gb), static_cast<void*>(m->d_lpart),
                    static_cast<void*>(m->d_wf), static_cast<void*>(m->d_wf_off), static_cast<void*>(m->d_b_off),
                    static_cast<void*>(m->d_aux), static_cast<void*>(m->d_ens), static_cast<void*>(m->d_wpart),
                    static_cast<void*>(m->d_bpart)})
        if (p) (void)hipFree(p);
    delete m;
    return SRP_OK;
}

}  // extern "C"
