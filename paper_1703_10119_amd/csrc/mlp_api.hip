// mlp_api.hip -- host side of the surface-flux surrogate (dfhm_mlp_* in
// include/dfhm.h).  Device memory: FP32 master weights, BF16 copies, AdamW
// moments, gradients, activations (BF16) and pre-activations (BF16) of every
// layer for the largest batch, split-K partials; and one file-scope device
// array, the scratch of the allocation-free inference call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "../../include/dfhm.h"
#include "mlp.hpp"

using namespace dfhm;

// rows per partial of the bias-gradient column sums
constexpr int kColsumRows = 256;

namespace {
constexpr int kOutPad = 32;   // output layer rows padded for the GEMM tiles

struct Layer {
    int K, N, Np;             // inputs, logical outputs, padded outputs
    size_t w_off, b_off;      // offsets into the flat FP32 parameter buffer
    size_t wb_off;            // offset of the BF16 weight operand [Np][K]
    size_t ws_off;            // offset of the same in fragment order (k_pack_swizzled)
};

// Scratch of dfhm_mlp_infer_noalloc: two hidden-activation buffers used in
// turn and the padded output layer, for at most kScratchBytes.  Every GPU the
// library runs on holds its own copy until the process ends.  Host code never
// uses the name `scratch` as an address: its device address is looked up once
// per device (hipGetSymbolAddress, with that device current) and kept in
// g_scratch.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) uint8_t scratch[kScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (the current device); nullptr
// and a message on failure.
void *scratch_on(int dev, std::string &msg)
{
    if (dev < 0 || dev >= kMaxDevices) { msg = "device index beyond the scratch table"; return nullptr; }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}
} // namespace

struct dfhm_mlp {
    dfhm_mlp_config cfg{};
    hipStream_t stream = nullptr;
    std::vector<Layer> layers;
    int64_t n_params = 0;      // logical parameters (exposed)
    int64_t n_dev = 0;         // device parameters (with padding)
    int64_t n_wb = 0;          // BF16 weight operands
    int64_t n_ws = 0;          // BF16 weight operands in fragment order
    int device = 0;            // device the network lives on
    void *scratch = nullptr;   // that device's address of `scratch` (nullptr: not available)
    std::string scratch_msg;   // why it is not
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    uint16_t *wb = nullptr;
    uint16_t *ws = nullptr;    // fragment-order copies (inference kernel)
    uint8_t *mask = nullptr;
    std::vector<uint16_t *> act;   // act[0] = input (caller's), act[l+1] = output of layer l [B][N]
    std::vector<uint16_t *> pre;   // pre-activations of hidden layers
    std::vector<uint16_t *> dact;  // gradients w.r.t. layer outputs (BF16)
    float *out = nullptr;          // output layer result [B][kOutPad] FP32
    float *part = nullptr;         // split-K partials / column sums
    size_t part_n = 0;
    float *loss_part = nullptr;
    int64_t step = 0;
    std::vector<void *> allocs;
    std::string err;
};

namespace {

dfhm_status mfail(dfhm_mlp *m, dfhm_status s, const std::string &msg)
{
    if (m) m->err = msg;
    return s;
}

#define MHIP(mm, call)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return mfail((mm), DFHM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// elements of a layer's fragment-order copy: ceil(Np / 16) x ceil(K / 32) tiles of 512
int64_t swizzled_size(const Layer &ly) { return (int64_t)((ly.Np + 15) / 16) * ((ly.K + 31) / 32) * 512; }

template <typename T>
dfhm_status dalloc(dfhm_mlp *m, T **p, size_t n)
{
    void *q = nullptr;
    if (hipMalloc(&q, sizeof(T) * (n ? n : 1)) != hipSuccess) return mfail(m, DFHM_E_NOMEM, "mlp buffers");
    m->allocs.push_back(q);
    *p = (T *)q;
    return DFHM_OK;
}

template <int LA, int LB, int EPI>
void gemm(dfhm_mlp *m, int M, int N, int K, const uint16_t *A, int lda, const uint16_t *B, int ldb,
          float *Cf, uint16_t *Cb, int ldc, const float *bias, const uint16_t *aux, uint16_t *pre,
          int nsplit)
{
    const int kchunk = ((K + nsplit - 1) / nsplit + GB_K - 1) / GB_K * GB_K;
    dim3 grid((N + GB_N - 1) / GB_N, (M + GB_M - 1) / GB_M, nsplit);
    hipLaunchKernelGGL((k_gemm_bf16<LA, LB, EPI>), grid, dim3(256), 0, m->stream, M, N, K, A, lda,
                       B, ldb, Cf, Cb, ldc, bias, aux, pre, kchunk);
}

int blocks_of(int64_t n, int t) { return (int)((n + t - 1) / t); }

// Forward pass over `batch` rows: layer l reads in(l) and writes its GELU
// output to out(l) (hidden layers; pre-activations to pre(l) when it is not
// null), the output layer writes y [batch][kOutPad] (FP32).
template <typename In, typename Out, typename Pre>
void forward_into(dfhm_mlp *m, int batch, In in, Out out, Pre pre, float *y)
{
    const int L = (int)m->layers.size();
    for (int l = 0; l < L; ++l) {
        const Layer &ly = m->layers[l];
        const uint16_t *W = m->wb + ly.wb_off;
        const float *b = m->w + ly.b_off;
        if (l < L - 1)
            gemm<OP_K, OP_K, EPI_BIAS_GELU>(m, batch, ly.N, ly.K, in(l), ly.K, W, ly.K, nullptr,
                                            out(l), ly.N, b, nullptr, pre(l), 1);
        else
            gemm<OP_K, OP_K, EPI_BIAS_F32>(m, batch, ly.Np, ly.K, in(l), ly.K, W, ly.K, y,
                                           nullptr, ly.Np, b, nullptr, nullptr, 1);
    }
}

// Whether the fused inference kernel covers this network: width a multiple
// of 128 up to 512 (8 waves x width / 8 columns), outputs within two tiles.
bool fused_ok(const dfhm_mlp *m)
{
    const int w = m->cfg.width;
    return w % 128 == 0 && w <= 512 && m->cfg.n_out <= 32;
}

template <int NJ>
void launch_fused(dfhm_mlp *m, const FusedNet &net, const uint16_t *x, int64_t batch, float *y)
{
    // above the default 64 KB of LDS; set on every call, so that every
    // device the library runs on and every thread sees it
    (void)hipFuncSetAttribute((const void *)k_mlp_infer_fused<NJ>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)fused_lds_bytes<NJ>());
    hipLaunchKernelGGL(k_mlp_infer_fused<NJ>, dim3((unsigned)((batch + FI_M - 1) / FI_M)),
                       dim3(64 * FI_NW), fused_lds_bytes<NJ>(), m->stream, net, x, m->cfg.n_in, batch,
                       y, kOutPad);
}

// Forward pass of inference in one launch (fused_ok): outputs y [batch][kOutPad]
// FP32 (the first 16 or 32 columns written).
void forward_fused(dfhm_mlp *m, const uint16_t *x, int64_t batch, float *y)
{
    FusedNet net{};
    const int L = (int)m->layers.size();
    const Layer &l0 = m->layers[0], &lo = m->layers[L - 1];
    net.W0 = m->ws + l0.ws_off;
    net.b0 = m->w + l0.b_off;
    net.Wo = m->ws + lo.ws_off;
    net.bo = m->w + lo.b_off;
    if (L > 2) {
        // hidden layers are equal in size, so they sit at a fixed stride
        net.Wh = m->ws + m->layers[1].ws_off;
        net.bh = m->w + m->layers[1].b_off;
        net.wh_stride = L > 3 ? (int64_t)(m->layers[2].ws_off - m->layers[1].ws_off) : 0;
        net.bh_stride = L > 3 ? (int64_t)(m->layers[2].b_off - m->layers[1].b_off) : 0;
    }
    net.depth = L - 1;
    net.n_in = m->cfg.n_in;
    net.n_outp = (m->cfg.n_out + 15) / 16 * 16;
    switch (m->cfg.width / 128) {
    case 1: launch_fused<1>(m, net, x, batch, y); break;
    case 2: launch_fused<2>(m, net, x, batch, y); break;
    case 3: launch_fused<3>(m, net, x, batch, y); break;
    default: launch_fused<4>(m, net, x, batch, y); break;
    }
}

// Forward pass through the network's own buffers (activations and
// pre-activations kept for the backward pass); output layer in m->out.
void forward(dfhm_mlp *m, const uint16_t *x, int batch)
{
    m->act[0] = const_cast<uint16_t *>(x);
    forward_into(m, batch, [m](int l) { return (const uint16_t *)m->act[l]; },
                 [m](int l) { return m->act[l + 1]; }, [m](int l) { return m->pre[l]; }, m->out);
}

// Backward pass from dact[L-1] (= dL/dz of the output layer, BF16 [B][Np])
// into m->g (FP32, device layout).
void backward(dfhm_mlp *m, int batch)
{
    const int L = (int)m->layers.size();
    for (int l = L - 1; l >= 0; --l) {
        const Layer &ly = m->layers[l];
        const int Nl = l == L - 1 ? ly.Np : ly.N;
        const uint16_t *dz = m->dact[l];
        // weight gradient dW[N][K] = dz^T [N][B] . act[l] [B][K] (the hi half of a pair),
        // split over the batch
        int nsplit = std::max(1, std::min(16, batch / 512));
        gemm<OP_MN, OP_MN, EPI_F32>(m, Nl, ly.K, batch, dz, Nl, m->act[l], ly.K, m->part, nullptr,
                                    ly.K, nullptr, nullptr, nullptr, nsplit);
        const int64_t nw = (int64_t)Nl * ly.K;
        hipLaunchKernelGGL(k_sum_partials, dim3(blocks_of(nw, 256)), dim3(256), 0, m->stream,
                           m->part, nsplit, nw, m->g + ly.w_off);
        // bias gradient: column sums of dz
        const int rchunk = kColsumRows;
        const int nrc = (batch + rchunk - 1) / rchunk;
        float *cs = m->part + (size_t)nsplit * nw;
        hipLaunchKernelGGL(k_colsum_bf16, dim3(blocks_of(Nl, 512), nrc), dim3(256), 0, m->stream, dz,
                           batch, Nl, rchunk, cs);
        hipLaunchKernelGGL(k_sum_partials, dim3(blocks_of(Nl, 256)), dim3(256), 0, m->stream, cs,
                           nrc, (int64_t)Nl, m->g + ly.b_off);
        // the log-variance outputs train the output layer only
        if (l == L - 1 && l > 0) {
            const int F = m->cfg.n_out / 2;
            hipLaunchKernelGGL(k_zero_cols, dim3(blocks_of((int64_t)batch * F, 256)), dim3(256), 0,
                               m->stream, m->dact[l], batch, Nl, F, 2 * F);
        }
        // input gradient through the previous GELU: dz_{l-1} = (dz . W) * gelu'(pre_{l-1})
        if (l > 0) {
            const uint16_t *W = m->wb + ly.wb_off;
            gemm<OP_K, OP_MN, EPI_GELU_BWD>(m, batch, ly.K, Nl, dz, Nl, W, ly.K, nullptr,
                                            m->dact[l - 1], ly.K, nullptr, m->pre[l - 1], nullptr, 1);
        }
    }
}

dfhm_status loss_and_grad(dfhm_mlp *m, const uint16_t *x, const float *y, int batch, float *loss)
{
    forward(m, x, batch);
    const int L = (int)m->layers.size();
    const int nb = blocks_of(batch, 256);
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, m->stream, m->out, kOutPad, y, batch,
                       m->cfg.n_out / 2, m->dact[L - 1], m->loss_part);
    backward(m, batch);
    MHIP(m, hipGetLastError());
    if (loss) {
        std::vector<float> p(nb);
        MHIP(m, hipMemcpyAsync(p.data(), m->loss_part, sizeof(float) * nb, hipMemcpyDeviceToHost, m->stream));
        MHIP(m, hipStreamSynchronize(m->stream));
        double s = 0;
        for (float q : p) s += q;
        *loss = (float)(s / batch);
    }
    return DFHM_OK;
}

// logical <-> device parameter layout (the output layer is padded)
void to_logical(const dfhm_mlp *m, const std::vector<float> &dev, float *out)
{
    size_t o = 0;
    for (const Layer &ly : m->layers) {
        for (int n = 0; n < ly.N; ++n)
            for (int k = 0; k < ly.K; ++k) out[o++] = dev[ly.w_off + (size_t)n * ly.K + k];
        for (int n = 0; n < ly.N; ++n) out[o++] = dev[ly.b_off + n];
    }
}
void to_device(const dfhm_mlp *m, const float *in, std::vector<float> &dev)
{
    std::fill(dev.begin(), dev.end(), 0.f);
    size_t o = 0;
    for (const Layer &ly : m->layers) {
        for (int n = 0; n < ly.N; ++n)
            for (int k = 0; k < ly.K; ++k) dev[ly.w_off + (size_t)n * ly.K + k] = in[o++];
        for (int n = 0; n < ly.N; ++n) dev[ly.b_off + n] = in[o++];
    }
}

// BF16 weight operands from the FP32 master weights
void pack_weights(dfhm_mlp *m)
{
    for (const Layer &ly : m->layers)
    {
        hipLaunchKernelGGL(k_pack_weights, dim3(blocks_of((int64_t)ly.Np * ly.K, 256)), dim3(256), 0,
                           m->stream, m->w + ly.w_off, m->wb + ly.wb_off, ly.Np, ly.K, ly.K);
        if (m->ws)
            hipLaunchKernelGGL(k_pack_swizzled, dim3(blocks_of(swizzled_size(ly), 256)),
                               dim3(256), 0, m->stream, m->w + ly.w_off, m->ws + ly.ws_off, ly.Np, ly.K);
    }
}

dfhm_status upload(dfhm_mlp *m, const std::vector<float> &dev)
{
    MHIP(m, hipMemcpyAsync(m->w, dev.data(), sizeof(float) * dev.size(), hipMemcpyHostToDevice, m->stream));
    pack_weights(m);
    MHIP(m, hipGetLastError());
    MHIP(m, hipStreamSynchronize(m->stream));
    return DFHM_OK;
}

} // namespace

extern "C" {

dfhm_status dfhm_mlp_create(const dfhm_mlp_config *cfg, dfhm_mlp **out)
{
    if (!out) return DFHM_E_INVAL;
    *out = nullptr;
    if (!cfg || cfg->n_in < 8 || cfg->n_in % 8 || cfg->width < 8 || cfg->width % 8 ||
        cfg->depth < 1 || cfg->depth > 16 || cfg->n_out < 1 || cfg->n_out > kOutPad ||
        cfg->max_batch < 1 || cfg->max_batch > (1 << 22))
        return DFHM_E_INVAL;
    dfhm_mlp *m = new (std::nothrow) dfhm_mlp();
    if (!m) return DFHM_E_NOMEM;
    m->cfg = *cfg;
    m->stream = (hipStream_t)cfg->stream;
    if (hipGetDevice(&m->device) != hipSuccess) { delete m; return DFHM_E_DEVICE; }
    m->scratch = scratch_on(m->device, m->scratch_msg);
    size_t o = 0, ob = 0, os = 0;
    int K = cfg->n_in;
    for (int l = 0; l <= cfg->depth; ++l) {
        Layer ly;
        ly.K = K;
        ly.N = l < cfg->depth ? cfg->width : cfg->n_out;
        ly.Np = l < cfg->depth ? ly.N : kOutPad;
        ly.w_off = o; o += (size_t)ly.Np * ly.K;
        ly.b_off = o; o += (size_t)ly.Np;
        ly.wb_off = ob; ob += (size_t)ly.Np * ly.K;
        ly.ws_off = os; os += (size_t)swizzled_size(ly);
        m->n_params += (int64_t)ly.N * ly.K + ly.N;
        m->layers.push_back(ly);
        K = ly.N;
    }
    m->n_dev = (int64_t)o;
    m->n_wb = (int64_t)ob;
    m->n_ws = (int64_t)os;
    const int B = cfg->max_batch, L = (int)m->layers.size();
    auto bail = [&](dfhm_status s) { dfhm_mlp_destroy(m); return s; };
    if (dalloc(m, &m->w, o) || dalloc(m, &m->m, o) || dalloc(m, &m->v, o) || dalloc(m, &m->g, o) ||
        dalloc(m, &m->wb, ob) || dalloc(m, &m->ws, os) || dalloc(m, &m->mask, o) || dalloc(m, &m->out, (size_t)B * kOutPad) ||
        dalloc(m, &m->loss_part, (size_t)(B + 255) / 256))
        return bail(DFHM_E_NOMEM);
    m->act.assign(L + 1, nullptr);
    m->pre.assign(L, nullptr);
    m->dact.assign(L, nullptr);
    size_t maxw = 0;
    for (int l = 0; l < L; ++l) {
        const Layer &ly = m->layers[l];
        const int Nl = l == L - 1 ? ly.Np : ly.N;
        if (l < L - 1) {
            if (dalloc(m, &m->act[l + 1], (size_t)B * ly.N) ||
                dalloc(m, &m->pre[l], (size_t)B * ly.N))
                return bail(DFHM_E_NOMEM);
        }
        if (dalloc(m, &m->dact[l], (size_t)B * Nl)) return bail(DFHM_E_NOMEM);
        maxw = std::max(maxw, (size_t)Nl * ly.K);
    }
    const size_t maxn = (size_t)std::max(cfg->width, kOutPad);
    m->part_n = 16 * maxw + (size_t)((B + kColsumRows - 1) / kColsumRows) * maxn + 1024;
    if (dalloc(m, &m->part, m->part_n)) return bail(DFHM_E_NOMEM);
    // He-style initialisation from the seed; biases zero; padding rows zero
    std::mt19937_64 rng(cfg->seed);
    std::vector<float> dev(o, 0.f);
    std::vector<uint8_t> mask(o, 0);
    for (int l = 0; l < L; ++l) {
        const Layer &ly = m->layers[l];
        std::normal_distribution<double> nd(0.0, std::sqrt((l < L - 1 ? 2.0 : 1.0) / ly.K));
        for (int n = 0; n < ly.N; ++n) {
            for (int k = 0; k < ly.K; ++k) {
                dev[ly.w_off + (size_t)n * ly.K + k] = (float)nd(rng);
                mask[ly.w_off + (size_t)n * ly.K + k] = 1;
            }
            mask[ly.b_off + n] = 1;
        }
    }
    if (hipMemsetAsync(m->m, 0, sizeof(float) * o, m->stream) != hipSuccess ||
        hipMemsetAsync(m->v, 0, sizeof(float) * o, m->stream) != hipSuccess ||
        hipMemsetAsync(m->g, 0, sizeof(float) * o, m->stream) != hipSuccess ||
        hipMemcpyAsync(m->mask, mask.data(), o, hipMemcpyHostToDevice, m->stream) != hipSuccess)
        return bail(DFHM_E_DEVICE);
    if (upload(m, dev)) return bail(DFHM_E_DEVICE);
    *out = m;
    return DFHM_OK;
}

int64_t dfhm_mlp_param_count(const dfhm_mlp *m) { return m ? m->n_params : -1; }

dfhm_status dfhm_mlp_get_params(dfhm_mlp *m, float *host)
{
    if (!m || !host) return DFHM_E_INVAL;
    std::vector<float> dev(m->n_dev);
    MHIP(m, hipMemcpyAsync(dev.data(), m->w, sizeof(float) * m->n_dev, hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    to_logical(m, dev, host);
    return DFHM_OK;
}

dfhm_status dfhm_mlp_set_params(dfhm_mlp *m, const float *host)
{
    if (!m || !host) return DFHM_E_INVAL;
    for (int64_t i = 0; i < m->n_params; ++i)
        if (!std::isfinite(host[i])) return mfail(m, DFHM_E_INVAL, "non-finite parameter");
    std::vector<float> dev(m->n_dev);
    to_device(m, host, dev);
    return upload(m, dev);
}

dfhm_status dfhm_mlp_forward(dfhm_mlp *m, const uint16_t *x, int64_t batch, float *y)
{
    if (!m || !x || !y) return DFHM_E_INVAL;
    if (batch < 1 || batch > m->cfg.max_batch) return mfail(m, DFHM_E_INVAL, "batch out of range");
    forward(m, x, (int)batch);
    // compact the padded output rows into y[batch][n_out]
    MHIP(m, hipMemcpy2DAsync(y, sizeof(float) * m->cfg.n_out, m->out, sizeof(float) * kOutPad,
                             sizeof(float) * m->cfg.n_out, batch, hipMemcpyDeviceToDevice, m->stream));
    MHIP(m, hipGetLastError());
    return DFHM_OK;
}

dfhm_status dfhm_mlp_gradients(dfhm_mlp *m, const uint16_t *x, const float *y, int64_t batch,
                               float *grad_host, float *loss)
{
    if (!m || !x || !y || !grad_host) return DFHM_E_INVAL;
    if (m->cfg.n_out % 2) return mfail(m, DFHM_E_STATE, "the training loss needs an even n_out");
    if (batch < 1 || batch > m->cfg.max_batch) return mfail(m, DFHM_E_INVAL, "batch out of range");
    dfhm_status s = loss_and_grad(m, x, y, (int)batch, loss);
    if (s) return s;
    std::vector<float> dev(m->n_dev);
    MHIP(m, hipMemcpyAsync(dev.data(), m->g, sizeof(float) * m->n_dev, hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    to_logical(m, dev, grad_host);
    return DFHM_OK;
}

dfhm_status dfhm_mlp_train_step(dfhm_mlp *m, const uint16_t *x, const float *y, int64_t batch,
                                float lr, float *loss)
{
    if (!m || !x || !y) return DFHM_E_INVAL;
    if (m->cfg.n_out % 2) return mfail(m, DFHM_E_STATE, "the training loss needs an even n_out");
    if (batch < 1 || batch > m->cfg.max_batch || !(lr >= 0.f))
        return mfail(m, DFHM_E_INVAL, "batch or learning rate out of range");
    dfhm_status s = loss_and_grad(m, x, y, (int)batch, loss);
    if (s) return s;
    m->step += 1;
    const float b1 = m->cfg.beta1, b2 = m->cfg.beta2;
    const float c1 = 1.0f / (1.0f - std::pow(b1, (float)m->step));
    const float c2 = 1.0f / (1.0f - std::pow(b2, (float)m->step));
    hipLaunchKernelGGL(k_adamw, dim3(blocks_of(m->n_dev, 256)), dim3(256), 0, m->stream, m->w, m->m,
                       m->v, m->g, m->mask, m->n_dev, lr, b1, b2, m->cfg.eps,
                       m->cfg.weight_decay, c1, c2);
    pack_weights(m);
    MHIP(m, hipGetLastError());
    return DFHM_OK;
}

dfhm_status dfhm_mlp_features(const int32_t *wall_dev, const double *t_dev, const double *sines_dev,
                              const float *params_dev, int64_t nsamp, const dfhm_feature_desc *fd,
                              uint16_t *x_dev, void *stream)
{
    if (!wall_dev || !t_dev || !sines_dev || !params_dev || !fd || !x_dev || nsamp < 0)
        return DFHM_E_INVAL;
    if (fd->n_hist < 1 || fd->stride < 2 * fd->n_hist + 8 || fd->stride % 8 || !(fd->dt_hist > 0.f))
        return DFHM_E_INVAL;
    if (nsamp == 0) return DFHM_OK;
    FeatDesc d;
    d.n_hist = fd->n_hist;
    d.stride = fd->stride;
    d.dt_hist = fd->dt_hist;
    d.T_mean = fd->T_mean; d.T_scale = fd->T_scale;
    d.RH_mean = fd->RH_mean; d.RH_scale = fd->RH_scale;
    for (int i = 0; i < 8; ++i) { d.p_mean[i] = fd->p_mean[i]; d.p_scale[i] = fd->p_scale[i]; }
    hipLaunchKernelGGL(k_features, dim3((unsigned)nsamp), dim3(256), 0, (hipStream_t)stream, wall_dev,
                       t_dev, sines_dev, params_dev, (int)nsamp, d, x_dev);
    return hipGetLastError() == hipSuccess ? DFHM_OK : DFHM_E_DEVICE;
}

static dfhm_status decode_nets(const DecodeNets &nets, int64_t batch, const float *scale, float tau,
                               float *flux_dev, float *err_dev, uint8_t *fallback_dev, void *stream)
{
    if (!scale || !flux_dev || batch < 0 || !(tau > 0.f)) return DFHM_E_INVAL;
    for (int k = 0; k < nets.n; ++k)
        if (!nets.y[k]) return DFHM_E_INVAL;
    if (batch == 0) return DFHM_OK;
    DecodeScale sc;
    for (int i = 0; i < 4; ++i) {
        sc.m[i] = scale[2 * i];
        sc.s[i] = scale[2 * i + 1];
        if (!std::isfinite(sc.m[i]) || !(sc.s[i] > 0.f) || !std::isfinite(sc.s[i])) return DFHM_E_INVAL;
    }
    hipLaunchKernelGGL(k_decode, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, nets, batch, sc, tau, flux_dev, err_dev, fallback_dev);
    return hipGetLastError() == hipSuccess ? DFHM_OK : DFHM_E_DEVICE;
}

dfhm_status dfhm_mlp_decode(const float *y_dev, int64_t batch, const float *scale, float tau,
                            float *flux_dev, uint8_t *fallback_dev, void *stream)
{
    if (!fallback_dev) return DFHM_E_INVAL;
    DecodeNets nets{};
    nets.y[0] = y_dev;
    nets.n = 1;
    nets.ld = 8;
    return decode_nets(nets, batch, scale, tau, flux_dev, nullptr, fallback_dev, stream);
}

dfhm_status dfhm_mlp_decode_ensemble(const float *const *y_dev, int32_t n_nets, int64_t batch,
                                     const float *scale, float tau, float *flux_dev,
                                     uint8_t *fallback_dev, void *stream)
{
    if (!y_dev || !fallback_dev || n_nets < 1 || n_nets > kMaxEnsemble) return DFHM_E_INVAL;
    DecodeNets nets{};
    for (int k = 0; k < n_nets; ++k) nets.y[k] = y_dev[k];
    nets.n = n_nets;
    nets.ld = 8;
    return decode_nets(nets, batch, scale, tau, flux_dev, nullptr, fallback_dev, stream);
}

// Shared checks of the two inference calls.
static dfhm_status infer_args(dfhm_mlp *m, const uint16_t *x, int64_t batch, const float *scale,
                              const float *flux, const float *err)
{
    if (!m) return DFHM_E_INVAL;
    if (!x || !scale || !flux || !err) return mfail(m, DFHM_E_INVAL, "null argument");
    if (m->cfg.n_out != 8) return mfail(m, DFHM_E_STATE, "inference decodes the 8-output flux head");
    if (batch < 1) return mfail(m, DFHM_E_INVAL, "batch out of range");
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(scale[2 * i]) || !(scale[2 * i + 1] > 0.f) || !std::isfinite(scale[2 * i + 1]))
            return mfail(m, DFHM_E_INVAL, "bad output scale");
    return DFHM_OK;
}

static dfhm_status infer_decode(dfhm_mlp *m, const float *y, int64_t batch, const float *scale,
                                float *flux, float *err)
{
    DecodeNets nets{};
    nets.y[0] = y;
    nets.n = 1;
    nets.ld = kOutPad;
    dfhm_status st = decode_nets(nets, batch, scale, 1.0f, flux, err, nullptr, m->stream);
    if (st) return mfail(m, st, "decode launch failed");
    return DFHM_OK;
}

dfhm_status dfhm_mlp_infer(dfhm_mlp *m, const uint16_t *x_dev, int64_t batch, const float *scale,
                           float *flux_dev, float *err_est_dev)
{
    dfhm_status st = infer_args(m, x_dev, batch, scale, flux_dev, err_est_dev);
    if (st) return st;
    if (batch > m->cfg.max_batch) return mfail(m, DFHM_E_INVAL, "batch above max_batch");
    if (fused_ok(m)) forward_fused(m, x_dev, batch, m->out);
    else forward(m, x_dev, (int)batch);
    MHIP(m, hipGetLastError());
    return infer_decode(m, m->out, batch, scale, flux_dev, err_est_dev);
}

dfhm_status dfhm_mlp_infer_ensemble(dfhm_mlp *const *nets, int32_t n_nets, const uint16_t *x_dev,
                                    int64_t batch, const float *scale, float *flux_dev,
                                    float *err_est_dev)
{
    if (!nets || n_nets < 1 || n_nets > kMaxEnsemble || !nets[0]) return DFHM_E_INVAL;
    dfhm_mlp *m0 = nets[0];
    DecodeNets dn{};
    for (int k = 0; k < n_nets; ++k) {
        dfhm_mlp *m = nets[k];
        if (!m) return mfail(m0, DFHM_E_INVAL, "null ensemble member");
        dfhm_status st = infer_args(m, x_dev, batch, scale, flux_dev, err_est_dev);
        if (st) return mfail(m0, st, "member " + std::to_string(k) + ": " + m->err);
        if (batch > m->cfg.max_batch) return mfail(m0, DFHM_E_INVAL, "batch above a member's max_batch");
        if (m->cfg.n_in != m0->cfg.n_in || m->stream != m0->stream || m->device != m0->device)
            return mfail(m0, DFHM_E_INVAL, "ensemble members differ in inputs, stream or device");
    }
    for (int k = 0; k < n_nets; ++k) {
        dfhm_mlp *m = nets[k];
        if (fused_ok(m)) forward_fused(m, x_dev, batch, m->out);
        else forward(m, x_dev, (int)batch);
        MHIP(m0, hipGetLastError());
        dn.y[k] = m->out;
    }
    dn.n = n_nets;
    dn.ld = kOutPad;
    dfhm_status st = decode_nets(dn, batch, scale, 1.0f, flux_dev, err_est_dev, nullptr, m0->stream);
    if (st) return mfail(m0, st, "decode launch failed");
    return DFHM_OK;
}

int64_t dfhm_mlp_noalloc_max_batch(const dfhm_mlp *m)
{
    if (!m) return -1;
    // the fused kernel keeps the hidden activations on chip: only the outputs
    const size_t per_row = (fused_ok(m) ? 0 : 2 * (size_t)m->cfg.width * sizeof(uint16_t)) +
                           kOutPad * sizeof(float);
    return (int64_t)((kScratchBytes - 1024) / per_row);
}

dfhm_status dfhm_mlp_infer_noalloc(dfhm_mlp *m, const uint16_t *x_dev, int64_t batch,
                                   const float *scale, float *flux_dev, float *err_est_dev)
{
    dfhm_status st = infer_args(m, x_dev, batch, scale, flux_dev, err_est_dev);
    if (st) return st;
    if (batch > dfhm_mlp_noalloc_max_batch(m))
        return mfail(m, DFHM_E_INVAL, "batch above the allocation-free limit (" +
                                          std::to_string(dfhm_mlp_noalloc_max_batch(m)) + " rows)");
    if (!m->scratch) return mfail(m, DFHM_E_DEVICE, "scratch not available: " + m->scratch_msg);
    if (fused_ok(m)) {
        // the outputs only, at the start of the array; every element the
        // decode reads is written by this call's forward pass
        float *y = (float *)m->scratch;
        forward_fused(m, x_dev, batch, y);
        MHIP(m, hipGetLastError());
        return infer_decode(m, y, batch, scale, flux_dev, err_est_dev);
    }
    // [hidden A][hidden B][output], each 256-byte aligned; every element a
    // kernel reads was written earlier in this call, so nothing is cleared
    const size_t hid = ((size_t)batch * m->cfg.width * sizeof(uint16_t) + 255) / 256 * 256;
    uint8_t *base = (uint8_t *)m->scratch;
    uint16_t *h[2] = {(uint16_t *)base, (uint16_t *)(base + hid)};
    float *y = (float *)(base + 2 * hid);
    forward_into(m, (int)batch,
                 [&](int l) { return l == 0 ? x_dev : (const uint16_t *)h[(l - 1) & 1]; },
                 [&](int l) { return h[l & 1]; }, [](int) { return (uint16_t *)nullptr; }, y);
    MHIP(m, hipGetLastError());
    return infer_decode(m, y, batch, scale, flux_dev, err_est_dev);
}

dfhm_status dfhm_mlp_get_intermediate(dfhm_mlp *m, int32_t kind, int32_t layer, int64_t rows,
                                      uint16_t *host)
{
    if (!m) return DFHM_E_INVAL;
    const int L = (int)m->layers.size();
    if (!host || rows < 1 || rows > m->cfg.max_batch) return mfail(m, DFHM_E_INVAL, "bad rows or buffer");
    const uint16_t *src = nullptr;
    size_t cols = 0;
    if (kind == DFHM_MLP_ACT && layer >= 0 && layer < L - 1) {
        src = m->act[layer + 1];
        cols = (size_t)m->layers[layer].N;
    } else if (kind == DFHM_MLP_PRE && layer >= 0 && layer < L - 1) {
        src = m->pre[layer];
        cols = (size_t)m->layers[layer].N;
    } else if (kind == DFHM_MLP_DZ && layer >= 0 && layer < L) {
        src = m->dact[layer];
        cols = (size_t)(layer == L - 1 ? m->layers[layer].Np : m->layers[layer].N);
    } else {
        return mfail(m, DFHM_E_INVAL, "bad kind or layer");
    }
    MHIP(m, hipMemcpyAsync(host, src, sizeof(uint16_t) * cols * (size_t)rows, hipMemcpyDeviceToHost,
                           m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    return DFHM_OK;
}

const char *dfhm_mlp_last_error(const dfhm_mlp *m) { return m ? m->err.c_str() : "null network"; }

void dfhm_mlp_destroy(dfhm_mlp *m)
{
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    else (void)hipDeviceSynchronize();
    for (void *p : m->allocs) (void)hipFree(p);
    delete m;
}

} // extern "C"
