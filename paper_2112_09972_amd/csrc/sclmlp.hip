// C-ABI host side of the droplet-shape surrogate.  Declarations and the contract
// of every call: sclmlp.h.  Kernels: mlp_kernels.hpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "mlp_kernels.hpp"
#include "sclmlp.h"

using namespace sclmlp;

namespace {

thread_local std::string g_err;

sclbm_status fail(sclbm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(SCLBM_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                          __FILE__, __LINE__);                                          \
    } while (0)

#define HIP_LAUNCHED()                                                                                  \
    do {                                                                                                \
        hipError_t e_ = hipGetLastError();                                                              \
        if (e_ != hipSuccess) return fail(SCLBM_EHIP, "kernel launch: %s (%s:%d)", hipGetErrorString(e_), \
                                          __FILE__, __LINE__);                                          \
    } while (0)

#define TRY(expr)                            \
    do {                                     \
        sclbm_status s_ = (expr);            \
        if (s_ != SCLBM_OK) return s_;       \
    } while (0)

constexpr size_t kAlign = 256;
size_t round_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// Byte offsets of every buffer inside the workspace for batches of up to mmax rows.
struct Layout {
    size_t p, g, m1, m2, norm, wb[NLAYER], wbt[NLAYER], wbf[3], x, xt, h[3], ht[3], dza, dzb, dzat, dzbt, dy, partial,
        loss, bad, total;
};

Layout make_layout(int64_t mmax) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = round_up(off + bytes);
        return o;
    };
    const size_t pb = sizeof(float) * NPARAM;
    L.p = take(pb);
    L.g = take(pb);
    L.m1 = take(pb);
    L.m2 = take(pb);
    L.norm = take(sizeof(float) * (2 * NIN + 2 * NOUT));
    const int rows[NLAYER] = {NHID, NHID, NHID, NOUT}, cols[NLAYER] = {NIN, NHID, NHID, NHID};
    for (int l = 0; l < NLAYER; ++l) L.wb[l] = take(sizeof(bf16) * rows[l] * cols[l]);
    L.wbt[0] = L.wbt[3] = 0;
    for (int l = 1; l < 3; ++l) L.wbt[l] = take(sizeof(bf16) * NHID * NHID);
    for (int l = 0; l < 3; ++l) L.wbf[l] = take(sizeof(bf16) * NHID * (l == 0 ? NIN : NHID));
    const size_t m = (size_t)mmax;
    L.x = take(sizeof(bf16) * m * NIN);
    L.xt = take(sizeof(bf16) * m * NIN);
    for (int l = 0; l < 3; ++l) {
        L.h[l] = take(sizeof(bf16) * m * NHID);
        L.ht[l] = take(sizeof(bf16) * m * NHID);
    }
    L.dza = take(sizeof(bf16) * m * NHID);
    L.dzb = take(sizeof(bf16) * m * NHID);
    L.dzat = take(sizeof(bf16) * m * NHID);
    L.dzbt = take(sizeof(bf16) * m * NHID);
    L.dy = take(sizeof(float) * m * NOUT);
    L.partial = take(sizeof(double) * 4 * (m / OUT_ROWS));
    L.loss = take(sizeof(double));
    L.bad = take(sizeof(unsigned));
    L.total = off;
    return L;
}

int64_t padded_rows(int64_t n) { return (n + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN; }

}  // namespace

struct sclmlp_ctx {
    int64_t max_batch = 0, mmax = 0;
    char *ws = nullptr;
    Layout lay{};
    hipStream_t stream = nullptr;
    int device = 0;
    int64_t step = 0;

    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    float *P() const { return at<float>(lay.p); }
    float *G() const { return at<float>(lay.g); }
    float *in_shift() const { return at<float>(lay.norm); }
    float *in_scale() const { return at<float>(lay.norm) + NIN; }
    float *out_shift() const { return at<float>(lay.norm) + 2 * NIN; }
    float *out_scale() const { return at<float>(lay.norm) + 2 * NIN + NOUT; }
    bf16 *wb(int l) const { return at<bf16>(lay.wb[l]); }
    bf16 *wbt(int l) const { return at<bf16>(lay.wbt[l]); }
    bf16 *wbf(int l) const { return at<bf16>(lay.wbf[l]); }
    bf16 *h(int l) const { return at<bf16>(lay.h[l]); }
    bf16 *ht(int l) const { return at<bf16>(lay.ht[l]); }
};

namespace {

// C = A B^T with the epilogue EPI.  Tiles of 64 x 128 (two waves down, two across, each
// 32 x 64) when the product has at least 1024 rows, else 64 x 64; K staged 64 columns at a
// time (measured on the 8192 x 512 x 576 and x 512 products: deeper stages and 128 x 128
// tiles were slower).
template <int EPI, bool AF32 = false>
sclbm_status gemm(const sclmlp_ctx *c, const GemmArgs &g) {
    if (g.K % 8 != 0 || g.K <= 0 || g.M <= 0 || g.N <= 0)
        return fail(SCLBM_EINVAL, "gemm shape %d x %d x %d", g.M, g.N, g.K);
    // 16-byte loads and stores: row strides in whole 8-element groups
    if (g.lda % 8 || g.ldb % 8 || (EPI != EPI_F32 && ((g.C && g.ldc % 8) || (g.CT && g.ldct % 8))))
        return fail(SCLBM_EINVAL, "gemm row strides must be multiples of 8");
    if (g.M >= 1024) {
        dim3 grid((g.N + 127) / 128, (g.M + 63) / 64);
        k_gemm_nt<64, 128, 64, EPI, AF32><<<grid, 256, 0, c->stream>>>(g);
    } else {
        dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
        k_gemm_nt<64, 64, 64, EPI, AF32><<<grid, 256, 0, c->stream>>>(g);
    }
    HIP_LAUNCHED();
    return SCLBM_OK;
}

GemmArgs gargs(const bf16 *A, int lda, const bf16 *B, int ldb, int M, int N, int K) {
    GemmArgs g{};
    g.A = A;
    g.B = B;
    g.lda = lda;
    g.ldb = ldb;
    g.M = M;
    g.N = N;
    g.K = K;
    return g;
}

// The three hidden layers (bias + ReLU); with `transposed` also the [unit][row] copies.
// With `windows` (inference) the first layer reads the n FP32 windows directly and normalises
// them while staging; otherwise it reads the BF16 inputs the preparation kernel wrote.
sclbm_status hidden_forward(const sclmlp_ctx *c, int Mp, bool transposed, const float *windows = nullptr,
                            int n = 0) {
    const float *P = c->P();
    const int boff[3] = {OFF_B1, OFF_B2, OFF_B3};
    for (int l = 0; l < 3; ++l) {
        const bf16 *A = l == 0 ? c->at<bf16>(c->lay.x) : c->h(l - 1);
        const int K = l == 0 ? NIN : NHID;
        GemmArgs g = gargs(A, K, c->wb(l), K, Mp, NHID, K);
        g.bias = P + boff[l];
        g.C = c->h(l);
        g.ldc = NHID;
        g.CT = transposed ? c->ht(l) : nullptr;
        g.ldct = Mp;
        if (l == 0 && windows) {
            g.A = nullptr;
            g.Af = windows;
            g.ashift = c->in_shift();
            g.ascale = c->in_scale();
            g.arows = n;
            TRY((gemm<EPI_RELU, true>(c, g)));
        } else {
            TRY(gemm<EPI_RELU>(c, g));
        }
    }
    return SCLBM_OK;
}

AdamArgs adam_args(const sclmlp_ctx *c) {
    AdamArgs a{};
    a.p = c->P();
    a.g = c->G();
    a.m = c->at<float>(c->lay.m1);
    a.v = c->at<float>(c->lay.m2);
    a.n = NPARAM;
    a.seg[0] = Seg{OFF_W1, NHID, NIN, c->wb(0), nullptr, c->wbf(0)};
    a.seg[1] = Seg{OFF_W2, NHID, NHID, c->wb(1), c->wbt(1), c->wbf(1)};
    a.seg[2] = Seg{OFF_W3, NHID, NHID, c->wb(2), c->wbt(2), c->wbf(2)};
    a.seg[3] = Seg{OFF_W4, NOUT, NHID, c->wb(3), nullptr, nullptr};
    return a;
}

sclbm_status refresh_copies(sclmlp_ctx *c) {
    AdamArgs a = adam_args(c);
    a.update = 0;
    k_adam<<<1024, 256, 0, c->stream>>>(a);
    HIP_LAUNCHED();
    return SCLBM_OK;
}

sclbm_status use_device(const sclmlp_ctx *c) {
    HIP_TRY(hipSetDevice(c->device));
    return SCLBM_OK;
}

}  // namespace

extern "C" {

sclbm_status sclmlp_workspace_bytes(int64_t max_batch, size_t *bytes) {
    if (!bytes) return fail(SCLBM_EINVAL, "null output");
    if (max_batch < 1 || max_batch > (1 << 24)) return fail(SCLBM_EINVAL, "max_batch must be in [1, 2^24]");
    *bytes = make_layout(padded_rows(max_batch)).total;
    return SCLBM_OK;
}

sclbm_status sclmlp_create(int64_t max_batch, void *dev_workspace, size_t bytes, void *hip_stream, sclmlp_ctx **out) {
    if (!out) return fail(SCLBM_EINVAL, "null output");
    *out = nullptr;
    size_t need = 0;
    TRY(sclmlp_workspace_bytes(max_batch, &need));
    if (!dev_workspace) return fail(SCLBM_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign) return fail(SCLBM_EINVAL, "workspace not 256-byte aligned");
    if (bytes < need) return fail(SCLBM_ESIZE, "workspace has %zu bytes, needs %zu", bytes, need);
    sclmlp_ctx *c = new sclmlp_ctx;
    c->max_batch = max_batch;
    c->mmax = padded_rows(max_batch);
    c->ws = static_cast<char *>(dev_workspace);
    c->lay = make_layout(c->mmax);
    c->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws, 0, c->lay.total, c->stream);
    if (e == hipSuccess) {
        std::vector<float> norm(2 * NIN + 2 * NOUT, 0.0f);
        for (int i = 0; i < NIN; ++i) norm[NIN + i] = 1.0f;
        for (int j = 0; j < NOUT; ++j) norm[2 * NIN + NOUT + j] = 1.0f;
        e = hipMemcpyAsync(c->in_shift(), norm.data(), norm.size() * sizeof(float), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e != hipSuccess) {
        delete c;
        return fail(SCLBM_EHIP, "create: %s", hipGetErrorString(e));
    }
    *out = c;
    return SCLBM_OK;
}

sclbm_status sclmlp_destroy(sclmlp_ctx *ctx) {
    delete ctx;
    return SCLBM_OK;
}

sclbm_status sclmlp_set_params(sclmlp_ctx *c, const float *params) {
    if (!c || !params) return fail(SCLBM_EINVAL, "null argument");
    for (int i = 0; i < NPARAM; ++i)
        if (!std::isfinite(params[i])) return fail(SCLBM_EINVAL, "parameter %d is not finite", i);
    TRY(use_device(c));
    HIP_TRY(hipMemcpyAsync(c->P(), params, sizeof(float) * NPARAM, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemsetAsync(c->at<float>(c->lay.m1), 0, sizeof(float) * NPARAM, c->stream));
    HIP_TRY(hipMemsetAsync(c->at<float>(c->lay.m2), 0, sizeof(float) * NPARAM, c->stream));
    TRY(refresh_copies(c));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->step = 0;
    return SCLBM_OK;
}

sclbm_status sclmlp_get_params(sclmlp_ctx *c, float *params) {
    if (!c || !params) return fail(SCLBM_EINVAL, "null argument");
    TRY(use_device(c));
    HIP_TRY(hipMemcpyAsync(params, c->P(), sizeof(float) * NPARAM, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SCLBM_OK;
}

sclbm_status sclmlp_get_grads(sclmlp_ctx *c, float *grads) {
    if (!c || !grads) return fail(SCLBM_EINVAL, "null argument");
    TRY(use_device(c));
    HIP_TRY(hipMemcpyAsync(grads, c->G(), sizeof(float) * NPARAM, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SCLBM_OK;
}

sclbm_status sclmlp_set_normalization(sclmlp_ctx *c, const float *in_shift, const float *in_scale,
                                      const float *out_shift, const float *out_scale) {
    if (!c || !in_shift || !in_scale || !out_shift || !out_scale) return fail(SCLBM_EINVAL, "null argument");
    std::vector<float> norm(2 * NIN + 2 * NOUT);
    for (int i = 0; i < NIN; ++i) {
        if (!std::isfinite(in_shift[i]) || !std::isfinite(in_scale[i]) || in_scale[i] == 0.0f)
            return fail(SCLBM_EINVAL, "input normalisation entry %d invalid", i);
        norm[i] = in_shift[i];
        norm[NIN + i] = in_scale[i];
    }
    for (int j = 0; j < NOUT; ++j) {
        if (!std::isfinite(out_shift[j]) || !std::isfinite(out_scale[j]) || out_scale[j] == 0.0f)
            return fail(SCLBM_EINVAL, "output normalisation entry %d invalid", j);
        norm[2 * NIN + j] = out_shift[j];
        norm[2 * NIN + NOUT + j] = out_scale[j];
    }
    TRY(use_device(c));
    HIP_TRY(hipMemcpyAsync(c->in_shift(), norm.data(), norm.size() * sizeof(float), hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SCLBM_OK;
}

sclbm_status sclmlp_predict(sclmlp_ctx *c, const float *dev_windows, int64_t n, float *dev_out) {
    if (!c) return fail(SCLBM_EINVAL, "null context");
    if (n < 0 || n > c->max_batch) return fail(SCLBM_EINVAL, "n = %lld outside [0, %lld]", (long long)n,
                                              (long long)c->max_batch);
    if (n == 0) return SCLBM_OK;
    if (!dev_windows || !dev_out) return fail(SCLBM_EINVAL, "null buffer");
    TRY(use_device(c));
    const int Mp = (int)padded_rows(n);
    if (reinterpret_cast<uintptr_t>(dev_windows) % 16 == 0) {
        // one launch: the four layers, activations in LDS (same results as the layer-by-layer path)
        ForwardArgs f{};
        f.win = dev_windows;
        f.n = (int)n;
        f.ashift = c->in_shift();
        f.ascale = c->in_scale();
        const int boff[3] = {OFF_B1, OFF_B2, OFF_B3};
        for (int l = 0; l < 3; ++l) {
            f.W[l] = c->wbf(l);
            f.bias[l] = c->P() + boff[l];
        }
        f.W4 = c->wb(3);
        f.b4 = c->P() + OFF_B4;
        f.oshift = c->out_shift();
        f.oscale = c->out_scale();
        f.out = dev_out;
        k_forward<<<Mp / FW_M, FW_T, 0, c->stream>>>(f);
        HIP_LAUNCHED();
        return SCLBM_OK;
    } else {
        k_prep<false><<<dim3(NIN / 64, Mp / 64), 256, 0, c->stream>>>(dev_windows, nullptr, nullptr, (int)n, (int)n,
                                                                        c->in_shift(), c->in_scale(),
                                                                        c->at<bf16>(c->lay.x), nullptr, Mp,
                                                                        c->at<unsigned>(c->lay.bad));
        HIP_LAUNCHED();
        TRY(hidden_forward(c, Mp, false));
    }
    k_out<true><<<Mp / OUT_ROWS, 256, 0, c->stream>>>(c->h(2), c->wb(3), c->P() + OFF_B4, (int)n, c->out_shift(),
                                                c->out_scale(), dev_out, nullptr, nullptr, nullptr, 0, nullptr,
                                                nullptr);
    HIP_LAUNCHED();
    return SCLBM_OK;
}

sclbm_status sclmlp_gradients(sclmlp_ctx *c, const float *dev_windows, const float *dev_targets,
                              const int32_t *dev_index, const int32_t *dev_sym, int64_t n, int64_t ndata,
                              double *dev_loss) {
    if (!c) return fail(SCLBM_EINVAL, "null context");
    if (n < 1 || n > c->max_batch) return fail(SCLBM_EINVAL, "n = %lld outside [1, %lld]", (long long)n,
                                              (long long)c->max_batch);
    if (ndata < 1 || ndata > INT32_MAX) return fail(SCLBM_EINVAL, "ndata must be in [1, 2^31)");
    if (!dev_index && ndata < n) return fail(SCLBM_EINVAL, "without an index ndata must be >= n");
    if (!dev_windows || !dev_targets) return fail(SCLBM_EINVAL, "null buffer");
    TRY(use_device(c));
    const int Mp = (int)padded_rows(n), nb = Mp / 64, nbo = Mp / OUT_ROWS;
    float *G = c->G();
    bf16 *dza = c->at<bf16>(c->lay.dza), *dzb = c->at<bf16>(c->lay.dzb);
    bf16 *dzat = c->at<bf16>(c->lay.dzat), *dzbt = c->at<bf16>(c->lay.dzbt);
    float *dy = c->at<float>(c->lay.dy);
    double *partial = c->at<double>(c->lay.partial);

    k_prep<true><<<dim3(NIN / 64, nb), 256, 0, c->stream>>>(dev_windows, dev_index, dev_sym, (int)n, (int)ndata,
                                                             c->in_shift(), c->in_scale(), c->at<bf16>(c->lay.x),
                                                             c->at<bf16>(c->lay.xt), Mp, c->at<unsigned>(c->lay.bad));
    HIP_LAUNCHED();
    TRY(hidden_forward(c, Mp, true));
    k_out<false><<<nbo, 256, 0, c->stream>>>(c->h(2), c->wb(3), c->P() + OFF_B4, (int)n, c->out_shift(),
                                            c->out_scale(), nullptr, dev_targets, dev_index, dev_sym, (int)ndata, dy,
                                            partial);
    HIP_LAUNCHED();
    k_loss_final<<<1, 256, 0, c->stream>>>(partial, nbo, (int)n, dev_loss ? dev_loss : c->at<double>(c->lay.loss),
                                          G + OFF_B4);
    HIP_LAUNCHED();

    // output layer: dZ3 = (dY W4) * relu'(z3); dW4 = dY^T H3 (db4 came with the loss)
    k_out_back<<<dim3(NHID / 64, nb), 256, 0, c->stream>>>(dy, c->wb(3), c->h(2), dza, dzat, Mp);
    HIP_LAUNCHED();
    k_rowdot<NOUT><<<NHID, 256, 0, c->stream>>>(c->ht(2), Mp, Mp, dy, G + OFF_W4, 1, NHID);
    HIP_LAUNCHED();

    // hidden layers 3, 2, 1: dW = dZ^T H_prev, db = sum_rows dZ, dZ_prev = (dZ W) * relu'(z_prev)
    const int woff[3] = {OFF_W1, OFF_W2, OFF_W3}, boff[3] = {OFF_B1, OFF_B2, OFF_B3};
    bf16 *cur = dza, *curT = dzat, *nxt = dzb, *nxtT = dzbt;
    for (int l = 2; l >= 0; --l) {
        const int K = l == 0 ? NIN : NHID;
        const bf16 *prevT = l == 0 ? c->at<bf16>(c->lay.xt) : c->ht(l - 1);
        GemmArgs gw = gargs(curT, Mp, prevT, Mp, NHID, K, Mp);
        gw.C = G + woff[l];
        gw.ldc = K;
        TRY(gemm<EPI_F32>(c, gw));
        k_rowdot<1><<<NHID, 256, 0, c->stream>>>(curT, Mp, Mp, nullptr, G + boff[l], 1, 0);
        HIP_LAUNCHED();
        if (l == 0) break;
        GemmArgs gx = gargs(cur, NHID, c->wbt(l), NHID, Mp, NHID, NHID);
        gx.mask = c->h(l - 1);
        gx.ldmask = NHID;
        gx.C = l - 1 > 0 ? nxt : nullptr;  // the first layer needs only the transposed copy
        gx.ldc = NHID;
        gx.CT = nxtT;
        gx.ldct = Mp;
        TRY(gemm<EPI_MASK>(c, gx));
        std::swap(cur, nxt);
        std::swap(curT, nxtT);
    }
    return SCLBM_OK;
}

sclbm_status sclmlp_adam(sclmlp_ctx *c, float lr, float beta1, float beta2, float eps) {
    if (!c) return fail(SCLBM_EINVAL, "null context");
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(SCLBM_EINVAL, "Adam hyper-parameters out of range");
    TRY(use_device(c));
    const int64_t t = c->step + 1;
    AdamArgs a = adam_args(c);
    a.update = 1;
    a.lr = lr;
    a.beta1 = beta1;
    a.beta2 = beta2;
    a.eps = eps;
    a.bc1 = (float)(1.0 - std::pow((double)beta1, (double)t));
    a.bc2 = (float)(1.0 - std::pow((double)beta2, (double)t));
    k_adam<<<1024, 256, 0, c->stream>>>(a);
    HIP_LAUNCHED();
    c->step = t;
    return SCLBM_OK;
}

sclbm_status sclmlp_train_step(sclmlp_ctx *c, const float *dev_windows, const float *dev_targets,
                               const int32_t *dev_index, const int32_t *dev_sym, int64_t n, int64_t ndata, float lr,
                               float beta1, float beta2, float eps, double *dev_loss) {
    if (!c) return fail(SCLBM_EINVAL, "null context");
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(SCLBM_EINVAL, "Adam hyper-parameters out of range");
    TRY(sclmlp_gradients(c, dev_windows, dev_targets, dev_index, dev_sym, n, ndata, dev_loss));
    return sclmlp_adam(c, lr, beta1, beta2, eps);
}

sclbm_status sclmlp_get_step(const sclmlp_ctx *c, int64_t *step) {
    if (!c || !step) return fail(SCLBM_EINVAL, "null argument");
    *step = c->step;
    return SCLBM_OK;
}

sclbm_status sclmlp_bad_rows(sclmlp_ctx *c, int64_t *count) {
    if (!c || !count) return fail(SCLBM_EINVAL, "null argument");
    TRY(use_device(c));
    unsigned v = 0;
    HIP_TRY(hipMemcpyAsync(&v, c->at<unsigned>(c->lay.bad), sizeof v, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *count = v;
    return SCLBM_OK;
}

const char *sclmlp_last_error(void) { return g_err.c_str(); }

}  // extern "C"
