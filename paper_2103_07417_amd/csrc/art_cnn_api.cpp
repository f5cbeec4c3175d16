// art_cnn_api.cpp -- C ABI of the learned refinement proposal network
// (creation, parameters, forward, gradients, one training step, features,
// labels).  The network's kernels live in art_cnn.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/art.h"
#include "art_cnn.hpp"

using namespace art;

namespace art {
int api_fail(int code, const char* fmt, ...);
}

namespace {

#define CNN_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return art::api_fail(ART_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr long long kMaxPositions = 1LL << 28;   // B * H * W of one call
constexpr int kLossBlocks = 1024;

// splitmix64 + Box-Muller: seeded He-normal initial weights.
struct Rng {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal()
    {
        const double u1 = uniform(), u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    }
};

void free_ptr(void* q)
{
    if (q) (void)hipFree(q);
}

void free_net(CnnNet& n)
{
    void* ptrs[] = { n.p, n.g, n.m, n.v, n.dz0, n.dz1, n.part, n.lossp, n.cntp, n.Wf[0], n.Wf[1], n.Wf[2],
                     n.Wf[3], n.Wb[0], n.Wb[1], n.Wb[2], n.Wb[3] };
    for (void* q : ptrs) free_ptr(q);
    cnn_work_free(&n.ws);
}

int pack(CnnNet& n, hipStream_t s)
{
    for (int l = 0; l < 4; ++l)
        CNN_TRY(cnn_pack(n.p + n.off_w[l], n.ci[l], n.co[l], n.cin_pad[l], n.cout_pad[l], n.Wf[l],
                         l > 0 ? n.Wb[l] : nullptr, s));
    return ART_OK;
}

int check_shape(int B, int H, int W)
{
    if (B < 1 || H < 1 || W < 1 || (long long)B * H * W > kMaxPositions)
        return api_fail(ART_EINVAL, "bad network input shape %d x %d x %d (at most 2^28 positions)", B, H, W);
    return ART_OK;
}

}  // namespace

namespace art {

void cnn_work_free(CnnWork* w)
{
    void* ptrs[] = { w->x, w->act[0], w->act[1], w->act[2], w->logits };
    for (void* q : ptrs) free_ptr(q);
    *w = CnnWork();
}

int cnn_work_reserve(CnnWork* w, long long P)
{
    if (P <= w->cap) return ART_OK;
    (void)hipDeviceSynchronize();
    cnn_work_free(w);
    void** bufs[] = { (void**)&w->x, (void**)&w->act[0], (void**)&w->act[1], (void**)&w->act[2],
                      (void**)&w->logits };
    const size_t per[] = { 8 * sizeof(uint16_t), 32 * sizeof(uint16_t), 32 * sizeof(uint16_t),
                           32 * sizeof(uint16_t), kCnnOut * sizeof(float) };
    for (int i = 0; i < 5; ++i)
        if (hipMalloc(bufs[i], per[i] * (size_t)P) != hipSuccess) {
            cnn_work_free(w);
            return api_fail(ART_ENOMEM, "hipMalloc(network workspace, %lld positions) failed", P);
        }
    w->cap = P;
    return ART_OK;
}

hipError_t cnn_net_forward(const CnnNet* n, CnnWork* w, const float* x_dev, int B, int H, int W, float* logits,
                           hipStream_t s)
{
    const long long HW = (long long)H * W;
    hipError_t e = x_dev ? cnn_input_bf16(x_dev, B, HW, w->x, s) : hipSuccess;
    if (e != hipSuccess) return e;
    const uint16_t* in = w->x;
    for (int l = 0; l < 3; ++l) {
        e = cnn_conv_fwd(in, n->cin_pad[l], B, H, W, n->Wf[l], 9 * n->cin_pad[l], n->p + n->off_b[l], n->co[l], 0,
                         w->act[l], nullptr, s);
        if (e != hipSuccess) return e;
        in = w->act[l];
    }
    return cnn_conv_fwd(in, n->cin_pad[3], B, H, W, n->Wf[3], 9 * n->cin_pad[3], n->p + n->off_b[3], n->co[3], 1,
                        logits, nullptr, s);
}

}  // namespace art

namespace {

// Forward, loss and backward over a batch; gradients land in net.g.  The
// loss is returned if loss_out != NULL (synchronises the stream).
int grads(CnnNet& n, const float* x, const uint8_t* lab, const uint8_t* val, int B, int H, int W, float pos_w,
          float* loss_out, hipStream_t s)
{
    const long long HW = (long long)H * W;
    const long long P = (long long)B * HW;
    int rc = cnn_work_reserve(&n.ws, P);
    if (rc) return rc;
    if (P > n.dz_cap) {
        (void)hipDeviceSynchronize();
        free_ptr(n.dz0);
        free_ptr(n.dz1);
        n.dz0 = n.dz1 = nullptr;
        n.dz_cap = 0;
        if (hipMalloc(&n.dz0, 32 * sizeof(uint16_t) * (size_t)P) != hipSuccess ||
            hipMalloc(&n.dz1, 32 * sizeof(uint16_t) * (size_t)P) != hipSuccess)
            return api_fail(ART_ENOMEM, "hipMalloc(gradient buffers) failed");
        n.dz_cap = P;
    }
    long long need = 0;
    for (int l = 0; l < 4; ++l) {
        const long long q = cnn_dw_part_floats(P, n.cin_pad[l]);
        need = q > need ? q : need;
    }
    if (need > n.part_cap) {
        (void)hipDeviceSynchronize();
        free_ptr(n.part);
        n.part = nullptr;
        n.part_cap = 0;
        if (hipMalloc(&n.part, sizeof(float) * need) != hipSuccess)
            return api_fail(ART_ENOMEM, "hipMalloc(gradient partials) failed");
        n.part_cap = need;
    }
    if (!n.lossp && hipMalloc(&n.lossp, sizeof(float) * (kLossBlocks + 1)) != hipSuccess)
        return api_fail(ART_ENOMEM, "hipMalloc(loss partials) failed");
    if (!n.cntp && hipMalloc(&n.cntp, sizeof(unsigned long long) * kLossBlocks) != hipSuccess)
        return api_fail(ART_ENOMEM, "hipMalloc(count partials) failed");
    CNN_TRY(cnn_net_forward(&n, &n.ws, x, B, H, W, n.ws.logits, s));
    // the loss is the mean over valid outputs of the whole batch
    CNN_TRY(cnn_count_valid(val, (long long)B * HW * kCnnOut, n.cntp, kLossBlocks, n.lossp + kLossBlocks, s));
    CNN_TRY(cnn_bce(n.ws.logits, lab, val, B, HW, pos_w, n.lossp + kLossBlocks, n.dz0, n.lossp, kLossBlocks, s));
    uint16_t* dz = n.dz0;
    uint16_t* dzn = n.dz1;
    for (int l = 3; l >= 0; --l) {
        const uint16_t* in = l > 0 ? n.ws.act[l - 1] : n.ws.x;
        CNN_TRY(cnn_conv_dw(in, n.ci[l], n.cin_pad[l], B, H, W, dz, n.co[l], n.cout_pad[l], n.part,
                            n.g + n.off_w[l], n.g + n.off_b[l], s));
        if (l > 0) {
            // gradient w.r.t. act[l-1] = conv(dZ, flipped W^T), masked by the ReLU
            CNN_TRY(cnn_conv_fwd(dz, n.cout_pad[l], B, H, W, n.Wb[l], 9 * n.cout_pad[l], nullptr, n.ci[l], 2, dzn,
                                 n.ws.act[l - 1], s));
            uint16_t* t = dz;
            dz = dzn;
            dzn = t;
        }
    }
    if (loss_out) {
        std::vector<float> hp(kLossBlocks);
        CNN_TRY(hipMemcpyAsync(hp.data(), n.lossp, sizeof(float) * kLossBlocks, hipMemcpyDeviceToHost, s));
        CNN_TRY(hipStreamSynchronize(s));
        double t = 0.0;
        for (int i = 0; i < kLossBlocks; ++i) t += hp[i];
        *loss_out = (float)t;
    }
    return ART_OK;
}

}  // namespace

extern "C" {

int art_cnn_num_params(void)
{
    CnnNet n;
    int t = 0;
    for (int l = 0; l < 4; ++l) t += n.co[l] * n.ci[l] * 9 + n.co[l];
    return t;
}

int art_cnn_create(uint64_t seed, art_cnn** out)
{
    if (!out) return api_fail(ART_EINVAL, "NULL output handle");
    *out = nullptr;
    art_cnn* c = new (std::nothrow) art_cnn();
    if (!c) return api_fail(ART_ENOMEM, "out of host memory");
    CnnNet& n = c->net;
    long long off = 0;
    for (int l = 0; l < 4; ++l) {
        n.off_w[l] = off;
        off += (long long)n.co[l] * n.ci[l] * 9;
        n.off_b[l] = off;
        off += n.co[l];
    }
    n.nparam = (int)off;
    std::vector<float> h(off, 0.0f);
    Rng r{ seed };
    for (int l = 0; l < 4; ++l) {
        const double sd = std::sqrt(2.0 / (9.0 * n.ci[l]));
        for (long long i = 0; i < (long long)n.co[l] * n.ci[l] * 9; ++i) h[n.off_w[l] + i] = (float)(sd * r.normal());
    }
    bool ok = hipMalloc(&n.p, sizeof(float) * off) == hipSuccess &&
              hipMalloc(&n.g, sizeof(float) * off) == hipSuccess &&
              hipMalloc(&n.m, sizeof(float) * off) == hipSuccess &&
              hipMalloc(&n.v, sizeof(float) * off) == hipSuccess;
    for (int l = 0; l < 4 && ok; ++l) {
        ok = hipMalloc(&n.Wf[l], sizeof(uint16_t) * 32 * 9 * n.cin_pad[l]) == hipSuccess;
        if (ok && l > 0) ok = hipMalloc(&n.Wb[l], sizeof(uint16_t) * 32 * 9 * n.cout_pad[l]) == hipSuccess;
    }
    if (!ok) {
        free_net(n);
        delete c;
        return api_fail(ART_ENOMEM, "hipMalloc(network parameters) failed");
    }
    if (hipMemcpy(n.p, h.data(), sizeof(float) * off, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(n.g, 0, sizeof(float) * off) != hipSuccess ||
        hipMemset(n.m, 0, sizeof(float) * off) != hipSuccess ||
        hipMemset(n.v, 0, sizeof(float) * off) != hipSuccess || pack(n, nullptr) != ART_OK ||
        hipStreamSynchronize(nullptr) != hipSuccess) {
        free_net(n);
        delete c;
        return api_fail(ART_EDEVICE, "network initialisation failed");
    }
    *out = c;
    return ART_OK;
}

int art_cnn_destroy(art_cnn* c)
{
    if (!c) return ART_OK;
    (void)hipDeviceSynchronize();
    free_net(c->net);
    delete c;
    return ART_OK;
}

int art_cnn_set_params(art_cnn* c, const float* host, int64_t n)
{
    if (!c || !host) return api_fail(ART_EINVAL, "NULL argument");
    if (n != c->net.nparam)
        return api_fail(ART_EINVAL, "expected %d parameters, got %lld", c->net.nparam, (long long)n);
    CNN_TRY(hipDeviceSynchronize());
    CNN_TRY(hipMemcpy(c->net.p, host, sizeof(float) * n, hipMemcpyHostToDevice));
    CNN_TRY(hipMemset(c->net.m, 0, sizeof(float) * n));
    CNN_TRY(hipMemset(c->net.v, 0, sizeof(float) * n));
    c->net.step = 0;
    int rc = pack(c->net, nullptr);
    if (rc) return rc;
    CNN_TRY(hipStreamSynchronize(nullptr));
    return ART_OK;
}

int art_cnn_get_params(art_cnn* c, float* host, int64_t n)
{
    if (!c || !host) return api_fail(ART_EINVAL, "NULL argument");
    if (n != c->net.nparam)
        return api_fail(ART_EINVAL, "expected %d parameters, got %lld", c->net.nparam, (long long)n);
    CNN_TRY(hipDeviceSynchronize());
    CNN_TRY(hipMemcpy(host, c->net.p, sizeof(float) * n, hipMemcpyDeviceToHost));
    return ART_OK;
}

int art_cnn_forward(art_cnn* c, const float* x_dev, int32_t B, int32_t H, int32_t W, float* logits_dev,
                    void* stream)
{
    if (!c || !x_dev || !logits_dev) return api_fail(ART_EINVAL, "NULL argument");
    int rc = check_shape(B, H, W);
    if (rc) return rc;
    rc = cnn_work_reserve(&c->net.ws, (long long)B * H * W);
    if (rc) return rc;
    CNN_TRY(cnn_net_forward(&c->net, &c->net.ws, x_dev, B, H, W, logits_dev, (hipStream_t)stream));
    return ART_OK;
}

int art_cnn_gradients(art_cnn* c, const float* x_dev, const uint8_t* labels_dev, const uint8_t* valid_dev,
                      int32_t B, int32_t H, int32_t W, float pos_weight, float* grad_host, float* loss_out,
                      void* stream)
{
    if (!c || !x_dev || !labels_dev || !valid_dev) return api_fail(ART_EINVAL, "NULL argument");
    int rc = check_shape(B, H, W);
    if (rc) return rc;
    if (!(pos_weight > 0.0f)) return api_fail(ART_EINVAL, "pos_weight must be > 0");
    hipStream_t s = (hipStream_t)stream;
    rc = grads(c->net, x_dev, labels_dev, valid_dev, B, H, W, pos_weight, loss_out, s);
    if (rc) return rc;
    if (grad_host) {
        CNN_TRY(hipMemcpyAsync(grad_host, c->net.g, sizeof(float) * c->net.nparam, hipMemcpyDeviceToHost, s));
        CNN_TRY(hipStreamSynchronize(s));
    }
    return ART_OK;
}

int art_cnn_train_step(art_cnn* c, const float* x_dev, const uint8_t* labels_dev, const uint8_t* valid_dev,
                       int32_t B, int32_t H, int32_t W, float lr, float pos_weight, float* loss_out, void* stream)
{
    if (!c || !x_dev || !labels_dev || !valid_dev) return api_fail(ART_EINVAL, "NULL argument");
    int rc = check_shape(B, H, W);
    if (rc) return rc;
    if (!(lr > 0.0f) || !(pos_weight > 0.0f)) return api_fail(ART_EINVAL, "lr and pos_weight must be > 0");
    hipStream_t s = (hipStream_t)stream;
    CnnNet& n = c->net;
    rc = grads(n, x_dev, labels_dev, valid_dev, B, H, W, pos_weight, loss_out, s);
    if (rc) return rc;
    n.step++;
    CNN_TRY(cnn_adam(n.p, n.g, n.m, n.v, n.nparam, lr, 0.9f, 0.999f, 1e-8f, n.step, s));
    return pack(n, s);
}

int art_cnn_features(const double* image_dev, const void* feat_dev, int32_t nx, int32_t ny, int32_t nx0,
                     int32_t ny0, int32_t levels, int32_t level, double n_abs, float* x_dev, void* stream)
{
    if (!image_dev || !x_dev) return api_fail(ART_EINVAL, "NULL argument");
    if (nx0 < 2 || ny0 < 2 || levels < 0 || levels > 20 || level < 0 || level > levels)
        return api_fail(ART_EINVAL, "bad level %d of %d or base grid %dx%d", level, levels, nx0, ny0);
    if ((1LL << levels) * (nx0 - 1) + 1 != nx || (1LL << levels) * (ny0 - 1) + 1 != ny)
        return api_fail(ART_EINVAL, "image %dx%d does not match the grid", nx, ny);
    if (!(n_abs > 0.0)) return api_fail(ART_EINVAL, "n_abs must be > 0");
    const int W = (1 << level) * (nx0 - 1) + 1, H = (1 << level) * (ny0 - 1) + 1;
    CNN_TRY(cnn_features(image_dev, (const RayFeat*)feat_dev, nx, 1 << (levels - level), H, W, n_abs, x_dev,
                         (hipStream_t)stream));
    return ART_OK;
}

int art_cnn_labels(const int8_t* level_dev, int32_t nx, int32_t ny, int32_t nx0, int32_t ny0, int32_t levels,
                   int32_t level, uint8_t* labels_dev, uint8_t* valid_dev, void* stream)
{
    if (!level_dev || !labels_dev || !valid_dev) return api_fail(ART_EINVAL, "NULL argument");
    if (nx0 < 2 || ny0 < 2 || levels < 1 || levels > 20 || level < 0 || level >= levels)
        return api_fail(ART_EINVAL, "bad level %d of %d or base grid %dx%d", level, levels, nx0, ny0);
    if ((1LL << levels) * (nx0 - 1) + 1 != nx || (1LL << levels) * (ny0 - 1) + 1 != ny)
        return api_fail(ART_EINVAL, "image %dx%d does not match the grid", nx, ny);
    CNN_TRY(cnn_labels(level_dev, nx, nx0, ny0, levels, level, labels_dev, valid_dev, (hipStream_t)stream));
    return ART_OK;
}

}  // extern "C"
