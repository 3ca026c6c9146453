// C ABI of the warm-start network kernels (include/lbm_nn.h): argument
// checks and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

#include "lbm.h"
#include "lbm_nn.h"
#include "nn_internal.h"

using namespace nn;

// Scratch of the allocation-free loss (nn_mse_noalloc): one float64 partial
// sum per 256 pixels.  Each GPU the library runs on holds its own copy until
// the process ends.  In host code the name below is only a stand-in for the
// device array; kernels get the address resolved per device by
// hipGetSymbolAddress (scratch_on_current_device).
constexpr long long MSE_SCRATCH_DOUBLES = 131072;                 // 1 MiB: up to 2^25 pixels
static __device__ __align__(256) double scratch[MSE_SCRATCH_DOUBLES];

namespace {

hipStream_t S(void* s) { return (hipStream_t)s; }

int status(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EDEVICE; }

bool conv_shape_ok(int n, int h, int w, int ci, int co) {
    return n > 0 && h > 0 && w > 0 && w % 64 == 0 && ci > 0 && ci % 32 == 0 && ci <= MAX_CH && co > 0 &&
           co % 32 == 0 && co <= MAX_CH;
}

// pixel chunks of the weight gradient: multiples of 256 pixels (so that
// every step size of the kernel divides them), about 256 chunks, a function
// of the sizes only (fixed summation order)
long long wgrad_chunk_pix(long long npix) {
    long long c = (npix + 255) / 256;
    c = ((c + 255) / 256) * 256;
    return c < 256 ? 256 : c;
}

// Device address of `scratch` on the current device, resolved once per
// device with that device current (each GPU has its own copy).
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};

int scratch_on_current_device(double** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return LBM_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBM_EDEVICE;
        g_scratch[dev] = (double*)ptr;
    }
    *out = g_scratch[dev];
    return LBM_OK;
}

ChanDesc desc_of(const lbm_params& p) {
    ChanDesc d;
    d.b = p.b;
    d.W = p.W;
    d.l = (double)p.nx / (double)p.n_waves;
    d.mu_a = p.mu_a;
    d.mu_b = p.mu_b;
    d.k_a = p.k_a;
    d.k_b = p.k_b;
    d.sigma_T = p.sigma_T;
    d.sigma_TT = p.sigma_TT;
    d.T_ref = p.T_ref;
    d.T_h = p.T_h;
    d.dT = p.dT;
    d.U_s = nn_velocity_scale(&p);
    return d;
}

// upload the per-channel table, run f(table), free; synchronous
template <class F>
int with_desc(const lbm_params* params, int n, hipStream_t st, F f) {
    if (!params || n <= 0) return LBM_EINVAL;
    for (int k = 1; k < n; ++k)
        if (params[k].nx != params[0].nx || params[k].ny != params[0].ny) return LBM_EINVAL;
    for (int k = 0; k < n; ++k)
        if (params[k].n_waves <= 0 || params[k].nx % params[k].n_waves != 0 || !(params[k].mu_b > 0) ||
            !(params[k].k_b > 0) || !(params[k].W > 0) || !(params[k].dT != 0))
            return LBM_EINVAL;
    std::vector<ChanDesc> h(n);
    for (int k = 0; k < n; ++k) h[k] = desc_of(params[k]);
    ChanDesc* d = nullptr;
    if (hipMalloc((void**)&d, sizeof(ChanDesc) * n) != hipSuccess) return LBM_ENOMEM;
    hipError_t e = hipMemcpyAsync(d, h.data(), sizeof(ChanDesc) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = f(d);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    return status(e);
}

}  // namespace

extern "C" {

double nn_velocity_scale(const lbm_params* p) {
    const double u = 0.01 * (std::fabs(p->sigma_T) + p->sigma_TT * std::fabs(p->dT)) * std::fabs(p->dT) / p->mu_b;
    return u > 1e-12 ? u : 1e-12;
}

int nn_conv3x3_fwd(const uint16_t* x, const uint16_t* w, const float* bias, uint16_t* y, float* y32,
                   int32_t y32_channels, int32_t n, int32_t h, int32_t wd, int32_t ci, int32_t co, int32_t relu,
                   void* stream) {
    if (!x || !w || (!y && !y32) || !conv_shape_ok(n, h, wd, ci, co)) return LBM_EINVAL;
    if (y32 && (y32_channels <= 0 || y32_channels > co)) return LBM_EINVAL;
    ConvArgs a{x, w, bias, y, y32, n, h, wd, ci, co, relu ? 1 : 0, y32 ? y32_channels : 0};
    return status(launch_conv_fwd(a, S(stream)));
}

int nn_set_conv_walk(int32_t steps) {
    if (steps < 0 || steps > 64) return LBM_EINVAL;
    set_conv_walk(steps);
    return LBM_OK;
}

int nn_conv3x3_bwd_data(const uint16_t* dy, const uint16_t* wflip, uint16_t* dx, int32_t n, int32_t h, int32_t wd,
                        int32_t ci, int32_t co, void* stream) {
    if (!dy || !wflip || !dx || !conv_shape_ok(n, h, wd, co, ci)) return LBM_EINVAL;
    // the forward convolution of dy with the flipped weights: ci <-> co
    ConvArgs a{dy, wflip, nullptr, dx, nullptr, n, h, wd, co, ci, 0, 0};
    return status(launch_conv_fwd(a, S(stream)));
}

int nn_conv3x3_wgrad_workspace(int32_t n, int32_t h, int32_t wd, int32_t ci, int32_t co, int64_t* bytes) {
    if (!bytes || !conv_shape_ok(n, h, wd, ci, co)) return LBM_EINVAL;
    const long long npix = (long long)n * h * wd;
    const long long cp = wgrad_chunk_pix(npix);
    const long long nc = (npix + cp - 1) / cp;
    *bytes = nc * ((long long)co * 9 * ci + co) * (long long)sizeof(float);
    return LBM_OK;
}

int nn_conv3x3_bwd_weight(const uint16_t* x, const uint16_t* dy, float* dw, float* db, void* work, int64_t work_bytes,
                          int32_t accumulate, int32_t n, int32_t h, int32_t wd, int32_t ci, int32_t co, void* stream) {
    int64_t need = 0;
    if (!x || !dy || !dw || !work || nn_conv3x3_wgrad_workspace(n, h, wd, ci, co, &need) != LBM_OK) return LBM_EINVAL;
    if (work_bytes < need) return LBM_EINVAL;
    WgradArgs a;
    a.x = x;
    a.dy = dy;
    a.dw = dw;
    a.db = db;
    a.npix = (long long)n * h * wd;
    a.chunk_pix = wgrad_chunk_pix(a.npix);
    a.n_chunks = (int)((a.npix + a.chunk_pix - 1) / a.chunk_pix);
    a.work = (float*)work;
    a.work_b = a.work + (size_t)a.n_chunks * co * 9 * ci;
    a.n = n;
    a.h = h;
    a.w = wd;
    a.ci = ci;
    a.co = co;
    a.accumulate = accumulate ? 1 : 0;
    return status(launch_conv_wgrad(a, S(stream)));
}

int nn_relu_bwd(const uint16_t* dy, const uint16_t* y, uint16_t* dx, int64_t count, void* stream) {
    if (!dy || !y || !dx || count < 0) return LBM_EINVAL;
    if (count == 0) return LBM_OK;
    return status(launch_relu_bwd(dy, y, dx, count, S(stream)));
}

int nn_add(const uint16_t* a, const uint16_t* b, uint16_t* out, int64_t count, void* stream) {
    if (!a || !b || !out || count < 0) return LBM_EINVAL;
    if (count == 0) return LBM_OK;
    return status(launch_add(a, b, out, count, S(stream)));
}

int nn_pool2(int32_t backward, const uint16_t* in, uint16_t* out, int32_t n, int32_t h, int32_t wd, int32_t c,
             void* stream) {
    if (!in || !out || n <= 0 || h <= 0 || wd <= 0 || c <= 0 || c % 8 || h % 2 || wd % 2) return LBM_EINVAL;
    if ((long long)n * h >= (1LL << 31) || (long long)wd * c >= (1LL << 31)) return LBM_EINVAL;
    return status(launch_pool(backward ? 1 : 0, in, out, n, h, wd, c, S(stream)));
}

int nn_up2(int32_t backward, const uint16_t* in, uint16_t* out, int32_t n, int32_t h, int32_t wd, int32_t c,
           void* stream) {
    if (!in || !out || n <= 0 || h <= 0 || wd <= 0 || c <= 0 || c % 8) return LBM_EINVAL;
    if ((long long)n * 2 * h >= (1LL << 31) || (long long)2 * wd * c >= (1LL << 31)) return LBM_EINVAL;
    return status(launch_up(backward ? 1 : 0, in, out, n, h, wd, c, S(stream)));
}

int nn_mse(const float* pred, const float* target, uint16_t* dpred, int32_t cpad, int64_t npix, int32_t nch,
           double* loss, void* work, int64_t work_bytes, void* stream) {
    if (!pred || !target || !loss || !work || npix <= 0 || nch <= 0 || (dpred && cpad < nch)) return LBM_EINVAL;
    if (work_bytes < 8 * ((npix + 255) / 256)) return LBM_EINVAL;
    return status(launch_mse(pred, target, dpred, (double*)work, loss, npix, nch, dpred ? cpad : 0, S(stream)));
}

int nn_mse_noalloc(const float* pred, const float* target, uint16_t* dpred, int32_t cpad, int64_t npix, int32_t nch,
                   double* loss, void* stream) {
    if (!pred || !target || !loss || npix <= 0 || nch <= 0 || (dpred && cpad < nch)) return LBM_EINVAL;
    if ((npix + 255) / 256 > MSE_SCRATCH_DOUBLES) return LBM_EINVAL;   // beyond the static scratch
    double* work = nullptr;
    const int rc = scratch_on_current_device(&work);
    if (rc) return rc;
    // every partial slot the launch reads is written first by the same launch:
    // nothing to clear
    return status(launch_mse(pred, target, dpred, work, loss, npix, nch, dpred ? cpad : 0, S(stream)));
}

int nn_adam(float* w, uint16_t* w16, uint16_t* wflip, const float* g, float* m, float* v, int64_t n, int32_t co,
            int32_t ci, int64_t step, float lr, float beta1, float beta2, float eps, float weight_decay,
            void* stream) {
    if (!w || !g || !m || !v || n <= 0 || step < 1) return LBM_EINVAL;
    if (wflip && (co <= 0 || ci <= 0 || (int64_t)co * 9 * ci != n)) return LBM_EINVAL;
    AdamArgs a;
    a.w = w;
    a.w16 = w16;
    a.wflip = wflip;
    a.g = g;
    a.m = m;
    a.v = v;
    a.n = n;
    a.co = co;
    a.ci = ci;
    a.lr = lr;
    a.b1 = beta1;
    a.b2 = beta2;
    a.eps = eps;
    a.wd = weight_decay;
    a.c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
    a.c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
    return status(launch_adam(a, S(stream)));
}

int nn_cast_weights(const float* w, uint16_t* w16, uint16_t* wflip, int32_t co, int32_t ci, void* stream) {
    if (!w || !w16 || co <= 0 || ci <= 0) return LBM_EINVAL;
    return status(launch_wcast(w, w16, wflip, co, ci, S(stream)));
}

int nn_features(const lbm_params* params, int32_t n, uint16_t* x, int32_t cpad, void* stream) {
    if (!x || cpad < NFEAT) return LBM_EINVAL;
    return with_desc(params, n, S(stream), [&](const ChanDesc* d) {
        return launch_features(d, x, n, params[0].ny, params[0].nx, cpad, S(stream));
    });
}

int nn_to_fields(const lbm_params* params, int32_t n, const float* pred, double* fields, int32_t phi_from_net,
                 void* stream) {
    if (!pred || !fields) return LBM_EINVAL;
    return with_desc(params, n, S(stream), [&](const ChanDesc* d) {
        return launch_to_fields(d, pred, fields, n, params[0].ny, params[0].nx, phi_from_net ? 1 : 0, S(stream));
    });
}

int nn_targets(const lbm_params* params, int32_t n, const double* fields, float* target, void* stream) {
    if (!fields || !target) return LBM_EINVAL;
    return with_desc(params, n, S(stream), [&](const ChanDesc* d) {
        return launch_targets(d, fields, target, n, params[0].ny, params[0].nx, S(stream));
    });
}

}  // extern "C"
