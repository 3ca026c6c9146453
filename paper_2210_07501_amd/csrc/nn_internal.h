// Internal declarations of the warm-start network kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace nn {

constexpr int MAX_CH = 96;               // widest layer (channels, padded to 32)
constexpr int NFEAT = 10;                // input planes
// The network's fourth output is the deviation of phi from the cold-start
// tanh profile, times PHI_DEV_SCALE, on the interface band |y - (b - 1/2)|
// <= PHI_BAND W (zero outside).  Steady deviations are a few 1e-3 to 1e-1.
constexpr double PHI_DEV_SCALE = 50.0;
constexpr double PHI_BAND = 3.0;

// Per-channel description for the feature and hand-off kernels.
struct ChanDesc {
    double b, W, l;                      // layer thickness, interface width, heating wavelength
    double mu_a, mu_b, k_a, k_b;
    double sigma_T, sigma_TT, T_ref, T_h, dT;
    double U_s;                          // velocity scale of the network outputs
};

struct ConvArgs {
    const uint16_t* x;                   // [n][h][w][ci] bf16
    const uint16_t* wt;                  // [co][9][ci] bf16
    const float* bias;                   // [co] or null
    uint16_t* y16;                       // [n][h][w][co] bf16 or null
    float* y32;                          // [n][h][w][y32_ch] float32 or null
    int n, h, w, ci, co, relu, y32_ch;
};

struct WgradArgs {
    const uint16_t* x;                   // [n][h][w][ci]
    const uint16_t* dy;                  // [n][h][w][co]
    float* dw;                           // [co][9][ci]
    float* db;                           // [co] or null
    float* work;                         // [n_chunks][co][9][ci]
    float* work_b;                       // [n_chunks][co]
    long long npix, chunk_pix;
    int n, h, w, ci, co, n_chunks, accumulate;
};

struct AdamArgs {
    float* w;
    uint16_t* w16;                       // bf16 copy or null
    uint16_t* wflip;                     // [ci][9][co] flipped copy or null
    const float* g;
    float* m;
    float* v;
    long long n;
    int co, ci;
    float lr, b1, b2, eps, wd, c1, c2;   // c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
};

hipError_t launch_conv_fwd(const ConvArgs& a, hipStream_t st);
hipError_t launch_conv_wgrad(const WgradArgs& a, hipStream_t st);
void set_conv_walk(int rs);
hipError_t launch_relu_bwd(const uint16_t* dy, const uint16_t* y, uint16_t* dx, long long n, hipStream_t st);
hipError_t launch_add(const uint16_t* a, const uint16_t* b, uint16_t* o, long long n, hipStream_t st);
hipError_t launch_pool(int dir, const uint16_t* in, uint16_t* out, int n, int h, int w, int c, hipStream_t st);
hipError_t launch_up(int dir, const uint16_t* in, uint16_t* out, int n, int h, int w, int c, hipStream_t st);
hipError_t launch_mse(const float* pred, const float* tgt, uint16_t* dpred, double* partial, double* out,
                      long long npix, int nch, int cpad, hipStream_t st);
hipError_t launch_adam(const AdamArgs& a, hipStream_t st);
hipError_t launch_wcast(const float* w, uint16_t* w16, uint16_t* wflip, int co, int ci, hipStream_t st);
hipError_t launch_features(const ChanDesc* d, uint16_t* x, int n, int h, int w, int cpad, hipStream_t st);
hipError_t launch_to_fields(const ChanDesc* d, const float* pred, double* fields, int n, int h, int w, int phi_net,
                            hipStream_t st);
hipError_t launch_targets(const ChanDesc* d, const double* fields, float* tgt, int n, int h, int w, hipStream_t st);

}  // namespace nn
