// Learned Newton initial guess: device state and host control (learned.hip).
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace bdm {

struct CnnGrid {
    int nx1, ny1, nz1;
    int64_t N;
};

// s_v, s_e (state inputs), s_dv, s_de (difference inputs), s_yv, s_ye (outputs)
constexpr int kScales = 6;

struct Predictor {
    bool ready = false, has_weights = false;
    CnnGrid g{};
    __half *X0 = nullptr, *Z[3] = {}, *H[3] = {}, *wh = nullptr;
    float *Y = nullptr, *G0 = nullptr, *G1 = nullptr, *w32 = nullptr, *mom1 = nullptr, *mom2 = nullptr;
    float *grad = nullptr, *bias = nullptr, *part = nullptr;
    double* lpart = nullptr;
    int *is_bias = nullptr, *bias_pos = nullptr;
    long woff[4] = {};
    int boff_[4] = {};
    int nchunk = 1;
    int64_t chunk = 1;
    double scale[kScales] = {1, 1, 1, 1, 1, 1};
    int adam_t = 0;

    static long n_params();
    std::string init(int64_t N, int nx1, int ny1, int nz1, void* (*alloc)(void*, size_t), void* ctx);
    void set(hipStream_t s, const float* host_params, const double sc[kScales]);
    void get(hipStream_t s, float* host_params, double sc[kScales]);
    // training forward pass (channel-major activations, kept for the backward pass)
    void forward(hipStream_t s, const double* vn, const double* uen, const double* vp, const double* uep);
    // inference forward pass on MFMA (node-major activations)
    void forward_mfma(hipStream_t s, const double* vn, const double* uen, const double* vp, const double* uep);
    void guess(hipStream_t s, const double* vn, const double* uen, const double* vp, const double* uep, double* out);
    double loss_grad(hipStream_t s, const double* s6);
    double train_step(hipStream_t s, const double* s6, double lr);
};

}  // namespace bdm
