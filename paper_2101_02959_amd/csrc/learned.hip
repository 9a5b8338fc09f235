// Learned Newton initial guess: a small 3-D convolutional network on the
// node grid (not part of the paper's method; it only supplies the starting
// point of Newton, and the converged Newton residual is unchanged).
//
// Network: four 3x3x3 zero-padded convolutions, channels 4 -> 16 -> 16 -> 16
// -> 2, GELU after the first three.  Inputs are (v^n / s_v, u_e^n / s_e,
// (v^n - v^{n-1}) / s_dv, (u_e^n - u_e^{n-1}) / s_de), the differences taken in
// FP64 before rounding to FP16; the output y gives the guess
//     u^{(0)} = u^n + (u^n - u^{n-1}) + (s_yv y_0, s_ye y_1),
// i.e. the network corrects the last-step extrapolation.  Weights and
// activations are stored in FP16, every sum accumulates in FP32, gradients and
// the Adam master weights are FP32.  Reductions over voxels use fixed-order
// two-stage sums, so training is deterministic.
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>

#include "learned.hpp"

namespace bdm {

namespace {

constexpr int BX = 64, BY = 4;

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.3989422804014327f;
}

// tap t = dx + 3 dy + 9 dz  <->  offset (dx-1, dy-1, dz-1)
__device__ inline bool tap_valid(const CnnGrid& g, int i, int j, int k, int t, int64_t& off) {
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    const int ii = i + dx, jj = j + dy, kk = k + dz;
    off = dx + (int64_t)g.nx1 * (dy + (int64_t)g.ny1 * dz);
    return ii >= 0 && ii < g.nx1 && jj >= 0 && jj < g.ny1 && kk >= 0 && kk < g.nz1;
}

__global__ void k_cnn_input(CnnGrid g, const double* __restrict__ vn, const double* __restrict__ uen,
                            const double* __restrict__ vp, const double* __restrict__ uep, double sv, double se,
                            double sdv, double sde, __half* __restrict__ X) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    X[n] = __float2half((float)(vn[n] / sv));
    X[g.N + n] = __float2half((float)(uen[n] / se));
    X[2 * g.N + n] = __float2half((float)((vn[n] - vp[n]) / sdv));
    X[3 * g.N + n] = __float2half((float)((uen[n] - uep[n]) / sde));
}

template <int CIN, int COUT, bool GELU>
__global__ __launch_bounds__(BX * BY) void k_conv_fwd(CnnGrid g, const __half* __restrict__ X,
                                                      const __half* __restrict__ W, const float* __restrict__ b,
                                                      __half* __restrict__ Z, __half* __restrict__ H,
                                                      float* __restrict__ Y) {
    // weights W[co][ci][t] staged as Ws[t][ci][co] (contiguous over co)
    __shared__ float Ws[COUT * CIN * 27];
    const int tid = threadIdx.x + BX * threadIdx.y;
    for (int q = tid; q < COUT * CIN * 27; q += BX * BY) {
        const int co = q / (CIN * 27), ci = (q / 27) % CIN, t = q % 27;
        Ws[(t * CIN + ci) * COUT + co] = __half2float(W[q]);
    }
    __syncthreads();
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx1 || j >= g.ny1) return;
    const int64_t n = i + (int64_t)g.nx1 * (j + (int64_t)g.ny1 * k);
    float acc[COUT];
#pragma unroll
    for (int co = 0; co < COUT; ++co) acc[co] = b[co];
    for (int t = 0; t < 27; ++t) {
        int64_t off;
        if (!tap_valid(g, i, j, k, t, off)) continue;
#pragma unroll
        for (int ci = 0; ci < CIN; ++ci) {
            const float x = __half2float(X[(int64_t)ci * g.N + n + off]);
#pragma unroll
            for (int co = 0; co < COUT; ++co) acc[co] = fmaf(Ws[(t * CIN + ci) * COUT + co], x, acc[co]);
        }
    }
#pragma unroll
    for (int co = 0; co < COUT; ++co) {
        if (GELU) {
            Z[(int64_t)co * g.N + n] = __float2half(acc[co]);
            H[(int64_t)co * g.N + n] = __float2half(gelu_f(acc[co]));
        } else {
            Y[(int64_t)co * g.N + n] = acc[co];
        }
    }
}

// Gin[ci][m] = sum_{co, t} W[co][ci][t] Gout[co][m - off(t)]  (times GELU'(Zin) when
// the layer input was an activation).
template <int CIN, int COUT, bool GELU_IN>
__global__ __launch_bounds__(BX * BY) void k_conv_bwd_data(CnnGrid g, const float* __restrict__ Gout,
                                                           const __half* __restrict__ W,
                                                           const __half* __restrict__ Zin, float* __restrict__ Gin) {
    // weights W[co][ci][t] staged as Ws[t][co][ci] (contiguous over ci)
    __shared__ float Ws[COUT * CIN * 27];
    const int tid = threadIdx.x + BX * threadIdx.y;
    for (int q = tid; q < COUT * CIN * 27; q += BX * BY) {
        const int co = q / (CIN * 27), ci = (q / 27) % CIN, t = q % 27;
        Ws[(t * COUT + co) * CIN + ci] = __half2float(W[q]);
    }
    __syncthreads();
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx1 || j >= g.ny1) return;
    const int64_t m = i + (int64_t)g.nx1 * (j + (int64_t)g.ny1 * k);
    float acc[CIN];
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci) acc[ci] = 0.0f;
    for (int t = 0; t < 27; ++t) {
        // output voxel n = m - off(t) must lie in the grid: reflect the tap
        int64_t off;
        if (!tap_valid(g, i, j, k, 26 - t, off)) continue;   // offset of tap t negated
#pragma unroll
        for (int co = 0; co < COUT; ++co) {
            const float gv = Gout[(int64_t)co * g.N + m + off];
#pragma unroll
            for (int ci = 0; ci < CIN; ++ci) acc[ci] = fmaf(Ws[(t * COUT + co) * CIN + ci], gv, acc[ci]);
        }
    }
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci) {
        float a = acc[ci];
        if (GELU_IN) a *= gelu_grad_f(__half2float(Zin[(int64_t)ci * g.N + m]));
        Gin[(int64_t)ci * g.N + m] = a;
    }
}

// Partial weight and bias gradients over one chunk of voxels:
// dW[co][ci][t] = sum_n Gout[co][n] X[ci][n + off(t)],  db[co] = sum_n Gout[co][n].
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_bwd_w(CnnGrid g, const float* __restrict__ Gout,
                                                    const __half* __restrict__ X, int64_t chunk,
                                                    float* __restrict__ part) {
    constexpr int NW = COUT * CIN * 27 + COUT;
    const int64_t n0 = (int64_t)blockIdx.x * chunk;
    const int64_t n1 = (n0 + chunk < g.N) ? n0 + chunk : g.N;
    for (int w = threadIdx.x; w < NW; w += 256) {
        float acc = 0.0f;
        if (w < COUT * CIN * 27) {
            const int co = w / (CIN * 27), ci = (w / 27) % CIN, t = w % 27;
            const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
            const int64_t off = dx + (int64_t)g.nx1 * (dy + (int64_t)g.ny1 * dz);
            int64_t q = n0 / g.nx1;
            int i = (int)(n0 - q * g.nx1);
            int k = (int)(q / g.ny1);
            int j = (int)(q - (int64_t)k * g.ny1);
            const float* gp = Gout + (int64_t)co * g.N;
            const __half* xp = X + (int64_t)ci * g.N;
            for (int64_t n = n0; n < n1; ++n) {
                const int ii = i + dx, jj = j + dy, kk = k + dz;
                if (ii >= 0 && ii < g.nx1 && jj >= 0 && jj < g.ny1 && kk >= 0 && kk < g.nz1)
                    acc = fmaf(gp[n], __half2float(xp[n + off]), acc);
                if (++i == g.nx1) {
                    i = 0;
                    if (++j == g.ny1) { j = 0; ++k; }
                }
            }
        } else {
            const float* gp = Gout + (int64_t)(w - COUT * CIN * 27) * g.N;
            for (int64_t n = n0; n < n1; ++n) acc += gp[n];
        }
        part[(int64_t)blockIdx.x * NW + w] = acc;
    }
}

__global__ void k_sum_chunks(int nchunk, int nw, const float* __restrict__ part, float* __restrict__ out) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nw) return;
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * nw + w];
    out[w] = s;
}

// Target of a training sample and the loss gradient:
// t = ((u^{n+1} - u^n) - (u^n - u^{n-1})) / s_y,  G = 2 (y - t) / (2N),
// per-block partial sums of (y - t)^2.
__global__ __launch_bounds__(256) void k_mse(CnnGrid g, const float* __restrict__ Y, const double* __restrict__ s6,
                                             double sdv, double sde, float* __restrict__ G,
                                             double* __restrict__ lpart) {
    const int64_t N = g.N;
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < 2 * N; n += (int64_t)gridDim.x * 256) {
        const int c = n >= N;
        const int64_t q = n - c * N;
        const double* cur = s6 + (c ? N : 0);          // v^n or u_e^n
        const double* prv = s6 + (c ? 3 * N : 2 * N);  // v^{n-1} or u_e^{n-1}
        const double* nxt = s6 + (c ? 5 * N : 4 * N);  // v^{n+1} or u_e^{n+1}
        const double t = ((nxt[q] - cur[q]) - (cur[q] - prv[q])) / (c ? sde : sdv);
        const double d = (double)Y[n] - t;
        G[n] = (float)(2.0 * d / (2.0 * N));
        acc += d * d;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_adam(int n, float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ gr, float lr, float b1, float b2, float eps, float c1, float c2,
                       __half* __restrict__ wh, float* __restrict__ bias_out, const int* __restrict__ is_bias,
                       const int* __restrict__ bias_pos) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mm = b1 * m[i] + (1.0f - b1) * g;
    const float vv = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mm;
    v[i] = vv;
    const float wn = w[i] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    w[i] = wn;
    if (is_bias[i]) bias_out[bias_pos[i]] = wn;
    else wh[i] = __float2half(wn);
}

// ------------------------------------------------- inference on MFMA
// The inference path holds activations node-major (the CIN channels of a
// node in consecutive halves) so that a convolution is an implicit GEMM on
// the 16x16x16 FP16 MFMA: 16 nodes along x (M) x 16 output channels (N),
// the inner dimension walked in blocks of 16 (K): one tap's 16 input
// channels (CIN = 16) or four taps' 4 channels (CIN = 4).  Operand lanes:
// A lane l holds A[l % 16][4 (l / 16) .. + 3], B lane l holds
// B[4 (l / 16) .. + 3][l % 16], accumulator register v of lane l holds
// C[4 (l / 16) + v][l % 16].  Taps outside the grid read zero (the network's
// zero padding); the sums accumulate in FP32 as in the training kernels, in
// a different order.
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float cf4 __attribute__((ext_vector_type(4)));
constexpr int CM_WAVES = 4;     // waves per workgroup
constexpr int CM_G = 4;         // 16-node groups per wave and pass (independent MFMA chains)

__global__ void k_cnn_input_nm(CnnGrid g, const double* __restrict__ vn, const double* __restrict__ uen,
                               const double* __restrict__ vp, const double* __restrict__ uep, double sv, double se,
                               double sdv, double sde, __half* __restrict__ X) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    h4 x;
    x[0] = (_Float16)(float)(vn[n] / sv);
    x[1] = (_Float16)(float)(uen[n] / se);
    x[2] = (_Float16)(float)((vn[n] - vp[n]) / sdv);
    x[3] = (_Float16)(float)((uen[n] - uep[n]) / sde);
    reinterpret_cast<h4*>(X)[n] = x;
}

// X node-major [N][CIN]; W as stored, [COUT][CIN][27]; GELU layers write H
// node-major [N][16], the last layer writes Y channel-major [COUT][N].  The
// node rows are cut into ngx groups of 16 nodes; the grid strides over the
// groups, CM_G per wave and pass.
template <int CIN, int COUT, bool GELU>
__global__ __launch_bounds__(64 * CM_WAVES) void k_conv_mfma(CnnGrid g, int ngx, int64_t ngroups,
                                                             const __half* __restrict__ X,
                                                             const __half* __restrict__ W,
                                                             const float* __restrict__ b, __half* __restrict__ H,
                                                             float* __restrict__ Y) {
    static_assert(CIN == 16 || CIN == 4, "input channels");
    static_assert(COUT <= 16, "output channels");
    constexpr int NK = CIN == 16 ? 27 : 7;   // K blocks of 16
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lr = lane & 15, lq = lane >> 4;
    // the weights as B operands, one register pair per K block
    h4 wb[NK];
#pragma unroll
    for (int q = 0; q < NK; ++q)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int t = CIN == 16 ? q : 4 * q + lq, ci = CIN == 16 ? 4 * lq + jj : jj;
            wb[q][jj] = (lr < COUT && t < 27) ? (_Float16)__half2float(W[((int64_t)lr * CIN + ci) * 27 + t])
                                              : (_Float16)0.0f;
        }
    const float bias = lr < COUT ? b[lr] : 0.0f;
    const h4* Xv = reinterpret_cast<const h4*>(X);
    const int64_t stride = (int64_t)gridDim.x * CM_WAVES * CM_G;
    for (int64_t g0 = ((int64_t)blockIdx.x * CM_WAVES + wv) * CM_G; g0 < ngroups; g0 += stride) {
        int gi[CM_G], gj[CM_G], gk[CM_G];
        bool gon[CM_G];
#pragma unroll
        for (int u = 0; u < CM_G; ++u) {
            const int64_t grp = min(g0 + u, ngroups - 1);
            const int64_t row = grp / ngx;
            gon[u] = g0 + u < ngroups;
            gi[u] = 16 * (int)(grp - row * ngx);
            gj[u] = (int)(row % g.ny1);
            gk[u] = (int)(row / g.ny1);
        }
        cf4 acc[CM_G];
#pragma unroll
        for (int u = 0; u < CM_G; ++u) acc[u] = (cf4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 3
        for (int q = 0; q < NK; ++q) {
            const int t = CIN == 16 ? q : 4 * q + lq;
            const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
            h4 a[CM_G];
#pragma unroll
            for (int u = 0; u < CM_G; ++u) {
                const int i = gi[u] + lr + dx, j = gj[u] + dy, k = gk[u] + dz;
                const bool ok = t < 27 && gi[u] + lr < g.nx1 && i >= 0 && i < g.nx1 && j >= 0 && j < g.ny1 &&
                                k >= 0 && k < g.nz1;
                const int64_t nn = ok ? i + (int64_t)g.nx1 * (j + (int64_t)g.ny1 * k) : 0;
                const h4 x = Xv[nn * (CIN / 4) + (CIN == 16 ? lq : 0)];
                a[u] = ok ? x : (h4){(_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f};
            }
#pragma unroll
            for (int u = 0; u < CM_G; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x16f16(a[u], wb[q], acc[u], 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < CM_G; ++u) {
            if (!gon[u] || lr >= COUT) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int io = gi[u] + 4 * lq + v;
                if (io >= g.nx1) continue;
                const int64_t n = io + (int64_t)g.nx1 * (gj[u] + (int64_t)g.ny1 * gk[u]);
                const float z = acc[u][v] + bias;
                if constexpr (GELU) H[n * 16 + lr] = __float2half(gelu_f(z));
                else Y[(int64_t)lr * g.N + n] = z;
            }
        }
    }
}

// guess = u^n + (u^n - u^{n-1}) + scale * y
__global__ void k_cnn_guess(CnnGrid g, const double* __restrict__ vn, const double* __restrict__ uen,
                            const double* __restrict__ vp, const double* __restrict__ uep, const float* __restrict__ Y,
                            double sdv, double sde, double* __restrict__ out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    out[n] = 2.0 * vn[n] - vp[n] + sdv * (double)Y[n];
    out[g.N + n] = 2.0 * uen[n] - uep[n] + sde * (double)Y[g.N + n];
}

inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// ------------------------------------------------------------------ host
static const int kCin[4] = {4, 16, 16, 16};
static const int kCout[4] = {16, 16, 16, 2};

long Predictor::n_params() {
    long s = 0;
    for (int L = 0; L < 4; ++L) s += (long)kCout[L] * kCin[L] * 27 + kCout[L];
    return s;
}

std::string Predictor::init(int64_t N_, int nx1, int ny1, int nz1, void* (*alloc)(void*, size_t), void* ctx) {
    g = CnnGrid{nx1, ny1, nz1, N_};
    const int64_t N = N_;
    auto A = [&](size_t bytes) { return alloc(ctx, bytes); };
    X0 = (__half*)A(4 * N * sizeof(__half));
    for (int L = 0; L < 3; ++L) {
        Z[L] = (__half*)A(16 * N * sizeof(__half));
        H[L] = (__half*)A(16 * N * sizeof(__half));
    }
    Y = (float*)A(2 * N * sizeof(float));
    G0 = (float*)A(16 * N * sizeof(float));
    G1 = (float*)A(16 * N * sizeof(float));
    const long np = n_params();
    w32 = (float*)A(np * sizeof(float));
    mom1 = (float*)A(np * sizeof(float));
    mom2 = (float*)A(np * sizeof(float));
    grad = (float*)A(np * sizeof(float));
    wh = (__half*)A(np * sizeof(__half));
    bias = (float*)A(64 * sizeof(float));
    nchunk = (int)std::min<int64_t>(2048, std::max<int64_t>(1, N / 128));
    chunk = (N + nchunk - 1) / nchunk;
    part = (float*)A((size_t)nchunk * (16 * 16 * 27 + 16) * sizeof(float));
    lpart = (double*)A(1024 * sizeof(double));
    std::vector<int> isb(np, 0), bpos(np, 0);
    long off = 0;
    int boff = 0;
    for (int L = 0; L < 4; ++L) {
        woff[L] = off;
        off += (long)kCout[L] * kCin[L] * 27;
        boff_[L] = boff;
        for (int c = 0; c < kCout[L]; ++c) {
            isb[off + c] = 1;
            bpos[off + c] = boff + c;
        }
        off += kCout[L];
        boff += kCout[L];
    }
    is_bias = (int*)A(np * sizeof(int));
    bias_pos = (int*)A(np * sizeof(int));
    if (!X0 || !Y || !G0 || !G1 || !w32 || !mom1 || !mom2 || !grad || !wh || !bias || !part || !lpart || !is_bias ||
        !bias_pos)
        return "device allocation failed (predictor)";
    for (int L = 0; L < 3; ++L)
        if (!Z[L] || !H[L]) return "device allocation failed (predictor)";
    hipMemcpy(is_bias, isb.data(), np * sizeof(int), hipMemcpyHostToDevice);
    hipMemcpy(bias_pos, bpos.data(), np * sizeof(int), hipMemcpyHostToDevice);
    ready = true;
    return "";
}

void Predictor::set(hipStream_t s, const float* host_params, const double sc[kScales]) {
    const long np = n_params();
    std::vector<__half> h(np);
    std::vector<float> b(64, 0.0f);
    for (int L = 0; L < 4; ++L) {
        const long nw = (long)kCout[L] * kCin[L] * 27;
        for (long q = 0; q < nw; ++q) h[woff[L] + q] = __float2half(host_params[woff[L] + q]);
        for (int c = 0; c < kCout[L]; ++c) b[boff_[L] + c] = host_params[woff[L] + nw + c];
    }
    hipMemcpyAsync(w32, host_params, np * sizeof(float), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(wh, h.data(), np * sizeof(__half), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(bias, b.data(), 64 * sizeof(float), hipMemcpyHostToDevice, s);
    hipMemsetAsync(mom1, 0, np * sizeof(float), s);
    hipMemsetAsync(mom2, 0, np * sizeof(float), s);
    hipStreamSynchronize(s);
    for (int q = 0; q < kScales; ++q) scale[q] = sc[q];
    adam_t = 0;
    has_weights = true;
}

void Predictor::get(hipStream_t s, float* host_params, double sc[kScales]) {
    hipMemcpyAsync(host_params, w32, n_params() * sizeof(float), hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    for (int q = 0; q < kScales; ++q) sc[q] = scale[q];
}

void Predictor::forward(hipStream_t s, const double* vn, const double* uen, const double* vp, const double* uep) {
    const int64_t N = g.N;
    hipLaunchKernelGGL(k_cnn_input, dim3(nb(N, 256)), dim3(256), 0, s, g, vn, uen, vp, uep, scale[0], scale[1],
                       scale[2], scale[3], X0);
    const dim3 grid(nb(g.nx1, BX), nb(g.ny1, BY), g.nz1), blk(BX, BY);
    hipLaunchKernelGGL((k_conv_fwd<4, 16, true>), grid, blk, 0, s, g, X0, wh + woff[0], bias + boff_[0], Z[0], H[0],
                       nullptr);
    hipLaunchKernelGGL((k_conv_fwd<16, 16, true>), grid, blk, 0, s, g, H[0], wh + woff[1], bias + boff_[1], Z[1],
                       H[1], nullptr);
    hipLaunchKernelGGL((k_conv_fwd<16, 16, true>), grid, blk, 0, s, g, H[1], wh + woff[2], bias + boff_[2], Z[2],
                       H[2], nullptr);
    hipLaunchKernelGGL((k_conv_fwd<16, 2, false>), grid, blk, 0, s, g, H[2], wh + woff[3], bias + boff_[3], nullptr,
                       nullptr, Y);
}

// Inference on MFMA, node-major activations in the training buffers X0,
// H[0] and H[1] (training rewrites them on its next forward pass).
void Predictor::forward_mfma(hipStream_t s, const double* vn, const double* uen, const double* vp,
                             const double* uep) {
    const int64_t N = g.N;
    hipLaunchKernelGGL(k_cnn_input_nm, dim3(nb(N, 256)), dim3(256), 0, s, g, vn, uen, vp, uep, scale[0], scale[1],
                       scale[2], scale[3], X0);
    const int ngx = (g.nx1 + 15) / 16;
    const int64_t ngroups = (int64_t)ngx * g.ny1 * g.nz1;
    const int64_t per_wg = (int64_t)CM_WAVES * CM_G;
    const dim3 grid((unsigned)std::min<int64_t>((ngroups + per_wg - 1) / per_wg, 4096)), blk(64 * CM_WAVES);
    hipLaunchKernelGGL((k_conv_mfma<4, 16, true>), grid, blk, 0, s, g, ngx, ngroups, X0, wh + woff[0],
                       bias + boff_[0], H[0], nullptr);
    hipLaunchKernelGGL((k_conv_mfma<16, 16, true>), grid, blk, 0, s, g, ngx, ngroups, H[0], wh + woff[1],
                       bias + boff_[1], H[1], nullptr);
    hipLaunchKernelGGL((k_conv_mfma<16, 16, true>), grid, blk, 0, s, g, ngx, ngroups, H[1], wh + woff[2],
                       bias + boff_[2], H[0], nullptr);
    hipLaunchKernelGGL((k_conv_mfma<16, 2, false>), grid, blk, 0, s, g, ngx, ngroups, H[0], wh + woff[3],
                       bias + boff_[3], nullptr, Y);
}

void Predictor::guess(hipStream_t s, const double* vn, const double* uen, const double* vp, const double* uep,
                      double* out) {
    forward_mfma(s, vn, uen, vp, uep);
    hipLaunchKernelGGL(k_cnn_guess, dim3(nb(g.N, 256)), dim3(256), 0, s, g, vn, uen, vp, uep, Y, scale[4], scale[5],
                       out);
}

template <int CIN, int COUT>
static void wgrad(hipStream_t s, const CnnGrid& g, const float* Gout, const __half* X, int nchunk, int64_t chunk,
                  float* part, float* dst) {
    constexpr int NW = COUT * CIN * 27 + COUT;
    hipLaunchKernelGGL((k_conv_bwd_w<CIN, COUT>), dim3(nchunk), dim3(256), 0, s, g, Gout, X, chunk, part);
    hipLaunchKernelGGL(k_sum_chunks, dim3(nb(NW, 256)), dim3(256), 0, s, nchunk, NW, part, dst);
}

// Loss and gradient of one sample s6 = [v^n, u_e^n, v^{n-1}, u_e^{n-1}, v^{n+1}, u_e^{n+1}].
double Predictor::loss_grad(hipStream_t s, const double* s6) {
    const int64_t N = g.N;
    forward(s, s6, s6 + N, s6 + 2 * N, s6 + 3 * N);
    const int nbl = 1024;
    hipLaunchKernelGGL(k_mse, dim3(nbl), dim3(256), 0, s, g, Y, s6, scale[4], scale[5], G0, lpart);
    const dim3 grid(nb(g.nx1, BX), nb(g.ny1, BY), g.nz1), blk(BX, BY);
    // layer 4 (16 -> 2): G0 holds dL/dY (2 channels)
    wgrad<16, 2>(s, g, G0, H[2], nchunk, chunk, part, grad + woff[3]);
    hipLaunchKernelGGL((k_conv_bwd_data<16, 2, true>), grid, blk, 0, s, g, G0, wh + woff[3], Z[2], G1);
    wgrad<16, 16>(s, g, G1, H[1], nchunk, chunk, part, grad + woff[2]);
    hipLaunchKernelGGL((k_conv_bwd_data<16, 16, true>), grid, blk, 0, s, g, G1, wh + woff[2], Z[1], G0);
    wgrad<16, 16>(s, g, G0, H[0], nchunk, chunk, part, grad + woff[1]);
    hipLaunchKernelGGL((k_conv_bwd_data<16, 16, true>), grid, blk, 0, s, g, G0, wh + woff[1], Z[0], G1);
    wgrad<4, 16>(s, g, G1, X0, nchunk, chunk, part, grad + woff[0]);
    std::vector<double> lp(nbl);
    hipMemcpyAsync(lp.data(), lpart, nbl * sizeof(double), hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    double l = 0.0;
    for (double x : lp) l += x;
    return l / (2.0 * (double)N);
}

double Predictor::train_step(hipStream_t s, const double* s6, double lr) {
    const double l = loss_grad(s, s6);
    ++adam_t;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)adam_t), c2 = 1.0f - std::pow(b2, (float)adam_t);
    const long np = n_params();
    hipLaunchKernelGGL(k_adam, dim3(nb(np, 256)), dim3(256), 0, s, (int)np, w32, mom1, mom2, grad, (float)lr, b1, b2,
                       1e-8f, c1, c2, wh, bias, is_bias, bias_pos);
    return l;
}

}  // namespace bdm
