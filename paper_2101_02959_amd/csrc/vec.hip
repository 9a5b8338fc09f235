// FP64 vector kernels of the Krylov and Newton loops.  Dot products use a
// fixed two-stage reduction (per-block partial sums, then one block), so
// they are deterministic.
#include "bddc_kernels.hpp"
#include "common.hpp"
#include "pcg_slots.hpp"

namespace bdm {

constexpr int kDotBlocks = 1024;
int dot_partials() { return kDotBlocks; }

namespace {

__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline double block_sum(double v) {
    __shared__ double red[kWG / 64];
    v = wsum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int q = 0; q < kWG / 64; ++q) t += red[q];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(kWG) void k_dot_partial(int64_t n, const double* __restrict__ x,
                                                    const double* __restrict__ y, double* __restrict__ part) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG)
        acc = fma(x[i], y[i], acc);
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kWG) void k_sum_partials(int np, const double* __restrict__ part,
                                                     double* __restrict__ out) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += kWG) acc += part[i];
    acc = block_sum(acc);
    if (threadIdx.x == 0) out[0] = acc;
}

__global__ void k_axpy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = fma(a, x[i], y[i]);
}

__global__ void k_scale_add(int64_t n, const double* __restrict__ z, double b, double* __restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = fma(b, p[i], z[i]);
}

__global__ void k_sub_scalar(int64_t n, const double* __restrict__ sum, double* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] -= sum[0] / (double)n;
}

__global__ __launch_bounds__(kWG) void k_sum_partial(int64_t n, const double* __restrict__ x,
                                                    double* __restrict__ part) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG)
        acc += x[i];
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Device-scalar variants for the graph-captured Krylov iteration.
__global__ void k_axpy_dev(int64_t n, const double* __restrict__ a, double sgn, const double* __restrict__ x,
                           double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = fma(sgn * a[0], x[i], y[i]);
}

__global__ void k_scale_add_dev(int64_t n, const double* __restrict__ z, const double* __restrict__ b,
                                double* __restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = fma(b[0], p[i], z[i]);
}

__global__ void k_fill(int64_t n, double v, double* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

template <typename T>
__global__ void k_fill_t(int64_t n, T v, T* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ void k_copy(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

// PCG scalar steps on device (slots in pcg_slots.hpp order).  Once the state
// is no longer PCG_RUNNING the iteration is frozen: alpha = beta = 0, so a
// replay after the stop leaves x and r unchanged.
__global__ void k_pcg_alpha(double* __restrict__ sc) {
    // a breakdown (p . q = 0) gives a non-finite alpha and residual, which the
    // check below reports as divergence, as the host-driven loop does
    sc[PCG_ALPHA] = (sc[PCG_STATE] == PCG_RUNNING) ? sc[PCG_RZ] / sc[PCG_PQ] : 0.0;
}

__global__ void k_pcg_check(double* __restrict__ sc, double* __restrict__ hist, double* __restrict__ ah,
                            int maxit) {
    if (sc[PCG_STATE] != PCG_RUNNING) return;
    const int it = (int)sc[PCG_IT];
    const double rn = sqrt(sc[PCG_RN2]);
    ah[it] = sc[PCG_ALPHA];
    hist[it + 1] = rn;
    sc[PCG_IT] = it + 1;
    if (!(rn == rn) || rn > sc[PCG_DTOL]) sc[PCG_STATE] = PCG_DIVERGED;
    else if (rn <= sc[PCG_TOL]) sc[PCG_STATE] = PCG_CONVERGED;
    else if (it + 1 >= maxit) sc[PCG_STATE] = PCG_MAXIT;
}

__global__ void k_pcg_beta(double* __restrict__ sc, double* __restrict__ bh) {
    double b = 0.0;
    if (sc[PCG_STATE] == PCG_RUNNING) {
        // Polak-Ribiere: (z_new . r_new - z_new . r_old) / (z_old . r_old)
        b = (sc[PCG_ZR] - sc[PCG_ZRO]) / sc[PCG_RZ];
        sc[PCG_RZ] = sc[PCG_ZR];
        bh[(int)sc[PCG_IT] - 1] = b;
    }
    sc[PCG_BETA] = b;
}

}  // namespace

static inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_axpy_dev(hipStream_t s, int64_t n, const double* a, double sgn, const double* x, double* y) {
    hipLaunchKernelGGL(k_axpy_dev, dim3(nb(n, 256)), dim3(256), 0, s, n, a, sgn, x, y);
}
void launch_scale_add_dev(hipStream_t s, int64_t n, const double* z, const double* b, double* p) {
    hipLaunchKernelGGL(k_scale_add_dev, dim3(nb(n, 256)), dim3(256), 0, s, n, z, b, p);
}
void launch_fill(hipStream_t s, int64_t n, double v, double* x) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(nb(n, 256)), dim3(256), 0, s, n, v, x);
}
template <typename T>
void launch_fill_t(hipStream_t s, int64_t n, T v, T* x) {
    if (n > 0) hipLaunchKernelGGL(k_fill_t<T>, dim3(nb(n, 256)), dim3(256), 0, s, n, v, x);
}
template void launch_fill_t<float>(hipStream_t, int64_t, float, float*);
template void launch_fill_t<double>(hipStream_t, int64_t, double, double*);
void launch_copy_kernel(hipStream_t s, int64_t n, const double* x, double* y) {
    if (n > 0) hipLaunchKernelGGL(k_copy, dim3(nb(n, 256)), dim3(256), 0, s, n, x, y);
}
void launch_pcg_alpha(hipStream_t s, double* sc) { hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(1), 0, s, sc); }
void launch_pcg_check(hipStream_t s, double* sc, double* hist, double* ah, int maxit) {
    hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(1), 0, s, sc, hist, ah, maxit);
}
void launch_pcg_beta(hipStream_t s, double* sc, double* bh) {
    hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(1), 0, s, sc, bh);
}

void launch_dot(hipStream_t s, int64_t n, const double* x, const double* y, double* partial, double* out) {
    hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(kWG), 0, s, n, x, y, partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kWG), 0, s, kDotBlocks, partial, out);
}
void launch_axpy(hipStream_t s, int64_t n, double a, const double* x, double* y) {
    hipLaunchKernelGGL(k_axpy, dim3(nb(n, 256)), dim3(256), 0, s, n, a, x, y);
}
void launch_copy(hipStream_t s, int64_t n, const double* x, double* y) {
    hipMemcpyAsync(y, x, n * sizeof(double), hipMemcpyDeviceToDevice, s);
}
void launch_scale_add(hipStream_t s, int64_t n, const double* z, double b, double* p) {
    hipLaunchKernelGGL(k_scale_add, dim3(nb(n, 256)), dim3(256), 0, s, n, z, b, p);
}
// x <- x - mean(x)
void launch_sub_mean(hipStream_t s, int64_t n, double* x, double* partial, double* tmp) {
    hipLaunchKernelGGL(k_sum_partial, dim3(kDotBlocks), dim3(kWG), 0, s, n, x, partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kWG), 0, s, kDotBlocks, partial, tmp);
    hipLaunchKernelGGL(k_sub_scalar, dim3(nb(n, 256)), dim3(256), 0, s, n, tmp, x);
}

}  // namespace bdm
