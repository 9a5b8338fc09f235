// FP64 vector kernels of the Krylov and Newton loops.
//
// Reductions are single launches: each workgroup sums its grid-stride share
// (64-lane shuffles, then the four waves in order) and stores a partial; the
// last workgroup to take a ticket (an integer atomic) adds the partials in
// workgroup order and writes the total.  The order of every floating-point
// addition is fixed by the grid size alone, so results are deterministic.
// The ticket is back at zero when the kernel ends, so the kernels can be
// replayed from a captured graph without a reset.
//
// One PCG iteration (Sec. 4.1 CG on the Newton system, or on the FETI-DP
// multiplier system, Sec. 4.3) is, besides the operator and the
// preconditioner: p.q (one pass), the fused update x += alpha p,
// r -= alpha q with ||r||^2 and the stopping test (one pass), the fused
// z.r and z.q with the Polak-Ribiere beta = -alpha (z.q) / (z_old.r_old)
// (one pass; r_new - r_old = -alpha q, so r_old need not be kept), and
// p = z + beta p.  The scalars live in device slots (pcg_slots.hpp).
#include "bddc_kernels.hpp"
#include "common.hpp"
#include "pcg_slots.hpp"

namespace bdm {

constexpr int kVecBlocks = 2048;   // workgroups of the reducing kernels
int dot_partials() { return 2 * kVecBlocks; }
int vec_tickets() { return 4; }
enum { TK_DOT = 0, TK_UPDATE = 1, TK_BETA = 2, TK_SUM = 3 };

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

// K workgroup partial sums: stored at part[k * gridDim.x + blockIdx.x]; the
// last workgroup to arrive returns true with the K totals in tot (in every
// one of its threads).  Every thread of the workgroup calls it.
template <int K>
__device__ bool reduce_last(const double (&acc)[K], double* __restrict__ part, unsigned* __restrict__ ticket,
                            double (&tot)[K]) {
    __shared__ double red[K][kWG / 64];
    __shared__ int last;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double v = wsum(acc[k]);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = 0.0;
            for (int q = 0; q < kWG / 64; ++q) t += red[k][q];
            part[(int64_t)k * gridDim.x + blockIdx.x] = t;
        }
        __threadfence();                               // partials visible device-wide
        last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();                                   // see every workgroup's partial
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double a = 0.0;
        for (int i = threadIdx.x; i < (int)gridDim.x; i += kWG)
            a += __hip_atomic_load(part + (int64_t)k * gridDim.x + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        tot[k] = block_sum(a);
    }
    if (threadIdx.x == 0) atomicExch(ticket, 0u);
    return true;
}

__global__ __launch_bounds__(kWG) void k_dot(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                                            double* __restrict__ part, unsigned* __restrict__ ticket,
                                            double* __restrict__ out) {
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG)
        acc[0] = fma(x[i], y[i], acc[0]);
    double tot[1];
    if (reduce_last<1>(acc, part, ticket, tot) && threadIdx.x == 0) out[0] = tot[0];
}

__global__ __launch_bounds__(kWG) void k_sum(int64_t n, const double* __restrict__ x, double* __restrict__ part,
                                            unsigned* __restrict__ ticket, double* __restrict__ out) {
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG)
        acc[0] += x[i];
    double tot[1];
    if (reduce_last<1>(acc, part, ticket, tot) && threadIdx.x == 0) out[0] = tot[0];
}

// x += alpha p, r -= alpha q with alpha = (z.r) / (p.q) from the slots, then
// ||r||^2 and the stopping test: the iteration count, residual and alpha
// histories and the state (diverged on a non-finite or too large residual,
// converged, iteration limit).  Once the state is not PCG_RUNNING the
// kernel leaves x, r and the slots unchanged.
__global__ __launch_bounds__(kWG) void k_pcg_update(int64_t n, double* __restrict__ sc, const double* __restrict__ p,
                                                   const double* __restrict__ q, double* __restrict__ x,
                                                   double* __restrict__ r, double* __restrict__ part,
                                                   unsigned* __restrict__ ticket, double* __restrict__ hist,
                                                   double* __restrict__ ah, int maxit) {
    const bool run = sc[PCG_STATE] == PCG_RUNNING;
    // a breakdown (p . q = 0) gives a non-finite alpha and residual, which the
    // test reports as divergence
    const double alpha = run ? sc[PCG_RZ] / sc[PCG_PQ] : 0.0;
    double acc[1] = {0.0};
    if (run) {
        for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG) {
            x[i] = fma(alpha, p[i], x[i]);
            const double ri = fma(-alpha, q[i], r[i]);
            r[i] = ri;
            acc[0] = fma(ri, ri, acc[0]);
        }
    }
    double tot[1];
    if (reduce_last<1>(acc, part, ticket, tot) && threadIdx.x == 0 && run) {
        const int it = (int)sc[PCG_IT];
        const double rn = sqrt(tot[0]);
        sc[PCG_ALPHA] = alpha;
        sc[PCG_RN2] = tot[0];
        ah[it] = alpha;
        hist[it + 1] = rn;
        sc[PCG_IT] = it + 1;
        if (!(rn == rn) || rn > sc[PCG_DTOL]) sc[PCG_STATE] = PCG_DIVERGED;
        else if (rn <= sc[PCG_TOL]) sc[PCG_STATE] = PCG_CONVERGED;
        else if (it + 1 >= maxit) sc[PCG_STATE] = PCG_MAXIT;
    }
}

// z.r and z.q in one pass, then the Polak-Ribiere beta
//   z_new.(r_new - r_old) / (z_old.r_old) = -alpha (z_new.q) / (z_old.r_old)
// (r_new = r_old - alpha q), its history, and z.r for the next alpha.
__global__ __launch_bounds__(kWG) void k_pcg_beta(int64_t n, double* __restrict__ sc, const double* __restrict__ z,
                                                 const double* __restrict__ r, const double* __restrict__ q,
                                                 double* __restrict__ part, unsigned* __restrict__ ticket,
                                                 double* __restrict__ bh) {
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG) {
        const double zi = z[i];
        acc[0] = fma(zi, r[i], acc[0]);
        acc[1] = fma(zi, q[i], acc[1]);
    }
    double tot[2];
    if (reduce_last<2>(acc, part, ticket, tot) && threadIdx.x == 0) {
        double b = 0.0;
        if (sc[PCG_STATE] == PCG_RUNNING) {
            b = -sc[PCG_ALPHA] * tot[1] / sc[PCG_RZ];
            sc[PCG_RZ] = tot[0];
            bh[(int)sc[PCG_IT] - 1] = b;
        }
        sc[PCG_ZR] = tot[0];
        sc[PCG_ZQ] = tot[1];
        sc[PCG_BETA] = b;
    }
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
void launch_pcg_update(hipStream_t s, int64_t n, double* sc, const double* p, const double* q, double* x, double* r,
                       double* partial, unsigned* tickets, double* hist, double* ah, int maxit) {
    hipLaunchKernelGGL(k_pcg_update, dim3(kVecBlocks), dim3(kWG), 0, s, n, sc, p, q, x, r, partial,
                       tickets + TK_UPDATE, hist, ah, maxit);
}
void launch_pcg_beta(hipStream_t s, int64_t n, double* sc, const double* z, const double* r, const double* q,
                     double* partial, unsigned* tickets, double* bh) {
    hipLaunchKernelGGL(k_pcg_beta, dim3(kVecBlocks), dim3(kWG), 0, s, n, sc, z, r, q, partial, tickets + TK_BETA, bh);
}

void launch_dot(hipStream_t s, int64_t n, const double* x, const double* y, double* partial, unsigned* tickets,
                double* out) {
    hipLaunchKernelGGL(k_dot, dim3(kVecBlocks), dim3(kWG), 0, s, n, x, y, partial, tickets + TK_DOT, out);
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
void launch_sub_mean(hipStream_t s, int64_t n, double* x, double* partial, unsigned* tickets, double* tmp) {
    hipLaunchKernelGGL(k_sum, dim3(kVecBlocks), dim3(kWG), 0, s, n, x, partial, tickets + TK_SUM, tmp);
    hipLaunchKernelGGL(k_sub_scalar, dim3(nb(n, 256)), dim3(256), 0, s, n, tmp, x);
}

}  // namespace bdm
