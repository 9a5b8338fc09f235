// FP64 coarse problem of BDDC / FETI-DP (paper Sec. 4.4): the assembled
// primal matrix S_PiPi over vertex values and edge averages.
//
// Ordered by position along x in the subdomain grid (the cut plane a and the
// slab a of x-edges form group a), S_PiPi is block tridiagonal: a subdomain
// in slab a only couples primal unknowns of groups a and a+1.  The solver
// uses the block LDL^T factorisation with explicit inverses of the block
// pivots,
//     Dt_0 = D_0,  C_g = E_g Dt_{g-1}^{-1},  Dt_g = D_g - C_g E_g^T,
// so every per-iteration solve is a sequence of dense GEMVs:
//     y_g = b_g - C_g y_{g-1},  z_g = Dt_g^{-1} y_g,  x_g = z_g - C_{g+1}^T x_{g+1}.
// The pivot inverses come from the block sweep (Gauss-Jordan) operator,
// which for an SPD matrix needs no pivoting.  All kernels are multi-workgroup.
#include <algorithm>
#include <vector>

#include "coarse.hpp"

namespace bdm {

namespace {

constexpr int TB = 64;     // GEMM tile
constexpr int TK = 32;     // GEMM k-step
constexpr int SB = 64;     // sweep block
constexpr int GV_ROWS = 256, GV_COLS = 128;   // GEMV stage-1 tile

typedef double f64x4 __attribute__((ext_vector_type(4)));

// C = beta C + alpha op(A) op(B); column-major; op = transpose when flag set.
// 64x64 tile per workgroup, k staged through LDS; each wave owns a 32x32
// quarter computed with 2x2 MFMA f64 16x16x4 blocks.  Operand lanes: A lane l
// holds A[l%16][l/16], B lane l holds B[l/16][l%16]; accumulator register v
// of lane l holds row l/16 + 4v of column l%16.
__global__ __launch_bounds__(256) void k_gemm(int m, int n, int k, double alpha, const double* __restrict__ A,
                                              int64_t lda, int ta, const double* __restrict__ B, int64_t ldb,
                                              int tb, double beta, double* __restrict__ C, int64_t ldc) {
    __shared__ double As[TK][TB + 1];
    __shared__ double Bs[TK][TB + 1];
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    const int wr = wv & 1, wc = wv >> 1;
    const int i0 = blockIdx.x * TB, j0 = blockIdx.y * TB;
    f64x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (f64x4){0, 0, 0, 0};
    for (int kk = 0; kk < k; kk += TK) {
        for (int idx = tid; idx < TK * TB; idx += 256) {
            int r, c;
            if (ta) { c = idx % TK; r = idx / TK; } else { r = idx % TB; c = idx / TB; }
            const int gi = i0 + r, gk = kk + c;
            double a = 0.0;
            if (gi < m && gk < k) a = ta ? A[gk + (int64_t)gi * lda] : A[gi + (int64_t)gk * lda];
            As[c][r] = a;
        }
        for (int idx = tid; idx < TK * TB; idx += 256) {
            int r, c;
            if (tb) { r = idx % TB; c = idx / TB; } else { c = idx % TK; r = idx / TK; }
            const int gj = j0 + r, gk = kk + c;
            double b = 0.0;
            if (gj < n && gk < k) b = tb ? B[gj + (int64_t)gk * ldb] : B[gk + (int64_t)gj * ldb];
            Bs[c][r] = b;
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < TK; c += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                av[q] = As[c + lk][wr * 32 + 16 * q + lr];
                bv[q] = Bs[c + lk][wc * 32 + 16 * q + lr];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int gj = j0 + wc * 32 + 16 * b + lr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = i0 + wr * 32 + 16 * a + lk + 4 * v;
                if (gi < m && gj < n) {
                    double* cp = C + gi + (int64_t)gj * ldc;
                    *cp = (beta == 0.0 ? 0.0 : beta * *cp) + alpha * acc[a][b][v];
                }
            }
        }
}

// Stage 1 of y = A x (A m x n): partial sums over column chunks of GV_COLS,
// threads along rows (coalesced); stage 2 adds the partials in a fixed order.
__global__ __launch_bounds__(GV_ROWS) void k_gemv_part(int m, int n, const double* __restrict__ A, int64_t lda,
                                                        const double* __restrict__ x, double* __restrict__ part) {
    __shared__ double xs[GV_COLS];
    const int c0 = blockIdx.y * GV_COLS;
    const int cn = min(GV_COLS, n - c0);
    for (int t = threadIdx.x; t < cn; t += GV_ROWS) xs[t] = x[c0 + t];
    __syncthreads();
    const int i = blockIdx.x * GV_ROWS + threadIdx.x;
    if (i >= m) return;
    const double* a = A + i + (int64_t)c0 * lda;
    double acc0 = 0.0, acc1 = 0.0;
    int j = 0;
    for (; j + 1 < cn; j += 2) {
        acc0 = fma(a[(int64_t)j * lda], xs[j], acc0);
        acc1 = fma(a[(int64_t)(j + 1) * lda], xs[j + 1], acc1);
    }
    if (j < cn) acc0 = fma(a[(int64_t)j * lda], xs[j], acc0);
    part[(int64_t)blockIdx.y * m + i] = acc0 + acc1;
}

__global__ void k_gemv_sum(int m, int nchunk, double alpha, const double* __restrict__ part, double beta,
                           double* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * m + i];
    y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + alpha * s;
}

// y = beta y + alpha op(A) x, one wave per output row block; deterministic.
__global__ __launch_bounds__(256) void k_gemv(int m, int n, double alpha, const double* __restrict__ A,
                                              int64_t lda, int ta, const double* __restrict__ x, double beta,
                                              double* __restrict__ y) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (!ta) {
        // y_i = sum_j A[i + j lda] x_j: threads over rows (coalesced), 4 waves split j
        __shared__ double part[4][64];
        const int i = blockIdx.x * 64 + lane;
        double acc = 0.0;
        if (i < m)
            for (int j = wv; j < n; j += 4) acc = fma(A[i + (int64_t)j * lda], x[j], acc);
        part[wv][lane] = acc;
        __syncthreads();
        if (wv == 0 && i < m) {
            const double s = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
            y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + alpha * s;
        }
    } else {
        // y_j = sum_i A[i + j lda] x_i: one wave per column, lanes over i
        const int j = blockIdx.x * 4 + wv;
        if (j >= m) return;
        double acc = 0.0;
        for (int i = lane; i < n; i += 64) acc = fma(A[i + (int64_t)j * lda], x[i], acc);
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) y[j] = (beta == 0.0 ? 0.0 : beta * y[j]) + alpha * acc;
    }
}

// B = inverse of the SB x SB diagonal block of A at (k0, k0) (size kb),
// by the sweep operator in LDS; writes B (kb x kb, ld SB).
__global__ __launch_bounds__(256) void k_block_inv(const double* __restrict__ A, int64_t lda, int k0, int kb,
                                                   double* __restrict__ B, int* __restrict__ info) {
    __shared__ double S[SB][SB + 1];
    const int tid = threadIdx.x;
    for (int idx = tid; idx < SB * SB; idx += 256) {
        const int i = idx % SB, j = idx / SB;
        S[i][j] = (i < kb && j < kb) ? A[(k0 + i) + (int64_t)(k0 + j) * lda] : (double)(i == j);
    }
    __syncthreads();
    for (int p = 0; p < kb; ++p) {
        const double d = S[p][p];
        __syncthreads();
        if (!(d > 0.0)) {
            if (tid == 0) info[0] = 1;
            return;
        }
        // sweep on pivot p: S_ij -= S_ip S_pj / d (i,j != p); S_ip /= d; S_pj /= d; S_pp = -1/d
        const double rd = 1.0 / d;
        double upd[SB * SB / 256];
        int cnt = 0;
        for (int idx = tid; idx < SB * SB; idx += 256, ++cnt) {
            const int i = idx % SB, j = idx / SB;
            const double v = S[i][j];
            upd[cnt] = (i != p && j != p) ? fma(-S[i][p], S[p][j] * rd, v) : ((i == p && j == p) ? -rd : v * rd);
        }
        __syncthreads();
        cnt = 0;
        for (int idx = tid; idx < SB * SB; idx += 256, ++cnt) S[idx % SB][idx / SB] = upd[cnt];
        __syncthreads();
    }
    // after sweeping every pivot S = -A^{-1}
    for (int idx = tid; idx < SB * SB; idx += 256) {
        const int i = idx % SB, j = idx / SB;
        B[i + j * SB] = -S[i][j];
    }
}

// After A -= T A[K,:]: A[:,K] = T, A[K,:] = T^T, A[K,K] = -B.
__global__ void k_sweep_fix(int n, double* __restrict__ A, int64_t lda, int k0, int kb,
                            const double* __restrict__ B, const double* __restrict__ T) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool inK = (i >= k0 && i < k0 + kb);
    for (int c = 0; c < kb; ++c) {
        const double t = inK ? -B[(i - k0) + c * SB] : T[i + (int64_t)c * n];
        A[i + (int64_t)(k0 + c) * lda] = t;
        A[(k0 + c) + (int64_t)i * lda] = t;
    }
}

__global__ void k_copy_rows(int n, const double* __restrict__ A, int64_t lda, int k0, int kb,
                            double* __restrict__ R) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    for (int c = 0; c < kb; ++c) R[c + (int64_t)j * SB] = A[(k0 + c) + (int64_t)j * lda];
}

__global__ void k_negate(int64_t n, double* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = -x[i];
}

// Assemble the local coarse matrices into the group blocks (one colour of
// subdomains per launch, so no two workgroups touch the same entry).
__global__ void k_assemble_blocks(const int* __restrict__ list, const int* __restrict__ nPv,
                                  const int64_t* __restrict__ P_off, const int* __restrict__ primal,
                                  const double* __restrict__ Sp, int sp_stride, CoarseMap cm,
                                  double* __restrict__ D, double* __restrict__ E) {
    const int s = list[blockIdx.x];
    const int nP = nPv[s];
    const int* pr = primal + P_off[s];
    const double* S = Sp + (int64_t)s * sp_stride;
    for (int idx = threadIdx.x; idx < nP * nP; idx += blockDim.x) {
        const int a = idx % nP, b = idx / nP;
        const int p = pr[a], q = pr[b];
        if (p == cm.pin || q == cm.pin) continue;
        const int gp = cm.grp[p], gq = cm.grp[q];
        const int ip = cm.pos[p], iq = cm.pos[q];
        if (gp == gq) D[cm.D_off[gp] + ip + (int64_t)iq * cm.ng[gp]] += S[a + b * nP];
        else if (gp == gq + 1) E[cm.E_off[gp] + ip + (int64_t)iq * cm.ng[gp]] += S[a + b * nP];
    }
}

__global__ void k_set_diag_one(double* __restrict__ D, int64_t idx) { D[idx] = 1.0; }

// Gather / scatter between the global primal numbering and group order.
__global__ void k_perm(int np, const int* __restrict__ grp, const int* __restrict__ pos,
                       const int64_t* __restrict__ goff, const double* __restrict__ in, double* __restrict__ out,
                       int to_groups) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int64_t k = goff[grp[p]] + pos[p];
    if (to_groups) out[k] = in[p];
    else out[p] = in[k];
}

inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void gemm(hipStream_t s, int m, int n, int k, double alpha, const double* A, int64_t lda, bool ta,
          const double* B, int64_t ldb, bool tb, double beta, double* C, int64_t ldc) {
    if (m <= 0 || n <= 0) return;
    dim3 grid(nb(m, TB), nb(n, TB));
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, m, n, k, alpha, A, lda, (int)ta, B, ldb, (int)tb, beta, C,
                       ldc);
}

void gemv(hipStream_t s, int m, int n, double alpha, const double* A, int64_t lda, bool ta, const double* x,
          double beta, double* y, double* part) {
    // ta = false: y (m) = A (m x n) x;  ta = true: y (m) = A^T x with A (n x m)
    if (m <= 0) return;
    if (!ta) {
        const int nch = (n + GV_COLS - 1) / GV_COLS;
        if (nch == 0) {
            hipLaunchKernelGGL(k_gemv_sum, dim3(nb(m, 256)), dim3(256), 0, s, m, 0, alpha, part, beta, y);
            return;
        }
        hipLaunchKernelGGL(k_gemv_part, dim3(nb(m, GV_ROWS), nch), dim3(GV_ROWS), 0, s, m, n, A, lda, x, part);
        hipLaunchKernelGGL(k_gemv_sum, dim3(nb(m, 256)), dim3(256), 0, s, m, nch, alpha, part, beta, y);
    } else {
        hipLaunchKernelGGL(k_gemv, dim3(nb(m, 4)), dim3(256), 0, s, m, n, alpha, A, lda, 1, x, beta, y);
    }
}

// In-place inverse of an SPD matrix (n x n, ld) by block sweeps.
void spd_inverse(hipStream_t s, int n, double* A, int64_t lda, double* Bwork, double* Twork, double* Rwork,
                 int* info) {
    for (int k0 = 0; k0 < n; k0 += SB) {
        const int kb = std::min(SB, n - k0);
        hipLaunchKernelGGL(k_block_inv, dim3(1), dim3(256), 0, s, A, lda, k0, kb, Bwork, info);
        // T = A[:, K] B
        gemm(s, n, kb, kb, 1.0, A + (int64_t)k0 * lda, lda, false, Bwork, SB, false, 0.0, Twork, n);
        // R = A[K, :] copied out (kb x n, ld SB) so the in-place update reads no row it writes
        hipLaunchKernelGGL(k_copy_rows, dim3(nb(n, 256)), dim3(256), 0, s, n, A, lda, k0, kb, Rwork);
        // A -= T R
        gemm(s, n, n, kb, -1.0, Twork, n, false, Rwork, SB, false, 1.0, A, lda);
        hipLaunchKernelGGL(k_sweep_fix, dim3(nb(n, 256)), dim3(256), 0, s, n, A, lda, k0, kb, Bwork, Twork);
    }
    // sweeping every pivot leaves -A^{-1}
    hipLaunchKernelGGL(k_negate, dim3(nb((int64_t)n * lda, 256)), dim3(256), 0, s, (int64_t)n * lda, A);
}

void CoarseSolver::factor(hipStream_t s, const int* color_list, const std::vector<int>& color_ptr,
                          const int* nPv, const int64_t* P_off, const int* primal, const double* Sp,
                          int sp_stride) {
    hipMemsetAsync(D, 0, nD * sizeof(double), s);
    if (nE) hipMemsetAsync(E, 0, nE * sizeof(double), s);
    hipMemsetAsync(info, 0, sizeof(int), s);
    for (size_t c = 0; c + 1 < color_ptr.size(); ++c) {
        const int cnt = color_ptr[c + 1] - color_ptr[c];
        if (cnt == 0) continue;
        hipLaunchKernelGGL(k_assemble_blocks, dim3(cnt), dim3(256), 0, s, color_list + color_ptr[c], nPv, P_off,
                           primal, Sp, sp_stride, map(), D, E);
    }
    const int gp = grp[pin];
    hipLaunchKernelGGL(k_set_diag_one, dim3(1), dim3(1), 0, s, D, D_off[gp] + (int64_t)pos[pin] * (ng[gp] + 1));
    for (int g = 0; g < G; ++g) {
        double* Dg = D + D_off[g];
        if (g > 0) {
            double* Cg = Cb + E_off[g];
            const double* Eg = E + E_off[g];
            // C_g = E_g Dinv_{g-1};  D_g -= C_g E_g^T
            gemm(s, ng[g], ng[g - 1], ng[g - 1], 1.0, Eg, ng[g], false, D + D_off[g - 1], ng[g - 1], false, 0.0,
                 Cg, ng[g]);
            gemm(s, ng[g], ng[g], ng[g - 1], -1.0, Cg, ng[g], false, Eg, ng[g], true, 1.0, Dg, ng[g]);
        }
        spd_inverse(s, ng[g], Dg, ng[g], Bw, Tw, Rw, info);
    }
}

void CoarseSolver::solve(hipStream_t s, double* b) {
    hipLaunchKernelGGL(k_perm, dim3(nb(np, 256)), dim3(256), 0, s, np, d_grp, d_pos, d_goff, b, yb, 1);
    for (int g = 1; g < G; ++g)
        gemv(s, ng[g], ng[g - 1], -1.0, Cb + E_off[g], ng[g], false, yb + goff[g - 1], 1.0, yb + goff[g], Pw);
    for (int g = 0; g < G; ++g)
        gemv(s, ng[g], ng[g], 1.0, D + D_off[g], ng[g], false, yb + goff[g], 0.0, zb + goff[g], Pw);
    for (int g = G - 2; g >= 0; --g)
        gemv(s, ng[g], ng[g + 1], -1.0, Cb + E_off[g + 1], ng[g + 1], true, zb + goff[g + 1], 1.0, zb + goff[g], Pw);
    hipLaunchKernelGGL(k_perm, dim3(nb(np, 256)), dim3(256), 0, s, np, d_grp, d_pos, d_goff, zb, b, 0);
}

std::string CoarseSolver::init(const std::vector<int>& grp_of, int pin_, int np_) {
    np = np_;
    pin = pin_;
    G = 0;
    for (int g : grp_of) G = std::max(G, g + 1);
    ng.assign(G, 0);
    pos.assign(np, 0);
    grp = grp_of;
    for (int p = 0; p < np; ++p) pos[p] = ng[grp[p]]++;
    D_off.assign(G, 0);
    E_off.assign(G, 0);
    goff.assign(G, 0);
    int64_t accD = 0, accE = 0, accg = 0;
    maxn = 0;
    for (int g = 0; g < G; ++g) {
        D_off[g] = accD; accD += (int64_t)ng[g] * ng[g];
        E_off[g] = accE; if (g > 0) accE += (int64_t)ng[g] * ng[g - 1];
        goff[g] = accg; accg += ng[g];
        maxn = std::max(maxn, ng[g]);
    }
    nD = accD;
    nE = accE;
    return "";
}

}  // namespace bdm
