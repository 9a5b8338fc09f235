// Batched dense linear algebra for the subdomain-local problems of BDDC /
// FETI-DP (paper Sec. 4.1, 4.2, 4.4): local matrix assembly, partial
// Cholesky (which yields the Dirichlet factor, the Schur complement S_Gamma
// and the constrained Neumann factor from one local matrix), extraction of
// the deluxe blocks, triangular solves, the small coarse-space algebra and
// the deluxe face / edge factors.
//
// One workgroup owns one matrix; matrices are column-major with a per-matrix
// leading dimension.  Templates are instantiated for double (plain path) and
// float (local factors in FP32 under the FP64 outer iteration).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace bdm {

constexpr int NB = 32;          // panel / block width

namespace {

// 16x16x4 MFMA helpers.  Operand lanes (both precisions): A lane l holds
// A[l%16][l/16], B lane l holds B[l/16][l%16].  Accumulator register v of
// lane l holds row 4*(l/16)+v (f32) or row l/16+4v (f64) of column l%16.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename T> struct Mfma;
template <> struct Mfma<float> {
    typedef f32x4 acc;
    static __device__ inline acc mac(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mfma<double> {
    typedef f64x4 acc;
    static __device__ inline acc mac(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

// -------------------------------------------------------------- assembly
// K^(j) of the Jacobian bilinear form restricted to Omega_j (Sec. 4.1) in
// the congruent (v, u_e) form: per node pair (P, Q) the 2x2 block
//   [[a_i + d_P delta_PQ, a_i], [a_i, a_i + a_e]],
// a_* = (tau A_*^(j))_PQ from the elements of the subdomain only, and
// d_P = m_P^(j) (chi C_m + tau dI_ion/dv) with the local lumped mass (the
// corner masses of the subdomain's elements around P).
template <typename T>
__global__ void k_assemble(BatchDesc d, FEParams p, const double* __restrict__ ke,
                           const double* __restrict__ v, const double* __restrict__ w,
                           T* __restrict__ K) {
    const int s = d.sub0 + blockIdx.y;
    const int* bx = d.box + 6 * s;
    const int ex0 = bx[0], ey0 = bx[1], ez0 = bx[2], Lx = bx[3], Ly = bx[4], Lz = bx[5];
    const int nbox = (Lx + 1) * (Ly + 1) * (Lz + 1);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int P = t / 27, dd = t % 27;
    if (P >= nbox) return;
    const int pi = P % (Lx + 1), pj = (P / (Lx + 1)) % (Ly + 1), pk = P / ((Lx + 1) * (Ly + 1));
    const int dx = dd % 3 - 1, dy = (dd / 3) % 3 - 1, dz = dd / 9 - 1;
    const int qi = pi + dx, qj = pj + dy, qk = pk + dz;
    if (qi < 0 || qi > Lx || qj < 0 || qj > Ly || qk < 0 || qk > Lz) return;
    double ai = 0.0, ae = 0.0, mloc = 0.0;
    int nel = 0;
    for (int oz = 0; oz < 2; ++oz)
        for (int oy = 0; oy < 2; ++oy)
            for (int ox = 0; ox < 2; ++ox) {
                const int ei = pi - 1 + ox, ej = pj - 1 + oy, ek = pk - 1 + oz;
                if (ei < 0 || ei >= Lx || ej < 0 || ej >= Ly || ek < 0 || ek >= Lz) continue;
                ++nel;
                const int a = (1 - ox) + 2 * (1 - oy) + 4 * (1 - oz);
                // element matrices per z-layer (box mesh) or per element (mapped mesh)
                const size_t e = p.mec ? (size_t)(ex0 + ei) + (size_t)p.nx * ((ey0 + ej) + (size_t)p.ny * (ez0 + ek))
                                       : (size_t)(ez0 + ek);
                if (p.mec) mloc += p.mec[e * 8 + a];
                const int bxl = 1 - ox + dx, byl = 1 - oy + dy, bzl = 1 - oz + dz;
                if (bxl < 0 || bxl > 1 || byl < 0 || byl > 1 || bzl < 0 || bzl > 1) continue;
                const int b = bxl + 2 * byl + 4 * bzl;
                ai += ke[(e * 2 + 0) * 64 + a * 8 + b];
                ae += ke[(e * 2 + 1) * 64 + a * 8 + b];
            }
    double dP = 0.0;
    if (dd == 13) {
        const int64_t g = (int64_t)(ex0 + pi) + (int64_t)p.nx1 * ((ey0 + pj) + (int64_t)p.ny1 * (ez0 + pk));
        const double m = p.mec ? mloc : p.h * p.hy * p.hz * 0.125 * nel;
        dP = m * (p.c + p.tau * rmc_diion(p, v[g], w[g]));
    }
    const int* lm = d.lmap + d.lmap_off[s];
    const int lP = lm[P];
    const int lQ = lm[qi + (Lx + 1) * (qj + (Ly + 1) * qk)];
    const int64_t ld = d.n[s];
    T* A = K + d.K_off[s];
    const int64_t r0 = 2 * lP, c0 = 2 * lQ;
    A[r0 + c0 * ld] = (T)(ai + dP);
    A[r0 + (c0 + 1) * ld] = (T)ai;
    A[r0 + 1 + c0 * ld] = (T)ai;
    A[r0 + 1 + (c0 + 1) * ld] = (T)(ai + ae);
}

// ------------------------------------------------------ partial Cholesky
constexpr int NBO = 128;        // outer panel width

// C[i][j] -= sum_{k in [k0,k1)} A[i][k] A[j][k] for j in [cb, ce), i in [j, re),
// 32x32 tiles (lower trapezoid), one wave per tile, 2x2 MFMA 16x16x4 blocks.
template <typename T>
__device__ void syrk_update(T* __restrict__ A, int64_t ld, int cb, int ce, int re, int k0, int k1) {
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    const int nct = (ce - cb + 31) / 32, nrt = (re - cb + 31) / 32;
    // tiles (ti >= tj): column tj has nrt - tj tiles
    const int ntiles = nct * nrt - nct * (nct - 1) / 2;
    for (int tile = wv; tile < ntiles; tile += kWG / 64) {
        // locate (tj, ti): columns are laid out one after another
        int tj = 0, rem = tile;
        while (rem >= nrt - tj) { rem -= nrt - tj; ++tj; }
        const int ti = tj + rem;
        const int I0 = cb + ti * 32, J0 = cb + tj * 32;
        typename Mfma<T>::acc acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = (typename Mfma<T>::acc){0, 0, 0, 0};
        // 32 inner indices at a time: every operand load of the chunk is
        // issued (clamped addresses, masked values) before its MFMAs, so
        // the chunk waits for global memory once rather than per step
        for (int kb = k0; kb < k1; kb += 32) {
            T av[8][2], bv[8][2];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = kb + 4 * u + lk;
                const bool cin = c < k1;
                const T* col = A + (int64_t)(cin ? c : k0) * ld;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int ra = I0 + 16 * q + lr, rb = J0 + 16 * q + lr;
                    const T x = col[min(ra, re - 1)], y = col[min(rb, ce - 1)];
                    av[u][q] = (cin && ra < re) ? x : (T)0;
                    bv[u][q] = (cin && rb < ce) ? y : (T)0;
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (kb + 4 * u >= k1) break;
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        if (!(ti == tj && a < b)) acc[a][b] = Mfma<T>::mac(av[u][a], bv[u][b], acc[a][b]);
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                if (ti == tj && a < b) continue;
                const int j = J0 + 16 * b + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = I0 + 16 * a + Mfma<T>::row(lane, v);
                    if (i < re && j < ce && i >= j) A[i + (int64_t)j * ld] -= acc[a][b][v];
                }
            }
    }
}

// Right-looking blocked Cholesky of columns [c0, c1) of a symmetric matrix
// (lower triangle).  Rows [c1, c2) below the eliminated block receive the
// panel L_GI = K_GI L_II^{-T}; the trailing updates stop at column c1, so the
// block [c1, c2)^2 is left untouched: k_syrk_schur turns it into the Schur
// complement K_GG - L_GI L_GI^T = K_GG - K_GI K_II^{-1} K_IG (Sec. 4.1) in one
// pass with the full inner dimension.
template <typename T>
__device__ __forceinline__ void potrf_body(T* __restrict__ A, int64_t ld, int cbeg, int cend, int c2,
                                           int* __restrict__ info, T* __restrict__ Wout = nullptr) {
    const int s = blockIdx.x;
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    __shared__ T D[NB][NB + 1];     // diagonal block, then its Cholesky factor
    __shared__ T W[NB][NB + 1];     // inverse of the factor
    __shared__ int bad;
    if (tid == 0) bad = 0;
    int p0 = cbeg;                  // start of the current outer panel
    for (int j0 = cbeg; j0 < cend; j0 += NB) {
        const int jb = min(NB, cend - j0);
        // 1. factor the diagonal block in LDS (identity padding beyond jb)
        for (int idx = tid; idx < NB * NB; idx += kWG) {
            const int i = idx % NB, j = idx / NB;
            D[i][j] = (i < jb && j < jb && j <= i) ? A[(j0 + i) + (j0 + j) * ld] : (T)(i == j);
        }
        __syncthreads();
        // One barrier per pivot: step k updates the trailing block with the
        // unscaled column, a_ij -= a_ik a_jk / a_kk (every thread reads the
        // pivot itself), and the columns are scaled once at the end,
        // l_kk = sqrt(a_kk), l_ik = a_ik / l_kk.  A pivot that is not positive
        // flags the matrix and is replaced by 1.
        for (int k = 0; k < jb; ++k) {
            T dk = D[k][k];
            if (!(dk > (T)0)) dk = (T)1;
            const T rk = (T)1 / dk;
            // thread (row NB-slot, column group): no division by the
            // trailing size
            const int i = tid % NB;
            if (i > k && i < jb) {
                const T lik = D[i][k] * rk;
                for (int j = k + 1 + tid / NB; j <= i; j += kWG / NB) D[i][j] -= lik * D[j][k];
            }
            __syncthreads();
        }
        if (tid < NB) {
            T dk = D[tid][tid];
            if (tid < jb && !(dk > (T)0)) { bad = 1; dk = (T)1; }
            W[tid][0] = sqrt(dk);   // pivots (W is rewritten below)
        }
        __syncthreads();
        for (int idx = tid; idx < NB * NB; idx += kWG) {
            const int i = idx % NB, k = idx / NB;
            if (i > k) D[i][k] /= W[k][0];
        }
        __syncthreads();
        if (tid < NB) D[tid][tid] = W[tid][0];
        __syncthreads();
        // W = D^{-1} (lower triangular), one column per thread, the column
        // in registers (no store-to-load dependence through LDS)
        // W = D^{-1} (lower triangular) by forward substitution.  FP32: column
        // c by the 8 lanes 8c .. 8c + 7: lane t keeps W[k][c] for k = t (mod 8)
        // in registers; per row, the lanes' partial dots are summed by xor
        // shuffles and the owning lane keeps the new entry.  FP64: one thread
        // per column through LDS (the register form costs FP64 occupancy
        // here).
        static_assert(kWG == 8 * NB, "eight lanes per column of the inverse");
        if constexpr (sizeof(T) == 8) {
            if (tid < NB) {
                const int c = tid;
                for (int i = 0; i < NB; ++i) {
                    T acc = (i == c) ? (T)1 : (T)0;
                    for (int k = c; k < i; ++k) acc -= D[i][k] * W[k][c];
                    W[i][c] = (i >= c) ? acc / D[i][i] : (T)0;
                }
            }
        } else {
            const int c = tid / 8, t = tid % 8;
            T w[NB / 8];
#pragma unroll
            for (int q = 0; q < NB / 8; ++q) w[q] = (T)0;
#pragma unroll 1
            for (int i0 = 0; i0 < NB; i0 += 8) {
#pragma unroll
                for (int ii = 0; ii < 8; ++ii) {
                    const int i = i0 + ii;
                    T part = (T)0;
#pragma unroll
                    for (int q = 0; q < NB / 8; ++q)
                        if (8 * q + t < i) part += D[i][8 * q + t] * w[q];
                    part += __shfl_xor(part, 1);
                    part += __shfl_xor(part, 2);
                    part += __shfl_xor(part, 4);
                    const T wi = (i >= c) ? (((i == c) ? (T)1 : (T)0) - part) / D[i][i] : (T)0;
#pragma unroll
                    for (int q = 0; q < NB / 8; ++q) w[q] = (t == ii && 8 * q == i0) ? wi : w[q];
                }
            }
#pragma unroll
            for (int q = 0; q < NB / 8; ++q) W[8 * q + t][c] = w[q];
        }
        for (int idx = tid; idx < jb * jb; idx += kWG) {
            const int i = idx % jb, j = idx / jb;
            if (j <= i) A[(j0 + i) + (j0 + j) * ld] = D[i][j];
        }
        __syncthreads();
        if (Wout) {
            T* Wb = Wout + (int64_t)((j0 - cbeg) / NB) * NB * NB;
            for (int idx = tid; idx < NB * NB; idx += kWG) {
                const int i = idx % NB, j = idx / NB;
                Wb[i + j * NB] = (i < jb && j < jb) ? W[i][j] : (T)0;
            }
        }
        // 2. panel below the block: X = P W^T on MFMA, 16-row tiles per wave
        const int t0 = j0 + jb;
        const int nrt = (c2 - t0 + 15) / 16;
        for (int tile = wv; tile < nrt; tile += kWG / 64) {
            const int R0 = t0 + 16 * tile;
            typename Mfma<T>::acc acc[2];
            acc[0] = (typename Mfma<T>::acc){0, 0, 0, 0};
            acc[1] = acc[0];
            const int r = R0 + lr;
            // the tile's 8 operand loads first (clamped addresses, masked values)
            T av[NB / 4];
#pragma unroll
            for (int u = 0; u < NB / 4; ++u) {
                const int k = 4 * u + lk;
                const T x = A[min(r, c2 - 1) + (int64_t)(j0 + min(k, jb - 1)) * ld];
                av[u] = (r < c2 && k < jb) ? x : (T)0;
            }
#pragma unroll
            for (int u = 0; u < NB / 4; ++u) {
                const int k = 4 * u + lk;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int j = 16 * h + lr;
                    const T b = (k < jb && j < jb) ? W[j][k] : (T)0;
                    acc[h] = Mfma<T>::mac(av[u], b, acc[h]);
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = R0 + Mfma<T>::row(lane, v), col = 16 * h + lr;
                    if (row < c2 && col < jb) A[row + (int64_t)(j0 + col) * ld] = acc[h][v];
                }
        }
        __syncthreads();
        // 3. trailing update.  Inner: only the remaining columns of the current
        //    outer panel; at the end of an outer panel: everything to its right
        //    with k = the whole outer panel (fewer passes over the matrix).
        const int pend = min(p0 + NBO, cend);
        if (t0 < pend) {
            syrk_update<T>(A, ld, t0, pend, c2, j0, j0 + jb);
        } else {
            syrk_update<T>(A, ld, t0, cend, c2, p0, pend);
            p0 = pend;
        }
        __syncthreads();
    }
    if (tid == 0 && bad) info[s] = 1;
}

// Factorisation of the local matrices' constrained Neumann block (columns
// [c0, c1), trailing update within them).
template <typename T>
__global__ __launch_bounds__(kWG) void k_potrf(T* __restrict__ A, const int64_t* __restrict__ off,
                                              const int* __restrict__ ld, const int* __restrict__ c0,
                                              const int* __restrict__ c1, const int* __restrict__ c2,
                                              int* __restrict__ info) {
    const int s = blockIdx.x;
    potrf_body<T>(A + off[s], ld[s], c0[s], c1[s], c2[s], info);
}

// One panel of the interior elimination, columns [J, J + w), w = min(NBO,
// nI - J), in two kernels:
//  k_panel_diag  one workgroup per matrix factors the w x w diagonal block
//                and stores the inverses W_b of its 32x32 diagonal factors;
//  k_panel_trsm  the rows below, [J + w, n), in blocks of PT_RB rows per
//                workgroup: X L_JJ^T = P by block forward substitution,
//                X_b = (P_b - sum_{c<b} X_c L_bc^T) W_b^T, on MFMA.
// The update of the columns right of the panel is left to k_syrk_batched.
constexpr int PT_RB = 64, PT_XS = NBO + 4, PT_XCD = 8;

static_assert(NB == PP_NB, "the packed factor blocks are the solve blocks");
// Rows [r0, r1) (all below ne) of the panel columns [J, J + w), read by
// get(row, column), into the panel-packed copy of the factor (the layout the
// per-iteration solves stream, pp_block): entries right of the diagonal or
// past column ne - 1 of a 32-column block are zero.  One workgroup.
template <typename T, typename Get>
__device__ inline void store_packed(T* __restrict__ P, int ne, int J, int w, int r0, int r1, Get get) {
    const int b0 = J / NB, b1 = (J + w + NB - 1) / NB;
    for (int b = b0; b < b1; ++b) {
        T* Pb = P + pp_block(ne, b);
        const int rb0 = max(r0, NB * b);
        for (int idx = threadIdx.x; idx < (r1 - rb0) * NB; idx += kWG) {
            const int r = rb0 + idx / NB, c = NB * b + idx % NB;
            Pb[(int64_t)(r - NB * b) * NB + (c - NB * b)] = (c <= r && c < J + w) ? get(r, c) : (T)0;
        }
    }
}

// The diagonal block's factor also goes to the packed copy (P, poff) when
// one is given: its columns are final once the panel is factored.
template <typename T>
__global__ __launch_bounds__(kWG) void k_panel_diag(T* __restrict__ A, const int64_t* __restrict__ off,
                                                   const int* __restrict__ ld, const int* __restrict__ nIv, int J,
                                                   T* __restrict__ Wbuf, int* __restrict__ info,
                                                   T* __restrict__ P, const int64_t* __restrict__ poff) {
    const int s = blockIdx.x;
    const int nI = nIv[s];
    if (J >= nI) return;
    const int w = min(NBO, nI - J);
    T* As = A + off[s];
    const int64_t lds = ld[s];
    potrf_body<T>(As, lds, J, J + w, J + w, info, Wbuf + (int64_t)s * NBO * NB);
    if (P) {
        __syncthreads();   // the block's factor has been written by every thread
        store_packed<T>(P + poff[s], nI, J, w, J, J + w,
                        [&](int r, int c) { return As[r + (int64_t)c * lds]; });
    }
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_panel_trsm(T* __restrict__ Abase, const int64_t* __restrict__ off,
                                                   const int* __restrict__ ldv, const int* __restrict__ nIv,
                                                   const int* __restrict__ nv, int nsub, int rowblocks, int J,
                                                   const T* __restrict__ Wbuf, T* __restrict__ Pk,
                                                   const int64_t* __restrict__ poff, const int* __restrict__ nIcv) {
    // FP32 stages every factor block of a column block (the L_bc, c < b, and
    // W_b) at once, two barriers per column block; FP64 stages one block at
    // a time (its LDS would otherwise halve the resident workgroups)
    constexpr int LSL = sizeof(T) == 4 ? NBO / NB : 1;
    __shared__ T Xs[PT_RB][PT_XS];
    __shared__ T Ls[LSL][NB][NB + 1];
    // all row blocks of one matrix run on one XCD (dispatch assigns
    // consecutive ids round robin to the 8 XCDs), so its factor blocks are
    // fetched from HBM once and then served by that XCD's L2
    const int g = blockIdx.x, q = g / PT_XCD;
    const int s = (q / rowblocks) * PT_XCD + g % PT_XCD;
    const int rb = q % rowblocks;
    if (s >= nsub) return;
    const int nI = nIv[s], n = nv[s];
    if (J >= nI) return;
    const int w = min(NBO, nI - J);
    const int R0 = J + w + rb * PT_RB;
    if (R0 >= n) return;
    // rows in [nI, n) of a panel inside the core: zero before, zero after
    if (nIcv && R0 >= nI && J + w <= nIcv[s]) return;
    const int rows = min(PT_RB, n - R0);
    T* A = Abase + off[s];
    const int64_t ld = ldv[s];
    const T* W = Wbuf + (int64_t)s * NBO * NB;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    const int nb = (w + NB - 1) / NB;   // 32-column blocks of this panel
    // Every global read is issued up front into registers: the rows of the
    // panel (XPT values per thread) and, for each 32-column block b, the
    // factor blocks L_bc (c < b) and the inverse W_b of the diagonal factor
    // (BPT values per thread and block).  Addresses are clamped into the
    // panel; out-of-range entries are zeroed when they are written to LDS.
    constexpr int XPT = PT_RB * NBO / kWG, BPT = NB * NB / kWG, NLB = NBO / NB * (NBO / NB - 1) / 2;
    T xr[XPT], lb[NLB][BPT], wb[NBO / NB][BPT];
#pragma unroll
    for (int e = 0; e < XPT; ++e) {
        const int idx = tid + e * kWG, r = idx % PT_RB, c = idx / PT_RB;
        xr[e] = A[(R0 + min(r, rows - 1)) + (int64_t)(J + min(c, w - 1)) * ld];
    }
#pragma unroll
    for (int b = 1; b < NBO / NB; ++b)
#pragma unroll
        for (int c = 0; c < b; ++c)
#pragma unroll
            for (int e = 0; e < BPT; ++e) {
                const int idx = tid + e * kWG, i = idx % NB, j = idx / NB;
                const int gi = min(NB * b + i, w - 1), gj = min(NB * c + j, w - 1);
                lb[b * (b - 1) / 2 + c][e] = A[(J + gi) + (int64_t)(J + gj) * ld];
            }
#pragma unroll
    for (int b = 0; b < NBO / NB; ++b)
#pragma unroll
        for (int e = 0; e < BPT; ++e) wb[b][e] = W[(int64_t)b * NB * NB + tid + e * kWG];
    // keep every load above this point (the blocks are all consumed below
    // without branches: blocks at or beyond nb are zero and never stored)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = 0; e < XPT; ++e) {
        const int idx = tid + e * kWG, r = idx % PT_RB, c = idx / PT_RB;
        Xs[r][c] = (r < rows && c < w) ? xr[e] : (T)0;
    }
    if constexpr (LSL > 1) {
        // Each wave owns rows 16 wv .. 16 wv + 15 of Xs, so between the
        // barriers that publish the staged blocks a wave only reads back what
        // it wrote itself (in order within the wave; the fences keep the
        // compiler from reordering those accesses).
        auto wave_sync = [] {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        __syncthreads();   // Xs is filled
#pragma unroll
        for (int b = 0; b < NBO / NB; ++b) {
            if (b > 0) __syncthreads();   // every wave is done with the previous blocks
#pragma unroll
            for (int c = 0; c < b; ++c)
#pragma unroll
                for (int e = 0; e < BPT; ++e) {
                    const int idx = tid + e * kWG, i = idx % NB, j = idx / NB;
                    Ls[c][i][j] = (NB * b + i < w && NB * c + j < w) ? lb[b * (b - 1) / 2 + c][e] : (T)0;
                }
#pragma unroll
            for (int e = 0; e < BPT; ++e) {
                const int idx = tid + e * kWG, i = idx % NB, j = idx / NB;
                Ls[LSL - 1][i][j] = (b < nb) ? wb[b][e] : (T)0;
            }
            __syncthreads();
            typename Mfma<T>::acc acc[2];
            acc[0] = (typename Mfma<T>::acc){0, 0, 0, 0};
            acc[1] = acc[0];
            // acc = sum_{c<b} X_c L_bc^T
#pragma unroll
            for (int c = 0; c < b; ++c)
#pragma unroll
                for (int kk = 0; kk < NB; kk += 4) {
                    const T a = Xs[16 * wv + lr][NB * c + kk + lk];
#pragma unroll
                    for (int h = 0; h < 2; ++h) acc[h] = Mfma<T>::mac(a, Ls[c][16 * h + lr][kk + lk], acc[h]);
                }
            // Y_b = P_b - acc in place; then X_b = Y_b W_b^T
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int v = 0; v < 4; ++v) Xs[16 * wv + Mfma<T>::row(lane, v)][NB * b + 16 * h + lr] -= acc[h][v];
            wave_sync();
            acc[0] = (typename Mfma<T>::acc){0, 0, 0, 0};
            acc[1] = acc[0];
#pragma unroll
            for (int kk = 0; kk < NB; kk += 4) {
                const T a = Xs[16 * wv + lr][NB * b + kk + lk];
#pragma unroll
                for (int h = 0; h < 2; ++h) acc[h] = Mfma<T>::mac(a, Ls[LSL - 1][16 * h + lr][kk + lk], acc[h]);
            }
            wave_sync();
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int v = 0; v < 4; ++v) Xs[16 * wv + Mfma<T>::row(lane, v)][NB * b + 16 * h + lr] = acc[h][v];
        }
    } else {
#pragma unroll
        for (int b = 0; b < NBO / NB; ++b) {
            typename Mfma<T>::acc acc[2];
            acc[0] = (typename Mfma<T>::acc){0, 0, 0, 0};
            acc[1] = acc[0];
            // acc = sum_{c<b} X_c L_bc^T  (wave wv: rows 16 wv .. 16 wv + 15, 32 columns)
#pragma unroll
            for (int c = 0; c < b; ++c) {
                __syncthreads();
#pragma unroll
                for (int e = 0; e < BPT; ++e) {
                    const int idx = tid + e * kWG, i = idx % NB, j = idx / NB;
                    Ls[0][i][j] = (NB * b + i < w && NB * c + j < w) ? lb[b * (b - 1) / 2 + c][e] : (T)0;
                }
                __syncthreads();
#pragma unroll
                for (int kk = 0; kk < NB; kk += 4) {
                    const T a = Xs[16 * wv + lr][NB * c + kk + lk];
#pragma unroll
                    for (int h = 0; h < 2; ++h) acc[h] = Mfma<T>::mac(a, Ls[0][16 * h + lr][kk + lk], acc[h]);
                }
            }
            __syncthreads();
            // Y_b = P_b - acc in place; then X_b = Y_b W_b^T
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int v = 0; v < 4; ++v) Xs[16 * wv + Mfma<T>::row(lane, v)][NB * b + 16 * h + lr] -= acc[h][v];
#pragma unroll
            for (int e = 0; e < BPT; ++e) {
                const int idx = tid + e * kWG, i = idx % NB, j = idx / NB;
                Ls[0][i][j] = (b < nb) ? wb[b][e] : (T)0;
            }
            __syncthreads();
            acc[0] = (typename Mfma<T>::acc){0, 0, 0, 0};
            acc[1] = acc[0];
#pragma unroll
            for (int kk = 0; kk < NB; kk += 4) {
                const T a = Xs[16 * wv + lr][NB * b + kk + lk];
#pragma unroll
                for (int h = 0; h < 2; ++h) acc[h] = Mfma<T>::mac(a, Ls[0][16 * h + lr][kk + lk], acc[h]);
            }
            __syncthreads();
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int v = 0; v < 4; ++v) Xs[16 * wv + Mfma<T>::row(lane, v)][NB * b + 16 * h + lr] = acc[h][v];
        }
    }
    __syncthreads();
    for (int idx = tid; idx < PT_RB * NBO; idx += kWG) {
        const int r = idx % PT_RB, c = idx / PT_RB;
        if (r < rows && c < w) A[(R0 + r) + (int64_t)(J + c) * ld] = Xs[r][c];
    }
    // rows of the factor proper (below nI) also go to the packed copy
    if (Pk && R0 < nI)
        store_packed<T>(Pk + poff[s], nI, J, w, R0, min(R0 + rows, nI),
                        [&](int r, int c) { return Xs[r - R0][c - J]; });
}

// Batched symmetric rank-k update C -= P P^T of a lower trapezoid of every
// local matrix: columns [cb, ce), rows [cb, re), lower part (row >= column),
// P = A[:, k0:k1).  Two uses, selected by mode:
//   SY_TRAIL  after the interior panel [J, J + NBO): cb = J + NBO, ce = nI,
//             re = n, k = the panel (K_II trailing block and the L_GI rows);
//   SY_SCHUR  after the last panel: cb = nI, ce = re = n, k = [0, nI), which
//             turns K_GG into S_Gamma = K_GG - L_GI L_GI^T (Sec. 4.1).
// TM x TM output tiles per workgroup (TM/2 x TM/2 per wave, in 16x16x4 MFMA
// blocks), the inner dimension staged through LDS in chunks of KC columns
// with a register prefetch of the next chunk; (TM, KC) is one of the tuned
// variants below.  The workgroup id is mapped so that all tiles of one
// subdomain run on the same XCD (dispatch assigns consecutive ids round
// robin to the 8 XCDs), which keeps P in that XCD's L2.
constexpr int SY_XCD = 8;
constexpr int SY_TRAIL = 0, SY_SCHUR = 1;
// variants (TM, KC): 0 = (128, 32), 1 = (128, 16), 2 = (64, 32), 3 = (64, 16),
// one LDS buffer and two barriers per chunk; 4 and 5 = (64, 16) with two LDS
// buffers and one barrier per chunk, 4 with the FP32 output tile read up
// front.
constexpr int SY_NVAR = 6;
__host__ __device__ constexpr int syrk_tm(int v) { return (v < 2) ? 128 : 64; }
__host__ __device__ constexpr int syrk_kc(int v) { return (v >= 4 || (v & 1)) ? 16 : 32; }

__host__ __device__ inline int trapezoid_tiles(int cb, int ce, int re, int TM) {
    if (ce <= cb || re <= cb) return 0;
    const int nct = (ce - cb + TM - 1) / TM, nrt = (re - cb + TM - 1) / TM;
    return nct * nrt - nct * (nct - 1) / 2;
}

template <typename T, int TM, int KC, bool DB = false, bool CP = false>
__global__ __launch_bounds__(kWG) void k_syrk_batched(T* __restrict__ Abase, const int64_t* __restrict__ off,
                                                      const int* __restrict__ ldv, const int* __restrict__ nIv,
                                                      const int* __restrict__ nv, const int* __restrict__ nIcv,
                                                      int nsub, int tiles, int mode, int J) {
    constexpr int LS = TM + 16;                // padded LDS row
    constexpr int KS = kWG / TM;               // inner indices staged per pass of the workgroup
    constexpr int EPT = TM * KC / kWG;         // staged elements per thread and operand
    constexpr int WT = TM / 2, NBK = WT / 16;  // wave tile and its MFMA blocks per side
    constexpr int NBUF = DB ? 2 : 1;
    __shared__ T As[NBUF][KC][LS];    // P rows of the output tile's rows (i)
    __shared__ T Bs[NBUF][KC][LS];    // P rows of the output tile's columns (j)
    const int g = blockIdx.x;
    const int q = g / SY_XCD;
    const int s = (q / tiles) * SY_XCD + g % SY_XCD;
    int tile = q % tiles;
    if (s >= nsub) return;
    T* A = Abase + off[s];
    const int64_t ld = ldv[s];
    const int nI = nIv[s], n = nv[s];
    int cb, ce, re, k0, k1;
    if (mode == SY_SCHUR) {
        cb = nI; ce = n; re = n; k0 = 0; k1 = nI;
    } else {
        cb = J + NBO; ce = nI; re = n; k0 = J; k1 = min(J + NBO, nI);
        // a panel inside the core leaves the interface rows as they are: the
        // trapezoid stops at nI (the launch is sized the same way)
        if (nIcv && k1 <= nIcv[s]) re = nI;
    }
    if (k1 <= k0 || tile >= trapezoid_tiles(cb, ce, re, TM)) return;
    const int nrt = (re - cb + TM - 1) / TM;
    int tj = 0;
    while (tile >= nrt - tj) { tile -= nrt - tj; ++tj; }
    const int ti = tj + tile;
    const int I0 = cb + ti * TM, J0 = cb + tj * TM;
    // rows of the tile all in [nI, n): their operand is zero left of the
    // core boundary c = nIc (the interface does not couple with the core),
    // so the inner indices start there, and a tile with none left keeps C.
    // A panel that straddles c (J < c < k1) gives these rows only the short
    // slice [c, k1), and only the next panel's columns take it at once
    // (that panel's row blocks need it); the columns beyond take the slice
    // with the next panel's own update, whose inner range then starts at c.
    if (nIcv && I0 >= nI) {
        const int c = nIcv[s];
        if (mode == SY_TRAIL && J < c && c < k1 && J0 >= J + 2 * NBO) return;
        k0 = (mode == SY_TRAIL && J - NBO < c && c < J) ? c : max(k0, c);
        if (k0 >= k1) return;
    }
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    const int wr = wv & 1, wc = wv >> 1;                 // wave's quadrant (rows i, cols j)
    const bool active = !(ti == tj && wr < wc);          // strictly upper quadrant of a diagonal tile
    // each thread stages EPT elements of each operand per chunk: row tid % TM, k = tid / TM + KS e.
    // The loads are branch-free: rows beyond the trapezoid are clamped to its
    // last row (they only reach outputs that are never stored) and the inner
    // index to k1 - 1; the k mask is applied when the chunk is written to LDS,
    // so no load has to complete before the next one is issued.
    const int lrow = tid % TM, lk0 = tid / TM;
    const int ri = min(I0 + lrow, re - 1), rj = min(J0 + lrow, ce - 1);
    T pa[EPT], pb[EPT];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t k = min(kc + lk0 + KS * e, k1 - 1);
            pa[e] = A[ri + k * ld];
            pb[e] = A[rj + k * ld];
        }
    };
    // FP64: the output tile starts from C, loaded in the accumulator layout
    // before the first chunk so that its latency overlaps the first fetch of
    // P; the column operand is staged negated, so the chunks add -P P^T and
    // the tile is stored without reading it again (this also keeps the
    // kernel at two waves per SIMD).  FP32: each chunk of SY_KC inner indices
    // is summed on its own and added to a running total that starts at zero
    // and is subtracted from C at the end, so rounding grows with the number
    // of chunks plus the chunk length rather than with the whole inner
    // dimension.
    constexpr bool two_level = std::is_same<T, float>::value;
    const T sgn = two_level ? (T)1 : (T)-1;
    typename Mfma<T>::acc acc[NBK][NBK], tot[NBK][NBK];
    auto c_at = [&](int a, int b, int v) -> T {       // C entry of accumulator (b, a, v), clamped address
        const int i = min(I0 + wr * WT + 16 * a + lr, re - 1);
        const int j = min(J0 + wc * WT + 16 * b + Mfma<T>::row(lane, v), ce - 1);
        return A[i + (int64_t)j * ld];
    };
    // CP, FP32: the output tile is read at the start (its latency hidden
    // behind the first chunks) instead of after the last one
    constexpr bool cpre = CP && two_level;
    T cv[cpre ? NBK : 1][cpre ? NBK : 1][4];
#pragma unroll
    for (int b = 0; b < NBK; ++b)
#pragma unroll
        for (int a = 0; a < NBK; ++a) {
            acc[b][a] = tot[b][a] = (typename Mfma<T>::acc){0, 0, 0, 0};
            if (!two_level && active) {
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[b][a][v] = c_at(a, b, v);
            }
            if constexpr (cpre) {
#pragma unroll
                for (int v = 0; v < 4; ++v) cv[b][a][v] = c_at(a, b, v);
            }
        }
    auto stage = [&](int buf, int kc) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const bool kin = kc + lk0 + KS * e < k1;
            As[buf][lk0 + KS * e][lrow] = kin ? pa[e] : (T)0;
            Bs[buf][lk0 + KS * e][lrow] = kin ? sgn * pb[e] : (T)0;
        }
    };
    auto chunk = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            T fa[NBK], fb[NBK];
#pragma unroll
            for (int a = 0; a < NBK; ++a) fa[a] = As[buf][kk + lk][wr * WT + 16 * a + lr];
#pragma unroll
            for (int b = 0; b < NBK; ++b) fb[b] = Bs[buf][kk + lk][wc * WT + 16 * b + lr];
            // output row index = j (A operand), column index = i (B operand), so
            // that the 16 lanes of an accumulator row hold consecutive i
#pragma unroll
            for (int b = 0; b < NBK; ++b)
#pragma unroll
                for (int a = 0; a < NBK; ++a) acc[b][a] = Mfma<T>::mac(fb[b], fa[a], acc[b][a]);
        }
        if (two_level) {
#pragma unroll
            for (int b = 0; b < NBK; ++b)
#pragma unroll
                for (int a = 0; a < NBK; ++a) {
                    tot[b][a] += acc[b][a];
                    acc[b][a] = (typename Mfma<T>::acc){0, 0, 0, 0};
                }
        }
    };
    fetch(k0);
    if constexpr (DB) {
        // chunk c is staged in buffer c & 1.  Each pass computes from one
        // buffer and stages the next chunk into the other; the single
        // barrier both publishes that chunk and ends every wave's reads of
        // the buffer the following pass overwrites.
        stage(0, k0);
        __syncthreads();
        if (k0 + KC < k1) fetch(k0 + KC);
        int buf = 0;
        for (int kc = k0; kc < k1; kc += KC) {
            if (active) chunk(buf);
            if (kc + KC < k1) {
                stage(buf ^ 1, kc + KC);
                __syncthreads();
                if (kc + 2 * KC < k1) fetch(kc + 2 * KC);
            }
            buf ^= 1;
        }
    } else {
        for (int kc = k0; kc < k1; kc += KC) {
            __syncthreads();
            stage(0, kc);
            __syncthreads();
            if (kc + KC < k1) fetch(kc + KC);
            if (active) chunk(0);
        }
    }
    if (!active) return;
    if (two_level) {
#pragma unroll
        for (int b = 0; b < NBK; ++b)
#pragma unroll
            for (int a = 0; a < NBK; ++a)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    T c;
                    if constexpr (cpre) c = cv[b][a][v];
                    else c = c_at(a, b, v);
                    tot[b][a][v] = c - tot[b][a][v];
                }
    }
#pragma unroll
    for (int b = 0; b < NBK; ++b)
#pragma unroll
        for (int a = 0; a < NBK; ++a) {
            const int i = I0 + wr * WT + 16 * a + lr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = J0 + wc * WT + 16 * b + Mfma<T>::row(lane, v);
                if (i < re && j < ce && j <= i) A[i + (int64_t)j * ld] = two_level ? tot[b][a][v] : acc[b][a][v];
            }
        }
}

// ------------------------------------------------------------- extraction
// Copy, from the Schur complement left in the trailing block after the
// interior elimination: the principal minors S_*^(j) of every face and edge
// (deluxe blocks, Sec. 4.2), the right-hand sides [C^T | -S_rV] of the
// coarse-basis problems, S_VV, and optionally S_rr.
template <typename T>
__global__ __launch_bounds__(kWG) void k_extract(BatchDesc d, const T* __restrict__ K, T* __restrict__ slots,
                                                T* __restrict__ F, double* __restrict__ Svv,
                                                T* __restrict__ Srr) {
    const int s = d.sub0 + blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t ld = d.n[s];
    const int nI = d.nI[s], nr = d.nr[s], nV = d.nV[s], nc = d.nc[s];
    const T* S = K + d.K_off[s] + (int64_t)nI * (ld + 1);   // S(a,b) = S[a + b*ld], a >= b valid
    auto Sat = [&](int a, int b) -> T { return a >= b ? S[a + (int64_t)b * ld] : S[b + (int64_t)a * ld]; };
    for (int64_t q = d.so_ptr[s]; q < d.so_ptr[s + 1]; ++q) {
        const int ro = d.so_roff[q], no = d.so_n[q];
        T* dst = slots + d.so_slot[q];
        for (int idx = tid; idx < no * no; idx += kWG) {
            const int i = idx % no, j = idx / no;
            dst[idx] = Sat(ro + i, ro + j);
        }
        const int e = d.so_eidx[q];   // constraint index of the object, or -1
        if (e >= 0) {
            const int nn = d.so_nnode[q];
            T* Fc = F + d.F_off[s];
            for (int idx = tid; idx < 2 * nn; idx += kWG) {
                const int f = idx & 1;
                Fc[(ro + idx) + (int64_t)(2 * e + f) * nr] = (T)(1.0 / nn);
            }
        }
    }
    T* Fv = F + d.F_off[s] + (int64_t)nc * nr;
    for (int idx = tid; idx < nr * nV; idx += kWG) {
        const int r = idx % nr, q = idx / nr;
        Fv[r + (int64_t)q * nr] = -Sat(nr + q, r);
    }
    double* sv = Svv + (int64_t)s * SVV_STRIDE;
    for (int idx = tid; idx < nV * nV; idx += kWG) {
        const int a = idx % nV, b = idx / nV;
        sv[idx] = (double)Sat(nr + a, nr + b);
    }
    if (Srr) {
        T* dst = Srr + d.Srr_off[s];
        for (int idx = tid; idx < nr * nr; idx += kWG) {
            const int a = idx % nr, b = idx / nr;
            dst[idx] = Sat(a, b);
        }
    }
}

// Row streaming of the single-RHS solves over a packed factor: TS_SEG
// entries (16 bytes) per lane, TS_LPR lanes per row, TS_RPI rows per wave
// load instruction, TS_U row groups per wave in flight.
template <typename T>
struct TSGeom {
    static constexpr int SEG = 16 / (int)sizeof(T), LPR = NB / SEG, RPI = 64 / LPR, U = 4;
};

// Loads of a packed factor row (NB entries) or of a contiguous M-entry
// segment of one, as 16-byte vector loads; p is 16-byte aligned (rows start
// on PP_NB-entry boundaries, segments on multiples of 4 floats / 2 doubles).
template <typename T, int M>
__device__ __forceinline__ void load_pseg(const T* __restrict__ p, T (&v)[M]) {
    if constexpr (sizeof(T) == 4) {
        static_assert(M % 4 == 0, "segment of whole float4");
#pragma unroll
        for (int q = 0; q < M / 4; ++q) {
            const float4 f = reinterpret_cast<const float4*>(p)[q];
            v[4 * q] = f.x; v[4 * q + 1] = f.y; v[4 * q + 2] = f.z; v[4 * q + 3] = f.w;
        }
    } else {
        static_assert(M % 2 == 0, "segment of whole double2");
#pragma unroll
        for (int q = 0; q < M / 2; ++q) {
            const double2 f = reinterpret_cast<const double2*>(p)[q];
            v[2 * q] = f.x; v[2 * q + 1] = f.y;
        }
    }
}
template <typename T>
__device__ __forceinline__ void load_prow(const T* __restrict__ p, T (&v)[NB]) {
    load_pseg<T, NB>(p, v);
}

// Zero the lower triangle (diagonal included) of every local matrix of a
// chunk before its assembly: the elimination and extraction read
// and write lower-triangle entries only.  Grid: (column blocks of CL_COLS,
// matrices).
constexpr int CL_COLS = 16;
// Each column segment [j, n) is written with 16-byte stores over its
// 16-byte aligned middle and single stores at the two ends.
template <typename T>
__global__ __launch_bounds__(kWG) void k_clear_lower(BatchDesc d, T* __restrict__ K) {
    constexpr int V = 16 / (int)sizeof(T);
    const int s = d.sub0 + blockIdx.y;
    const int n = d.n[s];
    T* A = K + d.K_off[s];
    const int tid = threadIdx.x;
    const int j1 = min(n, ((int)blockIdx.x + 1) * CL_COLS);
    for (int j = blockIdx.x * CL_COLS; j < j1; ++j) {
        T* c = A + (int64_t)j * n;
        const int head = (int)(((16 - ((uintptr_t)(c + j) & 15)) & 15) / sizeof(T));   // entries to the next 16-byte boundary
        const int a0 = min(j + head, n);            // first entry of the aligned middle
        const int nv = (n - a0) / V;                // 16-byte groups in it
        if (tid < a0 - j) c[j + tid] = (T)0;
        for (int q = tid; q < nv; q += kWG) reinterpret_cast<float4*>(c + a0)[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        const int t0 = a0 + nv * V;
        if (tid < n - t0) c[t0 + tid] = (T)0;
    }
}

// ----------------------------------------------------- multi-RHS forward
// L X = B in place (L lower n x n, panel-packed; B n x k, k <= 64).
template <typename T>
__global__ __launch_bounds__(kWG) void k_trsm_fwd(const T* __restrict__ Lb, const int64_t* __restrict__ Loff,
                                                 const int* __restrict__ nv, T* __restrict__ Bb,
                                                 const int64_t* __restrict__ Boff, const int* __restrict__ ldbv,
                                                 const int* __restrict__ kv) {
    const int s = blockIdx.x;
    const T* L = Lb + Loff[s];
    T* B = Bb + Boff[s];
    const int n = nv[s], k = kv[s];
    const int64_t ldb = ldbv[s];
    const int tid = threadIdx.x;
    __shared__ T D[NB][NB + 1];
    __shared__ T X[NB][64 + 1];
    __shared__ int live[64];
    for (int j0 = 0; j0 < n; j0 += NB) {
        const int jb = min(NB, n - j0);
        const T* Lp = L + pp_block(n, j0 / NB);   // row r of the block at Lp + (r - j0) NB
        for (int idx = tid; idx < NB * NB; idx += kWG) {
            const int i = idx / NB, j = idx % NB;
            D[i][j] = (i < jb && j <= i) ? Lp[i * NB + j] : (T)0;
        }
        for (int idx = tid; idx < NB * 64; idx += kWG) {
            const int i = idx % NB, c = idx / NB;
            X[i][c] = (i < jb && c < k) ? B[(j0 + i) + c * ldb] : (T)0;
        }
        __syncthreads();
        if (tid < k) {
            for (int i = 0; i < jb; ++i) {
                T acc = X[i][tid];
                for (int m = 0; m < i; ++m) acc -= D[i][m] * X[m][tid];
                X[i][tid] = acc / D[i][i];
            }
        }
        __syncthreads();
        for (int idx = tid; idx < jb * k; idx += kWG) {
            const int i = idx % jb, c = idx / jb;
            B[(j0 + i) + c * ldb] = X[i][c];
        }
        // columns whose solution is still zero (a right-hand side that starts
        // further down, such as a constraint column) need no update
        if (tid < 64) {
            bool nz = false;
            if (tid < k)
                for (int i = 0; i < jb; ++i) nz = nz || (X[i][tid] != (T)0);
            live[tid] = nz ? 1 : 0;
        }
        __syncthreads();
        // rows below the block: each thread loads its row of the column block
        // once and updates every live right-hand side
        const int t0 = j0 + jb;
        for (int r = t0 + tid; r < n; r += kWG) {
            T lv[NB];
            load_prow(Lp + (int64_t)(r - j0) * NB, lv);   // entries past column n-1 are zero
            for (int c = 0; c < k; ++c) {
                if (!live[c]) continue;
                T acc = (T)0;
#pragma unroll
                for (int m = 0; m < NB; ++m) acc += lv[m] * X[m][c];
                B[r + c * ldb] -= acc;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------- coarse algebra
// With Y = L_rr^{-1} C^T and X = -L_rr^{-1} S_rV (from k_trsm_fwd), the
// energy-minimising coarse basis of Sec. 4.4 under the average constraints
// (edges, and faces when the primal space has them) is Phi_r = L_rr^{-T} Z with
//   G = Y^T Y = C S_rr^{-1} C^T,  mu_V = G^{-1} Y^T X,
//   Z = [X - Y mu_V | Y G^{-1}]   (vertex primals, then average primals),
// and the local coarse matrix Phi^T S_Gamma Phi is
//   vertex rows: [-X^T Z + [S_VV | 0]],   average rows: [-mu_V | G^{-1}].
// With vertex primals only (no constraints) Z = X.  Every inner product the
// algebra needs is an entry of the Gram matrix of W = [Y | X]: G = Y^T Y,
// Y^T X, and X^T Z = [X^T X - (Y^T X)^T mu_V | (Y^T X)^T G^{-1}], so one pass
// over the rows of W (in FP64) replaces a pass per product.
template <typename T>
__global__ __launch_bounds__(kWG) void k_coarse_local(BatchDesc d, const T* __restrict__ Fb,
                                                     const double* __restrict__ Svv, T* __restrict__ Zb,
                                                     double* __restrict__ Spb,
                                                     int* __restrict__ info) {
    const int s = d.sub0 + blockIdx.x;
    const int tid = threadIdx.x;
    const int nr = d.nr[s], nV = d.nV[s], nc = d.nc[s], nP = nV + nc;
    const T* Y = Fb + d.F_off[s];
    const T* X = Y + (int64_t)nc * nr;
    T* Z = Zb + d.Z_off[s];
    __shared__ double G[MAXC][MAXC + 1];
    __shared__ double Gi[MAXC][MAXC + 1];
    __shared__ double YtX[MAXC][MAXV + 1];
    __shared__ double muV[MAXC][MAXV + 1];
    __shared__ double XtX[MAXV][MAXV + 1];
    // Gram matrix of W = [Y | X] (nr x nP, column-major: X follows Y): rows
    // in chunks of GR staged in LDS, each thread accumulating up to GP
    // lower-triangle entries in FP64, the rows in order.
    {
        constexpr int GR = 32, GP = (MAXP * (MAXP + 1) / 2 + kWG - 1) / kWG;
        __shared__ double wc[GR][MAXP + 1];
        const int npair = nP * (nP + 1) / 2;
        int pi[GP], pj[GP];
        double g[GP];
#pragma unroll
        for (int u = 0; u < GP; ++u) {
            const int p = tid + kWG * u;
            int i = 0;
            if (p < npair) {
                i = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
                while (i * (i + 1) / 2 > p) --i;
                while ((i + 1) * (i + 2) / 2 <= p) ++i;
            }
            pi[u] = i;
            pj[u] = p < npair ? p - i * (i + 1) / 2 : 0;
            g[u] = 0.0;
        }
        // the next chunk's rows are loaded into registers (clamped
        // addresses, masked values) while the current one is summed
        constexpr int GL = (GR * MAXP + kWG - 1) / kWG;
        T nxt[GL];
        auto load = [&](int r0) {
#pragma unroll
            for (int e = 0; e < GL; ++e) {
                const int idx = tid + kWG * e, rr = idx % GR, c = min(idx / GR, nP - 1);
                nxt[e] = Y[(int64_t)c * nr + min(r0 + rr, nr - 1)];
            }
        };
        load(0);
        for (int r0 = 0; r0 < nr; r0 += GR) {
            const int rows = min(GR, nr - r0);
            __syncthreads();   // the previous chunk has been consumed
#pragma unroll
            for (int e = 0; e < GL; ++e) {
                const int idx = tid + kWG * e, rr = idx % GR, c = idx / GR;
                if (c < nP) wc[rr][c] = (rr < rows) ? (double)nxt[e] : 0.0;
            }
            __syncthreads();
            if (r0 + GR < nr) load(r0 + GR);
#pragma unroll
            for (int u = 0; u < GP; ++u) {
                if (tid + kWG * u < npair) {
                    double a = g[u];
                    for (int rr = 0; rr < GR; ++rr) a += wc[rr][pi[u]] * wc[rr][pj[u]];
                    g[u] = a;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < GP; ++u) {
            if (tid + kWG * u >= npair) continue;
            const int i = pi[u], j = pj[u];   // i >= j
            if (i < nc) {
                G[i][j] = g[u];
                G[j][i] = g[u];
            } else if (j < nc) {
                YtX[j][i - nc] = g[u];
            } else {
                XtX[i - nc][j - nc] = g[u];
                XtX[j - nc][i - nc] = g[u];
            }
        }
    }
    __syncthreads();
    // Cholesky of the small constraint matrix (lower triangle of G): one
    // barrier per pivot, the trailing block updated with the unscaled column
    // by (row, column group) threads, the columns scaled at the end
    static_assert(MAXC <= 64, "one row slot per pivot row");
    for (int k = 0; k < nc; ++k) {
        double dk = G[k][k];
        if (!(dk > 0.0)) dk = 1.0;
        const int i = tid % 64;
        if (i > k && i < nc) {
            const double lik = G[i][k] / dk;
            for (int j = k + 1 + tid / 64; j <= i; j += kWG / 64) G[i][j] -= lik * G[j][k];
        }
        __syncthreads();
    }
    __shared__ double piv[MAXC];
    if (tid < nc) {
        double dk = G[tid][tid];
        if (!(dk > 0.0)) { info[s] = 2; dk = 1.0; }
        piv[tid] = sqrt(dk);
    }
    __syncthreads();
    for (int idx = tid; idx < nc * nc; idx += kWG) {
        const int i = idx % nc, k = idx / nc;
        if (i > k) G[i][k] /= piv[k];
    }
    __syncthreads();
    if (tid < nc) G[tid][tid] = piv[tid];
    __syncthreads();
    if (tid < nc) {   // column tid of G^{-1}, in registers (unrolled to MAXC)
        double y[MAXC];
#pragma unroll
        for (int i = 0; i < MAXC; ++i) {
            if (i < nc) {
                double a = (i == tid) ? 1.0 : 0.0;
#pragma unroll
                for (int m = 0; m < i; ++m) a -= G[i][m] * y[m];
                y[i] = a / G[i][i];
            } else {
                y[i] = 0.0;
            }
        }
#pragma unroll
        for (int i = MAXC - 1; i >= 0; --i) {
            if (i < nc) {
                double a = y[i];
#pragma unroll
                for (int m = i + 1; m < MAXC; ++m)
                    if (m < nc) a -= G[m][i] * y[m];
                y[i] = a / G[i][i];
            }
        }
#pragma unroll
        for (int i = 0; i < MAXC; ++i)
            if (i < nc) Gi[i][tid] = y[i];
    }
    __syncthreads();
    for (int idx = tid; idx < nc * nV; idx += kWG) {
        const int i = idx % nc, q = idx / nc;
        double acc = 0.0;
        for (int m = 0; m < nc; ++m) acc += Gi[i][m] * YtX[m][q];
        muV[i][q] = acc;
    }
    __syncthreads();
    for (int r = tid; r < nr; r += kWG) {
        double yr[MAXC];   // row r of Y, read once
#pragma unroll
        for (int m = 0; m < MAXC; ++m) yr[m] = (m < nc) ? (double)Y[r + (int64_t)m * nr] : 0.0;
        for (int q = 0; q < nV; ++q) {
            double acc = (double)X[r + (int64_t)q * nr];
#pragma unroll
            for (int m = 0; m < MAXC; ++m)
                if (m < nc) acc -= yr[m] * muV[m][q];
            Z[r + (int64_t)q * nr] = (T)acc;
        }
        for (int e = 0; e < nc; ++e) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < MAXC; ++m)
                if (m < nc) acc += yr[m] * Gi[m][e];
            Z[r + (int64_t)(nV + e) * nr] = (T)acc;
        }
    }
    __syncthreads();
    double* Sp = Spb + (int64_t)s * SP_STRIDE;
    const double* sv = Svv + (int64_t)s * SVV_STRIDE;
    for (int idx = tid; idx < nV * nP; idx += kWG) {
        const int q = idx % nV, pcol = idx / nV;
        double acc;   // X^T Z, column pcol
        if (pcol < nV) {
            acc = XtX[q][pcol];
            for (int m = 0; m < nc; ++m) acc -= YtX[m][q] * muV[m][pcol];
        } else {
            acc = 0.0;
            for (int m = 0; m < nc; ++m) acc += YtX[m][q] * Gi[m][pcol - nV];
        }
        Sp[q + (int64_t)pcol * nP] = -acc + (pcol < nV ? sv[q + pcol * nV] : 0.0);
    }
    for (int idx = tid; idx < nc * nP; idx += kWG) {
        const int e = idx % nc, pcol = idx / nc;
        Sp[(nV + e) + (int64_t)pcol * nP] = (pcol < nV) ? -muV[e][pcol] : Gi[e][pcol - nV];
    }
}

// The local coarse block S_PiPi^(j) = Phi^T S_Gamma^(j) Phi annihilates the
// primal vector k with 1 on every u_e primal (vertex value or average) and
// 0 on every v primal: Phi k is the constant u_e = 1, v = 0, which meets the
// constraints and has zero energy (Sec. 4.4; the kernel of the Jacobian,
// Sec. 3c).  Computed from rounded local factors the block only nearly
// does, and the assembled coarse matrix, which has a small eigenvalue along
// the pinned near-kernel (the u_e-constant mode of a large subdomain grid),
// amplifies the defect.  Replacing the block by P S P, P = I - k k^T /
// (k^T k), restores the exact kernel; it changes the block by the size of
// the defect.  Local primal order: (v, u_e) per vertex, then (v, u_e)
// averages per constraint object, so k is 1 on the odd local indices.
__global__ __launch_bounds__(kWG) void k_coarse_kernel_fix(int sub0, const int* __restrict__ nVv,
                                                          const int* __restrict__ ncv, double* __restrict__ Spb) {
    const int s = sub0 + blockIdx.x;
    const int nP = nVv[s] + ncv[s];
    double* S = Spb + (int64_t)s * SP_STRIDE;
    __shared__ double w[MAXP];
    __shared__ double sk;
    const int tid = threadIdx.x;
    if (tid < nP) {
        double a = 0.0;
        for (int j = 1; j < nP; j += 2) a += S[tid + (int64_t)j * nP];
        w[tid] = a;
    }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0;
        for (int i = 1; i < nP; i += 2) a += w[i];
        sk = a;
    }
    __syncthreads();
    const double kk = 0.5 * nP;
    for (int idx = tid; idx < nP * nP; idx += kWG) {
        const int i = idx % nP, j = idx / nP;
        const double ki = (i & 1) ? 1.0 : 0.0, kj = (j & 1) ? 1.0 : 0.0;
        S[i + (int64_t)j * nP] += -(w[i] * kj + ki * w[j]) / kk + sk * ki * kj / (kk * kk);
    }
}

// ------------------------------------------------- single-RHS triangular
// Forward L x = b or backward L^T x = b, in place, one workgroup per vector;
// x lives in LDS (dynamic, n values) for the whole solve.  Per 32-column
// block one wave solves the diagonal block from registers (lane i holds row i
// of the block for the forward solve, column i for the backward solve;
// reciprocal pivots; broadcasts by lane reads), then all waves stream the
// rows below: forward x_r -= L_r,blk x_blk, backward the dot products
// L_blk^T x_below that enter the block's right-hand side.
__device__ inline float lane_read(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double lane_read(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// Next matrix of a one-workgroup-per-matrix kernel: from the work queue when
// the launch is persistent, else the workgroup's own index (first pass only).
// Returns -1 when the workgroup is done; the last workgroup to finish resets
// the queue.  Contains barriers: every thread of the workgroup calls it.
__device__ inline int next_item(const int* __restrict__ order, int* __restrict__ ctr, int nb, int pass) {
    __shared__ int item;
    if (!ctr) return pass == 0 && (int)blockIdx.x < nb ? (order ? order[blockIdx.x] : (int)blockIdx.x) : -1;
    __syncthreads();                    // every thread has read the previous item
    if (threadIdx.x == 0) {
        int k = atomicAdd(&ctr[0], 1);
        if (k >= nb) {
            k = -1;
            if (atomicAdd(&ctr[1], 1) == (int)gridDim.x - 1) {   // last workgroup out
                atomicExch(&ctr[0], 0);
                atomicExch(&ctr[1], 0);
            }
        }
        item = k < 0 ? -1 : order[k];
    }
    __syncthreads();
    return item;
}

// Forward and backward solves of one subdomain on x staged in LDS (xl);
// every thread of the workgroup calls them, and each ends with a barrier.
template <typename T>
__device__ __forceinline__ void trsv_fwd_solve(const T* __restrict__ L, int n, T* xl, T* xs) {
    constexpr int TS_SEG = TSGeom<T>::SEG, TS_LPR = TSGeom<T>::LPR, TS_RPI = TSGeom<T>::RPI, TS_U = TSGeom<T>::U;
    const int tid = threadIdx.x, lane = tid & 63;
    // wave 0 holds the diagonal block of the current step in drow (lane i:
    // row i of the block, one packed row).  FP32: loaded during the previous
    // step's update so that its latency is hidden (at no cost in occupancy);
    // FP64: loaded at the step itself, which keeps the register count down.
    constexpr bool early = sizeof(T) == 4;
    T drow[NB], rdiag = (T)1;
    auto load_diag = [&](int j0) {
        const int jb = min(NB, n - j0), i = min(lane, jb - 1);
        load_prow(L + pp_block(n, j0 / NB) + (int64_t)i * NB, drow);
        rdiag = drow[0];
#pragma unroll
        for (int c = 1; c < NB; ++c) rdiag = (c == i) ? drow[c] : rdiag;
    };
    if (early && tid < 64) load_diag(0);
    for (int j0 = 0; j0 < n; j0 += NB) {
        const int jb = min(NB, n - j0);
        if (tid < 64) {
            if (!early) load_diag(j0);
            const T rinv = (lane < jb) ? (T)1 / rdiag : (T)0;
            T xv = (lane < jb) ? xl[j0 + lane] : (T)0;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                if (c < jb) {
                    const T xc = lane_read(xv, c) * lane_read(rinv, c);
                    xv = (lane == c) ? xc : ((lane > c) ? xv - drow[c] * xc : xv);
                }
            }
            if (lane < NB) xs[lane] = (lane < jb) ? xv : (T)0;
            if (lane < jb) xl[j0 + lane] = xv;
        }
        __syncthreads();
        if (early && tid < 64 && j0 + NB < n) load_diag(j0 + NB);
        // Rows below the block: LPR lanes share a packed row, one 16-byte
        // chunk each, so a load instruction reads RPI whole rows; TU row
        // groups per wave are in flight together.  Each lane dots its chunk
        // with x and the row's lanes sum by xor shuffles.  (xs and the
        // padding past column n-1 are zero.)
        const T* Lp = L + pp_block(n, j0 / NB);
        {
            const int q = lane % TS_LPR, rr = lane / TS_LPR;
            T xq[TS_SEG];
#pragma unroll
            for (int k = 0; k < TS_SEG; ++k) xq[k] = xs[q * TS_SEG + k];
            for (int r0 = j0 + jb + (tid >> 6) * TS_RPI * TS_U; r0 < n; r0 += (kWG / 64) * TS_RPI * TS_U) {
                T v[TS_U][TS_SEG];
#pragma unroll
                for (int u = 0; u < TS_U; ++u) {
                    const int rc = min(r0 + u * TS_RPI + rr, n - 1);
                    load_pseg<T, TS_SEG>(Lp + (int64_t)(rc - j0) * NB + q * TS_SEG, v[u]);
                }
#pragma unroll
                for (int u = 0; u < TS_U; ++u) {
                    T acc = (T)0;
#pragma unroll
                    for (int k = 0; k < TS_SEG; ++k) acc += v[u][k] * xq[k];
#pragma unroll
                    for (int m = 1; m < TS_LPR; m <<= 1) acc += __shfl_xor(acc, m);
                    const int r = r0 + u * TS_RPI + rr;
                    if (q == 0 && r < n) xl[r] -= acc;
                }
            }
        }
        __syncthreads();
    }
}

template <typename T>
__device__ __forceinline__ void trsv_bwd_solve(const T* __restrict__ L, int n, T* xl, T (*red)[NB]) {
    constexpr int TS_SEG = TSGeom<T>::SEG, TS_LPR = TSGeom<T>::LPR, TS_RPI = TSGeom<T>::RPI, TS_U = TSGeom<T>::U;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nblk = (n + NB - 1) / NB;
    for (int bi = nblk - 1; bi >= 0; --bi) {
        const int j0 = bi * NB, jb = min(NB, n - j0);
        const T* Lp = L + pp_block(n, bi);
        // L_blk^T x_below: the rows below the block as in the forward solve
        // (LPR lanes per packed row, one 16-byte chunk each, TU row groups in
        // flight); each lane accumulates its chunk's columns times x_r, the
        // lanes of one chunk position sum by xor shuffles, and the waves'
        // sums meet in LDS.
        {
            const int q = lane % TS_LPR, rr = lane / TS_LPR;
            T acc[TS_SEG];
#pragma unroll
            for (int k = 0; k < TS_SEG; ++k) acc[k] = (T)0;
            for (int r0 = j0 + jb + wv * TS_RPI * TS_U; r0 < n; r0 += (kWG / 64) * TS_RPI * TS_U) {
                T v[TS_U][TS_SEG], xr[TS_U];
#pragma unroll
                for (int u = 0; u < TS_U; ++u) {
                    const int r = r0 + u * TS_RPI + rr, rc = min(r, n - 1);
                    load_pseg<T, TS_SEG>(Lp + (int64_t)(rc - j0) * NB + q * TS_SEG, v[u]);
                    xr[u] = r < n ? xl[rc] : (T)0;
                }
#pragma unroll
                for (int u = 0; u < TS_U; ++u)
#pragma unroll
                    for (int k = 0; k < TS_SEG; ++k) acc[k] += v[u][k] * xr[u];
            }
#pragma unroll
            for (int k = 0; k < TS_SEG; ++k) {
#pragma unroll
                for (int m = TS_LPR; m < 64; m <<= 1) acc[k] += __shfl_xor(acc[k], m);
                if (rr == 0) red[wv][q * TS_SEG + k] = acc[k];
            }
        }
        __syncthreads();
        if (tid < 64) {
            const int i = min(lane, jb - 1);
            T dcol[NB];   // dcol[c] = L[j0 + c][j0 + i], used for c > i only
#pragma unroll
            for (int c = 0; c < NB; ++c) dcol[c] = Lp[(int64_t)min(c, jb - 1) * NB + i];
            const T rinv = (lane < jb) ? (T)1 / Lp[(int64_t)i * NB + i] : (T)0;
            T rhs = (T)0;
            if (lane < jb) rhs = xl[j0 + lane] - ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]));
#pragma unroll
            for (int c = NB - 1; c >= 0; --c) {
                if (c < jb) {
                    const T xc = lane_read(rhs, c) * lane_read(rinv, c);
                    rhs = (lane == c) ? xc : ((lane < c) ? rhs - dcol[c] * xc : rhs);
                }
            }
            if (lane < jb) xl[j0 + lane] = rhs;
        }
        __syncthreads();
    }
}

// One launch per solve: forward (FWD), backward (BWD) or both in turn on the
// same subdomain (FWD && BWD: the backward pass starts on the panels the
// forward pass streamed last, and x stays in LDS between them).  The
// arithmetic of each pass is the same in every form.
template <typename T, bool FWD, bool BWD>
__global__ __launch_bounds__(kWG) void k_trsv(const T* __restrict__ Lb, const int64_t* __restrict__ Loff,
                                             const int* __restrict__ nv, T* __restrict__ xb,
                                             const int64_t* __restrict__ xoff, int nb,
                                             const int* __restrict__ order, int* __restrict__ ctr) {
    extern __shared__ double trsv_lds[];
    T* xl = reinterpret_cast<T*>(trsv_lds);
    __shared__ T xs[FWD ? NB : 1];
    __shared__ T red[BWD ? kWG / 64 : 1][NB];
    for (int pass = 0;; ++pass) {
        const int s = next_item(order, ctr, nb, pass);
        if (s < 0) break;
        const T* L = Lb + Loff[s];
        T* x = xb + xoff[s];
        const int n = nv[s];
        for (int i = threadIdx.x; i < n; i += kWG) xl[i] = x[i];
        __syncthreads();
        if constexpr (FWD) trsv_fwd_solve<T>(L, n, xl, xs);
        if constexpr (BWD) trsv_bwd_solve<T>(L, n, xl, red);
        for (int i = threadIdx.x; i < n; i += kWG) x[i] = xl[i];
    }
}

// --------------------------------------------------------- deluxe operators
// Per face: S_F^j + S_F^k; per edge: sum_m S_E^(m) (Sec. 4.2).  The sum is
// inverted by the symmetric sweep (Gauss-Jordan) operator, which needs no
// pivoting for an SPD matrix: sweeping pivot k maps
//   a_ij -> a_ij - a_ik a_kj / a_kk,  a_ik, a_kj -> a_ik / a_kk,  a_kk -> -1 / a_kk,
// and sweeping every pivot leaves -(sum S)^{-1}; each step is one parallel
// pass over the matrix (the matrix is symmetric, so row k equals column k).
// Objects of up to 128 dofs sweep in registers (k_deluxe_small), edges and
// other small objects in LDS or, when the matrix does not fit, in the
// object's global workspace (k_deluxe_setup); larger faces sweep a block of
// pivots per pass (k_deluxe_blocked).  Then, for every sharing subdomain m, the
// operator E_m = S^(m) (sum S)^{-1} is formed: E_m g is the residual-side
// split and E_m^T u the value-side average term, so the per-iteration deluxe
// scaling is a set of dense GEMVs.  A non-positive pivot flags the object.
constexpr int DLX_MAXN = 1280;

// M = sum_m S^(m) over the shares of object ob (n x n, column-major), DS_U
// entries per thread and pass with all their loads issued together (clamped
// addresses, masked stores); called by the whole workgroup.
template <typename T>
__device__ void deluxe_sum(const ObjDesc& o, int ob, int n, T* M, const T* __restrict__ slots) {
    const int tid = threadIdx.x;
    {
        constexpr int DS_U = 8;
        const int nn = n * n;
        for (int base = 0; base < nn; base += kWG * DS_U) {
            T acc[DS_U];
#pragma unroll
            for (int u = 0; u < DS_U; ++u) acc[u] = (T)0;
            for (int q = o.sh_ptr[ob]; q < o.sh_ptr[ob + 1]; ++q) {
                const T* Sq = slots + o.sh_slot[q];
#pragma unroll
                for (int u = 0; u < DS_U; ++u) acc[u] += Sq[min(base + tid + u * kWG, nn - 1)];
            }
#pragma unroll
            for (int u = 0; u < DS_U; ++u)
                if (base + tid + u * kWG < nn) M[base + tid + u * kWG] = acc[u];
        }
    }
}

// E_m = S^(m) (sum S)^{-1} = -S^(m) M for the shares of object ob, given M =
// -(sum S)^{-1} (in LDS or global memory); called by the whole workgroup.
template <typename T, bool STRIP = true>
__device__ void deluxe_products(const ObjDesc& o, int ob, int n, const T* M, const T* __restrict__ slots,
                                T* __restrict__ dmat) {
    const int tid = threadIdx.x, wv0 = tid >> 6, lane0 = tid & 63;
    // M = -(sum S)^{-1};  E_m = S^(m) (sum S)^{-1} = -S^(m) M on MFMA 16x16x4
    // tiles (one wave per tile, S^(m) streamed from L2, M from LDS), for all
    // shares but the last; the E_m sum to the identity, which gives the last.
    const int wv = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    const int q0 = o.sh_ptr[ob], q1 = o.sh_ptr[ob + 1];
    const int nt = (n + 15) / 16;
    constexpr int DS_K = 32;   // k-steps of 4 held in registers: objects up to 128 dofs
    for (int q = q0; q < q1 - 1; ++q) {
        const T* S = slots + o.sh_slot[q];
        T* E = dmat + o.sh_slot[q];
        if (STRIP && n <= 4 * DS_K) {
            // one 16-row strip of S^(m) per wave, loaded into registers once
            // (one exposed latency) and reused for every column tile of E_m
            for (int ti = wv; ti < nt; ti += kWG / 64) {
                const int i = ti * 16 + lr, ic = min(i, n - 1);
                T a[DS_K];
#pragma unroll
                for (int s2 = 0; s2 < DS_K; ++s2) a[s2] = S[ic + (int64_t)min(4 * s2 + lk, n - 1) * n];
                for (int tj = 0; tj < nt; ++tj) {
                    const int j = tj * 16 + lr;
                    typename Mfma<T>::acc acc = {0, 0, 0, 0};
#pragma unroll
                    for (int s2 = 0; s2 < DS_K; ++s2) {
                        if (4 * s2 < n) {
                            const int k = 4 * s2 + lk;
                            const T av = (i < n && k < n) ? a[s2] : (T)0;
                            const T b = (k < n && j < n) ? M[k + j * n] : (T)0;
                            acc = Mfma<T>::mac(av, b, acc);
                        }
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = ti * 16 + Mfma<T>::row(lane, v);
                        if (r < n && j < n) E[r + j * n] = -acc[v];
                    }
                }
            }
            continue;
        }
        for (int tile = wv; tile < nt * nt; tile += kWG / 64) {
            const int i = (tile % nt) * 16 + lr, j = (tile / nt) * 16 + lr;
            typename Mfma<T>::acc acc = {0, 0, 0, 0};
            for (int k0 = 0; k0 < n; k0 += 4) {
                const int k = k0 + lk;
                const T a = (i < n && k < n) ? S[i + k * n] : (T)0;
                const T b = (k < n && j < n) ? M[k + j * n] : (T)0;
                acc = Mfma<T>::mac(a, b, acc);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = (tile % nt) * 16 + Mfma<T>::row(lane, v);
                if (r < n && j < n) E[r + j * n] = -acc[v];
            }
        }
    }
    __syncthreads();
    {
        T* E = dmat + o.sh_slot[q1 - 1];
        for (int j = wv0; j < n; j += kWG / 64)
            for (int i = lane0; i < n; i += 64) {
                const int64_t idx = i + (int64_t)j * n;
                T acc = (i == j) ? (T)1 : (T)0;
                for (int q = q0; q < q1 - 1; ++q) acc -= dmat[o.sh_slot[q] + idx];
                E[idx] = acc;
            }
    }
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_deluxe_setup(ObjDesc o, const T* __restrict__ slots,
                                                     T* __restrict__ fac, T* __restrict__ dmat,
                                                     int* __restrict__ info, int lds_cap, int ob0) {
    extern __shared__ double dlx_lds[];
    __shared__ T ck[DLX_MAXN];
    __shared__ int bad;
    const int ob = ob0 + blockIdx.x;
    const int n = o.n[ob];
    const int tid = threadIdx.x, wv0 = tid >> 6, lane0 = tid & 63;
    T* M = (n * n <= lds_cap) ? reinterpret_cast<T*>(dlx_lds) : fac + o.fac_off[ob];
    if (tid == 0) bad = 0;
    deluxe_sum<T>(o, ob, n, M, slots);
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        for (int i = tid; i < n; i += kWG) ck[i] = M[i + k * n];
        __syncthreads();
        T d = ck[k];
        if (!(d > (T)0)) {
            if (tid == 0) bad = 1;
            d = (T)1;
        }
        const T rd = (T)1 / d;
        // waves over columns, lanes over rows (no integer division per entry)
        for (int j = wv0; j < n; j += kWG / 64) {
            const T cj = ck[j];
            T* Mj = M + (int64_t)j * n;
            for (int i = lane0; i < n; i += 64) {
                const T ci = ck[i];
                T v;
                if (i == k) v = (j == k) ? -rd : cj * rd;
                else if (j == k) v = ci * rd;
                else v = Mj[i] - ci * cj * rd;
                Mj[i] = v;
            }
        }
        __syncthreads();
    }
    deluxe_products<T>(o, ob, n, M, slots, dmat);
    if (tid == 0 && bad) info[ob] = 1;
}

// Objects of more than DS_N dofs (faces of subdomains from H/h = 10 up):
// M = -(sum S)^{-1} by the sweep taken DB_W pivots at a time, with M in the
// object's global workspace.  For the pivot block K (D = M_KK, C = M_RK the
// rows R outside K) the sweep of all its pivots at once is
//   M_KK <- -D^{-1},  M_RK <- C D^{-1},  M_RR <- M_RR - C D^{-1} C^T,
// the composition of the single-pivot sweeps of K.  -D^{-1} comes from the
// scalar sweep of the small block in LDS; H = C (-D^{-1}) is staged in LDS
// (n x DB_W); M_RR gets the rank-DB_W update H C^T on MFMA 16x16x4 tiles
// (one wave per tile, C read from the untouched columns K), then the pivot
// rows and columns are written.  Each block reads and writes M once, where
// the single-pivot sweep does so per pivot.
template <typename T>
constexpr int deluxe_block_width() { return 64 / (int)sizeof(T); }   // 16 (FP32), 8 (FP64)

template <typename T>
__global__ __launch_bounds__(kWG) void k_deluxe_blocked(ObjDesc o, const T* __restrict__ slots,
                                                       T* __restrict__ fac, T* __restrict__ dmat,
                                                       int* __restrict__ info, int ob0) {
    constexpr int BW = deluxe_block_width<T>();
    extern __shared__ double dlx_lds[];
    T* H = reinterpret_cast<T*>(dlx_lds);            // [n][BW]
    __shared__ T Dk[BW][BW + 1];
    __shared__ int bad;
    const int ob = ob0 + blockIdx.x;
    const int n = o.n[ob];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    T* M = fac + o.fac_off[ob];
    if (tid == 0) bad = 0;
    deluxe_sum<T>(o, ob, n, M, slots);
    __syncthreads();
    const int nt = (n + 15) / 16;
    for (int k0 = 0; k0 < n; k0 += BW) {
        const int b = min(BW, n - k0);
        // D, padded with the identity beyond the object
        for (int e = tid; e < BW * BW; e += kWG) {
            const int i = e % BW, j = e / BW;
            Dk[i][j] = (i < b && j < b) ? M[(k0 + i) + (int64_t)(k0 + j) * n] : (i == j ? (T)1 : (T)0);
        }
        __syncthreads();
        // Dk <- -D^{-1}: one entry per thread (BW * BW <= kWG), two barriers per pivot
        {
            const int i = tid % BW, j = tid / BW;
            const bool mine = tid < BW * BW;
            for (int k = 0; k < BW; ++k) {
                T d = Dk[k][k], ci = mine ? Dk[i][k] : (T)0, cj = mine ? Dk[j][k] : (T)0, mij = mine ? Dk[i][j] : (T)0;
                if (!(d > (T)0)) {
                    if (tid == 0) bad = 1;
                    d = (T)1;
                }
                const T rd = (T)1 / d;
                __syncthreads();
                if (mine) {
                    T v;
                    if (i == k) v = (j == k) ? -rd : cj * rd;
                    else if (j == k) v = ci * rd;
                    else v = mij - ci * cj * rd;
                    Dk[i][j] = v;
                }
                __syncthreads();
            }
        }
        // H = C Dk (rows in K included; they are overwritten below)
        for (int r = tid; r < n; r += kWG) {
            T cr[BW];
#pragma unroll
            for (int j = 0; j < BW; ++j) cr[j] = j < b ? M[r + (int64_t)(k0 + j) * n] : (T)0;
#pragma unroll 1
            for (int c = 0; c < BW; ++c) {
                T acc = (T)0;
#pragma unroll
                for (int j = 0; j < BW; ++j) acc += cr[j] * Dk[j][c];
                H[r * BW + c] = acc;
            }
        }
        __syncthreads();
        // M_RR += H C^T on 16 x 16 tiles; entries in the rows or columns K are
        // left for the pivot write below (the columns K are only read here)
        // two tiles per wave and pass, their loads issued together
        constexpr int TP = 2, NW = kWG / 64;
        for (int t0 = wv; t0 < nt * nt; t0 += TP * NW) {
            typename Mfma<T>::acc acc[TP];
            T bk[TP][BW / 4];
#pragma unroll
            for (int u = 0; u < TP; ++u) {
                const int t = min(t0 + u * NW, nt * nt - 1);
                const int I0 = (t % nt) * 16, col = (t / nt) * 16 + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = I0 + Mfma<T>::row(lane, v);
                    acc[u][v] = M[min(row, n - 1) + (int64_t)min(col, n - 1) * n];
                }
#pragma unroll
                for (int kq = 0; kq < BW / 4; ++kq) {
                    const int k = 4 * kq + lk;
                    bk[u][kq] = M[min(col, n - 1) + (int64_t)(k0 + min(k, b - 1)) * n];
                }
            }
#pragma unroll
            for (int u = 0; u < TP; ++u) {
                const int t = t0 + u * NW;
                if (t >= nt * nt) continue;
                const int I0 = (t % nt) * 16, col = (t / nt) * 16 + lr;
#pragma unroll
                for (int kq = 0; kq < BW / 4; ++kq) {
                    const int k = 4 * kq + lk;
                    const T a = (I0 + lr < n) ? H[(I0 + lr) * BW + k] : (T)0;
                    const T bb = (k < b && col < n) ? bk[u][kq] : (T)0;
                    acc[u] = Mfma<T>::mac(a, bb, acc[u]);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = I0 + Mfma<T>::row(lane, v);
                    const bool rk = row >= k0 && row < k0 + b, ck = col >= k0 && col < k0 + b;
                    if (row < n && col < n && !rk && !ck) M[row + (int64_t)col * n] = acc[u][v];
                }
            }
        }
        __syncthreads();
        // pivot rows and columns: M_RK = -H, M_KR = -H^T, M_KK = Dk
        for (int e = tid; e < n * b; e += kWG) {
            const int r = e % n, c = e / n;
            const T v = (r >= k0 && r < k0 + b) ? Dk[r - k0][c] : -H[r * BW + c];
            M[r + (int64_t)(k0 + c) * n] = v;
            M[(k0 + c) + (int64_t)r * n] = v;
        }
        __syncthreads();
    }
    deluxe_products<T, false>(o, ob, n, M, slots, dmat);
    if (tid == 0 && bad) info[ob] = 1;
}

// Objects of DS_MIN < n <= DS_N dofs (the faces of subdomains up to H/h = 8,
// with their boundary nodes): the sweep runs in registers.  Thread (wave w,
// lane l) holds the entries (i = l + 64 a, j = w + 4 b) of sum S; for each
// pivot k the lane holding row k publishes it (the matrix stays symmetric,
// so row k is column k) into one of two LDS vectors, one barrier, and every
// thread updates its own entries.  The code is straight-line: indices are
// clamped into the object and entries beyond n are carried along but never
// stored.  The result -(sum S)^{-1} goes to LDS for the MFMA products
// E_m = -S^(m) M (per wave a 16-row strip of S^(m), per 16x16 tile all the
// strip's loads issued together); the last share's E is the identity minus
// the others, formed from the same product tiles without reading them back.
constexpr int DS_N = 128, DS_MIN = 32;

template <typename T>
__global__ __launch_bounds__(kWG, sizeof(T) == 4 ? 2 : 1) void k_deluxe_small(
    ObjDesc o, const T* __restrict__ slots, T* __restrict__ fac, T* __restrict__ dmat, int* __restrict__ info,
    int lds_cap, int ob0) {
    extern __shared__ double dlx_lds[];
    __shared__ T ck[2][DS_N];
    __shared__ int bad;
    constexpr int NA = DS_N / 64, NBW = DS_N / (kWG / 64), DS_K = DS_N / 4;
    const int ob = ob0 + blockIdx.x;
    const int n = o.n[ob];
    // the wave index is uniform within a wave: column indices, offsets and
    // tests derived from it stay in scalar registers
    const int tid = threadIdx.x, wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int wvv = tid >> 6;   // the same wave index as a per-lane value: tests on it compile to selects
    T* M = (n * n <= lds_cap) ? reinterpret_cast<T*>(dlx_lds) : fac + o.fac_off[ob];
    if (tid == 0) bad = 0;
    const int q0 = o.sh_ptr[ob], q1 = o.sh_ptr[ob + 1];
    int ri[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) ri[a] = min(lane + 64 * a, n - 1);
    T r[NA][NBW];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NBW; ++b) r[a][b] = (T)0;
    for (int q = q0; q < q1; ++q) {
        const T* Sq = slots + o.sh_slot[q];
#pragma unroll
        for (int b = 0; b < NBW; ++b) {
            const T* col = Sq + (int64_t)min(wv + 4 * b, n - 1) * n;
#pragma unroll
            for (int a = 0; a < NA; ++a) r[a][b] += col[ri[a]];
        }
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const int buf = k & 1;
        if (lane == (k & 63)) {
            const bool hi = k >= 64;
#pragma unroll
            for (int b = 0; b < NBW; ++b) ck[buf][wv + 4 * b] = hi ? r[NA - 1][b] : r[0][b];
        }
        __syncthreads();
        T d = ck[buf][k];
        if (!(d > (T)0)) {
            if (tid == 0) bad = 1;
            d = (T)1;
        }
        const T rd = (T)1 / d;
        T ci[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) ci[a] = ck[buf][ri[a]];
#pragma unroll
        for (int b = 0; b < NBW; ++b) {
            const T cj = ck[buf][min(wv + 4 * b, n - 1)];
            const bool jk = wvv + 4 * b == k;
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const bool ik = lane + 64 * a == k;
                const T v = r[a][b];
                const T g = v - ci[a] * cj * rd;                 // entries off row and column k
                const T e = ik ? (jk ? -rd : cj * rd) : ci[a] * rd;
                r[a][b] = (ik || jk) ? e : g;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NBW; ++b) {
            const int i = lane + 64 * a, j = wv + 4 * b;
            if (i < n && j < n) M[i + j * n] = r[a][b];
        }
    __syncthreads();
    const int nt = (n + 15) / 16;
    for (int ti = wv; ti < nt; ti += kWG / 64) {
        const int i = ti * 16 + lr, ic = min(i, n - 1);
        for (int tj = 0; tj < nt; ++tj) {
            const int j = tj * 16 + lr, jc = min(j, n - 1);
            typename Mfma<T>::acc esum = {0, 0, 0, 0};
            for (int q = q0; q < q1 - 1; ++q) {
                const T* S = slots + o.sh_slot[q];
                T av[DS_K];
#pragma unroll
                for (int s2 = 0; s2 < DS_K; ++s2) av[s2] = S[ic + (int64_t)min(4 * s2 + lk, n - 1) * n];
                typename Mfma<T>::acc acc = {0, 0, 0, 0};
#pragma unroll
                for (int s2 = 0; s2 < DS_K; ++s2) {
                    const int k = 4 * s2 + lk;
                    const T y = M[min(k, n - 1) + jc * n];
                    const bool in = k < n;
                    acc = Mfma<T>::mac((in && i < n) ? av[s2] : (T)0, (in && j < n) ? y : (T)0, acc);
                }
                T* E = dmat + o.sh_slot[q];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rr = ti * 16 + Mfma<T>::row(lane, v);
                    if (rr < n && j < n) E[rr + j * n] = -acc[v];
                }
                esum += acc;
            }
            T* E = dmat + o.sh_slot[q1 - 1];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = ti * 16 + Mfma<T>::row(lane, v);
                if (rr < n && j < n) E[rr + j * n] = (rr == j ? (T)1 : (T)0) + esum[v];
            }
        }
    }
    __syncthreads();
    if (tid == 0 && bad) info[ob] = 1;
}

}  // namespace

template <typename T>
void launch_assemble(hipStream_t s, const BatchDesc& d, int maxbox, const FEParams& p,
                     const double* ke, const double* v, const double* w, T* K) {
    dim3 grid((unsigned)((maxbox * 27 + kWG - 1) / kWG), (unsigned)d.nsub);
    hipLaunchKernelGGL(k_assemble<T>, grid, dim3(kWG), 0, s, d, p, ke, v, w, K);
}
template <typename T>
void launch_potrf(hipStream_t s, int nb, T* A, const int64_t* off, const int* ld, const int* c0,
                  const int* c1, const int* c2, int* info) {
    hipLaunchKernelGGL(k_potrf<T>, dim3(nb), dim3(kWG), 0, s, A, off, ld, c0, c1, c2, info);
}
template <typename T>
void launch_interior_panel(hipStream_t s, int nb, T* A, const int64_t* off, const int* ld, const int* nI,
                           const int* n, int J, T* Wbuf, int rowblocks, int* info, T* P, const int64_t* poff,
                           const int* nIc) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_panel_diag<T>, dim3(nb), dim3(kWG), 0, s, A, off, ld, nI, J, Wbuf, info, P, poff);
    if (rowblocks > 0) {
        const int groups = (nb + PT_XCD - 1) / PT_XCD;
        hipLaunchKernelGGL(k_panel_trsm<T>, dim3(groups * rowblocks * PT_XCD), dim3(kWG), 0, s, A, off, ld, nI, n, nb,
                           rowblocks, J, Wbuf, P, poff, nIc);
    }
}
template <typename T>
void launch_syrk_update(hipStream_t s, int nb, T* A, const int64_t* off, const int* ld, const int* nI, const int* n,
                        bool schur, int J, int tiles, int variant, const int* nIc) {
    if (nb <= 0 || tiles <= 0) return;
    const int groups = (nb + SY_XCD - 1) / SY_XCD;
    const dim3 grid(groups * tiles * SY_XCD);
    const int mode = schur ? SY_SCHUR : SY_TRAIL;
    switch (variant) {
        case 1: hipLaunchKernelGGL((k_syrk_batched<T, 128, 16>), grid, dim3(kWG), 0, s, A, off, ld, nI, n, nIc, nb, tiles, mode, J); break;
        case 2: hipLaunchKernelGGL((k_syrk_batched<T, 64, 32>), grid, dim3(kWG), 0, s, A, off, ld, nI, n, nIc, nb, tiles, mode, J); break;
        case 3: hipLaunchKernelGGL((k_syrk_batched<T, 64, 16>), grid, dim3(kWG), 0, s, A, off, ld, nI, n, nIc, nb, tiles, mode, J); break;
        case 4: hipLaunchKernelGGL((k_syrk_batched<T, 64, 16, true, true>), grid, dim3(kWG), 0, s, A, off, ld, nI, n, nIc, nb, tiles, mode, J); break;
        case 5: hipLaunchKernelGGL((k_syrk_batched<T, 64, 16, true>), grid, dim3(kWG), 0, s, A, off, ld, nI, n, nIc, nb, tiles, mode, J); break;
        default: hipLaunchKernelGGL((k_syrk_batched<T, 128, 32>), grid, dim3(kWG), 0, s, A, off, ld, nI, n, nIc, nb, tiles, mode, J);
    }
}
int syrk_variants() { return SY_NVAR; }
int syrk_variant_tm(int v) { return syrk_tm(v); }
int syrk_variant_kc(int v) { return syrk_kc(v); }
int interior_panel_width() { return NBO; }
int panel_wbuf_stride() { return NBO * NB; }
int panel_rowblocks(int J, int nI, int n, int nIc) {
    if (J >= nI) return 0;
    const int r0 = J + std::min(NBO, nI - J);
    const int re = r0 <= nIc ? nI : n;   // a core panel's interface row blocks have nothing to do
    return r0 < re ? (re - r0 + PT_RB - 1) / PT_RB : 0;
}
int syrk_tiles(bool schur, int J, int nI, int n, int variant, int nIc) {
    const int TM = syrk_tm(variant);
    if (schur) return trapezoid_tiles(nI, n, n, TM);
    if (J >= nI) return 0;
    return trapezoid_tiles(J + NBO, nI, std::min(J + NBO, nI) <= nIc ? nI : n, TM);
}
template <typename T>
void launch_extract(hipStream_t s, const BatchDesc& d, const T* K, T* slots, T* F, double* Svv, T* Srr) {
    hipLaunchKernelGGL(k_extract<T>, dim3(d.nsub), dim3(kWG), 0, s, d, K, slots, F, Svv, Srr);
}
template <typename T>
void launch_clear_lower(hipStream_t s, const BatchDesc& d, int maxn, T* K) {
    if (d.nsub <= 0 || maxn <= 0) return;
    hipLaunchKernelGGL(k_clear_lower<T>, dim3((unsigned)((maxn + CL_COLS - 1) / CL_COLS), (unsigned)d.nsub),
                       dim3(kWG), 0, s, d, K);
}
template <typename T>
void launch_trsm_fwd(hipStream_t s, int nb, const T* L, const int64_t* Loff, const int* n, T* B,
                     const int64_t* Boff, const int* ldb, const int* k) {
    hipLaunchKernelGGL(k_trsm_fwd<T>, dim3(nb), dim3(kWG), 0, s, L, Loff, n, B, Boff, ldb, k);
}
template <typename T>
void launch_coarse_local(hipStream_t s, const BatchDesc& d, const T* F, const double* Svv, T* Z,
                         double* Sp, int* info) {
    hipLaunchKernelGGL(k_coarse_local<T>, dim3(d.nsub), dim3(kWG), 0, s, d, F, Svv, Z, Sp, info);
    hipLaunchKernelGGL(k_coarse_kernel_fix, dim3(d.nsub), dim3(kWG), 0, s, d.sub0, d.nV, d.nc, Sp);
}
template <typename T, bool FWD, bool BWD>
void launch_trsv_kern(hipStream_t s, int nb, const T* L, const int64_t* Loff, const int* n, T* x,
                      const int64_t* xoff, int maxn, const WorkQueue& q) {
    if (nb <= 0 || maxn <= 0) return;
    const size_t lds = (size_t)maxn * sizeof(T);
    auto kern = k_trsv<T, FWD, BWD>;
    int grid = nb;
    if (q.order && q.counter) {
        // persistent: as many workgroups as are resident at once (at least one)
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kWG, lds) == hipSuccess)
            grid = std::max(1, std::min(nb, cus * per));
    }
    const int* ord = q.order;
    int* ctr = (q.order && q.counter) ? q.counter : nullptr;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWG), lds, s, L, Loff, n, x, xoff, nb, ord, ctr);
}
template <typename T>
void launch_trsv(hipStream_t s, int nb, bool trans, const T* L, const int64_t* Loff, const int* n, T* x,
                 const int64_t* xoff, int maxn, const WorkQueue& q) {
    if (trans) launch_trsv_kern<T, false, true>(s, nb, L, Loff, n, x, xoff, maxn, q);
    else launch_trsv_kern<T, true, false>(s, nb, L, Loff, n, x, xoff, maxn, q);
}
template <typename T>
void launch_trsv_fb(hipStream_t s, int nb, const T* L, const int64_t* Loff, const int* n, T* x,
                    const int64_t* xoff, int maxn, const WorkQueue& q) {
    launch_trsv_kern<T, true, true>(s, nb, L, Loff, n, x, xoff, maxn, q);
}
// Objects above DS_N dofs take the blocked sweep unless BDM_DELUXE_SCALAR=1
// (the single-pivot sweep of k_deluxe_setup, kept for comparison).
static bool deluxe_scalar_sweep() {
    static int v = -1;
    if (v < 0) {
        const char* e = std::getenv("BDM_DELUXE_SCALAR");
        v = (e && std::atoi(e) != 0) ? 1 : 0;
    }
    return v == 1;
}

template <typename T>
void launch_deluxe_setup(hipStream_t s, const ObjDesc& o, int ob0, int nob, int maxn, const T* slots, T* fac, T* dmat,
                         int* info) {
    if (nob <= 0) return;
    static int lds_max = -1;   // bytes of LDS a workgroup may use on this device
    if (lds_max < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 65536;
        lds_max = v;
    }
    if (maxn > DS_MIN && maxn <= DS_N) {
        // The register sweep is latency-bound, so the LDS kept for the inverse
        // is sized for several resident workgroups per CU rather than for the
        // largest face: objects whose inverse does not fit keep it in their
        // global workspace (same arithmetic).  BDM_DELUXE_WG_PER_CU (1-16)
        // overrides the target.
        static int lds_cu = -1, per_cu = -1;
        if (lds_cu < 0) {
            int dev = 0, v = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
                v <= 0)
                v = lds_max;
            lds_cu = v;
            per_cu = 6;
            if (const char* e = std::getenv("BDM_DELUXE_WG_PER_CU")) per_cu = std::min(16, std::max(1, std::atoi(e)));
        }
        const int stat = (int)(2 * DS_N * sizeof(T)) + 64;
        const int avail = std::min(lds_max, lds_cu / per_cu) - stat;
        const int cap = std::max(0, std::min(maxn * maxn, avail / (int)sizeof(T)));
        hipLaunchKernelGGL(k_deluxe_small<T>, dim3(nob), dim3(kWG), (size_t)cap * sizeof(T), s, o, slots, fac, dmat,
                           info, cap, ob0);
        return;
    }
    if (maxn > DS_N && !deluxe_scalar_sweep()) {
        hipLaunchKernelGGL(k_deluxe_blocked<T>, dim3(nob), dim3(kWG),
                           (size_t)maxn * deluxe_block_width<T>() * sizeof(T), s, o, slots, fac, dmat, info, ob0);
        return;
    }
    const int avail = lds_max - (int)(DLX_MAXN * sizeof(T)) - 64;
    const int cap = std::max(0, std::min(maxn * maxn, avail / (int)sizeof(T)));
    hipLaunchKernelGGL(k_deluxe_setup<T>, dim3(nob), dim3(kWG), (size_t)cap * sizeof(T), s, o, slots, fac, dmat,
                       info, cap, ob0);
}
int deluxe_max_object() { return DLX_MAXN; }

#define BDM_INST(T)                                                                                     \
    template void launch_assemble<T>(hipStream_t, const BatchDesc&, int, const FEParams&, const double*, \
                                     const double*, const double*, T*);                                \
    template void launch_potrf<T>(hipStream_t, int, T*, const int64_t*, const int*, const int*,         \
                                  const int*, const int*, int*);                                         \
    template void launch_interior_panel<T>(hipStream_t, int, T*, const int64_t*, const int*, const int*, \
                                           const int*, int, T*, int, int*, T*, const int64_t*,           \
                                           const int*);                                                   \
    template void launch_syrk_update<T>(hipStream_t, int, T*, const int64_t*, const int*, const int*,    \
                                        const int*, bool, int, int, int, const int*);                    \
    template void launch_extract<T>(hipStream_t, const BatchDesc&, const T*, T*, T*, double*, T*);      \
    template void launch_clear_lower<T>(hipStream_t, const BatchDesc&, int, T*);                       \
    template void launch_trsm_fwd<T>(hipStream_t, int, const T*, const int64_t*, const int*, T*,         \
                                     const int64_t*, const int*, const int*);                            \
    template void launch_coarse_local<T>(hipStream_t, const BatchDesc&, const T*, const double*, T*, \
                                         double*, int*);                                                 \
    template void launch_trsv<T>(hipStream_t, int, bool, const T*, const int64_t*, const int*, T*,      \
                                 const int64_t*, int, const WorkQueue&);                                 \
    template void launch_trsv_fb<T>(hipStream_t, int, const T*, const int64_t*, const int*, T*,      \
                                 const int64_t*, int, const WorkQueue&);                                 \
    template void launch_deluxe_setup<T>(hipStream_t, const ObjDesc&, int, int, int, const T*, T*, T*, int*);
BDM_INST(double)
BDM_INST(float)
#undef BDM_INST

}  // namespace bdm
