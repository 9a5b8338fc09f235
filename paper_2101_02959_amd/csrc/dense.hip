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
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace bdm {

constexpr int NB = 32;          // panel / block width
constexpr int MAXC = 24;        // edge constraints per subdomain (12 edges x 2)
constexpr int MAXV = 16;        // vertex dofs per subdomain (8 vertices x 2)
constexpr int MAXP = MAXC + MAXV;
constexpr int SVV_STRIDE = MAXV * MAXV;
constexpr int GI_STRIDE = MAXC * MAXC;
constexpr int SP_STRIDE = MAXP * MAXP;

namespace {

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// -------------------------------------------------------------- assembly
// K^(j) of the Jacobian bilinear form restricted to Omega_j (Sec. 4.1) in
// the congruent (v, u_e) form: per node pair (P, Q) the 2x2 block
//   [[a_i + d_P delta_PQ, a_i], [a_i, a_i + a_e]],
// a_* = (tau A_*^(j))_PQ from the elements of the subdomain only, and
// d_P = m_P^(j) (chi C_m + tau dI_ion/dv) with the local lumped mass.
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
    double ai = 0.0, ae = 0.0;
    int nel = 0;
    for (int oz = 0; oz < 2; ++oz)
        for (int oy = 0; oy < 2; ++oy)
            for (int ox = 0; ox < 2; ++ox) {
                const int ei = pi - 1 + ox, ej = pj - 1 + oy, ek = pk - 1 + oz;
                if (ei < 0 || ei >= Lx || ej < 0 || ej >= Ly || ek < 0 || ek >= Lz) continue;
                ++nel;
                const int bxl = 1 - ox + dx, byl = 1 - oy + dy, bzl = 1 - oz + dz;
                if (bxl < 0 || bxl > 1 || byl < 0 || byl > 1 || bzl < 0 || bzl > 1) continue;
                const int a = (1 - ox) + 2 * (1 - oy) + 4 * (1 - oz);
                const int b = bxl + 2 * byl + 4 * bzl;
                const int L = ez0 + ek;
                ai += ke[((size_t)L * 2 + 0) * 64 + a * 8 + b];
                ae += ke[((size_t)L * 2 + 1) * 64 + a * 8 + b];
            }
    double dP = 0.0;
    if (dd == 13) {
        const int64_t g = (int64_t)(ex0 + pi) + (int64_t)p.nx1 * ((ey0 + pj) + (int64_t)p.ny1 * (ez0 + pk));
        const double m = p.h * p.h * p.h * 0.125 * nel;
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
// Right-looking blocked Cholesky of columns [c0, c1) of a symmetric matrix
// (lower triangle), with the trailing update applied to rows/cols < c2.
// After eliminating the interior block the trailing block holds the Schur
// complement K_GG - K_GI K_II^{-1} K_IG (Sec. 4.1).
template <typename T>
__global__ __launch_bounds__(kWG) void k_potrf(T* __restrict__ Abase, const int64_t* __restrict__ off,
                                              const int* __restrict__ ldv, const int* __restrict__ c0v,
                                              const int* __restrict__ c1v, const int* __restrict__ c2v,
                                              int* __restrict__ info) {
    const int s = blockIdx.x;
    T* A = Abase + off[s];
    const int64_t ld = ldv[s];
    const int cbeg = c0v[s], cend = c1v[s], c2 = c2v[s];
    const int tid = threadIdx.x;
    __shared__ T D[NB][NB + 1];
    __shared__ int bad;
    if (tid == 0) bad = 0;
    for (int j0 = cbeg; j0 < cend; j0 += NB) {
        const int jb = min(NB, cend - j0);
        // 1. diagonal block
        for (int idx = tid; idx < NB * NB; idx += kWG) {
            const int i = idx % NB, j = idx / NB;
            T val = (T)0;
            if (i < jb && j < jb && j <= i) val = A[(j0 + i) + (j0 + j) * ld];
            else if (i == j) val = (T)1;
            D[i][j] = val;
        }
        __syncthreads();
        for (int k = 0; k < jb; ++k) {
            if (tid == 0) {
                T dk = D[k][k];
                if (!(dk > (T)0)) { bad = 1; dk = (T)1; }
                D[k][k] = sqrt(dk);
            }
            __syncthreads();
            const T piv = D[k][k];
            for (int i = k + 1 + tid; i < jb; i += kWG) D[i][k] /= piv;
            __syncthreads();
            const int m = jb - k - 1;
            for (int idx = tid; idx < m * m; idx += kWG) {
                const int i = k + 1 + idx % m, j = k + 1 + idx / m;
                if (j <= i) D[i][j] -= D[i][k] * D[j][k];
            }
            __syncthreads();
        }
        for (int idx = tid; idx < jb * jb; idx += kWG) {
            const int i = idx % jb, j = idx / jb;
            if (j <= i) A[(j0 + i) + (j0 + j) * ld] = D[i][j];
        }
        // 2. panel below: row r <- row r * L_d^{-T}
        const int t0 = j0 + jb;
        for (int r = t0 + tid; r < c2; r += kWG) {
            T x[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) x[c] = (c < jb) ? A[r + (j0 + c) * ld] : (T)0;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                T acc = x[c];
#pragma unroll
                for (int k = 0; k < c; ++k) acc -= x[k] * D[c][k];
                x[c] = acc / D[c][c];
            }
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < jb) A[r + (j0 + c) * ld] = x[c];
        }
        __syncthreads();
        // 3. trailing update (lower triangle), 32x32 tiles, one wave per tile
        const int nt = (c2 - t0 + 31) / 32;
        const int ntiles = nt * (nt + 1) / 2;
        const int wv = tid / 64, lane = tid % 64, tx = lane % 8, ty = lane / 8;
        for (int tile = wv; tile < ntiles; tile += kWG / 64) {
            int ti = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
            while (ti * (ti + 1) / 2 > tile) --ti;
            while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
            const int tj = tile - ti * (ti + 1) / 2;
            const int I0 = t0 + ti * 32 + 4 * ty, J0 = t0 + tj * 32 + 4 * tx;
            T acc[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = (T)0;
            for (int c = 0; c < jb; ++c) {
                const T* col = A + (j0 + c) * ld;
                T av[4], bv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    av[q] = (I0 + q < c2) ? col[I0 + q] : (T)0;
                    bv[q] = (J0 + q < c2) ? col[J0 + q] : (T)0;
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int i = I0 + a, j = J0 + b;
                    if (i < c2 && j < c2 && i >= j) A[i + (int64_t)j * ld] -= acc[a][b];
                }
        }
        __syncthreads();
    }
    if (tid == 0 && bad) info[s] = 1;
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
        const int e = d.so_eidx[q];
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

// Copy the lower triangles of the Dirichlet factor L_II and the Neumann
// factor L_rr out of the chunk workspace into compact square storage.
template <typename T>
__global__ __launch_bounds__(kWG) void k_copy_out(BatchDesc d, const T* __restrict__ K, T* __restrict__ LII,
                                                 const int64_t* __restrict__ LIIoff, T* __restrict__ Lrr,
                                                 const int64_t* __restrict__ Lrroff) {
    const int s = d.sub0 + blockIdx.x;
    const int64_t ld = d.n[s];
    const int nI = d.nI[s], nr = d.nr[s];
    const T* A = K + d.K_off[s];
    T* a = LII + LIIoff[s];
    for (int64_t idx = threadIdx.x; idx < (int64_t)nI * nI; idx += kWG) {
        const int i = (int)(idx % nI), j = (int)(idx / nI);
        a[idx] = (i >= j) ? A[i + (int64_t)j * ld] : (T)0;
    }
    const T* B = A + (int64_t)nI * (ld + 1);
    T* b = Lrr + Lrroff[s];
    for (int64_t idx = threadIdx.x; idx < (int64_t)nr * nr; idx += kWG) {
        const int i = (int)(idx % nr), j = (int)(idx / nr);
        b[idx] = (i >= j) ? B[i + (int64_t)j * ld] : (T)0;
    }
}

// ----------------------------------------------------- multi-RHS forward
// L X = B in place (L lower n x n, B n x k, k <= 64).
template <typename T>
__global__ __launch_bounds__(kWG) void k_trsm_fwd(const T* __restrict__ Lb, const int64_t* __restrict__ Loff,
                                                 const int* __restrict__ nv, const int* __restrict__ ldv,
                                                 T* __restrict__ Bb, const int64_t* __restrict__ Boff,
                                                 const int* __restrict__ ldbv, const int* __restrict__ kv) {
    const int s = blockIdx.x;
    const T* L = Lb + Loff[s];
    T* B = Bb + Boff[s];
    const int n = nv[s], k = kv[s];
    const int64_t ld = ldv[s], ldb = ldbv[s];
    const int tid = threadIdx.x;
    __shared__ T D[NB][NB + 1];
    __shared__ T X[NB][64 + 1];
    for (int j0 = 0; j0 < n; j0 += NB) {
        const int jb = min(NB, n - j0);
        for (int idx = tid; idx < NB * NB; idx += kWG) {
            const int i = idx % NB, j = idx / NB;
            D[i][j] = (i < jb && j <= i) ? L[(j0 + i) + (j0 + j) * ld] : (T)0;
        }
        for (int idx = tid; idx < jb * k; idx += kWG) {
            const int i = idx % jb, c = idx / jb;
            X[i][c] = B[(j0 + i) + c * ldb];
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
        const int t0 = j0 + jb, nrow = n - t0;
        for (int idx = tid; idx < nrow * k; idx += kWG) {
            const int r = t0 + idx % nrow, c = idx / nrow;
            T acc = (T)0;
            for (int m = 0; m < jb; ++m) acc += L[r + (j0 + m) * ld] * X[m][c];
            B[r + c * ldb] -= acc;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------- coarse algebra
// With Y = L_rr^{-1} C^T and X = -L_rr^{-1} S_rV (from k_trsm_fwd), the
// energy-minimising coarse basis of Sec. 4.4 under the edge-average
// constraints is Phi_r = L_rr^{-T} Z with
//   G = Y^T Y = C S_rr^{-1} C^T,  mu_V = G^{-1} Y^T X,
//   Z = [X - Y mu_V | Y G^{-1}]   (vertex primals, then edge primals),
// and the local coarse matrix Phi^T S_Gamma Phi is
//   vertex rows: [-X^T Z + [S_VV | 0]],   edge rows: [-mu_V | G^{-1}].
template <typename T>
__global__ __launch_bounds__(kWG) void k_coarse_local(BatchDesc d, const T* __restrict__ Fb,
                                                     const double* __restrict__ Svv, T* __restrict__ Zb,
                                                     T* __restrict__ Gib, double* __restrict__ Spb,
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
    // G = Y^T Y
    for (int idx = tid; idx < nc * nc; idx += kWG) {
        const int i = idx % nc, j = idx / nc;
        if (j > i) continue;
        double acc = 0.0;
        for (int r = 0; r < nr; ++r) acc += (double)Y[r + (int64_t)i * nr] * (double)Y[r + (int64_t)j * nr];
        G[i][j] = acc;
        G[j][i] = acc;
    }
    for (int idx = tid; idx < nc * nV; idx += kWG) {
        const int i = idx % nc, q = idx / nc;
        double acc = 0.0;
        for (int r = 0; r < nr; ++r) acc += (double)Y[r + (int64_t)i * nr] * (double)X[r + (int64_t)q * nr];
        YtX[i][q] = acc;
    }
    __syncthreads();
    if (tid == 0) {   // Cholesky of the small constraint matrix
        for (int k = 0; k < nc; ++k) {
            double dk = G[k][k];
            for (int m = 0; m < k; ++m) dk -= G[k][m] * G[k][m];
            if (!(dk > 0.0)) { info[s] = 2; dk = 1.0; }
            dk = sqrt(dk);
            G[k][k] = dk;
            for (int i = k + 1; i < nc; ++i) {
                double a = G[i][k];
                for (int m = 0; m < k; ++m) a -= G[i][m] * G[k][m];
                G[i][k] = a / dk;
            }
        }
    }
    __syncthreads();
    if (tid < nc) {   // column tid of G^{-1}
        double y[MAXC];
        for (int i = 0; i < nc; ++i) {
            double a = (i == tid) ? 1.0 : 0.0;
            for (int m = 0; m < i; ++m) a -= G[i][m] * y[m];
            y[i] = a / G[i][i];
        }
        for (int i = nc - 1; i >= 0; --i) {
            double a = y[i];
            for (int m = i + 1; m < nc; ++m) a -= G[m][i] * y[m];
            y[i] = a / G[i][i];
        }
        for (int i = 0; i < nc; ++i) Gi[i][tid] = y[i];
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
        for (int q = 0; q < nV; ++q) {
            double acc = (double)X[r + (int64_t)q * nr];
            for (int m = 0; m < nc; ++m) acc -= (double)Y[r + (int64_t)m * nr] * muV[m][q];
            Z[r + (int64_t)q * nr] = (T)acc;
        }
        for (int e = 0; e < nc; ++e) {
            double acc = 0.0;
            for (int m = 0; m < nc; ++m) acc += (double)Y[r + (int64_t)m * nr] * Gi[m][e];
            Z[r + (int64_t)(nV + e) * nr] = (T)acc;
        }
    }
    T* gi = Gib + (int64_t)s * GI_STRIDE;
    for (int idx = tid; idx < nc * nc; idx += kWG) gi[idx] = (T)Gi[idx % nc][idx / nc];
    __syncthreads();
    double* Sp = Spb + (int64_t)s * SP_STRIDE;
    const double* sv = Svv + (int64_t)s * SVV_STRIDE;
    for (int idx = tid; idx < nV * nP; idx += kWG) {
        const int q = idx % nV, pcol = idx / nV;
        double acc = 0.0;
        for (int r = 0; r < nr; ++r) acc += (double)X[r + (int64_t)q * nr] * (double)Z[r + (int64_t)pcol * nr];
        double val = -acc + (pcol < nV ? sv[q + pcol * nV] : 0.0);
        Sp[q + (int64_t)pcol * nP] = val;
    }
    for (int idx = tid; idx < nc * nP; idx += kWG) {
        const int e = idx % nc, pcol = idx / nc;
        Sp[(nV + e) + (int64_t)pcol * nP] = (pcol < nV) ? -muV[e][pcol] : Gi[e][pcol - nV];
    }
}

// ------------------------------------------------- single-RHS triangular
// Forward L x = b or backward L^T x = b, in place, one workgroup per vector.
template <typename T>
__global__ __launch_bounds__(kWG) void k_trsv_fwd(const T* __restrict__ Lb, const int64_t* __restrict__ Loff,
                                                 const int* __restrict__ nv, const int* __restrict__ ldv,
                                                 T* __restrict__ xb, const int64_t* __restrict__ xoff) {
    const int s = blockIdx.x;
    const T* L = Lb + Loff[s];
    T* x = xb + xoff[s];
    const int n = nv[s];
    const int64_t ld = ldv[s];
    const int tid = threadIdx.x, lane = tid & 63;
    __shared__ T D[NB][NB + 1];
    __shared__ T xs[NB];
    for (int j0 = 0; j0 < n; j0 += NB) {
        const int jb = min(NB, n - j0);
        // stage the diagonal block (coalesced along columns)
        for (int idx = tid; idx < NB * NB; idx += kWG) {
            const int i = idx % NB, j = idx / NB;
            D[i][j] = (i < jb && j < jb && j <= i) ? L[(j0 + i) + (j0 + j) * ld] : (T)(i == j);
        }
        __syncthreads();
        if (tid < 64) {
            T xv = (lane < jb) ? x[j0 + lane] : (T)0;
            for (int c = 0; c < jb; ++c) {
                const T xc = __shfl(xv, c) / D[c][c];
                if (lane == c) xv = xc;
                else if (lane > c && lane < NB) xv -= D[lane][c] * xc;
            }
            if (lane < jb) { xs[lane] = xv; x[j0 + lane] = xv; }
        }
        __syncthreads();
        for (int r = j0 + jb + tid; r < n; r += kWG) {
            T acc = (T)0;
            for (int c = 0; c < jb; ++c) acc += L[r + (j0 + c) * ld] * xs[c];
            x[r] -= acc;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_trsv_bwd(const T* __restrict__ Lb, const int64_t* __restrict__ Loff,
                                                 const int* __restrict__ nv, const int* __restrict__ ldv,
                                                 T* __restrict__ xb, const int64_t* __restrict__ xoff) {
    const int s = blockIdx.x;
    const T* L = Lb + Loff[s];
    T* x = xb + xoff[s];
    const int n = nv[s];
    const int64_t ld = ldv[s];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    __shared__ T red[kWG / 64][NB];
    __shared__ T D[NB][NB + 1];
    const int nblk = (n + NB - 1) / NB;
    for (int bi = nblk - 1; bi >= 0; --bi) {
        const int j0 = bi * NB, jb = min(NB, n - j0);
        for (int idx = tid; idx < NB * NB; idx += kWG) {
            const int i = idx % NB, j = idx / NB;
            D[i][j] = (i < jb && j < jb && j <= i) ? L[(j0 + i) + (j0 + j) * ld] : (T)(i == j);
        }
        T acc[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[c] = (T)0;
        for (int r = j0 + jb + tid; r < n; r += kWG) {
            const T xr = x[r];
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < jb) acc[c] += L[r + (j0 + c) * ld] * xr;
        }
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const T sred = wave_sum(acc[c]);
            if (lane == 0) red[wv][c] = sred;
        }
        __syncthreads();
        if (tid < 64) {
            T rhs = (T)0;
            if (lane < jb) {
                rhs = x[j0 + lane];
                for (int q = 0; q < kWG / 64; ++q) rhs -= red[q][lane];
            }
            for (int c = jb - 1; c >= 0; --c) {
                const T xc = __shfl(rhs, c) / D[c][c];
                if (lane == c) rhs = xc;
                else if (lane < c) rhs -= D[c][lane] * xc;
            }
            if (lane < jb) x[j0 + lane] = rhs;
        }
        __syncthreads();
    }
}

// --------------------------------------------------------- deluxe factors
// Per face: S_F^j + S_F^k; per edge: sum_m S_E^(m) (Sec. 4.2); then an
// unblocked Cholesky (objects hold at most a few hundred dofs).
template <typename T>
__global__ __launch_bounds__(kWG) void k_deluxe_setup(ObjDesc o, const T* __restrict__ slots,
                                                     T* __restrict__ fac, int* __restrict__ info) {
    const int ob = blockIdx.x;
    const int n = o.n[ob];
    T* A = fac + o.fac_off[ob];
    const int tid = threadIdx.x;
    for (int idx = tid; idx < n * n; idx += kWG) {
        T acc = (T)0;
        for (int q = o.sh_ptr[ob]; q < o.sh_ptr[ob + 1]; ++q) acc += slots[o.sh_slot[q] + idx];
        A[idx] = acc;
    }
    __syncthreads();
    __shared__ int bad;
    if (tid == 0) bad = 0;
    for (int k = 0; k < n; ++k) {
        if (tid == 0) {
            T dk = A[k + k * n];
            if (!(dk > (T)0)) { bad = 1; dk = (T)1; }
            A[k + k * n] = sqrt(dk);
        }
        __syncthreads();
        const T piv = A[k + k * n];
        for (int i = k + 1 + tid; i < n; i += kWG) A[i + k * n] /= piv;
        __syncthreads();
        const int m = n - k - 1;
        for (int idx = tid; idx < m * m; idx += kWG) {
            const int i = k + 1 + idx % m, j = k + 1 + idx / m;
            if (j <= i) A[i + j * n] -= A[i + k * n] * A[j + k * n];
        }
        __syncthreads();
    }
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
void launch_extract(hipStream_t s, const BatchDesc& d, const T* K, T* slots, T* F, double* Svv, T* Srr) {
    hipLaunchKernelGGL(k_extract<T>, dim3(d.nsub), dim3(kWG), 0, s, d, K, slots, F, Svv, Srr);
}
template <typename T>
void launch_copy_out(hipStream_t s, const BatchDesc& d, int nb, const T* K, T* LII, const int64_t* LIIoff, T* Lrr,
                     const int64_t* Lrroff) {
    hipLaunchKernelGGL(k_copy_out<T>, dim3(nb), dim3(kWG), 0, s, d, K, LII, LIIoff, Lrr, Lrroff);
}
template <typename T>
void launch_trsm_fwd(hipStream_t s, int nb, const T* L, const int64_t* Loff, const int* n, const int* ld,
                     T* B, const int64_t* Boff, const int* ldb, const int* k) {
    hipLaunchKernelGGL(k_trsm_fwd<T>, dim3(nb), dim3(kWG), 0, s, L, Loff, n, ld, B, Boff, ldb, k);
}
template <typename T>
void launch_coarse_local(hipStream_t s, const BatchDesc& d, const T* F, const double* Svv, T* Z, T* Gi,
                         double* Sp, int* info) {
    hipLaunchKernelGGL(k_coarse_local<T>, dim3(d.nsub), dim3(kWG), 0, s, d, F, Svv, Z, Gi, Sp, info);
}
template <typename T>
void launch_trsv(hipStream_t s, int nb, bool trans, const T* L, const int64_t* Loff, const int* n,
                 const int* ld, T* x, const int64_t* xoff) {
    if (trans)
        hipLaunchKernelGGL(k_trsv_bwd<T>, dim3(nb), dim3(kWG), 0, s, L, Loff, n, ld, x, xoff);
    else
        hipLaunchKernelGGL(k_trsv_fwd<T>, dim3(nb), dim3(kWG), 0, s, L, Loff, n, ld, x, xoff);
}
template <typename T>
void launch_deluxe_setup(hipStream_t s, const ObjDesc& o, const T* slots, T* fac, int* info) {
    hipLaunchKernelGGL(k_deluxe_setup<T>, dim3(o.nobj), dim3(kWG), 0, s, o, slots, fac, info);
}

#define BDM_INST(T)                                                                                     \
    template void launch_assemble<T>(hipStream_t, const BatchDesc&, int, const FEParams&, const double*, \
                                     const double*, const double*, T*);                                \
    template void launch_potrf<T>(hipStream_t, int, T*, const int64_t*, const int*, const int*,         \
                                  const int*, const int*, int*);                                         \
    template void launch_extract<T>(hipStream_t, const BatchDesc&, const T*, T*, T*, double*, T*);      \
    template void launch_copy_out<T>(hipStream_t, const BatchDesc&, int, const T*, T*, const int64_t*, T*,    \
                                     const int64_t*);                                                    \
    template void launch_trsm_fwd<T>(hipStream_t, int, const T*, const int64_t*, const int*, const int*, \
                                     T*, const int64_t*, const int*, const int*);                        \
    template void launch_coarse_local<T>(hipStream_t, const BatchDesc&, const T*, const double*, T*, T*, \
                                         double*, int*);                                                 \
    template void launch_trsv<T>(hipStream_t, int, bool, const T*, const int64_t*, const int*,          \
                                 const int*, T*, const int64_t*);                                        \
    template void launch_deluxe_setup<T>(hipStream_t, const ObjDesc&, const T*, T*, int*);
BDM_INST(double)
BDM_INST(float)
#undef BDM_INST

}  // namespace bdm
