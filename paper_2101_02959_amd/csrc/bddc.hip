// Per-iteration kernels of the BDDC and FETI-DP deluxe preconditioners
// (paper Sec. 4.2 - 4.4): gathers / scatters between the global (v, u_e)
// vectors and the per-subdomain local vectors, deluxe averaging on faces
// and edges, the coarse right-hand side and prolongation, and the FETI-DP
// jump operators.  Every reduction runs in a fixed order, so results are
// bitwise reproducible from run to run.
#include "bddc_kernels.hpp"
#include "common.hpp"

namespace bdm {


namespace {

__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Pairwise sum of N partial sums (N a power of two), the order fixed by N.
template <int N>
__device__ __forceinline__ double tree_sum(const double (&a)[N]) {
    if constexpr (N == 1) {
        return a[0];
    } else {
        double h[N / 2];
#pragma unroll
        for (int k = 0; k < N / 2; ++k) h[k] = a[2 * k] + a[2 * k + 1];
        return tree_sum<N / 2>(h);
    }
}

template <typename T>
__global__ void k_gather_I(int n, const int* __restrict__ list, int64_t N, const double* __restrict__ r,
                           const double* __restrict__ q, T* __restrict__ x) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t g = list[t];
    double a = r[g], b = r[N + g];
    if (q) { a -= q[g]; b -= q[N + g]; }
    x[2 * (int64_t)t] = (T)a;
    x[2 * (int64_t)t + 1] = (T)b;
}

template <typename T>
__global__ void k_scatter_I(int n, const int* __restrict__ list, int64_t N, const T* __restrict__ x,
                            double* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t g = list[t];
    out[g] = (double)x[2 * (int64_t)t];
    out[N + g] = (double)x[2 * (int64_t)t + 1];
}

// Residual side of the deluxe scaling, E_D^T: for every share m of the
// object, y^(m) = E_m g (g gathered once into LDS).  The scaling matrices of
// an object sum to the identity, so the last share's split is g minus the
// others' and its matrix is never read (half the matrix traffic of a face).
// One thread per (share, row) pair, four independent accumulators along the
// row, so the reads of E_m are coalesced across the rows.
// Objects of at most DLX_SMALL dofs (every face and edge of subdomains up to
// H/h = 16) stage their vectors in static LDS of fixed stride; BIG launches
// take dynamic LDS sized by the largest object of the mesh.
constexpr int DLX_SMALL = 512;
constexpr int DV_SH = 4;   // shares per object: 2 on a face, up to 4 on an edge

template <typename T, bool BIG>
__global__ __launch_bounds__(kWG) void k_deluxe_res(ObjDesc o, int64_t N, const double* __restrict__ g,
                                                   const T* __restrict__ dmat, T* __restrict__ xr,
                                                   const int64_t* __restrict__ xoff) {
    constexpr int NA = 4;   // independent accumulators along the row
    const int ob = blockIdx.x, tid = threadIdx.x;
    const int n = o.n[ob];
    extern __shared__ double r_dyn[];   // BIG: DV_SH rows of o.maxn values (g, then the splits)
    __shared__ double r_st[BIG ? 1 : DV_SH * DLX_SMALL];
    double* h = BIG ? r_dyn : r_st;
    const int64_t ld = BIG ? (int64_t)o.maxn : (int64_t)DLX_SMALL;
    double* ys = h + ld;                // splits of the shares before the last
    const int* nodes = o.nodes + o.node_off[ob];
    for (int i = tid; i < n; i += kWG) h[i] = g[(i & 1) * N + nodes[i >> 1]];
    __syncthreads();
    const int q0 = o.sh_ptr[ob], nm = o.sh_ptr[ob + 1] - q0 - 1;
    for (int t = tid; t < nm * n; t += kWG) {
        const int qq = t / n, i = t % n, q = q0 + qq;
        const T* E = dmat + o.sh_slot[q] + i;
        double a[NA];
#pragma unroll
        for (int u = 0; u < NA; ++u) a[u] = 0.0;
        int j = 0;
        for (; j + NA <= n; j += NA) {
#pragma unroll
            for (int u = 0; u < NA; ++u) a[u] += (double)E[(int64_t)(j + u) * n] * h[j + u];
        }
        for (; j < n; ++j) a[0] += (double)E[(int64_t)j * n] * h[j];
        const double y = tree_sum<NA>(a);
        ys[qq * ld + i] = y;
        xr[xoff[o.sh_sub[q]] + o.sh_roff[q] + i] = (T)y;
    }
    __syncthreads();
    const int ql = q0 + nm;
    for (int i = tid; i < n; i += kWG) {
        double y = h[i];
        for (int qq = 0; qq < nm; ++qq) y -= ys[qq * ld + i];
        xr[xoff[o.sh_sub[ql]] + o.sh_roff[ql] + i] = (T)y;
    }
}

// Value side of the deluxe scaling, E_D: u = (sum S)^{-1} sum_m S^(m) u^(m)
// = sum_m E_m^T u^(m) = u^(last) + sum_{m < last} E_m^T (u^(m) - u^(last)),
// since the matrices sum to the identity; the transposes E_m^T are stored
// beside E_m (Et), so the reads are coalesced across the output rows.  The
// differences and u^(last) are staged in LDS (DV_SH rows of o.maxn values);
// threads take (row, half of the inner range), four accumulators each, and
// the two halves are added through LDS.
template <typename T, bool BIG>
__global__ __launch_bounds__(kWG) void k_deluxe_val(ObjDesc o, int64_t N, const T* __restrict__ Et,
                                                   const T* __restrict__ xr, const int64_t* __restrict__ xoff,
                                                   double* __restrict__ z) {
    constexpr int NA = 4;   // independent accumulators along the inner range
    const int ob = blockIdx.x, tid = threadIdx.x;
    const int n = o.n[ob];
    const int* nodes = o.nodes + o.node_off[ob];
    const int q0 = o.sh_ptr[ob], nsh = o.sh_ptr[ob + 1] - q0;
    extern __shared__ double us_dyn[];   // BIG: [DV_SH][o.maxn]
    __shared__ double us_st[BIG ? 1 : DV_SH * DLX_SMALL];
    __shared__ double part[kWG];
    double* us = BIG ? us_dyn : us_st;
    const int64_t ld = BIG ? (int64_t)o.maxn : (int64_t)DLX_SMALL;
    const int nm = nsh - 1;
    double* ul = us + nm * ld;   // u^(last)
    for (int j = tid; j < n; j += kWG) ul[j] = (double)xr[xoff[o.sh_sub[q0 + nm]] + o.sh_roff[q0 + nm] + j];
    __syncthreads();
    for (int t = tid; t < nm * n; t += kWG) {
        const int q = t / n, j = t % n;
        us[q * ld + j] = (double)xr[xoff[o.sh_sub[q0 + q]] + o.sh_roff[q0 + q] + j] - ul[j];
    }
    __syncthreads();
    const int half = (n + 1) / 2, hp = tid / (kWG / 2), il = tid % (kWG / 2);
    for (int i0 = 0; i0 < n; i0 += kWG / 2) {
        const int i = i0 + il;
        double a[NA];
#pragma unroll
        for (int v = 0; v < NA; ++v) a[v] = 0.0;
        if (i < n) {
            const int jb = hp * half, je = min(n, jb + half);
            for (int q = 0; q < nm; ++q) {
                const T* F = Et + o.sh_slot[q0 + q] + i;
                const double* u = us + q * ld;
                int j = jb;
                for (; j + NA <= je; j += NA) {
#pragma unroll
                    for (int v = 0; v < NA; ++v) a[v] += (double)F[(int64_t)(j + v) * n] * u[j + v];
                }
                for (; j < je; ++j) a[0] += (double)F[(int64_t)j * n] * u[j];
            }
        }
        part[tid] = tree_sum<NA>(a);
        __syncthreads();
        if (hp == 0 && i < n) z[(i & 1) * N + nodes[i >> 1]] = (part[tid] + part[tid + kWG / 2]) + ul[i];
        __syncthreads();
    }
}

// E_m^T beside every E_m (one workgroup per object, 32 x 32 tiles through
// LDS so that reads and writes are both coalesced).
template <typename T>
__global__ __launch_bounds__(kWG) void k_deluxe_transpose(ObjDesc o, const T* __restrict__ dmat, T* __restrict__ Et) {
    __shared__ T tl[32][33];
    const int ob = blockIdx.x, tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
    const int n = o.n[ob];
    for (int q = o.sh_ptr[ob]; q < o.sh_ptr[ob + 1]; ++q) {
        const T* E = dmat + o.sh_slot[q];
        T* F = Et + o.sh_slot[q];
        for (int bj = 0; bj < n; bj += 32)
            for (int bi = 0; bi < n; bi += 32) {
                for (int y = ty; y < 32; y += kWG / 32) {
                    const int i = bi + tx, j = bj + y;
                    if (i < n && j < n) tl[y][tx] = E[i + (int64_t)j * n];
                }
                __syncthreads();
                for (int y = ty; y < 32; y += kWG / 32) {
                    const int j = bj + tx, i = bi + y;   // F(j, i) = E(i, j), F column-major
                    if (i < n && j < n) F[j + (int64_t)i * n] = tl[tx][y];
                }
                __syncthreads();
            }
    }
}

// rho scaling (Sec. 4.2): the scaling matrix of share q of an object is
// diagonal, w_q^v on the v dofs and w_q^e on the u_e dofs (dofs interleaved
// per node), so the residual split and the value average run through the
// same per-share matrices as the deluxe scaling.  Written into both the
// matrix and its transpose (equal); one workgroup per object.
template <typename T>
__global__ __launch_bounds__(kWG) void k_rho_fill(ObjDesc o, const double* __restrict__ w, T* __restrict__ dmat,
                                                 T* __restrict__ dmatT) {
    const int ob = blockIdx.x, tid = threadIdx.x;
    const int n = o.n[ob];
    for (int q = o.sh_ptr[ob]; q < o.sh_ptr[ob + 1]; ++q) {
        const T wv = (T)w[2 * q], we = (T)w[2 * q + 1];
        T* E = dmat + o.sh_slot[q];
        T* F = dmatT + o.sh_slot[q];
        for (int64_t idx = tid; idx < (int64_t)n * n; idx += kWG) {
            const int i = (int)(idx % n), j = (int)(idx / n);
            const T v = (i == j) ? ((i & 1) ? we : wv) : (T)0;
            E[idx] = v;
            F[idx] = v;
        }
    }
}

// Per subdomain after the forward Neumann solve x1 = L_rr^{-1} g_r:
//   cP = Z^T x1 (the local coarse right-hand side Phi^T g),
//   mu = G^{-1} Y^T x1 (multipliers of the average constraints).
// The constraint columns of Z are Y G^{-1}, so mu is the constraint part of
// cP and Y is not read.
template <typename T>
__global__ __launch_bounds__(kWG) void k_coarse_rhs_local(SubVecDesc d, const T* __restrict__ xr,
                                                         const T* __restrict__ Zb, double* __restrict__ cP,
                                                         double* __restrict__ mu) {
    const int s = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nr = d.nr[s], nV = d.nV[s], nc = d.nc[s], nP = nV + nc;
    const T* x = xr + d.xoff[s];
    const T* Z = Zb + d.Z_off[s];
    for (int o = wv; o < nP; o += kWG / 64) {
        const T* col = Z + (int64_t)o * nr;
        // rows of the lane in flight: four in FP32 (0.61 against 0.87 ms per
        // apply at 17M dofs); FP64 is no faster with more
        constexpr int U = sizeof(T) == 4 ? 4 : 1;
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = 0.0;
        int r = lane;
        for (; r + 64 * (U - 1) < nr; r += 64 * U) {
#pragma unroll
            for (int u = 0; u < U; ++u) a[u] += (double)col[r + 64 * u] * (double)x[r + 64 * u];
        }
        for (; r < nr; r += 64) a[0] += (double)col[r] * (double)x[r];
        double acc = wsum(tree_sum<U>(a));
        if (lane == 0) {
            cP[(int64_t)s * MAXP + o] = acc;
            if (o >= nV) mu[(int64_t)s * MAXC + (o - nV)] = acc;
        }
    }
}

// Coarse right-hand side: the assembled vertex residual plus the gathered
// local contributions Phi_j^T g^(j) (fixed order per primal dof).
__global__ void k_coarse_rhs_gather(CoarseDesc c, int64_t N, const double* __restrict__ g,
                                    const double* __restrict__ cP, double* __restrict__ b) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= c.np) return;
    double acc = (p < 2 * c.nverts) ? g[(p & 1) * N + c.vnode[p >> 1]] : 0.0;
    for (int q = c.cp_ptr[p]; q < c.cp_ptr[p + 1]; ++q) acc += cP[(int64_t)c.cp_sub[q] * MAXP + c.cp_loc[q]];
    b[p] = acc;
}

// Remove the kernel component (u_e-primal constant) and pin one u_e primal.
__global__ void k_coarse_project(int np, int pin, double* __restrict__ b) {
    const int tid = threadIdx.x;
    double part = 0.0;
    for (int p = 1 + 2 * tid; p < np; p += 2 * kWG) part += b[p];
    part = wsum(part);
    __shared__ double red[kWG / 64];
    if ((tid & 63) == 0) red[tid >> 6] = part;
    __syncthreads();
    double tot = 0.0;
    for (int q = 0; q < kWG / 64; ++q) tot += red[q];
    const double mean = tot / (np / 2);
    for (int p = 1 + 2 * tid; p < np; p += 2 * kWG) b[p] -= mean;
    __syncthreads();
    if (tid == 0) b[pin] = 0.0;
}

// x_r <- x1 - Y mu + Z u_c(primal of s): right-hand side of the combined
// backward solve that yields the Neumann correction plus the coarse
// prolongation Phi_r u_c.
template <typename T>
__global__ __launch_bounds__(kWG) void k_neumann_rhs(SubVecDesc d, const T* __restrict__ Fb,
                                                    const T* __restrict__ Zb, const double* __restrict__ mu,
                                                    const double* __restrict__ uc, T* __restrict__ xr,
                                                    int with_mu) {
    const int s = blockIdx.x, tid = threadIdx.x;
    const int nr = d.nr[s], nV = d.nV[s], nc = d.nc[s], nP = nV + nc;
    const T* Y = Fb + d.F_off[s];
    const T* Z = Zb + d.Z_off[s];
    const int* prim = d.primal + d.P_off[s];
    __shared__ double m[MAXC];
    __shared__ double u[MAXP];
    if (tid < nc) m[tid] = with_mu ? mu[(int64_t)s * MAXC + tid] : 0.0;
    if (tid < nP) u[tid] = uc ? uc[prim[tid]] : 0.0;
    __syncthreads();
    T* x = xr + d.xoff[s];
    for (int r = tid; r < nr; r += kWG) {
        double acc = (double)x[r];
        for (int e = 0; e < nc; ++e) acc -= (double)Y[r + (int64_t)e * nr] * m[e];
        for (int p = 0; p < nP; ++p) acc += (double)Z[r + (int64_t)p * nr] * u[p];
        x[r] = (T)acc;
    }
}

__global__ void k_vertex_val(int nv, const int* __restrict__ vnode, int64_t N, const double* __restrict__ uc,
                             double* __restrict__ z) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    z[vnode[v]] = uc[2 * v];
    z[N + vnode[v]] = uc[2 * v + 1];
}

// ------------------------------------------------------------- FETI-DP
// Multiplier blocks: (object, pair a < b); lam_ab = w^(a) - w^(b) on the
// object's dofs.  B^T: subdomain m receives sum_{(m,b)} lam - sum_{(a,m)} lam.
template <typename T>
__global__ __launch_bounds__(kWG) void k_feti_BT(ObjDesc o, FetiDesc f, const double* __restrict__ lam,
                                                T* __restrict__ xr, const int64_t* __restrict__ xoff) {
    const int ob = blockIdx.x, tid = threadIdx.x;
    const int n = o.n[ob];
    for (int q = o.sh_ptr[ob]; q < o.sh_ptr[ob + 1]; ++q) {
        const int m = o.sh_sub[q];
        T* dst = xr + xoff[m] + o.sh_roff[q];
        for (int i = tid; i < n; i += kWG) {
            double acc = 0.0;
            for (int pq = f.pr_ptr[ob]; pq < f.pr_ptr[ob + 1]; ++pq) {
                const double l = lam[f.pr_off[pq] + i];
                if (f.pr_a[pq] == m) acc += l;
                else if (f.pr_b[pq] == m) acc -= l;
            }
            dst[i] = (T)acc;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_feti_B(ObjDesc o, FetiDesc f, const T* __restrict__ xr,
                                               const int64_t* __restrict__ xoff, double* __restrict__ lam) {
    const int ob = blockIdx.x, tid = threadIdx.x;
    const int n = o.n[ob];
    for (int pq = f.pr_ptr[ob]; pq < f.pr_ptr[ob + 1]; ++pq) {
        const T* wa = xr + xoff[o.sh_sub[f.pr_qa[pq]]] + o.sh_roff[f.pr_qa[pq]];
        const T* wb = xr + xoff[o.sh_sub[f.pr_qb[pq]]] + o.sh_roff[f.pr_qb[pq]];
        for (int i = tid; i < n; i += kWG) lam[f.pr_off[pq] + i] = (double)wa[i] - (double)wb[i];
    }
}

// B_D^T: subdomain m receives sum_{(m,b)} D^(b) lam_mb - sum_{(a,m)} D^(a) lam_am,
// D^(x) = (sum S)^{-1} S^(x) = E_x^T; one wave per output entry.
template <typename T>
__global__ __launch_bounds__(kWG) void k_feti_BDT(ObjDesc o, FetiDesc f, const double* __restrict__ lam,
                                                 const T* __restrict__ dmat, T* __restrict__ xr,
                                                 const int64_t* __restrict__ xoff) {
    const int ob = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = o.n[ob];
    for (int q = o.sh_ptr[ob]; q < o.sh_ptr[ob + 1]; ++q) {
        const int m = o.sh_sub[q];
        T* dst = xr + xoff[m] + o.sh_roff[q];
        for (int i = wv; i < n; i += kWG / 64) {
            double acc = 0.0;
            for (int pq = f.pr_ptr[ob]; pq < f.pr_ptr[ob + 1]; ++pq) {
                int other;
                double sgn;
                if (f.pr_a[pq] == m) { other = f.pr_qb[pq]; sgn = 1.0; }
                else if (f.pr_b[pq] == m) { other = f.pr_qa[pq]; sgn = -1.0; }
                else continue;
                const T* E = dmat + o.sh_slot[other] + (int64_t)i * n;
                const double* l = lam + f.pr_off[pq];
                double a = 0.0;
                for (int j = lane; j < n; j += 64) a += (double)E[j] * l[j];
                acc += sgn * a;
            }
            acc = wsum(acc);
            if (lane == 0) dst[i] = (T)acc;
        }
    }
}

// B_D: lam_ab = D^(b)T w^(a) - D^(a)T w^(b) = E_b w^(a) - E_a w^(b).
template <typename T>
__global__ __launch_bounds__(kWG) void k_feti_BD(ObjDesc o, FetiDesc f, const T* __restrict__ xr,
                                                const int64_t* __restrict__ xoff, const T* __restrict__ dmat,
                                                double* __restrict__ lam) {
    const int ob = blockIdx.x, tid = threadIdx.x;
    const int n = o.n[ob];
    for (int pq = f.pr_ptr[ob]; pq < f.pr_ptr[ob + 1]; ++pq) {
        const int qa = f.pr_qa[pq], qb = f.pr_qb[pq];
        const T* Ea = dmat + o.sh_slot[qa];
        const T* Eb = dmat + o.sh_slot[qb];
        const T* wa = xr + xoff[o.sh_sub[qa]] + o.sh_roff[qa];
        const T* wb = xr + xoff[o.sh_sub[qb]] + o.sh_roff[qb];
        for (int i = tid; i < n; i += kWG) {
            double acc = 0.0;
            for (int j = 0; j < n; ++j)
                acc += (double)Eb[i + (int64_t)j * n] * (double)wa[j] - (double)Ea[i + (int64_t)j * n] * (double)wb[j];
            lam[f.pr_off[pq] + i] = acc;
        }
    }
}

// y_r = S_rr x_r per subdomain (dense saved copy of the Schur block).
template <typename T>
__global__ __launch_bounds__(kWG) void k_schur_mv(SubVecDesc d, const T* __restrict__ Srr,
                                                 const int64_t* __restrict__ Soff, const T* __restrict__ x,
                                                 T* __restrict__ y) {
    const int s = blockIdx.x, tid = threadIdx.x;
    const int nr = d.nr[s];
    const T* S = Srr + Soff[s];
    const T* xs = x + d.xoff[s];
    T* ys = y + d.xoff[s];
    for (int i = tid; i < nr; i += kWG) {
        double acc = 0.0;
        for (int j = 0; j < nr; ++j) acc += (double)S[i + (int64_t)j * nr] * (double)xs[j];
        ys[i] = (T)acc;
    }
}

// Split the condensed residual 1/|N_x| over the sharing subdomains (f~ of
// the FETI-DP right-hand side): every share of an object gets g / nshare.
template <typename T>
__global__ __launch_bounds__(kWG) void k_split_res(ObjDesc o, int64_t N, const double* __restrict__ g,
                                                  T* __restrict__ xr, const int64_t* __restrict__ xoff) {
    const int ob = blockIdx.x, tid = threadIdx.x;
    const int n = o.n[ob];
    const int* nodes = o.nodes + o.node_off[ob];
    const int ns = o.sh_ptr[ob + 1] - o.sh_ptr[ob];
    for (int q = o.sh_ptr[ob]; q < o.sh_ptr[ob + 1]; ++q) {
        T* dst = xr + xoff[o.sh_sub[q]] + o.sh_roff[q];
        for (int i = tid; i < n; i += kWG) dst[i] = (T)(g[(i & 1) * N + nodes[i >> 1]] / ns);
    }
}

// Recovered interface values: every share of a continuous solution holds
// the same values; take the first share's.
template <typename T>
__global__ __launch_bounds__(kWG) void k_take_first(ObjDesc o, int64_t N, const T* __restrict__ xr,
                                                   const int64_t* __restrict__ xoff, double* __restrict__ z) {
    const int ob = blockIdx.x, tid = threadIdx.x;
    const int n = o.n[ob];
    const int* nodes = o.nodes + o.node_off[ob];
    const int q = o.sh_ptr[ob];
    const T* u = xr + xoff[o.sh_sub[q]] + o.sh_roff[q];
    for (int i = tid; i < n; i += kWG) z[(i & 1) * N + nodes[i >> 1]] = (double)u[i];
}

}  // namespace

static inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
void launch_gather_I(hipStream_t s, int n, const int* list, int64_t N, const double* r, const double* q, T* x) {
    hipLaunchKernelGGL(k_gather_I<T>, dim3(nb(n, 256)), dim3(256), 0, s, n, list, N, r, q, x);
}
template <typename T>
void launch_scatter_I(hipStream_t s, int n, const int* list, int64_t N, const T* x, double* out) {
    hipLaunchKernelGGL(k_scatter_I<T>, dim3(nb(n, 256)), dim3(256), 0, s, n, list, N, x, out);
}
template <typename T>
void launch_deluxe_res(hipStream_t s, const ObjDesc& o, int64_t N, const double* g, const T* dmat, T* xr,
                       const int64_t* xoff) {
    if (o.maxn <= DLX_SMALL)
        hipLaunchKernelGGL((k_deluxe_res<T, false>), dim3(o.nobj), dim3(kWG), 0, s, o, N, g, dmat, xr, xoff);
    else
        hipLaunchKernelGGL((k_deluxe_res<T, true>), dim3(o.nobj), dim3(kWG), (size_t)DV_SH * o.maxn * sizeof(double), s,
                           o, N, g, dmat, xr, xoff);
}
template <typename T>
void launch_deluxe_val(hipStream_t s, const ObjDesc& o, int64_t N, const T* dmatT, const T* xr,
                       const int64_t* xoff, double* z) {
    if (o.maxn <= DLX_SMALL)
        hipLaunchKernelGGL((k_deluxe_val<T, false>), dim3(o.nobj), dim3(kWG), 0, s, o, N, dmatT, xr, xoff, z);
    else
        hipLaunchKernelGGL((k_deluxe_val<T, true>), dim3(o.nobj), dim3(kWG), (size_t)DV_SH * o.maxn * sizeof(double),
                           s, o, N, dmatT, xr, xoff, z);
}
template <typename T>
void launch_deluxe_transpose(hipStream_t s, const ObjDesc& o, const T* dmat, T* dmatT) {
    hipLaunchKernelGGL(k_deluxe_transpose<T>, dim3(o.nobj), dim3(kWG), 0, s, o, dmat, dmatT);
}
int deluxe_max_shares() { return DV_SH; }
template <typename T>
void launch_rho_fill(hipStream_t s, const ObjDesc& o, const double* w, T* dmat, T* dmatT) {
    if (o.nobj <= 0) return;
    hipLaunchKernelGGL(k_rho_fill<T>, dim3(o.nobj), dim3(kWG), 0, s, o, w, dmat, dmatT);
}
template <typename T>
void launch_coarse_rhs_local(hipStream_t s, const SubVecDesc& d, const T* xr, const T* Z, double* cP, double* mu) {
    hipLaunchKernelGGL(k_coarse_rhs_local<T>, dim3(d.nsub), dim3(kWG), 0, s, d, xr, Z, cP, mu);
}
void launch_coarse_rhs_gather(hipStream_t s, const CoarseDesc& c, int64_t N, const double* g,
                              const double* cP, double* b) {
    hipLaunchKernelGGL(k_coarse_rhs_gather, dim3(nb(c.np, 256)), dim3(256), 0, s, c, N, g, cP, b);
}
void launch_coarse_project(hipStream_t s, int np, int pin, double* b) {
    hipLaunchKernelGGL(k_coarse_project, dim3(1), dim3(kWG), 0, s, np, pin, b);
}
template <typename T>
void launch_neumann_rhs(hipStream_t s, const SubVecDesc& d, const T* F, const T* Z, const double* mu,
                        const double* uc, T* xr, int with_mu) {
    hipLaunchKernelGGL(k_neumann_rhs<T>, dim3(d.nsub), dim3(kWG), 0, s, d, F, Z, mu, uc, xr, with_mu);
}
void launch_vertex_val(hipStream_t s, int nv, const int* vnode, int64_t N, const double* uc, double* z) {
    if (nv > 0) hipLaunchKernelGGL(k_vertex_val, dim3(nb(nv, 256)), dim3(256), 0, s, nv, vnode, N, uc, z);
}
template <typename T>
void launch_feti_BT(hipStream_t s, const ObjDesc& o, const FetiDesc& f, const double* lam, T* xr,
                    const int64_t* xoff) {
    hipLaunchKernelGGL(k_feti_BT<T>, dim3(o.nobj), dim3(kWG), 0, s, o, f, lam, xr, xoff);
}
template <typename T>
void launch_feti_B(hipStream_t s, const ObjDesc& o, const FetiDesc& f, const T* xr, const int64_t* xoff,
                   double* lam) {
    hipLaunchKernelGGL(k_feti_B<T>, dim3(o.nobj), dim3(kWG), 0, s, o, f, xr, xoff, lam);
}
template <typename T>
void launch_feti_BDT(hipStream_t s, const ObjDesc& o, const FetiDesc& f, const double* lam, const T* dmat, T* xr,
                     const int64_t* xoff) {
    hipLaunchKernelGGL(k_feti_BDT<T>, dim3(o.nobj), dim3(kWG), 0, s, o, f, lam, dmat, xr, xoff);
}
template <typename T>
void launch_feti_BD(hipStream_t s, const ObjDesc& o, const FetiDesc& f, const T* xr, const int64_t* xoff,
                    const T* dmat, double* lam) {
    hipLaunchKernelGGL(k_feti_BD<T>, dim3(o.nobj), dim3(kWG), 0, s, o, f, xr, xoff, dmat, lam);
}
template <typename T>
void launch_schur_mv(hipStream_t s, const SubVecDesc& d, const T* Srr, const int64_t* Soff, const T* x, T* y) {
    hipLaunchKernelGGL(k_schur_mv<T>, dim3(d.nsub), dim3(kWG), 0, s, d, Srr, Soff, x, y);
}
template <typename T>
void launch_split_res(hipStream_t s, const ObjDesc& o, int64_t N, const double* g, T* xr, const int64_t* xoff) {
    hipLaunchKernelGGL(k_split_res<T>, dim3(o.nobj), dim3(kWG), 0, s, o, N, g, xr, xoff);
}
template <typename T>
void launch_take_first(hipStream_t s, const ObjDesc& o, int64_t N, const T* xr, const int64_t* xoff, double* z) {
    hipLaunchKernelGGL(k_take_first<T>, dim3(o.nobj), dim3(kWG), 0, s, o, N, xr, xoff, z);
}

#define BDM_INST(T)                                                                                         \
    template void launch_gather_I<T>(hipStream_t, int, const int*, int64_t, const double*, const double*, T*); \
    template void launch_scatter_I<T>(hipStream_t, int, const int*, int64_t, const T*, double*);            \
    template void launch_deluxe_res<T>(hipStream_t, const ObjDesc&, int64_t, const double*, const T*, T*,   \
                                       const int64_t*);                                                     \
    template void launch_deluxe_val<T>(hipStream_t, const ObjDesc&, int64_t, const T*, const T*,            \
                                       const int64_t*, double*);                                            \
    template void launch_deluxe_transpose<T>(hipStream_t, const ObjDesc&, const T*, T*);                   \
    template void launch_rho_fill<T>(hipStream_t, const ObjDesc&, const double*, T*, T*);                    \
    template void launch_coarse_rhs_local<T>(hipStream_t, const SubVecDesc&, const T*, const T*, double*, double*); \
    template void launch_neumann_rhs<T>(hipStream_t, const SubVecDesc&, const T*, const T*, const double*,  \
                                        const double*, T*, int);                                            \
    template void launch_feti_BT<T>(hipStream_t, const ObjDesc&, const FetiDesc&, const double*, T*,        \
                                    const int64_t*);                                                        \
    template void launch_feti_B<T>(hipStream_t, const ObjDesc&, const FetiDesc&, const T*, const int64_t*,  \
                                   double*);                                                                \
    template void launch_feti_BDT<T>(hipStream_t, const ObjDesc&, const FetiDesc&, const double*, const T*, \
                                     T*, const int64_t*);                                                   \
    template void launch_feti_BD<T>(hipStream_t, const ObjDesc&, const FetiDesc&, const T*, const int64_t*, \
                                    const T*, double*);                                                     \
    template void launch_schur_mv<T>(hipStream_t, const SubVecDesc&, const T*, const int64_t*, const T*, T*); \
    template void launch_split_res<T>(hipStream_t, const ObjDesc&, int64_t, const double*, T*, const int64_t*); \
    template void launch_take_first<T>(hipStream_t, const ObjDesc&, int64_t, const T*, const int64_t*, double*);
BDM_INST(double)
BDM_INST(float)
#undef BDM_INST

}  // namespace bdm
