// Pointwise ionic kernels and the matrix-free Q1 stencils of the Bidomain
// Jacobian and residual (paper Sec. 2, 3a-c).
//
// The stiffness of a structured Q1 mesh with one conductivity tensor per
// z-layer is a 27-point stencil whose coefficients depend only on the node's
// z-level k and on whether it sits on the low / interior / high boundary in x
// and in y (nine classes).  The host builds these tables once, scaled by tau,
// for both media; the kernels stage the tables of one z-level at a time in
// LDS.
#include <cmath>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace bdm {

// ---------------------------------------------------------------- host side
// Closed-form Q1 element stiffness on a box of sizes hd[0..2] for a constant
// tensor D: integrals factor per axis d into
//   int psi_a' psi_b' = s_a s_b / h_d,  int psi_a psi_b = h_d/3 (a==b) or h_d/6,
//   int psi_a' psi_b  = s_a / 2,        s_0 = -1, s_1 = +1.
void element_stiffness(const double D[3][3], const double hd[3], double Ke[8][8]) {
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
            const int ad[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
            const int bd[3] = {b & 1, (b >> 1) & 1, (b >> 2) & 1};
            double acc = 0.0;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) {
                    double prod = 1.0;
                    for (int d = 0; d < 3; ++d) {
                        const double sa = ad[d] ? 1.0 : -1.0, sb = bd[d] ? 1.0 : -1.0;
                        double f;
                        if (d == p && d == q) f = sa * sb / hd[d];
                        else if (d == p) f = 0.5 * sa;
                        else if (d == q) f = 0.5 * sb;
                        else f = (ad[d] == bd[d]) ? hd[d] / 3.0 : hd[d] / 6.0;
                        prod *= f;
                    }
                    acc += D[p][q] * prod;
                }
            Ke[a][b] = acc;
        }
}

void conductivity_tensor(const double sig[3], double theta, double D[3][3]) {
    const double c = std::cos(theta), s = std::sin(theta);
    D[0][0] = sig[0] * c * c + sig[1] * s * s;
    D[1][1] = sig[0] * s * s + sig[1] * c * c;
    D[0][1] = D[1][0] = (sig[0] - sig[1]) * c * s;
    D[0][2] = D[2][0] = D[1][2] = D[2][1] = 0.0;
    D[2][2] = sig[2];
}

// tau-scaled element matrices per z-layer: ke[(layer*2 + medium)*64 + a*8 + b]
// (nz * 128 doubles, caller's buffer), box elements of sizes hd[0..2]
void layer_matrices_into(int nz, const double hd[3], double tau, const double sig_i[3], const double sig_e[3],
                         double th0, double th1, double* ke) {
    for (int L = 0; L < nz; ++L) {
        const double th = th0 + (th1 - th0) * (L + 0.5) / nz;
        for (int m = 0; m < 2; ++m) {
            double D[3][3], K[8][8];
            conductivity_tensor(m == 0 ? sig_i : sig_e, th, D);
            element_stiffness(D, hd, K);
            for (int a = 0; a < 8; ++a)
                for (int b = 0; b < 8; ++b) ke[((size_t)L * 2 + m) * 64 + a * 8 + b] = tau * K[a][b];
        }
    }
}

std::vector<double> layer_matrices(int nz, const double hd[3], double tau, const double sig_i[3],
                                   const double sig_e[3], double th0, double th1) {
    std::vector<double> ke((size_t)nz * 128);
    layer_matrices_into(nz, hd, tau, sig_i, sig_e, th0, th1, ke.data());
    return ke;
}

// 27-point tables st[((k*9 + xc + 3*yc)*2 + m)*27 + d], d = (dx+1) + 3(dy+1) + 9(dz+1):
// the sum over the elements adjacent to both the node and its neighbour
// ((nz + 1) * 486 doubles, caller's buffer).
void stencil_tables_into(int nz, const double* ke, double* st) {
    for (size_t i = 0; i < (size_t)(nz + 1) * 9 * 2 * 27; ++i) st[i] = 0.0;
    for (int k = 0; k <= nz; ++k)
        for (int yc = 0; yc < 3; ++yc)
            for (int xc = 0; xc < 3; ++xc)
                for (int m = 0; m < 2; ++m) {
                    double* t = &st[(((size_t)k * 9 + xc + 3 * yc) * 2 + m) * 27];
                    for (int oz = 0; oz < 2; ++oz) {
                        const int L = k - 1 + oz;
                        if (L < 0 || L >= nz) continue;
                        for (int oy = 0; oy < 2; ++oy) {
                            if ((yc == 0 && oy == 0) || (yc == 2 && oy == 1)) continue;
                            for (int ox = 0; ox < 2; ++ox) {
                                if ((xc == 0 && ox == 0) || (xc == 2 && ox == 1)) continue;
                                const int a = (1 - ox) + 2 * (1 - oy) + 4 * (1 - oz);
                                for (int bz = 0; bz < 2; ++bz)
                                    for (int by = 0; by < 2; ++by)
                                        for (int bx = 0; bx < 2; ++bx) {
                                            const int b = bx + 2 * by + 4 * bz;
                                            const int dx = bx - (1 - ox), dy = by - (1 - oy),
                                                      dz = bz - (1 - oz);
                                            t[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] +=
                                                ke[((size_t)L * 2 + m) * 64 + a * 8 + b];
                                        }
                            }
                        }
                    }
                }
}

std::vector<double> stencil_tables(int nz, const std::vector<double>& ke) {
    std::vector<double> st((size_t)(nz + 1) * 9 * 2 * 27);
    stencil_tables_into(nz, ke.data(), st.data());
    return st;
}

// --------------------------------------------------------------- device side
namespace {


__device__ inline double lumped_mass(const FEParams& p, int i, int j, int k) {
    const double fx = (i == 0 || i == p.nx) ? 0.5 : 1.0;
    const double fy = (j == 0 || j == p.ny) ? 0.5 : 1.0;
    const double fz = (k == 0 || k == p.nz) ? 0.5 : 1.0;
    return p.h * p.hy * p.hz * fx * fy * fz;
}

enum { ST_JAC = 0, ST_RES_MINUS_JAC = 1, ST_RESIDUAL = 2 };

// One fused 27-point stencil pass over the mesh.  si = (tau A_i)(xv + xe),
// se = (tau A_e) xe; then
//   ST_JAC:            y = [d xv + si ; si + se]
//   ST_RES_MINUS_JAC:  y = r - [d xv + si ; si + se]
//   ST_RESIDUAL:       y = [m (c (v - v^n) + tau (I_ion - I_s)) + si ; si + se]
// A block owns an SX x SY column of nodes and walks SZ z-levels (the tile
// shape is one of the autotuned variants below).  The planes k-1, k, k+1 of
// (xv + xe) and xe, with a one-node halo, live in a rotating LDS buffer, so
// each input value is fetched from memory about once; the coefficient tables
// of level k (9 boundary classes x 2 media) are staged too.
constexpr int ST_XCD = 8;

template <int MODE, int SX, int SY, int SZ>
__global__ __launch_bounds__(SX * SY) void k_stencil(FEParams p, const double* __restrict__ st,
                                                     const double* __restrict__ dg, const double* __restrict__ xv,
                                                     const double* __restrict__ xe, const double* __restrict__ rv,
                                                     const double* __restrict__ re, const double* __restrict__ vn,
                                                     const double* __restrict__ w, const double* __restrict__ Is,
                                                     double stim, double* __restrict__ yv, double* __restrict__ ye) {
    constexpr int PX = SX + 2, PY = SY + 2;
    constexpr int NT = SX * SY, NPT = (PX * PY + NT - 1) / NT, TABN = 9 * 2 * 27, NTB = (TABN + NT - 1) / NT;
    __shared__ double tab[TABN];
    __shared__ double ps[3][PY][PX];
    __shared__ double pe[3][PY][PX];
    // Tile of this workgroup: the launch is one-dimensional and consecutive
    // ids go round robin to the 8 XCDs, so XCD x takes the contiguous run of
    // tiles [x * per, (x + 1) * per) in x-fastest order; tiles that share halo
    // rows then share that XCD's L2 and are processed close together.
    const int gx = (p.nx1 + SX - 1) / SX, gy = (p.ny1 + SY - 1) / SY, gz = (p.nz + 1 + SZ - 1) / SZ;
    const int ntile = gx * gy * gz, per = (ntile + ST_XCD - 1) / ST_XCD;
    const int tile = ((int)blockIdx.x % ST_XCD) * per + (int)blockIdx.x / ST_XCD;
    if (tile >= ntile) return;
    const int bxi = tile % gx, byi = (tile / gx) % gy, bzi = tile / (gx * gy);
    const int tid = threadIdx.x + SX * threadIdx.y;
    const int i0 = bxi * SX, j0 = byi * SY;
    const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
    const int kbeg = bzi * SZ;
    const int kend = min(kbeg + SZ, p.nz + 1);
    const bool act = (i <= p.nx) && (j <= p.ny);
    const int xc = (i == 0) ? 0 : (i == p.nx ? 2 : 1);
    const int yc = (j == 0) ? 0 : (j == p.ny ? 2 : 1);
    const int cls = xc + 3 * yc;
    const int64_t plane = (int64_t)p.nx1 * p.ny1;
    // A block whose nodes all lie off the x and y boundaries has one
    // boundary class (the interior one): its coefficients are read at a
    // wave-uniform address (scalar loads) instead of being staged in LDS and
    // read per lane, which halves the LDS reads per node.
    const bool inner = i0 >= 1 && i0 + SX <= p.nx && j0 >= 1 && j0 + SY <= p.ny;
    // Planes are fetched into registers one iteration ahead and stored into a
    // three-plane LDS ring (with the level's coefficient table) after the
    // compute of the previous plane.  The loads are branch free (clamped
    // index, mask applied at the LDS store), so they stay in flight across
    // the compute instead of being waited for inside a bounds branch.
    double ra[NPT], rb[NPT], rt[NTB];
    bool rok[NPT];
    auto fetch = [&](int k) {
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const int t = tid + q * NT;
            const int lx = t % PX, ly = t / PX;
            const int gi = i0 - 1 + lx, gj = j0 - 1 + ly;
            const bool ok = t < PX * PY && k >= 0 && k <= p.nz && gi >= 0 && gi <= p.nx && gj >= 0 && gj <= p.ny;
            const int64_t n = ok ? gi + (int64_t)p.nx1 * gj + plane * k : 0;
            ra[q] = xv[n];
            rb[q] = xe[n];
            rok[q] = ok;
        }
    };
    auto store = [&](int k) {
        const int sl = (k + 3) % 3;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const int t = tid + q * NT;
            if (t < PX * PY) {
                ps[sl][t / PX][t % PX] = rok[q] ? ra[q] + rb[q] : 0.0;
                pe[sl][t / PX][t % PX] = rok[q] ? rb[q] : 0.0;
            }
        }
    };
    auto fetch_tab = [&](int k) {
#pragma unroll
        for (int q = 0; q < NTB; ++q) {
            const int t = tid + q * NT;
            const bool ok = t < TABN && k <= p.nz;
            rt[q] = st[ok ? (int64_t)k * TABN + t : 0];
        }
    };
    fetch(kbeg - 1);
    store(kbeg - 1);
    fetch(kbeg);
    store(kbeg);
    fetch(kbeg + 1);
    if (!inner) fetch_tab(kbeg);
    for (int k = kbeg; k < kend; ++k) {
        store(k + 1);
        if (!inner) {
#pragma unroll
            for (int q = 0; q < NTB; ++q)
                if (tid + q * NT < TABN) tab[tid + q * NT] = rt[q];
        }
        if (k + 1 < kend) {
            fetch(k + 2);
            if (!inner) fetch_tab(k + 1);
        }
        __syncthreads();
        if (act) {
            double ai = 0.0, ae = 0.0;
            auto sum27 = [&](const double* ti, const double* te) {
#pragma unroll
                for (int dz = 0; dz < 3; ++dz) {
                    const int sl = (k + dz + 2) % 3;
#pragma unroll
                    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                        for (int dx = 0; dx < 3; ++dx) {
                            const int d = dx + 3 * dy + 9 * dz;
                            ai = fma(ti[d], ps[sl][threadIdx.y + dy][threadIdx.x + dx], ai);
                            ae = fma(te[d], pe[sl][threadIdx.y + dy][threadIdx.x + dx], ae);
                        }
                }
            };
            if (inner) {
                const double* tg = st + (int64_t)k * TABN + 4 * 54;   // class 4: interior in x and y
                sum27(tg, tg + 27);
            } else {
                sum27(tab + cls * 54, tab + cls * 54 + 27);
            }
            const int64_t n = i + (int64_t)p.nx1 * j + plane * k;
            if (MODE == ST_RESIDUAL) {
                const double vv = xv[n];
                const double m = lumped_mass(p, i, j, k);
                const double is = (stim != 0.0 && Is) ? Is[n] : 0.0;
                yv[n] = m * (p.c * (vv - vn[n]) + p.tau * (rmc_iion(p, vv, w[n]) - is)) + ai;
                ye[n] = ai + ae;
            } else {
                const double a = dg[n] * xv[n] + ai, b = ai + ae;
                if (MODE == ST_JAC) {
                    yv[n] = a;
                    ye[n] = b;
                } else {
                    yv[n] = rv[n] - a;
                    ye[n] = re[n] - b;
                }
            }
        }
        __syncthreads();
    }
}

// The same stencil pass without LDS or barriers.  A wave spans 64
// consecutive x columns and each thread owns RY consecutive rows in y.  The
// thread marches up z over SZ levels: per plane it loads its RY + 2 rows of
// (v, u_e) (coalesced along x), takes the x neighbours from the adjacent
// lanes over DPP wave shifts (the two columns beyond the wave come from one
// extra load per row, at one address for lanes 0-62 and another for lane
// 63), and adds the plane to three running sums per
// row: the node below (its dz = +1 coefficients), the node itself (dz = 0)
// and the node above (dz = -1); node m - 1 is complete once plane m is in.
// Each sum takes the 27 products in the order of k_stencil, and planes
// outside the mesh add nothing there (their values are zero), so the two
// kernels agree bitwise.
//
// The launch has two parts.  Boundary tiles (first, so their short
// latency-bound columns start early) give one thread to each node column on
// the x or y faces, ZB levels deep, and read the coefficients of its class
// per lane.  Interior tiles cover the x-y interior 1..nx-1 x 1..ny-1, where
// every neighbour is inside the mesh and all nodes share one boundary class,
// so their coefficients are read at wave-uniform addresses (scalar loads).
template <int MODE>
__device__ __forceinline__ void stencil_out(const FEParams& p, int i, int j, int k, int64_t n, double ai, double ae,
                                            const double* __restrict__ dg, const double* __restrict__ xv,
                                            const double* __restrict__ rv, const double* __restrict__ re,
                                            const double* __restrict__ vn, const double* __restrict__ w,
                                            const double* __restrict__ Is, double stim, double* __restrict__ yv,
                                            double* __restrict__ ye) {
    if (MODE == ST_RESIDUAL) {
        const double vv = xv[n];
        const double mm = lumped_mass(p, i, j, k);
        const double is = (stim != 0.0 && Is) ? Is[n] : 0.0;
        yv[n] = mm * (p.c * (vv - vn[n]) + p.tau * (rmc_iion(p, vv, w[n]) - is)) + ai;
        ye[n] = ai + ae;
    } else {
        const double a = dg[n] * xv[n] + ai, b = ai + ae;
        if (MODE == ST_JAC) {
            yv[n] = a;
            ye[n] = b;
        } else {
            yv[n] = rv[n] - a;
            ye[n] = re[n] - b;
        }
    }
}

// Per-node operands of the stencil output besides the sums, loaded one plane
// ahead in the register march: JAC the diagonal; RES_MINUS_JAC the diagonal
// and both right-hand sides; RESIDUAL the previous potential, the gating
// variable and the stimulus.  out_store computes what stencil_out does.
struct OutOps {
    double a = 0.0, b = 0.0, c = 0.0;
};

template <int MODE>
__device__ __forceinline__ void out_load(OutOps& o, int64_t n, const double* __restrict__ dg,
                                         const double* __restrict__ rv, const double* __restrict__ re,
                                         const double* __restrict__ vn, const double* __restrict__ w,
                                         const double* __restrict__ Is, double stim) {
    if (MODE == ST_RESIDUAL) {
        o.a = vn[n];
        o.b = w[n];
        o.c = (stim != 0.0 && Is) ? Is[n] : 0.0;
    } else {
        o.a = dg[n];
        if (MODE == ST_RES_MINUS_JAC) {
            o.b = rv[n];
            o.c = re[n];
        }
    }
}

template <int MODE>
__device__ __forceinline__ void out_store(const FEParams& p, int i, int j, int k, int64_t n, double xvn,
                                          const OutOps& o, double ai, double ae, double* __restrict__ yv,
                                          double* __restrict__ ye) {
    if (MODE == ST_RESIDUAL) {
        const double mm = lumped_mass(p, i, j, k);
        yv[n] = mm * (p.c * (xvn - o.a) + p.tau * (rmc_iion(p, xvn, o.b) - o.c)) + ai;
        ye[n] = ai + ae;
    } else {
        const double a = o.a * xvn + ai, b = ai + ae;
        if (MODE == ST_JAC) {
            yv[n] = a;
            ye[n] = b;
        } else {
            yv[n] = o.b - a;
            ye[n] = o.c - b;
        }
    }
}

// DPP wave shifts of a double: dpp_lo(x) holds lane l - 1's x, dpp_hi(x)
// lane l + 1's (lanes without a source get 0).
template <int CTRL>
__device__ __forceinline__ double dpp64(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double dpp_lo(double x) { return dpp64<0x138>(x); }   // wave_shr:1
__device__ __forceinline__ double dpp_hi(double x) { return dpp64<0x130>(x); }   // wave_shl:1

constexpr int ZM_OUT = 64;   // output columns per wave
constexpr int ZM_ZB = 2;     // levels per boundary thread

struct ZmGrid {
    int gx, gy, gz, nbnd, nbt, gzb, nboundary, ntile, per;
};

template <int RY, int W, int SZ>
__host__ __device__ inline ZmGrid zm_grid(const FEParams& p) {
    ZmGrid g;
    g.gx = (p.nx - 1 + ZM_OUT - 1) / ZM_OUT;   // interior columns 1..nx-1
    g.gy = (p.ny - 1 + RY * W - 1) / (RY * W);
    g.gz = (p.nz + 1 + SZ - 1) / SZ;
    g.nbnd = 2 * (p.ny + 1) + 2 * (p.nx - 1);   // node columns on the x and y faces
    g.nbt = (g.nbnd + 64 * W - 1) / (64 * W);
    g.gzb = (p.nz + 1 + ZM_ZB - 1) / ZM_ZB;
    g.nboundary = g.nbt * g.gzb;
    g.ntile = g.nboundary + g.gx * g.gy * g.gz;
    g.per = (g.ntile + ST_XCD - 1) / ST_XCD;
    return g;
}

// One boundary node column (x or y face) of the register march: thread b
// of the boundary columns walks levels [ZM_ZB bzi, ZM_ZB (bzi + 1)) and
// reads the coefficients of its boundary class per lane.
template <int MODE>
__device__ void zm_boundary(const FEParams& p, const double* __restrict__ st, int b, int bzi, int nbnd,
                            const double* __restrict__ dg, const double* __restrict__ xv,
                            const double* __restrict__ xe, const double* __restrict__ rv,
                            const double* __restrict__ re, const double* __restrict__ vn,
                            const double* __restrict__ w, const double* __restrict__ Is, double stim,
                            double* __restrict__ yv, double* __restrict__ ye) {
    constexpr int TABN = 9 * 2 * 27;
    const int64_t plane = (int64_t)p.nx1 * p.ny1;
    const bool act = b < nbnd;
    const int bb = act ? b : 0;
    int i, j;
    if (bb < p.ny + 1) {
        i = 0; j = bb;
    } else if (bb < 2 * (p.ny + 1)) {
        i = p.nx; j = bb - (p.ny + 1);
    } else if (bb < 2 * (p.ny + 1) + (p.nx - 1)) {
        j = 0; i = 1 + bb - 2 * (p.ny + 1);
    } else {
        j = p.ny; i = 1 + bb - 2 * (p.ny + 1) - (p.nx - 1);
    }
    const int xc = (i == 0) ? 0 : (i == p.nx ? 2 : 1);
    const int yc = (j == 0) ? 0 : (j == p.ny ? 2 : 1);
    const int c54 = (xc + 3 * yc) * 54;
    const int kbeg = bzi * ZM_ZB, kend = min(kbeg + ZM_ZB, p.nz + 1);
    double aAi = 0.0, aAe = 0.0, aBi = 0.0, aBe = 0.0, aCi = 0.0, aCe = 0.0;   // nodes m - 1, m, m + 1
    for (int m = max(kbeg - 1, 0); m <= min(kend, p.nz); ++m) {
        const double* tC = st + (int64_t)min(m + 1, p.nz) * TABN + c54;
        const double* tB = st + (int64_t)m * TABN + c54 + 9;
        const double* tA = st + (int64_t)max(m - 1, 0) * TABN + c54 + 18;
#pragma unroll 1
        for (int dy = 0; dy < 3; ++dy) {
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int d = dx + 3 * dy;
                const int gi = i - 1 + dx, gj = j - 1 + dy;
                const bool ok = gi >= 0 && gi <= p.nx && gj >= 0 && gj <= p.ny;
                const int64_t n = ok ? gi + (int64_t)p.nx1 * gj + plane * m : 0;
                const double e0 = xe[n], v0 = xv[n];
                const double e = ok ? e0 : 0.0, v = ok ? v0 + e0 : 0.0;
                aCi = fma(tC[d], v, aCi);
                aCe = fma(tC[27 + d], e, aCe);
                aBi = fma(tB[d], v, aBi);
                aBe = fma(tB[27 + d], e, aBe);
                aAi = fma(tA[d], v, aAi);
                aAe = fma(tA[27 + d], e, aAe);
            }
        }
        const int k = m - 1;
        if (act && k >= kbeg && k < kend)
            stencil_out<MODE>(p, i, j, k, i + (int64_t)p.nx1 * j + plane * k, aAi, aAe, dg, xv, rv, re, vn, w,
                              Is, stim, yv, ye);
        aAi = aBi; aAe = aBe;
        aBi = aCi; aBe = aCe;
        aCi = 0.0; aCe = 0.0;
    }
    // the top node of the mesh has no plane above it
    if (act && kend == p.nz + 1)
        stencil_out<MODE>(p, i, j, p.nz, i + (int64_t)p.nx1 * j + plane * p.nz, aAi, aAe, dg, xv, rv, re, vn, w,
                          Is, stim, yv, ye);
}

template <int MODE, int RY, int W, int SZ, int PF>
__global__ __launch_bounds__(64 * W) void k_stencil_zm(FEParams p, const double* __restrict__ st,
                                                       const double* __restrict__ dg, const double* __restrict__ xv,
                                                       const double* __restrict__ xe, const double* __restrict__ rv,
                                                       const double* __restrict__ re, const double* __restrict__ vn,
                                                       const double* __restrict__ w, const double* __restrict__ Is,
                                                       double stim, double* __restrict__ yv,
                                                       double* __restrict__ ye) {
    constexpr int TABN = 9 * 2 * 27;
    const ZmGrid g = zm_grid<RY, W, SZ>(p);
    // consecutive ids go round robin to the 8 XCDs; XCD x takes the run of
    // tiles [x * per, (x + 1) * per) so neighbouring tiles share its L2
    const int tile = ((int)blockIdx.x % ST_XCD) * g.per + (int)blockIdx.x / ST_XCD;
    if (tile >= g.ntile) return;
    const int64_t plane = (int64_t)p.nx1 * p.ny1;
    if (tile < g.nboundary) {
        zm_boundary<MODE>(p, st, (tile % g.nbt) * (64 * W) + (int)(threadIdx.x + 64 * threadIdx.y), tile / g.nbt,
                          g.nbnd, dg, xv, xe, rv, re, vn, w, Is, stim, yv, ye);
        return;
    }
    const int t = tile - g.nboundary;
    const int bxi = t % g.gx, byi = (t / g.gx) % g.gy, bzi = t / (g.gx * g.gy);
    const int lane = (int)threadIdx.x;
    const int i = 1 + bxi * ZM_OUT + lane;
    const bool xout = i <= p.nx - 1;
    const int ic = min(i, p.nx);
    // halo column: left of lane 0 for lanes 0-62, right of lane 63 for 63
    const int hc = lane == 63 ? min(1 + bxi * ZM_OUT + 64, p.nx) : bxi * ZM_OUT;
    const int jb = 1 + RY * ((int)threadIdx.y + W * byi);   // first output row (wave-uniform)
    const int kbeg = bzi * SZ, kend = min(kbeg + SZ, p.nz + 1);
    double aAi[RY], aAe[RY], aBi[RY], aBe[RY], aCi[RY], aCe[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) aAi[r] = aAe[r] = aBi[r] = aBe[r] = aCi[r] = aCe[r] = 0.0;
    // rows jb - 1 .. jb + RY of a plane (rows past ny only feed unused sums)
    // and their halo values; planes are fetched two ahead of the one summed
    const int m0 = max(kbeg - 1, 0), m1 = min(kend, p.nz);
    int64_t roff[RY + 2], hoff[RY + 2];
#pragma unroll
    for (int q = 0; q < RY + 2; ++q) {
        roff[q] = ic + (int64_t)p.nx1 * min(jb - 1 + q, p.ny);
        hoff[q] = hc + (int64_t)p.nx1 * min(jb - 1 + q, p.ny);
    }
    struct Plane {
        double v[RY + 2], e[RY + 2], hv[RY + 2], he[RY + 2];
    };
    Plane nv_, n2_;
    auto fetch = [&](Plane& b, int m) {
#pragma unroll
        for (int q = 0; q < RY + 2; ++q) {
            b.v[q] = xv[roff[q] + plane * m];
            b.e[q] = xe[roff[q] + plane * m];
            b.hv[q] = xv[hoff[q] + plane * m];
            b.he[q] = xe[hoff[q] + plane * m];
        }
    };
    // output operands of node m are fetched with plane m + 1; the potential
    // at the output node is the centre row value of the previous plane
    OutOps onx[RY], ocur[RY];
    double xprev[RY];
    auto fetch_out = [&](int m) {
#pragma unroll
        for (int r = 0; r < RY; ++r)
            out_load<MODE>(onx[r], roff[r + 1] + plane * m, dg, rv, re, vn, w, Is, stim);
    };
#pragma unroll
    for (int r = 0; r < RY; ++r) xprev[r] = 0.0;
    fetch(nv_, m0);
    if (PF == 2) fetch(n2_, min(m0 + 1, m1));
    for (int m = m0; m <= m1; ++m) {
        const double* tC = st + (int64_t)min(m + 1, p.nz) * TABN + 4 * 54;
        const double* tB = st + (int64_t)m * TABN + 4 * 54 + 9;
        const double* tA = st + (int64_t)max(m - 1, 0) * TABN + 4 * 54 + 18;
        double vx[RY + 2][3], ex[RY + 2][3], xcen[RY];
#pragma unroll
        for (int q = 0; q < RY + 2; ++q) {
            const double sv = nv_.v[q] + nv_.e[q], hs = nv_.hv[q] + nv_.he[q];   // v + u_e (intracellular)
            const double lv = dpp_lo(sv), rv2 = dpp_hi(sv), le = dpp_lo(nv_.e[q]), re2 = dpp_hi(nv_.e[q]);
            vx[q][0] = lane == 0 ? hs : lv;
            vx[q][1] = sv;
            vx[q][2] = lane == 63 ? hs : rv2;
            ex[q][0] = lane == 0 ? nv_.he[q] : le;
            ex[q][1] = nv_.e[q];
            ex[q][2] = lane == 63 ? nv_.he[q] : re2;
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            xcen[r] = nv_.v[r + 1];
            ocur[r] = onx[r];
        }
        fetch_out(m);
        if (PF == 2) {
            nv_ = n2_;
            fetch(n2_, min(m + 2, m1));
        } else {
            fetch(nv_, min(m + 1, m1));
        }
        // One target level at a time, so only its 18 coefficients are live:
        // the empty asm statements route the table pointer and the finished
        // sums through the (ordered) volatile statements, so the scalar loads
        // of one target cannot be hoisted above the previous target's
        // products and the products cannot sink into the store branch.
        // Without them all 54 coefficients are loaded at the top of the
        // plane, more than the scalar register file holds.
        // The table is read-only during the kernel, so it is read through
        // the constant address space, which keeps the loads scalar.
        auto add = [&](const double* tb, double (&si)[RY], double (&se)[RY]) {
            asm volatile("" : "+s"(tb));
            const __attribute__((address_space(4))) double* tk =
                (const __attribute__((address_space(4))) double*)tb;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const int d = dx + 3 * dy;
                    const double ci = tk[d], ce = tk[27 + d];
#pragma unroll
                    for (int r = 0; r < RY; ++r) {
                        si[r] = fma(ci, vx[r + dy][dx], si[r]);
                        se[r] = fma(ce, ex[r + dy][dx], se[r]);
                    }
                }
#pragma unroll
            for (int r = 0; r < RY; ++r) asm volatile("" : "+v"(si[r]), "+v"(se[r]));
        };
        add(tC, aCi, aCe);
        add(tB, aBi, aBe);
        add(tA, aAi, aAe);
        const int k = m - 1;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int j = jb + r;
            if (xout && j <= p.ny - 1 && k >= kbeg && k < kend)
                out_store<MODE>(p, i, j, k, i + (int64_t)p.nx1 * j + plane * k, xprev[r], ocur[r], aAi[r], aAe[r],
                                yv, ye);
            xprev[r] = xcen[r];
            aAi[r] = aBi[r]; aAe[r] = aBe[r];
            aBi[r] = aCi[r]; aBe[r] = aCe[r];
            aCi[r] = 0.0; aCe[r] = 0.0;
        }
    }
    if (kend == p.nz + 1) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int j = jb + r;
            if (xout && j <= p.ny - 1)
                out_store<MODE>(p, i, j, p.nz, i + (int64_t)p.nx1 * j + plane * p.nz, xprev[r], onx[r], aAi[r],
                                aAe[r], yv, ye);
        }
    }
}

__global__ void k_ionic_update(int64_t N, double tau, double eta2, double vp,
                               const double* __restrict__ v, double* __restrict__ w) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    w[n] = (w[n] + tau * eta2 * v[n] / vp) / (1.0 + tau * eta2);
}

__global__ void k_reaction_diag(FEParams p, const double* __restrict__ v, const double* __restrict__ w,
                                double* __restrict__ dg, int* __restrict__ bad) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= p.N) return;
    const int64_t t = n / p.nx1;
    const int i = (int)(n - t * p.nx1);
    const int k = (int)(t / p.ny1);
    const int j = (int)(t - (int64_t)k * p.ny1);
    const double m = p.mnode ? p.mnode[n] : lumped_mass(p, i, j, k);
    const double d = m * (p.c + p.tau * rmc_diion(p, v[n], w[n]));
    dg[n] = d;
    if (!(d > 0.0)) atomicOr(bad, 1);
}

// ------------------------------------------------------ mapped (curved) meshes
// The stencil pass of k_stencil on a mesh whose coefficients differ at every
// node: one thread per node (x fastest), the 2 x 27 coefficients read from
// the node-major tables (consecutive lanes read consecutive addresses), the
// neighbour values from memory through the caches.  The coefficient tables
// are the dominant traffic: 432 bytes per node against 40 for the vectors.
// Consecutive workgroup ids go round robin to the 8 XCDs, so XCD x takes the
// contiguous run of node blocks [x * per, (x + 1) * per): the y and z
// neighbours of its nodes are then mostly its own, already in its L2.
constexpr int GEN_WG = 256;

template <int MODE>
__global__ __launch_bounds__(GEN_WG) void k_stencil_gen(FEParams p, const double* __restrict__ dg,
                                                     const double* __restrict__ xv, const double* __restrict__ xe,
                                                     const double* __restrict__ rv, const double* __restrict__ re,
                                                     const double* __restrict__ vn, const double* __restrict__ w,
                                                     const double* __restrict__ Is, double stim,
                                                     double* __restrict__ yv, double* __restrict__ ye) {
    const int64_t nblk = (p.N + GEN_WG - 1) / GEN_WG, per = (nblk + ST_XCD - 1) / ST_XCD;
    const int64_t blk = (int64_t)(blockIdx.x % ST_XCD) * per + blockIdx.x / ST_XCD;
    const int64_t n = blk * GEN_WG + threadIdx.x;
    if (blk >= nblk || n >= p.N) return;
    const int64_t plane = (int64_t)p.nx1 * p.ny1;
    const int k = (int)(n / plane);
    const int64_t t = n - (int64_t)k * plane;
    const int j = (int)(t / p.nx1), i = (int)(t - (int64_t)j * p.nx1);
    const double* __restrict__ ci = p.stn + n;
    const double* __restrict__ ce = p.stn + 27 * p.N + n;
    double ai = 0.0, ae = 0.0;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (i + dx < 0 || i + dx > p.nx || j + dy < 0 || j + dy > p.ny || k + dz < 0 || k + dz > p.nz)
                    continue;
                const int d = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
                const int64_t q = n + dx + (int64_t)dy * p.nx1 + (int64_t)dz * plane;
                const double xeq = xe[q];
                ai = fma(ci[(int64_t)d * p.N], xv[q] + xeq, ai);
                ae = fma(ce[(int64_t)d * p.N], xeq, ae);
            }
    if (MODE == ST_RESIDUAL) {
        const double vv = xv[n];
        const double is = (stim != 0.0 && Is) ? Is[n] : 0.0;
        yv[n] = p.mnode[n] * (p.c * (vv - vn[n]) + p.tau * (rmc_iion(p, vv, w[n]) - is)) + ai;
        ye[n] = ai + ae;
    } else {
        const double a = dg[n] * xv[n] + ai, b = ai + ae;
        if (MODE == ST_JAC) {
            yv[n] = a;
            ye[n] = b;
        } else {
            yv[n] = rv[n] - a;
            ye[n] = re[n] - b;
        }
    }
}

// Truncated ellipsoid (Sec. 6): point of the parametric map and the
// orthonormal frame (e1 along dX/dphi, e2 along dX/dtheta orthogonalised
// against e1, n = e1 x e2).
__device__ inline void ell_axes(const EllGeom& g, double r, double& a, double& b, double& c) {
    a = g.p[0] + r * (g.p[1] - g.p[0]);
    b = g.p[2] + r * (g.p[3] - g.p[2]);
    c = g.p[4] + r * (g.p[5] - g.p[4]);
}

__device__ inline void ell_node(const FEParams& p, const EllGeom& g, int i, int j, int k, double X[3]) {
    const double ph = g.p[8] + (g.p[9] - g.p[8]) * (double)i / p.nx;
    const double th = g.p[6] + (g.p[7] - g.p[6]) * (double)j / p.ny;
    double a, b, c;
    ell_axes(g, (double)k / p.nz, a, b, c);
    X[0] = a * cos(th) * cos(ph);
    X[1] = b * cos(th) * sin(ph);
    X[2] = c * sin(th);
}

// Per element (one thread each): the isoparametric Q1 stiffness of both
// media, tau-scaled, into ke[(e * 2 + m) * 64 + a * 8 + b], and the corner
// masses int_e phi_a into mec[e * 8 + a], by 2x2x2 Gauss quadrature on the
// trilinear map; a non-positive Jacobian determinant sets *bad.  The tensor
// of medium m is sum sigma_* a_* a_*^T in the frame at the element's
// parametric centre with the fibre at angle th0 + (th1 - th0) r_c.
__global__ void k_iso_elements(FEParams p, EllGeom g, IsoMedia md, double* __restrict__ ke,
                               double* __restrict__ mec, int* __restrict__ bad) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ne = (int64_t)p.nx * p.ny * p.nz;
    if (e >= ne) return;
    const int ex = (int)(e % p.nx), ey = (int)((e / p.nx) % p.ny), ez = (int)(e / ((int64_t)p.nx * p.ny));
    double X[8][3];
#pragma unroll
    for (int a = 0; a < 8; ++a) ell_node(p, g, ex + (a & 1), ey + ((a >> 1) & 1), ez + (a >> 2), X[a]);
    // frame and tensors at the parametric centre
    const double rc = (ez + 0.5) / p.nz;
    const double ph = g.p[8] + (g.p[9] - g.p[8]) * (ex + 0.5) / p.nx;
    const double th = g.p[6] + (g.p[7] - g.p[6]) * (ey + 0.5) / p.ny;
    double aa, bb, cc;
    ell_axes(g, rc, aa, bb, cc);
    double e1[3] = {-aa * cos(th) * sin(ph), bb * cos(th) * cos(ph), 0.0};
    double t2[3] = {-aa * sin(th) * cos(ph), -bb * sin(th) * sin(ph), cc * cos(th)};
    const double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int d = 0; d < 3; ++d) e1[d] /= n1;
    const double pr = t2[0] * e1[0] + t2[1] * e1[1] + t2[2] * e1[2];
    for (int d = 0; d < 3; ++d) t2[d] -= pr * e1[d];
    const double n2 = sqrt(t2[0] * t2[0] + t2[1] * t2[1] + t2[2] * t2[2]);
    for (int d = 0; d < 3; ++d) t2[d] /= n2;
    const double nn[3] = {e1[1] * t2[2] - e1[2] * t2[1], e1[2] * t2[0] - e1[0] * t2[2], e1[0] * t2[1] - e1[1] * t2[0]};
    const double al = md.th0 + (md.th1 - md.th0) * rc;
    double fl[3], ft[3];
    for (int d = 0; d < 3; ++d) {
        fl[d] = cos(al) * e1[d] + sin(al) * t2[d];
        ft[d] = -sin(al) * e1[d] + cos(al) * t2[d];
    }
    double D[2][3][3];
    for (int m = 0; m < 2; ++m) {
        const double* sg = m ? md.sig_e : md.sig_i;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) D[m][r][c] = sg[0] * fl[r] * fl[c] + sg[1] * ft[r] * ft[c] + sg[2] * nn[r] * nn[c];
    }
    double* Ke = ke + e * 128;
    double* Me = mec + e * 8;
    for (int q = 0; q < 128; ++q) Ke[q] = 0.0;
    for (int a = 0; a < 8; ++a) Me[a] = 0.0;
    const double gp[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
    for (int qp = 0; qp < 8; ++qp) {
        const double s = gp[qp & 1], tt = gp[(qp >> 1) & 1], u = gp[qp >> 2];
        double val[8], gr[8][3];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
            const double fx = ax ? s : 1.0 - s, fy = ay ? tt : 1.0 - tt, fz = az ? u : 1.0 - u;
            const double sx = ax ? 1.0 : -1.0, sy = ay ? 1.0 : -1.0, sz = az ? 1.0 : -1.0;
            val[a] = fx * fy * fz;
            gr[a][0] = sx * fy * fz;
            gr[a][1] = fx * sy * fz;
            gr[a][2] = fx * fy * sz;
        }
        double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};   // J[d][r] = dx_d / dxi_r
#pragma unroll
        for (int a = 0; a < 8; ++a)
            for (int d = 0; d < 3; ++d)
                for (int r = 0; r < 3; ++r) J[d][r] += X[a][d] * gr[a][r];
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        if (!(det > 0.0)) {
            atomicOr(bad, 1);
            return;
        }
        // inverse: Ji[r][d] = cofactor(d, r) / det
        double Ji[3][3];
        Ji[0][0] = c00 / det;
        Ji[1][0] = c01 / det;
        Ji[2][0] = c02 / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        double G[8][3];
#pragma unroll
        for (int a = 0; a < 8; ++a)
            for (int d = 0; d < 3; ++d) G[a][d] = gr[a][0] * Ji[0][d] + gr[a][1] * Ji[1][d] + gr[a][2] * Ji[2][d];
        const double wq = det / 8.0;
        for (int m = 0; m < 2; ++m) {
            double DG[8][3];
#pragma unroll
            for (int b = 0; b < 8; ++b)
                for (int d = 0; d < 3; ++d)
                    DG[b][d] = D[m][d][0] * G[b][0] + D[m][d][1] * G[b][1] + D[m][d][2] * G[b][2];
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int b = 0; b < 8; ++b)
                    Ke[m * 64 + a * 8 + b] +=
                        md.tau * wq * (G[a][0] * DG[b][0] + G[a][1] * DG[b][1] + G[a][2] * DG[b][2]);
        }
#pragma unroll
        for (int a = 0; a < 8; ++a) Me[a] += wq * val[a];
    }
}

// Per node (one thread each): the 27-point stencil rows of both media and the
// lumped mass, summed over the (up to 8) elements around the node in a fixed
// order.
__global__ __launch_bounds__(256) void k_node_stencil(FEParams p, const double* __restrict__ ke,
                                                      const double* __restrict__ mec, double* __restrict__ stn,
                                                      double* __restrict__ mnode) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= p.N) return;
    const int64_t plane = (int64_t)p.nx1 * p.ny1;
    const int k = (int)(n / plane);
    const int64_t t = n - (int64_t)k * plane;
    const int j = (int)(t / p.nx1), i = (int)(t - (int64_t)j * p.nx1);
    double acc[2][27];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int d = 0; d < 27; ++d) acc[m][d] = 0.0;
    double mass = 0.0;
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy)
#pragma unroll
            for (int ox = 0; ox < 2; ++ox) {
                const int ei = i - 1 + ox, ej = j - 1 + oy, ek = k - 1 + oz;
                if (ei < 0 || ei >= p.nx || ej < 0 || ej >= p.ny || ek < 0 || ek >= p.nz) continue;
                const int64_t e = ei + (int64_t)p.nx * (ej + (int64_t)p.ny * ek);
                const int a = (1 - ox) + 2 * (1 - oy) + 4 * (1 - oz);
                mass += mec[e * 8 + a];
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const int dx = (b & 1) - (1 - ox), dy = ((b >> 1) & 1) - (1 - oy), dz = (b >> 2) - (1 - oz);
                    const int d = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
                    acc[0][d] += ke[(e * 2 + 0) * 64 + a * 8 + b];
                    acc[1][d] += ke[(e * 2 + 1) * 64 + a * 8 + b];
                }
            }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int d = 0; d < 27; ++d) stn[(int64_t)(m * 27 + d) * p.N + n] = acc[m][d];
    mnode[n] = mass;
}

// tile variants (SX, SY, SZ)
// Variants: 0-6 the LDS kernel with tiles (SX, SY, SZ) = (32, 8, 8),
// (32, 8, 16), (64, 4, 8), (32, 4, 16), (16, 16, 8), (32, 8, 4), (16, 16, 4);
// 7-10 the register march with (RY, W, SZ) = (1, 4, 8), (2, 4, 8),
// (2, 4, 16), (4, 4, 8).
constexpr int ST_NVAR = 11;

template <int MODE, int SX, int SY, int SZ, typename... Args>
void launch_stencil_shape(hipStream_t s, const FEParams& p, Args... args) {
    const int ntile = ((p.nx1 + SX - 1) / SX) * ((p.ny1 + SY - 1) / SY) * ((p.nz + 1 + SZ - 1) / SZ);
    const int per = (ntile + ST_XCD - 1) / ST_XCD;
    hipLaunchKernelGGL((k_stencil<MODE, SX, SY, SZ>), dim3((unsigned)(per * ST_XCD)), dim3(SX, SY), 0, s, p, args...);
}

template <int MODE, int RY, int W, int SZ, int PF, typename... Args>
void launch_stencil_zm(hipStream_t s, const FEParams& p, Args... args) {
    const ZmGrid g = zm_grid<RY, W, SZ>(p);
    hipLaunchKernelGGL((k_stencil_zm<MODE, RY, W, SZ, PF>), dim3((unsigned)(g.per * ST_XCD)), dim3(64, W), 0, s, p,
                       args...);
}

template <int MODE, typename... Args>
void launch_stencil(hipStream_t s, const FEParams& p, const double* st, Args... args) {
    if (p.stn) {
        const int64_t nblk = (p.N + GEN_WG - 1) / GEN_WG, per = (nblk + ST_XCD - 1) / ST_XCD;
        hipLaunchKernelGGL(k_stencil_gen<MODE>, dim3((unsigned)(per * ST_XCD)), dim3(GEN_WG), 0, s, p, args...);
        return;
    }
    switch (p.stencil_variant) {
        case 1: launch_stencil_shape<MODE, 32, 8, 16>(s, p, st, args...); break;
        case 2: launch_stencil_shape<MODE, 64, 4, 8>(s, p, st, args...); break;
        case 3: launch_stencil_shape<MODE, 32, 4, 16>(s, p, st, args...); break;
        case 4: launch_stencil_shape<MODE, 16, 16, 8>(s, p, st, args...); break;
        case 5: launch_stencil_shape<MODE, 32, 8, 4>(s, p, st, args...); break;
        case 6: launch_stencil_shape<MODE, 16, 16, 4>(s, p, st, args...); break;
        case 7: launch_stencil_zm<MODE, 1, 4, 8, 1>(s, p, st, args...); break;
        case 8: launch_stencil_zm<MODE, 1, 4, 16, 2>(s, p, st, args...); break;
        case 9: launch_stencil_zm<MODE, 2, 4, 16, 1>(s, p, st, args...); break;
        case 10: launch_stencil_zm<MODE, 2, 4, 16, 2>(s, p, st, args...); break;
        default: launch_stencil_shape<MODE, 32, 8, 8>(s, p, st, args...);
    }
}

}  // namespace

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_ionic_update(hipStream_t s, const FEParams& p, const double* v, double* w) {
    hipLaunchKernelGGL(k_ionic_update, dim3(nblk(p.N, 256)), dim3(256), 0, s, p.N, p.tau, p.eta2,
                       p.vp, v, w);
}

void launch_residual(hipStream_t s, const FEParams& p, const double* st, const double* v,
                     const double* ue, const double* vn, const double* w, const double* Is,
                     double stim, double* Rv, double* Re) {
    launch_stencil<ST_RESIDUAL>(s, p, st, (const double*)nullptr, v, ue, (const double*)nullptr,
                                (const double*)nullptr, vn, w, Is, stim, Rv, Re);
}

void launch_reaction_diag(hipStream_t s, const FEParams& p, const double* v, const double* w,
                          double* dg, int* bad) {
    hipLaunchKernelGGL(k_reaction_diag, dim3(nblk(p.N, 256)), dim3(256), 0, s, p, v, w, dg, bad);
}

void launch_jac_apply(hipStream_t s, const FEParams& p, const double* st, const double* dg,
                      const double* x, double* y) {
    launch_stencil<ST_JAC>(s, p, st, dg, x, x + p.N, (const double*)nullptr, (const double*)nullptr,
                           (const double*)nullptr, (const double*)nullptr, (const double*)nullptr, 0.0, y, y + p.N);
}

void launch_res_minus_jac(hipStream_t s, const FEParams& p, const double* st, const double* dg,
                          const double* x, const double* r, double* y) {
    launch_stencil<ST_RES_MINUS_JAC>(s, p, st, dg, x, x + p.N, r, r + p.N, (const double*)nullptr,
                                     (const double*)nullptr, (const double*)nullptr, 0.0, y, y + p.N);
}

int stencil_variants() { return ST_NVAR; }

void launch_mapped_mesh(hipStream_t s, const FEParams& p, const EllGeom& g, const IsoMedia& md, double* ke,
                        double* mec, double* stn, double* mnode, int* bad) {
    const int64_t ne = (int64_t)p.nx * p.ny * p.nz;
    hipLaunchKernelGGL(k_iso_elements, dim3(nblk(ne, 64)), dim3(64), 0, s, p, g, md, ke, mec, bad);
    hipLaunchKernelGGL(k_node_stencil, dim3(nblk(p.N, 256)), dim3(256), 0, s, p, (const double*)ke,
                       (const double*)mec, stn, mnode);
}

}  // namespace bdm
