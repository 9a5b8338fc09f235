// Shared definitions for the HIP kernels and the host orchestration.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace bdm {

// Threads per workgroup for batched per-subdomain kernels (4 wave64).
constexpr int kWG = 256;

// Primal unknowns of one box subdomain (Sec. 4.4): the (v, u_e) values at
// its 8 vertices, and two averages over each of its 12 edges and 6 faces
// (the richest primal space, vertices + edges + faces).
constexpr int MAXV = 16;                    // vertex dofs
constexpr int MAXC = 36;                    // average constraints
constexpr int MAXP = MAXC + MAXV;           // primal dofs
constexpr int SVV_STRIDE = MAXV * MAXV;     // per-subdomain S_VV block
constexpr int SP_STRIDE = MAXP * MAXP;      // per-subdomain coarse block

// Pointwise and stencil parameters of the Bidomain step.
struct FEParams {
    int nx, ny, nz;             // elements per axis
    int nx1, ny1;               // nodes per axis (x, y)
    int64_t N;                  // nodes
    double h, tau, c;           // element size along x, time step, chi*C_m
    double hy = 0.0, hz = 0.0;  // element sizes along y and z
    double chiG, chieta1, eta2, vth, vp;
    int stencil_variant = 0;    // tile shape of the stencil kernel (autotuned)
    // Mapped (curved) meshes: per-node 27-point stencils of tau A_i and tau A_e
    // (stn[(m * 27 + d) * N + n], d = (dx+1) + 3(dy+1) + 9(dz+1)), per-node
    // lumped masses, and per-element corner masses mec[e * 8 + a]; the element
    // matrices are then per element (e = ex + nx (ey + ny ez)) instead of per
    // z-layer.  All null on box meshes.
    const double* stn = nullptr;
    const double* mnode = nullptr;
    const double* mec = nullptr;
};

__host__ __device__ inline double rmc_iion(const FEParams& p, double v, double w) {
    return p.chiG * v * (1.0 - v / p.vth) * (1.0 - v / p.vp) + p.chieta1 * v * w;
}

// d(chi I_ion)/dv = chi G (1 - 2v/v_th - 2v/v_p + 3 v^2/(v_th v_p)) + chi eta_1 w
__host__ __device__ inline double rmc_diion(const FEParams& p, double v, double w) {
    const double a = 1.0 / p.vth, b = 1.0 / p.vp;
    return p.chiG * (1.0 - 2.0 * v * (a + b) + 3.0 * v * v * a * b) + p.chieta1 * w;
}

}  // namespace bdm
