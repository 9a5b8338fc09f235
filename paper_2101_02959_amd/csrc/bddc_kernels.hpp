// Launch wrappers of the per-iteration BDDC / FETI-DP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace bdm {

// Per-subdomain local vectors (device arrays, length nsub).
struct SubVecDesc {
    int nsub;
    const int* nr;
    const int* nV;
    const int* nc;
    const int64_t* xoff;    // start of the subdomain's local r-vector
    const int64_t* F_off;   // Y = L_rr^{-1} C^T (first nc columns of F)
    const int64_t* Z_off;
    const int64_t* P_off;   // start of the subdomain's primal list
    const int* primal;      // local primal -> global primal
};

// Coarse right-hand side gather.
struct CoarseDesc {
    int np;                 // global primal dofs
    int nverts;
    const int* vnode;       // vertex -> global node
    const int* cp_ptr;      // primal dof -> contributions (CSR)
    const int* cp_sub;
    const int* cp_loc;
};

// FETI-DP multiplier blocks: per object, the pairs (a < b) of sharing
// subdomains (CSR over objects).
struct FetiDesc {
    const int* pr_ptr;
    const int* pr_a;        // subdomain ids
    const int* pr_b;
    const int* pr_qa;       // share indices (into the object's share list)
    const int* pr_qb;
    const int64_t* pr_off;  // offset of the block in lambda
    const int64_t* sh_yoff; // staging offset per share
};

template <typename T>
void launch_gather_I(hipStream_t s, int n, const int* list, int64_t N, const double* r, const double* q, T* x);
template <typename T>
void launch_scatter_I(hipStream_t s, int n, const int* list, int64_t N, const T* x, double* out);
template <typename T>
void launch_deluxe_res(hipStream_t s, const ObjDesc& o, int64_t N, const double* g, const T* dmat, T* xr,
                       const int64_t* xoff);
template <typename T>
void launch_deluxe_val(hipStream_t s, const ObjDesc& o, int64_t N, const T* dmatT, const T* xr,
                       const int64_t* xoff, double* z);
// dmatT <- the transpose of every E_m block of dmat (same offsets), for the
// value side; deluxe_max_shares() bounds the shares of one object.
template <typename T>
void launch_deluxe_transpose(hipStream_t s, const ObjDesc& o, const T* dmat, T* dmatT);
int deluxe_max_shares();
// rho scaling: every share's matrix (and its transpose) set to the diagonal
// of its weights, w[2q] on the v dofs and w[2q + 1] on the u_e dofs.
template <typename T>
void launch_rho_fill(hipStream_t s, const ObjDesc& o, const double* w, T* dmat, T* dmatT);
template <typename T>
void launch_coarse_rhs_local(hipStream_t s, const SubVecDesc& d, const T* xr, const T* Z, double* cP, double* mu);
void launch_coarse_rhs_gather(hipStream_t s, const CoarseDesc& c, int64_t N, const double* g,
                              const double* cP, double* b);
void launch_coarse_project(hipStream_t s, int np, int pin, double* b);
template <typename T>
void launch_neumann_rhs(hipStream_t s, const SubVecDesc& d, const T* F, const T* Z, const double* mu,
                        const double* uc, T* xr, int with_mu);
void launch_vertex_val(hipStream_t s, int nv, const int* vnode, int64_t N, const double* uc, double* z);
template <typename T>
void launch_feti_BT(hipStream_t s, const ObjDesc& o, const FetiDesc& f, const double* lam, T* xr,
                    const int64_t* xoff);
template <typename T>
void launch_feti_B(hipStream_t s, const ObjDesc& o, const FetiDesc& f, const T* xr, const int64_t* xoff,
                   double* lam);
template <typename T>
void launch_feti_BDT(hipStream_t s, const ObjDesc& o, const FetiDesc& f, const double* lam, const T* dmat, T* xr,
                     const int64_t* xoff);
template <typename T>
void launch_feti_BD(hipStream_t s, const ObjDesc& o, const FetiDesc& f, const T* xr, const int64_t* xoff,
                    const T* dmat, double* lam);
template <typename T>
void launch_schur_mv(hipStream_t s, const SubVecDesc& d, const T* Srr, const int64_t* Soff, const T* x, T* y);
template <typename T>
void launch_split_res(hipStream_t s, const ObjDesc& o, int64_t N, const double* g, T* xr, const int64_t* xoff);
template <typename T>
void launch_take_first(hipStream_t s, const ObjDesc& o, int64_t N, const T* xr, const int64_t* xoff, double* z);

// ---- vec.hip: FP64 vector kernels with deterministic two-stage reductions
// Reductions take a partial buffer of dot_partials() doubles and a ticket
// array of vec_tickets() zero-initialised unsigned ints (vec.hip).
void launch_dot(hipStream_t s, int64_t n, const double* x, const double* y, double* partial, unsigned* tickets,
                double* out);
void launch_axpy(hipStream_t s, int64_t n, double a, const double* x, double* y);
void launch_copy(hipStream_t s, int64_t n, const double* x, double* y);
// device-scalar and capture-safe vector operations (PCG)
void launch_axpy_dev(hipStream_t s, int64_t n, const double* a, double sgn, const double* x, double* y);
void launch_scale_add_dev(hipStream_t s, int64_t n, const double* z, const double* b, double* p);
void launch_fill(hipStream_t s, int64_t n, double v, double* x);
template <typename T>
void launch_fill_t(hipStream_t s, int64_t n, T v, T* x);
void launch_copy_kernel(hipStream_t s, int64_t n, const double* x, double* y);
// x += alpha p, r -= alpha q, ||r||^2 and the stopping test (slots sc)
void launch_pcg_update(hipStream_t s, int64_t n, double* sc, const double* p, const double* q, double* x, double* r,
                       double* partial, unsigned* tickets, double* hist, double* ah, int maxit);
// z.r, z.q and the Polak-Ribiere beta (slots sc)
void launch_pcg_beta(hipStream_t s, int64_t n, double* sc, const double* z, const double* r, const double* q,
                     double* partial, unsigned* tickets, double* bh);
void launch_scale_add(hipStream_t s, int64_t n, const double* z, double b, double* p);  // p = z + b p
void launch_sub_mean(hipStream_t s, int64_t n, double* x, double* partial, unsigned* tickets, double* tmp);
int dot_partials();
int vec_tickets();

}  // namespace bdm
