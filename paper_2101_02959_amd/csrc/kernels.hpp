// Launch wrappers of the HIP kernels (host-callable).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "common.hpp"

namespace bdm {

// ---- fe.hip
// element sizes hd = (hx, hy, hz)
std::vector<double> layer_matrices(int nz, const double hd[3], double tau, const double sig_i[3],
                                   const double sig_e[3], double th0, double th1);
std::vector<double> stencil_tables(int nz, const std::vector<double>& ke);
// the same into caller buffers: ke of nz * 128 doubles, st of (nz + 1) * 486
void layer_matrices_into(int nz, const double hd[3], double tau, const double sig_i[3], const double sig_e[3],
                         double th0, double th1, double* ke);
void stencil_tables_into(int nz, const double* ke, double* st);
void launch_ionic_update(hipStream_t s, const FEParams& p, const double* v, double* w);
void launch_residual(hipStream_t s, const FEParams& p, const double* st, const double* v,
                     const double* ue, const double* vn, const double* w, const double* Is,
                     double stim, double* Rv, double* Re);
void launch_reaction_diag(hipStream_t s, const FEParams& p, const double* v, const double* w,
                          double* dg, int* bad);
void launch_jac_apply(hipStream_t s, const FEParams& p, const double* st, const double* dg,
                      const double* x, double* y);
void launch_res_minus_jac(hipStream_t s, const FEParams& p, const double* st, const double* dg,
                          const double* x, const double* r, double* y);
// Truncated-ellipsoid parameters {a1, a2, b1, b2, c1, c2, theta_min,
// theta_max, phi_min, phi_max} and the media of the isoparametric elements.
struct EllGeom {
    double p[10];
};
struct IsoMedia {
    double sig_i[3], sig_e[3], th0, th1, tau;
};
// Mapped mesh set-up: per-element tau-scaled stiffness ke (nx ny nz * 128
// doubles) and corner masses mec (* 8), then the per-node stencils stn
// (54 N) and lumped masses mnode (N); *bad is set on a non-positive
// Jacobian determinant.
void launch_mapped_mesh(hipStream_t s, const FEParams& p, const EllGeom& g, const IsoMedia& md, double* ke,
                        double* mec, double* stn, double* mnode, int* bad);
// Variants of the stencil pass (FEParams::stencil_variant: LDS tile shapes
// and register z-march shapes, all with the same summation order); the
// autotuner picks one per mesh.
int stencil_variants();

// ---- dense.hip: batched dense linear algebra, one workgroup per matrix.
// Per-subdomain layout descriptor (device arrays, length nsub).
struct BatchDesc {
    int nsub;
    int sub0;              // first subdomain of the batch (chunked setup)
    const int* n;          // local dofs nI + nG (= leading dimension of K)
    const int* nI;
    const int* nr;
    const int* nV;
    const int* nc;
    const int64_t* K_off;  // start of the local matrix K in the (chunk) K buffer
    const int* box;        // ex0, ey0, ez0, Lx, Ly, Lz per subdomain
    const int64_t* lmap_off;
    const int* lmap;       // box node -> local node index in [I | r | V]
    const int64_t* F_off;  // start of the nr x (nc + nV) RHS / solution block
    const int64_t* Z_off;  // start of Z (nr x nP)
    const int64_t* Gi_off; // start of G^{-1} (nc x nc)
    const int64_t* Sp_off; // start of the local coarse matrix (nP x nP, double)
    const int64_t* so_ptr; // per-subdomain object list (CSR) ...
    const int* so_roff;    //   object offset in the local r-dofs
    const int* so_n;       //   object dofs
    const int64_t* so_slot;//   start of this subdomain's copy of the object block
    const int* so_kind;    //   0 face, 1 edge
    const int* so_nnode;   //   object nodes (for the constraint rows)
    const int* so_eidx;    //   constraint index c of the object (rows 2c, 2c+1
                           //   of C) or -1 when the primal space leaves it free
    const int64_t* Srr_off;// start of the saved S_rr copy (FETI-DP) or null
};

template <typename T>
void launch_assemble(hipStream_t s, const BatchDesc& d, int maxbox, const FEParams& p,
                     const double* ke, const double* v, const double* w, T* K);
// Cholesky of columns [c0, c1) of each local matrix (trailing update within them).
template <typename T>
void launch_potrf(hipStream_t s, int nb, T* A, const int64_t* off, const int* ld, const int* c0,
                  const int* c1, const int* c2, int* info);
// Interior elimination, right looking in panels of interior_panel_width()
// columns: for J = 0, w, 2w, ...: the panel (diagonal block, then the rows
// below; Wbuf holds panel_wbuf_stride() values per matrix, rowblocks = max
// over the batch of panel_rowblocks(...)), then the trailing update
// (schur = false); finally the Schur update of the interface block
// (schur = true).  tiles = max over the batch of syrk_tiles(...) for the
// same variant of the rank-k kernel (its output tile and inner chunk; the
// variants are chosen by the autotuner, 0 is the default).
template <typename T>
// P, poff: when P is given, the rows below nI of the panel columns are also
// written to the panel-packed copy of the factor at P + poff[matrix].
// nIc (optional): per matrix, the leading columns [0, nIc[m]) whose rows
// [nI, n) are zero in the assembled matrix; they stay zero in the factor,
// so row blocks wholly in [nI, n) skip panels inside [0, nIc).
void launch_interior_panel(hipStream_t s, int nb, T* A, const int64_t* off, const int* ld, const int* nI,
                           const int* n, int J, T* Wbuf, int rowblocks, int* info, T* P = nullptr,
                           const int64_t* poff = nullptr, const int* nIc = nullptr);
// nIc as above: tiles whose rows lie in [nI, n) take only the inner
// indices k >= nIc[m], where their operand is not zero.
template <typename T>
void launch_syrk_update(hipStream_t s, int nb, T* A, const int64_t* off, const int* ld, const int* nI, const int* n,
                        bool schur, int J, int tiles, int variant = 0, const int* nIc = nullptr);
int interior_panel_width();
int panel_wbuf_stride();
// row blocks of k_panel_trsm and trailing tiles of the rank-k update for
// the panel at J of one matrix (nIc: its core columns, 0 for none)
int panel_rowblocks(int J, int nI, int n, int nIc = 0);
int syrk_tiles(bool schur, int J, int nI, int n, int variant = 0, int nIc = 0);
int syrk_variants();          // number of rank-k variants
int syrk_variant_tm(int v);   // output tile edge of variant v
int syrk_variant_kc(int v);   // inner chunk of variant v
template <typename T>
void launch_extract(hipStream_t s, const BatchDesc& d, const T* K, T* slots, T* F, double* Svv,
                    T* Srr);
// Zero the lower triangles of the chunk's local matrices (maxn bounds n).
template <typename T>
void launch_clear_lower(hipStream_t s, const BatchDesc& d, int maxn, T* K);
// Panel-packed storage of the Dirichlet and Neumann factors, which the
// per-iteration solves stream: column blocks of PP_NB; block b holds the rows
// b PP_NB .. n-1, each as PP_NB consecutive entries (the row's part of the
// block's columns; entries right of the diagonal or past column n-1 are
// zero).  Every row starts on a PP_NB-entry boundary, so the solves read
// whole cache lines only, and the storage holds the lower triangle only.
constexpr int PP_NB = 32;
__host__ __device__ inline int64_t pp_block(int n, int b) {   // first entry of block b
    return (int64_t)PP_NB * ((int64_t)b * n - (int64_t)PP_NB * b * (b - 1) / 2);
}
__host__ __device__ inline int64_t pp_size(int n) { return pp_block(n, (n + PP_NB - 1) / PP_NB); }

// Multi-right-hand-side forward solve L X = B with panel-packed L.
template <typename T>
void launch_trsm_fwd(hipStream_t s, int nb, const T* L, const int64_t* Loff, const int* n,
                     T* B, const int64_t* Boff, const int* ldb, const int* k);
template <typename T>
void launch_coarse_local(hipStream_t s, const BatchDesc& d, const T* F, const double* Svv, T* Z,
                         double* Sp, int* info);
// Schedule of a batched one-workgroup-per-matrix kernel over uneven matrices.
// With order and counter set, the launch is persistent (as many workgroups
// as fit on the device) and each workgroup draws the next matrix from the
// counter, in the given order (largest cost first: LPT); the last workgroup
// to finish resets the two counters to zero for the next launch.  Without
// them, one workgroup per matrix in index order.
struct WorkQueue {
    const int* order = nullptr;   // device: nb matrix indices, decreasing cost
    int* counter = nullptr;       // device: 2 ints (next item, finished workgroups), zero between launches
};
// Batched triangular solves with the panel-packed n x n lower factor of each
// matrix, in place on x; maxn bounds n over the batch.
template <typename T>
void launch_trsv(hipStream_t s, int nb, bool trans, const T* L, const int64_t* Loff, const int* n,
                 T* x, const int64_t* xoff, int maxn, const WorkQueue& q);
// Forward then backward solve of every subdomain in one launch (x kept in
// LDS between the two passes); the same arithmetic as the two launches.
template <typename T>
void launch_trsv_fb(hipStream_t s, int nb, const T* L, const int64_t* Loff, const int* n,
                 T* x, const int64_t* xoff, int maxn, const WorkQueue& q);

// Deluxe objects (faces and edges), one workgroup per object.
struct ObjDesc {
    int nobj;
    const int* n;          // dofs of the object (2 per node)
    const int64_t* node_off;
    const int* nodes;      // global node ids
    const int64_t* fac_off;// factor of sum_m S^(m) (n x n)
    const int* sh_ptr;     // shares (CSR over objects)
    const int* sh_sub;     // sharing subdomain
    const int* sh_roff;    // offset of the object in that subdomain's r-dofs
    const int64_t* sh_slot;// that subdomain's block S^(m) (n x n)
    int maxn = 0;          // largest object (dofs): sizes the LDS of the deluxe applies
};
// Deluxe setup of the objects [ob0, ob0 + nob): E_m = S^(m) (sum S)^{-1}
// into dmat; maxn bounds their sizes (at most deluxe_max_object()) and sets
// the LDS each workgroup reserves, so faces and edges are launched
// separately; fac is the per-object workspace for objects too large for LDS.
template <typename T>
void launch_deluxe_setup(hipStream_t s, const ObjDesc& o, int ob0, int nob, int maxn, const T* slots, T* fac,
                         T* dmat, int* info);
int deluxe_max_object();

}  // namespace bdm
