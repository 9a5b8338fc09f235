// FP64 coarse problem of BDDC / FETI-DP: multifrontal Cholesky of the
// assembled primal matrix S_PiPi in a nested-dissection order of the
// subdomain grid (see coarse.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "topology.hpp"

namespace bdm {

struct CoarseSolver {
    // ---- symbolic structure (host), fronts numbered height by height
    int np = 0, pin = 0, nfront = 0, H = 0, maxp = 0;
    std::vector<int> hptr;                       // fronts of height h: [hptr[h], hptr[h+1])
    std::vector<int> ne, m, ld, parent;          // per front: eliminated dofs, dofs, rows (m + ne)
    std::vector<int64_t> foff, zoff, pmoff;      // matrix, vector and parent-map offsets
    std::vector<int> vars, pmap;                 // front dofs (eliminated first); child boundary -> parent position
    std::vector<std::vector<int>> kids[2];       // per height: children of its fronts, by child slot
    std::vector<int> maxne, maxm, maxnb, schur_tiles;
    std::vector<std::vector<int>> trail_tiles, panel_rows;
    std::vector<int> sub_pos;                    // subdomain s, local primal a -> position in its leaf front (-1: pin)
    std::vector<int> sub_front;                  // subdomain -> leaf front
    int pin_front = -1, pin_pos = -1;
    int64_t nF = 0, nZ = 0;
    int maxnf = 0;

    // ---- device
    double *F = nullptr, *z = nullptr, *z2 = nullptr, *Wbuf = nullptr;
    int* info = nullptr;       // [0]: any failure; [1..]: per-front flags of the height being factored
    int64_t *d_foff = nullptr, *d_zoff = nullptr, *d_pmoff = nullptr;
    int *d_ne = nullptr, *d_m = nullptr, *d_ld = nullptr, *d_parent = nullptr, *d_vars = nullptr, *d_pmap = nullptr;
    int *d_sub_pos = nullptr, *d_sub_front = nullptr;
    std::vector<int*> d_kids[2];

    // Nested dissection of the subdomain grid of topo; primal dof p belongs to
    // object p / 2.  maxp bounds the primal dofs per subdomain.  Returns an
    // empty string on success.
    std::string init(const Topology& topo, int pin, int maxp);
    // Device buffers, through alloc(ctx, bytes) (nullptr on failure).
    std::string alloc(void* (*alloc_fn)(void*, size_t), void* ctx, hipStream_t s);
    // Assemble the subdomain blocks Sp (nP x nP, stride sp_stride) colour by
    // colour, then factor; info[0] != 0 on a non-positive pivot.
    void factor(hipStream_t s, const int* color_list, const std::vector<int>& color_ptr, const int* nPv,
                const double* Sp, int sp_stride);
    // b <- S_PiPi^{-1} b (global primal numbering; b already projected)
    void solve(hipStream_t s, double* b);
    int64_t factor_bytes() const { return nF * (int64_t)sizeof(double); }
};

}  // namespace bdm
