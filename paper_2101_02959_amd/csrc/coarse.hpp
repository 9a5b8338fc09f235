// FP64 block-tridiagonal coarse solver (see coarse.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace bdm {

struct CoarseMap {
    int pin;
    const int* grp;         // primal -> group
    const int* pos;         // primal -> position in its group
    const int64_t* D_off;   // group -> start of its diagonal block
    const int64_t* E_off;   // group -> start of its sub-diagonal block (rows g, cols g-1)
    const int* ng;          // group sizes
};

void gemm(hipStream_t s, int m, int n, int k, double alpha, const double* A, int64_t lda, bool ta,
          const double* B, int64_t ldb, bool tb, double beta, double* C, int64_t ldc);
// part: workspace of m * ceil(n / 128) doubles (non-transposed case)
void gemv(hipStream_t s, int m, int n, double alpha, const double* A, int64_t lda, bool ta, const double* x,
          double beta, double* y, double* part);
constexpr int kCoarseSweepBlock = 64;
void spd_inverse(hipStream_t s, int n, double* A, int64_t lda, double* Bwork, double* Twork, double* Rwork,
                 int* info);

struct CoarseSolver {
    int np = 0, pin = 0, G = 0, maxn = 0;
    std::vector<int> grp, pos, ng;
    std::vector<int64_t> D_off, E_off, goff;
    int64_t nD = 0, nE = 0;
    // device
    double *D = nullptr, *E = nullptr, *Cb = nullptr, *yb = nullptr, *zb = nullptr;
    double *Bw = nullptr, *Tw = nullptr, *Rw = nullptr, *Pw = nullptr;
    int *d_grp = nullptr, *d_pos = nullptr, *d_ng = nullptr, *info = nullptr;
    int64_t *d_Doff = nullptr, *d_Eoff = nullptr, *d_goff = nullptr;

    std::string init(const std::vector<int>& grp_of, int pin, int np);
    CoarseMap map() const { return CoarseMap{pin, d_grp, d_pos, d_Doff, d_Eoff, d_ng}; }
    // assemble (colour by colour), factor
    void factor(hipStream_t s, const int* color_list, const std::vector<int>& color_ptr, const int* nPv,
                const int64_t* P_off, const int* primal, const double* Sp, int sp_stride);
    // x = S_PiPi^{-1} b in place (global primal numbering), b already projected
    void solve(hipStream_t s, double* b);
};

}  // namespace bdm
