// Solver context: topology, device workspace and the host-side control of
// the Newton-Krylov BDDC / FETI-DP deluxe iteration.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/bidomain.h"
#include "bddc_kernels.hpp"
#include "coarse.hpp"
#include "learned.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "topology.hpp"
#include "tune.hpp"

namespace bdm {

struct KrylovOut {
    int its = 0;
    int status = 0;            // 0 converged, 1 maxit, 2 diverged
    std::vector<double> alpha, beta, hist;
    double cond = 1.0;
};

class Context {
  public:
    Context() = default;
    ~Context();
    int create(const bdm_mesh* m, const bdm_physics* ph, const bdm_opts* o, hipStream_t s);

    int set_state(const double* v, const double* ue, const double* w, double t, bool dev);
    int get_state(double* v, double* ue, double* w, double* t, bool dev);
    int set_stimulus(const double* Is, int on, int off, bool dev);
    int ionic_update();
    int residual(const double* v, const double* ue, double* Rv, double* Re);
    int linearize(const double* v, const double* w);
    int jacobian_apply(const double* x, double* y);
    int bddc_apply(const double* r, double* z);
    int fetidp_apply(int op, const double* in, double* out);
    int step(int nsteps, bdm_step_stats* st);
    int profile_kernel(int kernel, int reps, double* avg_ms, double* work);
    // A right-looking elimination over the columns [0, ne) of a view of each
    // local matrix (offset off, leading dimension the matrix size, n rows),
    // with launch sizes per 128-column panel and, when schur > 0, the Schur
    // update of the trailing block [ne, n)^2.
    struct ElimPlan {
        const int64_t* off = nullptr;
        const int* ne = nullptr;
        const int* n = nullptr;
        const int* nIc = nullptr;           // core columns (interior plan), see launch_syrk_update
        std::vector<int> trail, rows;
        int schur = 0;
        int variant = 0;        // rank-k kernel variant (autotuned)
        void* packed = nullptr;             // panel-packed copy of the factor (element type T)
        const int64_t* poff = nullptr;      // its per-subdomain offsets
    };
    ElimPlan plan_int_, plan_rr_;
    void build_plan(ElimPlan& pl, bool interior, int variant);
    // autotuner: stencil tile shape at creation, rank-k variants of the two
    // elimination plans at the first linearisation (timed on the first chunk)
    Tuner tuner_;
    std::string tune_path_;
    bool syrk_tuned_ = false;
    int tune_stencil();
    template <typename T>
    int tune_syrk();
    int save_tuning();
    std::string tune_report() const { return tuner_.report(); }
    template <typename T>
    int eliminate(T* K, int s0, int cnt, const ElimPlan& pl, double* tm);
    int predictor_set(const float* params, const double* scales);
    int predictor_get(float* params, double* scales);
    int predictor_guess(const double* vn, const double* uen, const double* vp, const double* uep, double* out);
    int predictor_loss_grad(const double* sample, float* grad, double* loss);
    int predictor_train(const double* samples, int nsamples, const int* order, int nsteps, double lr,
                        double* losses);
    long n_lambda() const { return nlam_; }

    Topology topo;
    FEParams fp{};
    bdm_opts opts{};
    bdm_physics phys{};
    int64_t N = 0;

  private:
    template <typename T> int alloc_local();
    template <typename T> int profile_t(int kernel, int reps, double* avg_ms, double* work);
    template <typename T> int linearize_t();
    template <typename T> void dirichlet(const double* r, const double* q, double* out);
    template <typename T> void condense(const double* r, double* g);
    template <typename T> void stilde_inv(T* xr, const double* gvert, double* uc);
    template <typename T> void interior_extend(const double* r, double* zbuf);
    template <typename T> int bddc_apply_t(const double* r, double* z, bool interior_free = false);
    template <typename T> int fetidp_apply_t(int op, const double* in, double* out);
    int pcg(int n, const double* b, double* x, bool feti, KrylovOut& out, bool reduced = false, double rref = 0.0);
    int krylov(int n, const double* b, double* x, bool feti, KrylovOut& out, bool reduced = false, double rref = 0.0);
    int newton_solve(const double* b, double* s, KrylovOut& out);
    int sync();
    double dot(int64_t n, const double* x, const double* y);
    void* dalloc(size_t bytes);
    template <typename V> V* upload(const std::vector<V>& h);

    hipStream_t stream_ = nullptr;
    std::vector<void*> allocs_;
    bool linearized_ = false;
    int prec_ = 0;
    size_t tsize_ = 8;

    // fe
    double *st_ = nullptr, *ke_ = nullptr;
    double *v_ = nullptr, *ue_ = nullptr, *w_ = nullptr, *vn_ = nullptr;
    double *vprev_ = nullptr, *ueprev_ = nullptr, *Is_ = nullptr;
    double *dg_ = nullptr, *vlin_ = nullptr, *wlin_ = nullptr;
    int* bad_ = nullptr;
    int stim_on_ = 0, stim_off_ = 0, nstep_ = 0;
    bool have_prev_ = false, have_stim_ = false;
    double t_ = 0.0;

    // batched local storage (element type per precision)
    void *K_ = nullptr, *slots_ = nullptr, *F_ = nullptr, *Z_ = nullptr;
    // second setup workspace (when the device has room): the next chunk is
    // cleared and assembled into it on the side stream while the current
    // chunk is eliminated
    void* K2_ = nullptr;
    bool setup_overlap_ = true;
    void *fac_ = nullptr, *Srr_ = nullptr, *xI_ = nullptr, *xr_ = nullptr, *xr2_ = nullptr;
    double *Svv_ = nullptr, *Sp_ = nullptr, *cP_ = nullptr, *mu_ = nullptr;
    double *cb_ = nullptr, *ybuf_ = nullptr;
    void *LIIs_ = nullptr, *Lrrs_ = nullptr;   // compact Dirichlet / Neumann factors
    void *inv_ = nullptr, *dmat_ = nullptr;    // deluxe (sum S)^{-1} and E_m = S^(m) (sum S)^{-1}
    void* dmatT_ = nullptr;                    // E_m^T (value side of the scaling)
    CoarseSolver coarse_;
    Predictor pred_;
    int ensure_predictor();
    std::vector<std::pair<int, int>> chunks_;  // subdomain ranges of the chunked setup
    const int64_t* Kc_off_ = nullptr;           // chunk-relative offsets of the local matrices
    int64_t nKwork_ = 0, nLII_ = 0, nLrr_ = 0;
    int *info_sub_ = nullptr, *info_obj_ = nullptr, *info_c_ = nullptr;

    // descriptors (device arrays) and host copies of sizes
    BatchDesc bd_{};
    ObjDesc od_{};
    SubVecDesc sv_{};
    CoarseDesc cd_{};
    FetiDesc fd_{};
    int maxbox_ = 0, maxG_ = 0, maxnI_ = 0, maxnr_ = 0, maxobjn_ = 0, nInodes_ = 0;
    int nface_obj_ = 0, maxface_n_ = 0, maxedge_n_ = 0;   // objects: faces [0, nface_obj_), then edges
    double* rho_w_ = nullptr;   // rho scaling weights per share: (v, u_e)
    bool fused_dirichlet_ = true;   // forward and backward Dirichlet solves in one launch
    int maxn_ = 0;                                         // largest local matrix (n = nI + nGamma)
    void* Wbuf_ = nullptr;
    int *Ilist_ = nullptr;
    int64_t *LII_off_ = nullptr, *Lrr_off_ = nullptr, *xI_off_ = nullptr, *xr_off_ = nullptr;
    const int64_t *Srr_off_ = nullptr;
    const int *nI_ = nullptr, *nr_ = nullptr, *ld_ = nullptr, *kF_ = nullptr, *nP_ = nullptr;
    int *st1c0_ = nullptr, *st1c1_ = nullptr, *st1c2_ = nullptr, *st2c1_ = nullptr;
    std::vector<std::vector<int>> colors_;   // subdomains per colour (disjoint primal sets)
    int *color_list_ = nullptr;
    std::vector<int> color_ptr_;
    int *cpin_ = nullptr;
    int64_t *zero64_ = nullptr;
    int *one_ = nullptr, *np_ = nullptr;
    int64_t nK_ = 0, nslot_ = 0, nF_ = 0, nZ_ = 0, nfac_ = 0, nSrr_ = 0, nxI_ = 0, nxr_ = 0, nyb_ = 0;
    int pin_ = 1;
    long nlam_ = 0;

    // Krylov / Newton workspace (2N or n_lambda doubles)
    double *kx_ = nullptr, *kr_ = nullptr, *kz_ = nullptr, *kp_ = nullptr, *kq_ = nullptr;
    double *t1_ = nullptr, *t2_ = nullptr, *t3_ = nullptr, *gzero_ = nullptr;
    double *R_ = nullptr, *S_ = nullptr, *U_ = nullptr, *Rt_ = nullptr;
    double *part_ = nullptr, *scal_ = nullptr;
    unsigned* tick_ = nullptr;   // reduction tickets (vec.hip), zero between launches
    bool hip_err_ = false;       // a host read-back of a reduction failed
    // PCG: device scalars and histories, the cached graphs
    double *kry_sc_ = nullptr, *kry_hist_ = nullptr, *kry_ah_ = nullptr, *kry_bh_ = nullptr;
    int kry_hcap_ = 0, kry_key_ = -1;
    double* kry_x_ = nullptr;
    hipGraphExec_t kry_exec_[2] = {nullptr, nullptr};   // operator half, preconditioner half
    // persistent LPT work queues of the Dirichlet and Neumann triangular solves
    int* qctr_ = nullptr;
    WorkQueue qI_, qr_;
    hipStream_t kry_stream_ = nullptr;
    // side stream of the setup: the deluxe factors run on it concurrently
    // with the coarse chain (forward solves, local products, factorization)
    hipStream_t side_stream_ = nullptr;
    hipEvent_t ev_fork_ = nullptr, ev_join_ = nullptr;
    hipEvent_t ev_free_ = nullptr, ev_ready_ = nullptr;   // workspace hand-over between the streams
    int side_stream_init();
};

void set_error(const std::string& msg);

}  // namespace bdm
