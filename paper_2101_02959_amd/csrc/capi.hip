// extern "C" entry points of libbidomain (declared in include/bidomain.h).
// No C++ exception crosses this boundary.
#include <cstring>
#include <exception>
#include <new>

#include "solver.hpp"

namespace bdm {
const char* last_error();
}

struct bdm_ctx {
    bdm::Context c;
};

#define GUARD(expr)                                   \
    try {                                             \
        return (expr);                                \
    } catch (const std::bad_alloc&) {                 \
        bdm::set_error("host allocation failed");     \
        return BDM_E_OOM;                             \
    } catch (const std::exception& e) {               \
        bdm::set_error(e.what());                     \
        return BDM_E_ARG;                             \
    } catch (...) {                                   \
        bdm::set_error("unknown error");              \
        return BDM_E_ARG;                             \
    }

#define NEED(p)                                                   \
    if (!(p)) {                                                   \
        bdm::set_error("null argument: " #p);                     \
        return BDM_E_ARG;                                         \
    }

extern "C" {

int bdm_create(const bdm_mesh* mesh, const bdm_physics* phys, const bdm_opts* opts, void* hip_stream,
               bdm_ctx** out) {
    NEED(mesh); NEED(phys); NEED(opts); NEED(out);
    NEED(mesh->cuts_x); NEED(mesh->cuts_y); NEED(mesh->cuts_z);
    *out = nullptr;
    try {
        bdm_ctx* c = new bdm_ctx();
        int rc = c->c.create(mesh, phys, opts, (hipStream_t)hip_stream);
        if (rc) {
            delete c;
            return rc;
        }
        *out = c;
        return 0;
    } catch (const std::bad_alloc&) {
        bdm::set_error("host allocation failed");
        return BDM_E_OOM;
    } catch (const std::exception& e) {
        bdm::set_error(e.what());
        return BDM_E_ARG;
    }
}

int bdm_destroy(bdm_ctx* ctx) {
    NEED(ctx);
    delete ctx;
    return 0;
}

int bdm_set_state(bdm_ctx* ctx, const double* v, const double* ue, const double* w, double t, int on_device) {
    NEED(ctx);
    GUARD(ctx->c.set_state(v, ue, w, t, on_device != 0));
}

int bdm_get_state(bdm_ctx* ctx, double* v, double* ue, double* w, double* t, int on_device) {
    NEED(ctx);
    GUARD(ctx->c.get_state(v, ue, w, t, on_device != 0));
}

int bdm_set_stimulus(bdm_ctx* ctx, const double* Is, int step_on, int step_off, int on_device) {
    NEED(ctx);
    GUARD(ctx->c.set_stimulus(Is, step_on, step_off, on_device != 0));
}

int bdm_ionic_update(bdm_ctx* ctx) {
    NEED(ctx);
    GUARD(ctx->c.ionic_update());
}

int bdm_residual(bdm_ctx* ctx, const double* v, const double* ue, double* Rv, double* Re) {
    NEED(ctx); NEED(v); NEED(ue); NEED(Rv); NEED(Re);
    GUARD(ctx->c.residual(v, ue, Rv, Re));
}

int bdm_linearize(bdm_ctx* ctx, const double* v_lin, const double* w_lin) {
    NEED(ctx); NEED(v_lin); NEED(w_lin);
    GUARD(ctx->c.linearize(v_lin, w_lin));
}

int bdm_jacobian_apply(bdm_ctx* ctx, const double* x, double* y) {
    NEED(ctx); NEED(x); NEED(y);
    GUARD(ctx->c.jacobian_apply(x, y));
}

int bdm_bddc_apply(bdm_ctx* ctx, const double* r, double* z) {
    NEED(ctx); NEED(r); NEED(z);
    GUARD(ctx->c.bddc_apply(r, z));
}

int bdm_fetidp_size(bdm_ctx* ctx, long* n_lambda) {
    NEED(ctx); NEED(n_lambda);
    *n_lambda = ctx->c.n_lambda();
    return 0;
}

int bdm_fetidp_apply(bdm_ctx* ctx, int op, const double* in, double* out) {
    NEED(ctx); NEED(in); NEED(out);
    GUARD(ctx->c.fetidp_apply(op, in, out));
}

int bdm_step(bdm_ctx* ctx, int nsteps, bdm_step_stats* stats) {
    NEED(ctx);
    if (nsteps < 0) {
        bdm::set_error("nsteps < 0");
        return BDM_E_ARG;
    }
    GUARD(ctx->c.step(nsteps, stats));
}

int bdm_profile_kernel(bdm_ctx* ctx, int kernel, int reps, double* avg_ms, double* work) {
    NEED(ctx); NEED(avg_ms); NEED(work);
    GUARD(ctx->c.profile_kernel(kernel, reps, avg_ms, work));
}

int bdm_tune_report(bdm_ctx* ctx, char* buf, long cap, long* len) {
    NEED(ctx); NEED(len);
    try {
        const std::string r = ctx->c.tune_report();
        *len = (long)r.size();
        if (!buf || cap <= (long)r.size()) {
            bdm::set_error("bdm_tune_report: buffer too small");
            return BDM_E_ARG;
        }
        std::memcpy(buf, r.c_str(), r.size() + 1);
        return BDM_OK;
    } catch (...) {
        bdm::set_error("host allocation failed");
        return BDM_E_OOM;
    }
}

long bdm_predictor_size(void) { return bdm::Predictor::n_params(); }

int bdm_predictor_set(bdm_ctx* ctx, const float* params, const double* scales) {
    NEED(ctx); NEED(params); NEED(scales);
    GUARD(ctx->c.predictor_set(params, scales));
}

int bdm_predictor_get(bdm_ctx* ctx, float* params, double* scales) {
    NEED(ctx); NEED(params); NEED(scales);
    GUARD(ctx->c.predictor_get(params, scales));
}

int bdm_predictor_guess(bdm_ctx* ctx, const double* vn, const double* uen, const double* vprev, const double* ueprev,
                        double* guess) {
    NEED(ctx); NEED(vn); NEED(uen); NEED(vprev); NEED(ueprev); NEED(guess);
    GUARD(ctx->c.predictor_guess(vn, uen, vprev, ueprev, guess));
}

int bdm_predictor_loss_grad(bdm_ctx* ctx, const double* sample, float* grad, double* loss) {
    NEED(ctx); NEED(sample); NEED(grad); NEED(loss);
    GUARD(ctx->c.predictor_loss_grad(sample, grad, loss));
}

int bdm_predictor_train(bdm_ctx* ctx, const double* samples, int nsamples, const int* order, int nsteps, double lr,
                        double* losses) {
    NEED(ctx); NEED(samples); NEED(order);
    if (nsamples <= 0 || nsteps < 0 || !(lr > 0)) {
        bdm::set_error("bdm_predictor_train: nsamples > 0, nsteps >= 0 and lr > 0 required");
        return BDM_E_ARG;
    }
    GUARD(ctx->c.predictor_train(samples, nsamples, order, nsteps, lr, losses));
}

int bdm_sizes(bdm_ctx* ctx, long* n_nodes, long* n_sub, long* n_primal) {
    NEED(ctx);
    if (n_nodes) *n_nodes = (long)ctx->c.N;
    if (n_sub) *n_sub = (long)ctx->c.topo.subs.size();
    if (n_primal) *n_primal = (long)ctx->c.topo.nprimal;
    return 0;
}

const char* bdm_last_error(void) { return bdm::last_error(); }

}  // extern "C"
