// bdm_residual_noalloc: the Step-2 residual of bdm_residual without a
// context and without any device allocation, for callers that cannot
// allocate (declared in include/bidomain.h).
//
// The residual's kernels read one device buffer besides their inputs and
// outputs: the tau-scaled 27-point coefficient tables, (nz + 1) levels of
// 9 boundary classes x 2 media x 27 coefficients.  A context allocates them
// at bdm_create; here they live in the file-scope array `scratch` below,
// sized for nz + 1 <= NA_MAX_LEVELS (about 4 MB per GPU, held until the
// process ends).  The host builds the tables into a static host buffer and
// copies them into that GPU's array.  Every call on one GPU rewrites the
// part it uses before the residual kernel reads it; a mutex serialises the
// host side and each call synchronises its stream before it releases the
// mutex, so calls from several threads do not interleave on the array.
// Work that other code enqueues itself on the same GPU while a call runs is
// not ordered against it.
#include <mutex>

#include "../../include/bidomain.h"
#include "common.hpp"
#include "kernels.hpp"

namespace bdm {
void set_error(const std::string& msg);
}

namespace {

constexpr int NA_MAX_LEVELS = 1024;          // nz + 1 levels of coefficients at most
constexpr int NA_LEVEL = 9 * 2 * 27;          // doubles per level
constexpr int NA_MAX_DEVICES = 64;

static __device__ __align__(256) double scratch[NA_MAX_LEVELS * NA_LEVEL];

std::mutex g_mu;
double g_ke[(NA_MAX_LEVELS - 1) * 128];        // element matrices per layer (host)
double g_st[NA_MAX_LEVELS * NA_LEVEL];         // coefficient tables (host)
double* g_scratch[NA_MAX_DEVICES] = {};        // device address of `scratch`, per device

}  // namespace

extern "C" int bdm_residual_noalloc(const bdm_mesh* mesh, const bdm_physics* ph, double dt, const double* v,
                                    const double* ue, const double* vn, const double* w, const double* Is,
                                    int stim_on, double* Rv, double* Re, void* hip_stream) {
    using bdm::set_error;
    if (!mesh || !ph || !v || !ue || !vn || !w || !Rv || !Re || (stim_on && !Is)) {
        set_error("bdm_residual_noalloc: null argument");
        return BDM_E_ARG;
    }
    if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1 || !(mesh->h > 0.0) || !(dt > 0.0)) {
        set_error("bdm_residual_noalloc: mesh sizes and h must be positive, dt positive");
        return BDM_E_ARG;
    }
    if (mesh->geometry != BDM_GEOM_BOX) {
        set_error("bdm_residual_noalloc: box meshes only (a mapped mesh needs per-node coefficient arrays)");
        return BDM_E_ARG;
    }
    if (mesh->nz + 1 > NA_MAX_LEVELS) {
        set_error("bdm_residual_noalloc: nz + 1 exceeds the " + std::to_string(NA_MAX_LEVELS) +
                  " coefficient levels of the static device buffer");
        return BDM_E_ARG;
    }
    const hipStream_t s = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lock(g_mu);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= NA_MAX_DEVICES)) {
        set_error("bdm_residual_noalloc: device index beyond the per-device table");
        return BDM_E_ARG;
    }
    if (e == hipSuccess && !g_scratch[dev]) {
        // first call on this device (the current one): the array's device address
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e == hipSuccess) g_scratch[dev] = (double*)ptr;
    }
    if (e != hipSuccess) {
        set_error(std::string("bdm_residual_noalloc: ") + hipGetErrorString(e));
        return BDM_E_HIP;
    }
    double* tab = g_scratch[dev];
    const int nz = mesh->nz;
    const double hd[3] = {mesh->h, mesh->hy > 0.0 ? mesh->hy : mesh->h, mesh->hz > 0.0 ? mesh->hz : mesh->h};
    bdm::layer_matrices_into(nz, hd, dt, ph->sigma_i, ph->sigma_e, ph->theta0, ph->theta1, g_ke);
    bdm::stencil_tables_into(nz, g_ke, g_st);
    bdm::FEParams p{};
    p.nx = mesh->nx; p.ny = mesh->ny; p.nz = nz;
    p.nx1 = mesh->nx + 1; p.ny1 = mesh->ny + 1;
    p.N = (int64_t)p.nx1 * p.ny1 * (nz + 1);
    p.h = hd[0]; p.hy = hd[1]; p.hz = hd[2]; p.tau = dt; p.c = ph->chi * ph->Cm;
    p.chiG = ph->chi * ph->G; p.chieta1 = ph->chi * ph->eta1; p.eta2 = ph->eta2;
    p.vth = ph->vth; p.vp = ph->vp;
    p.stencil_variant = 0;   // every variant takes the same sums in the same order
    e = hipMemcpyAsync(tab, g_st, (size_t)(nz + 1) * NA_LEVEL * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        bdm::launch_residual(s, p, tab, v, ue, vn, w, Is, stim_on ? 1.0 : 0.0, Rv, Re);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // g_st and the array are reused by the next call
    if (e != hipSuccess) {
        set_error(std::string("bdm_residual_noalloc: ") + hipGetErrorString(e));
        return BDM_E_HIP;
    }
    return 0;
}
