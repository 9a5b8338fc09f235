// Device scalar slots of the PCG iteration (vec.hip, solver.hip).
#pragma once

namespace bdm {

enum PcgSlot {
    PCG_RZ = 0,      // z . r of the current iterate
    PCG_PQ,          // p . q
    PCG_ALPHA,
    PCG_RN2,         // r . r after the update
    PCG_ZR,          // z_new . r_new
    PCG_ZQ,          // z_new . q
    PCG_BETA,
    PCG_STATE,       // PCG_RUNNING, PCG_CONVERGED, PCG_DIVERGED, PCG_MAXIT
    PCG_IT,          // completed iterations
    PCG_TOL,         // rtol * ||r_0||
    PCG_DTOL,        // dtol * ||r_0||
    PCG_NSLOT
};
constexpr double PCG_RUNNING = 0.0, PCG_CONVERGED = 1.0, PCG_DIVERGED = 2.0, PCG_MAXIT = 3.0;

}  // namespace bdm
