// eqs_launch.h -- host-side launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>

#include "eqs_internal.h"

namespace eqs {

enum Kern {
    K_SETUP,    // r = b - A x, r^ = r, (b,b), (r,r), a_P check; initialises the state
    K_RECHECK,  // true residual after recursive convergence (restart if above tol)
    K_REPORT,   // true residual of the final iterate (no writes)
    K_K1,       // p update + Jacobi + product + (r^, v)
    K_K2,       // s + Jacobi + product + (t,s), (t,t), (s,s)
    K_K3,       // x and r updates + (r^, r), (r, r)
    K_CAST,     // FP64 -> FP32 coefficients, (b,b), a_P check (FP32 forms)
    K_OUTER,    // FP64 residual -> scaled FP32 inner right-hand side (FP32 forms)
    K_UPDATE,   // x += d / scale (FP32 forms)
    K_ZERO,     // x = 0 (b = 0, or forced)
    K_GRAD,     // adjoint gradients
    K_APPLY     // y = A x or A^T x
};

// LDS bytes of a march kernel (three plane buffers of Q + 2 nx values)
size_t march_lds_bytes(int cpt, int max_nx, int elem);

// halo cells per thread per plane (1, 2, 4 or 8), or -1 if nx is too wide
int halo_slots(int max_nx);

// Launch kernel k: march kernels over ntiles blocks (the sum of the sets'
// tile counts), pointwise kernels over nflat blocks (the sum of their nflat).
hipError_t launch_kernel(Kern k, const LaunchSets &ls, int ntiles, int nflat, int cpt, int max_nx, bool fp32,
                         bool trans, hipStream_t stream, const double *x, double *y, int arg);

}  // namespace eqs
