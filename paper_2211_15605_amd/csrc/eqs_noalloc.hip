// eqs_noalloc.hip -- eqsolve_solve_noalloc: the FP64 solve on a static device array.
//
// For callers that cannot allocate.  The workspace every kernel of the solve
// uses (Krylov vectors, scaled coefficients, reduction partials, the ticket
// counter, the set table and the state block) lives in `scratch`, a static
// device array of EQS_NOALLOC_BYTES bytes, one instance per GPU.  Host code
// never passes the array's name to a kernel or a copy: on the first call on a
// device its device address is taken with hipGetSymbolAddress (with that
// device current) and kept per device, and only that address is used.

#include <hip/hip_runtime.h>

#include "eqs_static.h"
#include "eqsolve.h"

namespace {

constexpr size_t kScratchBytes = EQS_NOALLOC_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kDevices = 64;
void *g_scratch_ptr[kDevices];  // device address of `scratch` on each device, once taken

bool diag_args_ok(const double *const diag[7], const double *b, const double *x) {
    if (!diag || !b || !x) return false;
    for (int k = 0; k < 7; ++k)
        if (!diag[k] || (const void *)diag[k] == (const void *)x) return false;
    return (const void *)b != (const void *)x;
}

}  // namespace

extern "C" int eqsolve_solve_noalloc(const eqs_grid *grid, const double *const diag[7], const double *b, double *x,
                                     double tol, int32_t maxit, eqs_info *info, void *hip_stream) {
    if (!grid || !diag_args_ok(diag, b, x)) return EQS_ERR_ARG;
    if (!(tol > 0.0 && tol < 1.0) || maxit < 1) return EQS_ERR_ARG;
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || grid->nx > 1024) return EQS_ERR_ARG;
    const long long n = (long long)grid->nx * grid->ny * grid->nz;
    if (n > EQS_NOALLOC_MAX_CELLS) return EQS_ERR_SIZE;
    const size_t need = eqs::static_solve_bytes(*grid);
    if (need == 0) return EQS_ERR_ARG;
    if (need > kScratchBytes) return EQS_ERR_SIZE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return EQS_ERR_HIP;
    }
    if (dev < 0 || dev >= kDevices) return EQS_ERR_STATE;
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return EQS_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    return eqs::static_solve(g_scratch_ptr[dev], kScratchBytes, dev, *grid, diag, b, x, tol, maxit, info, hip_stream);
}
