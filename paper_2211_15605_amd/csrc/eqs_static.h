// eqs_static.h -- FP64 solve of one set on a workspace lent by the caller (no allocation).
#pragma once

#include <stddef.h>

#include "eqsolve.h"

namespace eqs {

// Bytes of workspace static_solve needs for grid g (0 if the grid's rows are too wide).
size_t static_solve_bytes(const eqs_grid &g);

// The FP64 solve of eqsolve_solve on workspace ws (cap bytes, 256-byte aligned, device memory
// of `device`): its set table and state block are the first two 256-byte-aligned slots, the
// vectors follow.  The whole part a call uses is cleared by a fill kernel first.  Returns the
// EQS_* code (EQS_ERR_SIZE if the grid needs more than cap bytes).
int static_solve(void *ws, size_t cap, int device, const eqs_grid &g, const double *const diag[7], const double *b,
                 double *x, double tol, int32_t maxit, eqs_info *info, void *hip_stream);

}  // namespace eqs
