// Internal helpers shared by the translation units of the library (not part of the ABI).
#pragma once
#include "lbm.h"

// Record a thread-local error message (printf format) and return `code`.
lbm_status lbm_fail(lbm_status code, const char* fmt, ...);

// a_i alpha_i(T) of each component (Sec. 3.2), float64.
void lbm_internal_aalpha(const lbm_mixture* mix, double T, double* aa_out);
