// Philox4x32-10 Gaussian start vectors for the multigrid setup.
#pragma once

#include "wcmg_internal.h"

namespace wcmg {
// full-lattice FP64 spinor (internal layout, both parities)
void random_fine_vector(void* out, uint64_t seed, int vec, int level, const Geom& g, hipStream_t st);
// coarse FP64 vector [internal site][n], perm: device array lex -> internal
void random_coarse_vector(void* out, uint64_t seed, int vec, int level, const int* perm, int V, int n,
                          hipStream_t st);
}  // namespace wcmg
