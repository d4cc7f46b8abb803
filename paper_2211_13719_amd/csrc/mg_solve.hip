// Placeholder translation unit for the multigrid solver state.
#include "mg_internal.h"

namespace mrhs {
void mg_solver_release(mrhs_mg) {}
}  // namespace mrhs
