// Poisson solve (placeholder until the solver lands).
#include "dgwm_internal.h"

using namespace dgwm;

extern "C" {

int64_t dg_solve_workspace_bytes(const dg_mesh* m, const dg_solve_params* sp) {
  (void)m;
  (void)sp;
  return set_error(DG_ERR_UNSUPPORTED, "solver not built");
}

int dg_solve_poisson(const dg_mesh* m, const dg_solve_params* sp, const double* b, double* x, void* ws,
                     size_t ws_bytes, dg_solve_stats* st, void* stream) {
  (void)m; (void)sp; (void)b; (void)x; (void)ws; (void)ws_bytes; (void)st; (void)stream;
  return set_error(DG_ERR_UNSUPPORTED, "solver not built");
}
}
