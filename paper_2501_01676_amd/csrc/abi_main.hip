// Placeholder entry points (replaced by the full context implementation).
#include "internal.h"
extern "C" {
int abddc_assemble(const abddc_problem*, const abddc_device*, abddc_ctx**) { return ABDDC_ESTATE; }
int abddc_setup_coarse_space(abddc_ctx*, const abddc_options*, abddc_counts*) { return ABDDC_ESTATE; }
int abddc_apply_bddc(abddc_ctx*, const double*, double*) { return ABDDC_ESTATE; }
int abddc_apply_schur(abddc_ctx*, const double*, double*) { return ABDDC_ESTATE; }
int abddc_get_rhs(abddc_ctx*, double*) { return ABDDC_ESTATE; }
int abddc_gmres_solve(abddc_ctx*, int32_t, double, int32_t, double*, abddc_solve_info*) { return ABDDC_ESTATE; }
int abddc_query(const abddc_ctx*, int64_t*, int64_t*, int32_t*, int32_t*, int32_t*) { return ABDDC_ESTATE; }
int64_t abddc_get_stage(abddc_ctx*, int32_t, int32_t, double*, int64_t) { return ABDDC_ESTATE; }
int abddc_phase_times(const abddc_ctx*, double*, int32_t) { return ABDDC_ESTATE; }
void abddc_destroy(abddc_ctx*) {}
}
