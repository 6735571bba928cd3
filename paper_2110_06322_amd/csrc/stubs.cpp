// Entry points not implemented yet: they fail with CPM_ERR_STATE.
#include "internal.h"
using namespace cpm;
static cpm_status ni(const char* f) { set_error(std::string(f) + " is not implemented yet"); return CPM_ERR_STATE; }
cpm_status cpm_precond_create(const cpm_operator*, const cpm_precond_opts*, cpm_precond**) { return ni("cpm_precond_create"); }
cpm_status cpm_precond_get_info(const cpm_precond*, cpm_precond_info*) { return ni("cpm_precond_get_info"); }
cpm_status cpm_precond_export_partition(const cpm_precond*, int32_t*, int64_t*, int32_t*) { return ni("export"); }
cpm_status cpm_precond_apply(const cpm_precond*, const double*, double*, int32_t, void*) { return ni("cpm_precond_apply"); }
void cpm_precond_destroy(cpm_precond*) {}
cpm_status cpm_solve_opts_default(cpm_solve_opts*) { return ni("opts"); }
cpm_status cpm_precond_opts_default(cpm_precond_opts*) { return ni("opts"); }
cpm_status cpm_solve(const cpm_operator*, const cpm_precond*, const double*, double*, int32_t, const cpm_solve_opts*, cpm_solve_stats*, void*) { return ni("cpm_solve"); }
cpm_status cpm_batch_create(int32_t, const cpm_operator* const*, const cpm_precond* const*, const int32_t*, cpm_batch**) { return ni("batch"); }
cpm_status cpm_batch_solve(cpm_batch*, const double* const*, double* const*, const cpm_solve_opts*, cpm_solve_stats*, void*) { return ni("batch"); }
cpm_status cpm_batch_apply(cpm_batch*, const double* const*, double* const*, void*) { return ni("batch"); }
void cpm_batch_destroy(cpm_batch*) {}
