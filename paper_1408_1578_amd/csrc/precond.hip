// placeholder, replaced below
#include "dp_internal.hpp"
namespace dp {
struct Precond {};
int precond_build(dp_problem* p, const dp_precond_opts* o) { set_error("not built"); return DP_ESTATE; }
int precond_apply(dp_problem* p, int nrhs, const cplx* v, cplx* z) { set_error("not built"); return DP_ESTATE; }
void precond_destroy(Precond* pc) { delete pc; }
int precond_info(dp_problem* p, dp_precond_info* info) { return DP_ESTATE; }
int precond_export(dp_problem* p, int64_t* a, int64_t* b, int64_t* c, double* d) { return DP_ESTATE; }
}
