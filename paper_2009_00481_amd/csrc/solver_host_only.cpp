// Solver entry points of the host-only test build (libbddmp_host*.so): the problem, plan, primal
// search and export calls of the C-ABI are the library's own, every call that needs the device
// fails with BDDMP_DEVICE. This build exists to run the host code (builder, planner, primal search,
// argument checks) under the CPU sanitizers; the product library is libbddmp.so.
#include <string>

#include "internal.h"
#include "solver.h"

namespace bddmp {

namespace {
int32_t no_device() { return set_error(BDDMP_DEVICE, "host-only test build: no device code"); }
}  // namespace

int32_t solver_bind(const Plan &, void *, size_t, void *, Solver *&out) {
  out = nullptr;
  return no_device();
}
int32_t solver_reset(Solver &) { return no_device(); }
int32_t solver_iterate(Solver &, int32_t) { return no_device(); }
int32_t solver_iterate_until(Solver &, int32_t, double, int32_t, int32_t *, int32_t *, double *) { return no_device(); }
int32_t solver_lower_bound(Solver &, double *, double *, double *) { return no_device(); }
int32_t solver_instance_bounds(Solver &, double *, int32_t) { return no_device(); }
int32_t solver_lb_history(Solver &, double *, int32_t, int32_t *) { return no_device(); }
int32_t solver_min_marginals(Solver &, float *, float *) { return no_device(); }
int32_t solver_get_lambda(Solver &, float *) { return no_device(); }
int32_t solver_set_lambda(Solver &, const float *) { return no_device(); }
int32_t solver_copy_duals(Solver &, bool, float *, float *, float *, float *) { return no_device(); }
int32_t solver_round_primal(Solver &, float *, int8_t *, double *, int64_t *) { return no_device(); }
int32_t solver_set_graphs(Solver &, int32_t) { return no_device(); }
int32_t solver_set_launch(Solver &, int32_t, int32_t) { return no_device(); }
int32_t solver_get_launch(const Solver &, int32_t *, int32_t *) { return no_device(); }
int32_t solver_set_groups(Solver &, const int32_t *) { return no_device(); }
int32_t solver_get_groups(const Solver &, int32_t *) { return no_device(); }
int32_t solver_autotune(Solver &, int32_t, int32_t *) { return no_device(); }
int32_t solver_time_kernels(Solver &, int32_t, bddmp_kernel_times *) { return no_device(); }
int32_t solver_smooth_workspace(const Plan &, int32_t, size_t *) { return no_device(); }
int32_t solver_smooth_run(Solver &, float, int32_t, void *, size_t) { return no_device(); }
int32_t solver_smooth_grad(Solver &, float, int32_t, void *, size_t, double, float *) { return no_device(); }
int32_t solver_smooth_grad_noalloc(Solver &, float, int32_t, double, float *) { return no_device(); }
int32_t solver_set_costs(Solver &, const double *) { return no_device(); }
void solver_destroy(Solver *) {}

}  // namespace bddmp
