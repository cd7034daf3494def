// Solver entry points shared by the C-ABI layer and the HIP translation unit.
#pragma once

#include <cstddef>
#include <cstdint>

#include "bddmp.h"

namespace bddmp {

struct Plan;
struct Solver;

int32_t solver_bind(const Plan &P, void *arena, size_t bytes, void *stream, Solver *&out);
int32_t solver_reset(Solver &S);
int32_t solver_iterate(Solver &S, int32_t n);
int32_t solver_iterate_until(Solver &S, int32_t max_iters, double rel, int32_t every, int32_t *done, int32_t *at,
                             double *lb);
int32_t solver_lower_bound(Solver &S, double *lb, double *residual, double *any_lambda_bound);
int32_t solver_instance_bounds(Solver &S, double *lb_host, int32_t n);
int32_t solver_lb_history(Solver &S, double *out, int32_t cap, int32_t *n_out);
int32_t solver_min_marginals(Solver &S, float *m0, float *m1);
int32_t solver_get_lambda(Solver &S, float *lam);
int32_t solver_set_lambda(Solver &S, const float *lam);
int32_t solver_copy_duals(Solver &S, bool out, float *mu_bar, float *mu, float *dfw, float *dbw);
int32_t solver_round_primal(Solver &S, float *M_dev, int8_t *x_host, double *obj, int64_t *nviol);
int32_t solver_set_graphs(Solver &S, int32_t enable);
int32_t solver_set_launch(Solver &S, int32_t mode, int32_t chunk);
int32_t solver_get_launch(const Solver &S, int32_t *mode, int32_t *chunk);
int32_t solver_set_groups(Solver &S, const int32_t *lanes);
int32_t solver_get_groups(const Solver &S, int32_t *lanes);
int32_t solver_autotune(Solver &S, int32_t iters, int32_t *lanes);
int32_t solver_time_kernels(Solver &S, int32_t n, bddmp_kernel_times *out);
int32_t solver_smooth_workspace(const Plan &P, int32_t T, size_t *bytes);
int32_t solver_smooth_run(Solver &S, float alpha, int32_t T, void *ws, size_t bytes);
int32_t solver_smooth_grad(Solver &S, float alpha, int32_t T, void *ws, size_t bytes, double dlb, float *grad);
int32_t solver_set_costs(Solver &S, const double *cost_dev);
// bytes of the static scratch that solver_smooth_grad_noalloc uses as its workspace
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
int32_t solver_smooth_grad_noalloc(Solver &S, float alpha, int32_t T, double dlb, float *grad);
void solver_destroy(Solver *S);

}  // namespace bddmp
