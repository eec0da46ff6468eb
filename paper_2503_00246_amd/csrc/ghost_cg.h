// Conjugate-gradient driver on (M + G) x = b over the active lattice nodes.
#pragma once

#include <hip/hip_runtime_api.h>

#include "ghost.h"
#include "ghost_device.h"

namespace ghost {

struct CgWork;
void cg_free(CgWork *w);
int cg_solve(ghost_ctx *ctx, const double *b, double *x, const ghost_cg_opts &opts, ghost_cg_result &res,
             hipStream_t s);

// Accessors into the context (defined with the C ABI).
int set_error(int code, const char *msg);
const DevPlan &dev_plan(const ghost_ctx *c);
const Plan &host_plan(const ghost_ctx *c);
CgWork *&cg_slot(ghost_ctx *c);
int ctx_device(const ghost_ctx *c);

}  // namespace ghost
