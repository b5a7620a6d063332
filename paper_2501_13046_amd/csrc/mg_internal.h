// Solver functions used by the network runtime in the same library; not part
// of the C ABI.
#pragma once

#include "grtmg.h"

namespace grtmg {

// Residual norms of the zero state (u = 0, W_i = 0), in two halves so that the
// caller can queue other work on its own stream in between: begin zeroes d_u
// and d_W (cells and 3 x cells doubles) and queues the evaluation on the
// solver's internal stream, ordered after the work queued on the solver's
// caller stream so far but not after anything queued there later; end waits
// for it, returns the norms as mg_residual_norm does, and orders the caller
// stream after it.  d_u and d_W must not be used by other work in between.
// Every successful begin must be followed by an end.
mg_status zero_norms_begin(mg_ctx *c, double *d_u, double *d_W);
mg_status zero_norms_end(mg_ctx *c, double out[4]);

// Forgets the state the last solve left, so that mg_solve_constraints_continue
// refuses it (its arrays were changed outside the solver).
void cancel_continue(mg_ctx *c);

// Shape of a solver context for callers that hand it arrays sized elsewhere:
// cells per axis of the finest level, boundary rule, whether it solves the
// momentum equation, whether psi is data (CTTK), and the caller stream given at setup.
struct SolverShape {
    int n, bc;
    bool momentum;
    bool cttk; // psi is data (MG_FLAG_CTTK)
    void *user_stream;
};
SolverShape solver_shape(const mg_ctx *c);

// One outer iteration from (d_u, d_W) as mg_solve_constraints(tol 1e-300,
// max_outer 1) does it, with the iteration enqueued before the starting state's
// norms are read (no tolerance can stop it there); rep as that call fills it.
mg_status check_iteration(mg_ctx *c, double *d_u, double *d_W, mg_report *rep);

} // namespace grtmg
