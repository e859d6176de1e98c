// Internal interface between the solver (solver.hip) and the batch engine (batch.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/fde.h"

namespace fde {

// Starts one CN step of h from u_prev (device FP64) with sources sum_k phi[k] S[k]: right-hand
// side, first restart cycle and a state read are issued on the handle's stream; nothing waits.
int async_step_start(fde_handle* h, const double* u_prev, int nsrc, const double* phi, const double* const* S);
// Non-blocking: *finished = 1 once the step's solve has converged or stopped (stats filled, return
// code as fde_step's); otherwise issues the next cycle when the previous one has completed.
int async_poll(fde_handle* h, int* finished, fde_stats* stats);
// Device address of the last solution (valid until the next async_step_start).
const double* async_result(const fde_handle* h);
hipStream_t handle_stream(const fde_handle* h);
// Graph capture of the restart cycle (on by default).
void async_use_graph(fde_handle* h, bool on);
// Device bytes a handle for problem p needs (0 if p is invalid).
size_t footprint_bytes(const fde_problem* p);
// Sets the message fde_last_error(NULL) returns on this thread.
void set_global_error(const char* msg);

}  // namespace fde
