// Internal interface between the solver (solver.hip) and the batch engine (batch.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/fde.h"
#include "common.h"

namespace fde {

// Starts one CN step of h from u_prev (device FP64) with sources sum_k phi[k] S[k]: right-hand
// side, first restart cycle and a state read are issued on the handle's stream; nothing waits.
// With defer the first cycle is held instead (issued by async_issue).
int async_step_start(fde_handle* h, const double* u_prev, int nsrc, const double* phi, const double* const* S,
                     bool defer = false);
// Non-blocking: *finished = 1 once the step's solve has converged or stopped (stats filled, return
// code as fde_step's); otherwise issues the next cycle when the previous one has completed, or with
// defer holds it (async_held) until async_issue.
int async_poll(fde_handle* h, int* finished, fde_stats* stats, bool defer = false);
// Issues the held cycle of h.
int async_issue(fde_handle* h);
// True if h has a step in flight whose next cycle is held.
bool async_held(const fde_handle* h);
// Issues each restart cycle in pieces of `steps` Arnoldi steps plus a tail (0: one piece); the host
// stops issuing pieces once the cycle is done.  Not while a step is in flight.
int async_set_piece(fde_handle* h, int steps);
// Device address of the last solution (valid until the next async_step_start).
const double* async_result(const fde_handle* h);
hipStream_t handle_stream(const fde_handle* h);
// Graph capture of the restart cycle (on by default).
void async_use_graph(fde_handle* h, bool on);
// Device bytes a handle for problem p needs (0 if p is invalid).
size_t footprint_bytes(const fde_problem* p);
// Sets the message fde_last_error(NULL) returns on this thread.
void set_global_error(const char* msg);

// ---- batched groups (batch.hip): handles of one shape in equal slots of one device region ----------
// fde_setup with every buffer carved, in a fixed order, from [base, base + cap): handles of the same
// shape built in equal slots have identical layouts, `cap` bytes apart.
int group_setup(const fde_problem* p, const double* dp, const double* dm, const double* ep, const double* em,
                hipStream_t stream, void* base, size_t cap, fde_handle** out);
// Byte offset of the handle's solver state within its slot.
long long group_state_offset(const fde_handle* h);
// Starts a CN step of one member on its stream: right-hand side, x = 0 and the norm of b (no cycle).
int group_step_start(fde_handle* h, const double* u_prev, int nsrc, const double* phi, const double* const* S);
// A restart cycle runs as group_pieces(h) pieces of Arnoldi steps (each skips its steps on the device
// once the cycle is done, so the host may stop issuing them) and a tail, piece group_pieces(h):
// x += Z y and the true residual.
int group_pieces(const fde_handle* h);
// Captures one piece of the cycle as a graph whose every launch has grid z extent nz: the launches
// carry the pointers of h's slot, and workgroup z works on the slot ztab[z] bytes away (device table
// of nz entries, read when the graph runs; kZSkip entries are padding).
int group_capture_piece(fde_handle* h, int nz, const long long* ztab, int piece, hipGraph_t* graph,
                        hipGraphExec_t* gexec);
// After a cycle: *finished = 1 if the member's solve stopped (stats filled, fde_step's return code).
int group_step_result(fde_handle* h, const GmresState& s, int cycles, int* finished, fde_stats* stats);
// Whether problems of this shape can be advanced by batched launches.
bool group_eligible(const fde_problem* p, int max_n);

}  // namespace fde
