// Batching and serving: many independent CN time-stepping requests (each its own sizes, orders,
// coefficients and source) resident on one GPU and advanced together (the CN recursion of
// eq. (CNWSGD) / (system), one solve per step, applied to independent problems).
//
// Every request owns a solver handle on its own HIP stream (default priority): its Toeplitz symbols,
// hierarchy and Krylov storage stay resident until the request is released.  A step is a chain of
// restart cycles replayed from a captured HIP graph; the host only starts steps and reads the solver
// state between cycles, without blocking, so the cycles of all requests overlap on the device.
// Requests are admitted against a device-memory budget and may join or leave between calls to
// fde_batch_step (continuous batching).  The kernels a request runs, and their order, do not depend
// on the other requests, so its result is the same alone and in the mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fde.h"
#include "common.h"
#include "engine.h"

using namespace fde;

namespace {

enum ReqState { RS_START = 0, RS_RUNNING = 1, RS_DONE = 2, RS_FAILED = 3 };

struct Request {
  fde_handle* h = nullptr;
  hipStream_t stream = nullptr;
  fde_problem p{};
  size_t N = 0;
  double* u[2] = {nullptr, nullptr};
  int cur = 0;
  int nsrc = 0;
  double coef[kMaxSrc] = {}, rate[kMaxSrc] = {};
  double* S[kMaxSrc] = {};
  int nsteps = 0, steps_done = 0;
  double t0 = 0;
  int state = RS_START;
  int err = 0;
  int64_t iters = 0;
  int noconv = 0;  // steps that stopped at the iteration limit (their last iterate is kept)
  size_t bytes = 0;
};

void release(Request& r) {
  if (r.stream) (void)hipStreamSynchronize(r.stream);
  if (r.h) fde_destroy(r.h);
  for (double*& p : r.u)
    if (p) (void)hipFree(p);
  for (int k = 0; k < kMaxSrc; ++k)
    if (r.S[k]) (void)hipFree(r.S[k]);
  if (r.stream) (void)hipStreamDestroy(r.stream);
  r = Request{};
}

}  // namespace

struct fde_batch {
  size_t budget = 0;
  size_t used = 0;
  int next_id = 0;
  std::map<int, Request> reqs;
  std::string err;
};

extern "C" {

size_t fde_footprint(const fde_problem* p) { return footprint_bytes(p); }

int fde_batch_create(size_t budget_bytes, void* stream, fde_batch** out) {
  (void)stream;  // every request runs on a stream of its own
  if (!out) return FDE_EINVAL;
  *out = new fde_batch();
  (*out)->budget = budget_bytes;
  return FDE_OK;
}

void fde_batch_destroy(fde_batch* b) {
  if (!b) return;
  for (auto& kv : b->reqs) release(kv.second);
  delete b;
}

int fde_batch_admit(fde_batch* b, const fde_problem* p, const double* dp, const double* dm, const double* ep,
                    const double* em, const double* u0, int32_t nsteps, double t0, int32_t nsrc,
                    const double* coef, const double* rate, const double* const* S) {
  if (!b || !p || !u0 || nsteps < 1) return FDE_EINVAL;
  if (nsrc < 0 || nsrc > kMaxSrc || (nsrc > 0 && (!coef || !rate || !S))) return FDE_EINVAL;
  const size_t core = footprint_bytes(p);
  if (core == 0) return FDE_EINVAL;
  const size_t N = (size_t)p->n1 * p->n2;
  const size_t need = core + (2 + (size_t)nsrc) * N * sizeof(double);
  if (b->used + need > b->budget) return FDE_EAGAIN;
  Request r;
  r.p = *p;
  r.N = N;
  r.nsteps = nsteps;
  r.t0 = t0;
  r.nsrc = nsrc;
  r.bytes = need;
  auto fail = [&](int code, const char* msg) {
    b->err = msg;
    release(r);
    return code;
  };
  if (hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking) != hipSuccess)
    return fail(FDE_EDEVICE, "stream creation failed");
  const int rc = fde_setup(p, dp, dm, ep, em, r.stream, &r.h);
  if (rc != FDE_OK) {
    b->err = fde_last_error(nullptr);
    release(r);
    return rc;
  }
  for (double*& q : r.u)
    if (hipMalloc(&q, N * sizeof(double)) != hipSuccess) return fail(FDE_ENOMEM, "device allocation failed");
  if (hipMemcpyAsync(r.u[0], u0, N * sizeof(double), hipMemcpyDeviceToDevice, r.stream) != hipSuccess)
    return fail(FDE_EDEVICE, "copy of u0 failed");
  for (int k = 0; k < nsrc; ++k) {
    if (!S[k]) return fail(FDE_EINVAL, "source field is NULL");
    r.coef[k] = coef[k];
    r.rate[k] = rate[k];
    if (hipMalloc(&r.S[k], N * sizeof(double)) != hipSuccess) return fail(FDE_ENOMEM, "device allocation failed");
    if (hipMemcpyAsync(r.S[k], S[k], N * sizeof(double), hipMemcpyDeviceToDevice, r.stream) != hipSuccess)
      return fail(FDE_EDEVICE, "copy of a source field failed");
  }
  // the caller may free or reuse its arrays once this returns
  if (hipStreamSynchronize(r.stream) != hipSuccess) return fail(FDE_EDEVICE, "stream synchronisation failed");
  const int id = b->next_id++;
  b->used += need;
  b->reqs.emplace(id, r);
  return id;
}

int fde_batch_step(fde_batch* b) {
  if (!b) return FDE_EINVAL;
  int completed = 0;
  while (true) {
    int active = 0;
    for (auto& kv : b->reqs) {
      Request& r = kv.second;
      if (r.state == RS_START) {
        // source amplitudes at the half step t^(m-1/2), m = steps_done + 1
        const double t = r.t0 + (r.steps_done + 0.5) * r.p.tau;
        double phi[kMaxSrc];
        for (int k = 0; k < r.nsrc; ++k) phi[k] = r.coef[k] * std::exp(r.rate[k] * t);
        const int rc = async_step_start(r.h, r.u[r.cur], r.nsrc, phi, r.S);
        if (rc != FDE_OK) {
          r.state = RS_FAILED;
          r.err = rc;
          ++completed;
          continue;
        }
        r.state = RS_RUNNING;
      }
      if (r.state != RS_RUNNING) continue;
      ++active;
      int fin = 0;
      fde_stats st{};
      const int rc = async_poll(r.h, &fin, &st);
      if (!fin && rc == FDE_OK) continue;
      ++completed;
      r.iters += st.iters;
      if (rc == FDE_ENOCONV) {
        ++r.noconv;
      } else if (rc != FDE_OK) {
        r.state = RS_FAILED;
        r.err = rc;
        continue;
      }
      const int nxt = 1 - r.cur;
      if (hipMemcpyAsync(r.u[nxt], async_result(r.h), r.N * sizeof(double), hipMemcpyDeviceToDevice, r.stream) !=
          hipSuccess) {
        r.state = RS_FAILED;
        r.err = FDE_EDEVICE;
        continue;
      }
      r.cur = nxt;
      ++r.steps_done;
      r.state = (r.steps_done >= r.nsteps) ? RS_DONE : RS_START;
    }
    if (completed > 0 || active == 0) break;
    std::this_thread::yield();
  }
  int running = 0;
  for (auto& kv : b->reqs)
    if (kv.second.state == RS_START || kv.second.state == RS_RUNNING) ++running;
  return running;
}

int fde_batch_poll(fde_batch* b, int id, double* u_out, int64_t* iters_out) {
  if (!b) return FDE_EINVAL;
  auto it = b->reqs.find(id);
  if (it == b->reqs.end()) return FDE_EINVAL;
  Request& r = it->second;
  if (iters_out) *iters_out = r.iters;
  if (r.state == RS_FAILED) {
    const int e = r.err;
    b->used -= r.bytes;
    release(r);
    b->reqs.erase(it);
    return e;
  }
  if (r.state != RS_DONE) return 0;
  const int done_code = r.noconv ? 2 : 1;
  if (u_out) {
    if (hipMemcpyAsync(u_out, r.u[r.cur], r.N * sizeof(double), hipMemcpyDeviceToDevice, r.stream) != hipSuccess ||
        hipStreamSynchronize(r.stream) != hipSuccess)
      return FDE_EDEVICE;
    b->used -= r.bytes;
    release(r);
    b->reqs.erase(it);
  }
  return done_code;
}

int fde_batch_cancel(fde_batch* b, int id) {
  if (!b) return FDE_EINVAL;
  auto it = b->reqs.find(id);
  if (it == b->reqs.end()) return FDE_EINVAL;
  b->used -= it->second.bytes;
  release(it->second);
  b->reqs.erase(it);
  return FDE_OK;
}

int fde_batch_info(const fde_batch* b, int32_t* active, size_t* bytes_in_use) {
  if (!b) return FDE_EINVAL;
  int n = 0;
  for (auto& kv : b->reqs)
    if (kv.second.state == RS_START || kv.second.state == RS_RUNNING) ++n;
  if (active) *active = n;
  if (bytes_in_use) *bytes_in_use = b->used;
  return FDE_OK;
}

}  // extern "C"
