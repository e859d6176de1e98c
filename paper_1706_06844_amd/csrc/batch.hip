// Batching and serving: many independent CN time-stepping requests (each its own sizes, orders,
// coefficients and source) resident on one GPU and advanced together (the CN recursion of
// eq. (CNWSGD) / (system), one solve per step, applied to independent problems).
//
// Every request owns a solver handle on its own HIP stream (default priority; or on one of the batch's
// lanes, fde_batch_set_lanes): its Toeplitz symbols, hierarchy and Krylov storage stay resident until
// the request is released.  A step is a chain of restart cycles replayed from captured HIP graphs,
// whole or in pieces of Arnoldi steps (fde_batch_set_policy); the host only starts steps and reads the
// solver state between cycles (or pieces), without blocking, so the work of all requests overlaps on
// the device.  With a cap on the requests in flight the host hands each free place to the waiting
// request with the least work left.
// Requests are admitted against a device-memory budget and may join or leave between calls to
// fde_batch_step (continuous batching).  The kernels a request runs, and their order, do not depend
// on the other requests, so its result is the same alone and in the mix.
//
// Grouped mode (fde_batch_set_grouping): requests of one shape (sizes, precision, multigrid settings)
// up to a size limit share a group: one device region cut into equal slots and one stream.  The
// group's restart cycle (each of its pieces) is captured once per z extent of a short ladder (1, 2,
// 3, 4, 6, 8, 12, ..., and the slot count); before each cycle the host writes the slot offsets of the members that are
// solving into a small device table and replays the smallest capture that holds them, so every kernel
// of the cycle is one launch over exactly the solving members (plus at most a third of padding, whose
// workgroups exit at once).  Each member starts its CN steps on its own (right-hand side, norm of b)
// between cycles.  A member whose solve stops inside a cycle skips the rest of it (done flag), and a
// slot without a member is marked idle, so each member runs exactly the arithmetic it runs alone.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
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
  int group = -1;  // index of its group in grouped mode (the stream then belongs to the group)
  bool own_stream = false;  // the stream was created for this request
  int lane = -1;            // index of its lane when the batch has lanes
  int slot = -1;
  int cycles = 0;  // restart cycles of the solve in flight (grouped mode)
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
  if (r.stream && r.own_stream) (void)hipStreamDestroy(r.stream);
  r = Request{};
}

// One capture of the group cycle: z extent nz, launches carrying the pointers of slot `base`, one
// graph per piece (the Arnoldi pieces, then the tail).
struct CycleGraph {
  int nz = 0;
  int base = 0;
  std::vector<hipGraph_t> graph;
  std::vector<hipGraphExec_t> gexec;
};

// A group: `nslots` slots of `slot_bytes` in one allocation, members by slot, the captured cycles.
struct Group {
  fde_problem shape{};
  int nslots = 0;
  size_t slot_bytes = 0;
  char* arena = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;  // the stream was created for this group (not a lane of the batch)
  std::vector<int> member;  // request id per slot, -1 if empty
  long long st_off = 0;     // offset of the solver state within a slot
  std::vector<CycleGraph> cycles;  // by increasing nz; the last one has nz = nslots
  int npieces = 0;                 // Arnoldi pieces of a cycle (the tail is piece npieces)
  int cg = 0;                      // the capture the piece in flight runs
  int piece = 0;                   // the piece in flight
  std::vector<int> cyc;            // slots of the members in the cycle in flight
  long long* zt_dev = nullptr;     // slot offsets of the next cycle (nslots entries)
  long long* zt_host = nullptr;    // pinned staging of zt_dev
  hipEvent_t ev = nullptr;
  GmresState* hst = nullptr;  // pinned: the states' host-read prefix of every slot after a cycle
  GmresState* idle = nullptr;  // pinned: the state written into an empty slot
  bool inflight = false;
};

// The part of the state the host reads after a cycle (the configuration fields follow it).
constexpr size_t kStatePrefix = offsetof(GmresState, rtol);

bool same_shape(const fde_problem& a, const fde_problem& b) {
  return a.n1 == b.n1 && a.n2 == b.n2 && a.precision == b.precision && a.mg_variant == b.mg_variant &&
         a.nu_pre == b.nu_pre && a.nu_post == b.nu_post && a.coarsest_n == b.coarsest_n && a.restart == b.restart &&
         a.omega == b.omega;
}

// The z extents a group's cycle is captured for: 1, 2, 3, 4, 6, 8, 12, 16, 24, ... below nslots,
// then nslots (consecutive extents differ by at most 1.5x).
std::vector<int> nz_ladder(int nslots) {
  std::vector<int> v;
  for (int a = 1; a < nslots; a *= 2) {
    v.push_back(a);
    if (a >= 2 && a + a / 2 < nslots) v.push_back(a + a / 2);
  }
  std::sort(v.begin(), v.end());
  v.push_back(nslots);
  return v;
}

void destroy_group(Group& g) {
  if (g.stream) (void)hipStreamSynchronize(g.stream);
  for (CycleGraph& c : g.cycles) {
    for (hipGraphExec_t e : c.gexec)
      if (e) (void)hipGraphExecDestroy(e);
    for (hipGraph_t e : c.graph)
      if (e) (void)hipGraphDestroy(e);
  }
  if (g.zt_dev) (void)hipFree(g.zt_dev);
  if (g.zt_host) (void)hipHostFree(g.zt_host);
  if (g.ev) (void)hipEventDestroy(g.ev);
  if (g.hst) (void)hipHostFree(g.hst);
  if (g.idle) (void)hipHostFree(g.idle);
  if (g.arena) (void)hipFree(g.arena);
  if (g.stream && g.own_stream) (void)hipStreamDestroy(g.stream);
  g = Group{};
}

// Marks slot `s` empty on the device: every kernel of the group cycle skips it from now on.
hipError_t mark_idle(Group& g, int s) {
  return hipMemcpyAsync(g.arena + (size_t)s * g.slot_bytes + g.st_off, g.idle, sizeof(GmresState),
                        hipMemcpyHostToDevice, g.stream);
}

}  // namespace

struct fde_batch {
  size_t budget = 0;
  size_t used = 0;
  int next_id = 0;
  std::map<int, Request> reqs;
  std::string err;
  int group_max_n = 0;  // 0: grouping off
  int group_slots = 0;
  std::vector<Group> groups;
  int max_running = 0;  // ungrouped requests with a cycle in flight at once (0: no limit)
  int piece_steps = 0;  // Arnoldi steps per issued piece of a restart cycle (0: whole cycles)
  int busy_running = -1;  // ungrouped requests with a piece in flight while a group has work (-1: max_running)
  // lanes: streams created together at set-up (so that they map to distinct hardware queues): the
  // first half for the ungrouped requests (dealt in turn, at most one piece in flight per lane), the
  // others dealt to the groups in turn; empty: a stream per request and per group
  std::vector<hipStream_t> lanes;
  int groups_made = 0;
  int ungrouped_made = 0;
};

extern "C" {

size_t fde_footprint(const fde_problem* p) { return footprint_bytes(p); }

int fde_batch_create(size_t budget_bytes, void* stream, fde_batch** out) {
  (void)stream;  // requests and groups get streams of their own, or the batch's lanes
  if (!out) return FDE_EINVAL;
  *out = new fde_batch();
  (*out)->budget = budget_bytes;
  return FDE_OK;
}

void fde_batch_destroy(fde_batch* b) {
  if (!b) return;
  for (Group& g : b->groups)
    if (g.stream) (void)hipStreamSynchronize(g.stream);
  for (auto& kv : b->reqs) release(kv.second);
  for (Group& g : b->groups) destroy_group(g);
  for (hipStream_t s : b->lanes) (void)hipStreamDestroy(s);
  delete b;
}

int fde_batch_set_lanes(fde_batch* b, int32_t lanes) {
  if (!b || lanes < 0 || lanes == 1 || lanes > 16) return FDE_EINVAL;
  if (!b->reqs.empty() || !b->groups.empty()) return FDE_EINVAL;
  for (hipStream_t s : b->lanes) (void)hipStreamDestroy(s);
  b->lanes.clear();
  for (int k = 0; k < lanes; ++k) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t t : b->lanes) (void)hipStreamDestroy(t);
      b->lanes.clear();
      return FDE_EDEVICE;
    }
    b->lanes.push_back(s);
  }
  return FDE_OK;
}

int fde_batch_set_grouping(fde_batch* b, int32_t max_n, int32_t slots) {
  if (!b || max_n < 0 || slots < 0 || (max_n > 0 && slots < 1) || slots > 1024) return FDE_EINVAL;
  if (!b->reqs.empty()) return FDE_EINVAL;
  b->group_max_n = slots > 0 ? max_n : 0;
  b->group_slots = slots;
  return FDE_OK;
}

int fde_batch_set_policy(fde_batch* b, int32_t max_running, int32_t piece_steps, int32_t busy_running) {
  if (!b || max_running < 0 || piece_steps < 0 || busy_running < -1) return FDE_EINVAL;
  if (piece_steps != b->piece_steps && !b->reqs.empty()) return FDE_EINVAL;
  b->max_running = max_running;
  b->piece_steps = piece_steps;
  b->busy_running = busy_running;
  return FDE_OK;
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
  fde_problem pf = *p;  // the defaults filled in, so that equal shapes compare equal
  {
    fde_problem q{};
    fde_problem_default(&q, p->alpha, p->beta, p->n1, p->n2, p->tau);
    if (pf.nu_pre < 0) pf.nu_pre = q.nu_pre;
    if (pf.nu_post < 0) pf.nu_post = q.nu_post;
    if (pf.coarsest_n == 0) pf.coarsest_n = q.coarsest_n;
    if (pf.restart == 0) pf.restart = q.restart;
  }
  if (b->group_max_n > 0 && group_eligible(&pf, b->group_max_n)) {
    // a free slot of a group of this shape, or a new group
    int gi = -1, si = -1;
    for (int k = 0; k < (int)b->groups.size() && gi < 0; ++k) {
      Group& g = b->groups[k];
      if (!g.arena || !same_shape(g.shape, pf)) continue;
      for (int s = 0; s < g.nslots; ++s)
        if (g.member[s] < 0) {
          gi = k;
          si = s;
          break;
        }
    }
    const size_t extra = (2 + (size_t)nsrc) * N * sizeof(double);
    if (gi < 0) {
      Group g;
      g.shape = pf;
      g.nslots = b->group_slots;
      g.slot_bytes = (core + 4095) / 4096 * 4096;
      const size_t gbytes = g.slot_bytes * (size_t)g.nslots;
      if (b->used + gbytes + extra > b->budget) return FDE_EAGAIN;
      g.member.assign(g.nslots, -1);
      if (hipMalloc(&g.arena, gbytes) != hipSuccess) return FDE_ENOMEM;
      if (!b->lanes.empty()) {
        const int nb = (int)b->lanes.size() / 2;
        g.stream = b->lanes[nb + b->groups_made % ((int)b->lanes.size() - nb)];
      } else if (hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) == hipSuccess) {
        g.own_stream = true;
      }
      ++b->groups_made;
      if (!g.stream || hipEventCreateWithFlags(&g.ev, hipEventDisableTiming) != hipSuccess ||
          hipHostMalloc((void**)&g.hst, sizeof(GmresState) * g.nslots, hipHostMallocDefault) != hipSuccess ||
          hipHostMalloc((void**)&g.idle, sizeof(GmresState), hipHostMallocDefault) != hipSuccess ||
          hipHostMalloc((void**)&g.zt_host, sizeof(long long) * g.nslots, hipHostMallocDefault) != hipSuccess ||
          hipMalloc(&g.zt_dev, sizeof(long long) * g.nslots) != hipSuccess) {
        destroy_group(g);
        return FDE_EDEVICE;
      }
      std::memset(g.idle, 0, sizeof(GmresState));
      g.idle->done = 1;
      g.idle->conv = 1;
      g.idle->idle = 1;
      b->used += gbytes;
      b->groups.push_back(g);
      gi = (int)b->groups.size() - 1;
      si = 0;
    } else if (b->used + extra > b->budget) {
      return FDE_EAGAIN;
    }
    Group& g = b->groups[gi];
    r.group = gi;
    r.slot = si;
    r.stream = g.stream;
    r.bytes = extra;
    const int rc = group_setup(&pf, dp, dm, ep, em, g.stream, g.arena + (size_t)si * g.slot_bytes, g.slot_bytes, &r.h);
    if (rc != FDE_OK) {
      b->err = fde_last_error(nullptr);
      release(r);
      return rc;
    }
    if (async_set_piece(r.h, b->piece_steps) != FDE_OK) return fail(FDE_EINVAL, "piece setting failed");
    if (g.cycles.empty()) {
      // the group's first member lays out the slots: the others get the idle state, and every piece
      // of the cycle is captured for every z extent of the ladder, with this member's pointers
      g.st_off = group_state_offset(r.h);
      for (int s = 1; s < g.nslots; ++s)
        if (mark_idle(g, s) != hipSuccess) return fail(FDE_EDEVICE, "initialising the slots failed");
      g.npieces = group_pieces(r.h);
      for (int nz : nz_ladder(g.nslots)) {
        g.cycles.emplace_back();
        CycleGraph& c = g.cycles.back();
        c.nz = nz;
        c.base = si;
        c.graph.assign(g.npieces + 1, nullptr);
        c.gexec.assign(g.npieces + 1, nullptr);
        for (int pc = 0; pc <= g.npieces; ++pc) {
          const int cr = group_capture_piece(r.h, nz, g.zt_dev, pc, &c.graph[pc], &c.gexec[pc]);
          if (cr != FDE_OK) {
            b->err = fde_last_error(r.h);
            for (CycleGraph& d : g.cycles) {
              for (hipGraphExec_t e : d.gexec)
                if (e) (void)hipGraphExecDestroy(e);
              for (hipGraph_t e : d.graph)
                if (e) (void)hipGraphDestroy(e);
            }
            g.cycles.clear();
            release(r);
            return cr;
          }
        }
      }
    }
  } else {
    if (!b->lanes.empty()) {
      r.lane = b->ungrouped_made++ % ((int)b->lanes.size() / 2);
      r.stream = b->lanes[r.lane];
    } else {
      if (hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking) != hipSuccess)
        return fail(FDE_EDEVICE, "stream creation failed");
      r.own_stream = true;
    }
    const int rc = fde_setup(p, dp, dm, ep, em, r.stream, &r.h);
    if (rc != FDE_OK) {
      b->err = fde_last_error(nullptr);
      release(r);
      return rc;
    }
    if (async_set_piece(r.h, b->piece_steps) != FDE_OK) return fail(FDE_EINVAL, "piece setting failed");
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
  b->used += r.bytes;
  if (r.group >= 0) b->groups[r.group].member[r.slot] = id;
  b->reqs.emplace(id, r);
  return id;
}

}  // extern "C"

namespace {

// Index of the smallest capture whose z extent holds n members.
int capture_for(const Group& g, int n) {
  for (int c = 0; c < (int)g.cycles.size(); ++c)
    if (g.cycles[c].nz >= n) return c;
  return (int)g.cycles.size() - 1;
}

// Selects the capture for the members in `slots` and writes their slot offsets (then padding) into
// the device table, ordered before the next launch on the group's stream.
hipError_t set_table(Group& g, const std::vector<int>& slots) {
  g.cg = capture_for(g, (int)slots.size());
  const CycleGraph& cg = g.cycles[g.cg];
  for (int z = 0; z < cg.nz; ++z)
    g.zt_host[z] = z < (int)slots.size() ? (long long)(slots[z] - cg.base) * (long long)g.slot_bytes : kZSkip;
  return hipMemcpyAsync(g.zt_dev, g.zt_host, sizeof(long long) * cg.nz, hipMemcpyHostToDevice, g.stream);
}

// Issues piece pc of the group's current cycle and the read-back of the slots' states.
hipError_t launch_piece(Group& g, int pc) {
  g.piece = pc;
  hipError_t e = hipGraphLaunch(g.cycles[g.cg].gexec[pc], g.stream);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(g.hst, sizeof(GmresState), g.arena + g.st_off, g.slot_bytes, kStatePrefix, g.nslots,
                         hipMemcpyDeviceToHost, g.stream);
  if (e == hipSuccess) e = hipEventRecord(g.ev, g.stream);
  return e;
}

// Advances the grouped requests: after an Arnoldi piece of the group cycle the next one is issued
// while a member's cycle goes on (else the tail); a finished cycle is read out (members whose solve
// stopped complete their step), members waiting for a step start it, and the next cycle is issued.
// Returns the number of steps completed; *active counts the groups with work in flight.
int step_groups(fde_batch* b, int* active) {
  int completed = 0;
  for (int gi = 0; gi < (int)b->groups.size(); ++gi) {
    Group& g = b->groups[gi];
    if (!g.arena || g.cycles.empty()) continue;
    if (g.inflight) {
      hipError_t q = hipEventQuery(g.ev);
      if (q == hipErrorNotReady) {
        ++*active;
        continue;
      }
      g.inflight = false;
      if (q == hipSuccess && g.piece < g.npieces) {
        // the members whose cycle goes on: the next Arnoldi piece runs over them alone (a smaller
        // capture once they fit one), the tail over every member of the cycle
        std::vector<int> act;
        for (int s : g.cyc)
          if (g.member[s] >= 0 && b->reqs.at(g.member[s]).state == RS_RUNNING && !g.hst[s].done) act.push_back(s);
        if (!act.empty() && g.piece + 1 < g.npieces) {
          if (capture_for(g, (int)act.size()) < g.cg) q = set_table(g, act);
          if (q == hipSuccess) q = launch_piece(g, g.piece + 1);
        } else {
          if (capture_for(g, (int)g.cyc.size()) != g.cg) q = set_table(g, g.cyc);
          if (q == hipSuccess) q = launch_piece(g, g.npieces);
        }
        if (q == hipSuccess) {
          g.inflight = true;
          ++*active;
          continue;
        }
      }
      for (int s = 0; s < g.nslots; ++s) {
        if (g.member[s] < 0) continue;
        Request& r = b->reqs.at(g.member[s]);
        if (r.state != RS_RUNNING) continue;
        if (q != hipSuccess) {
          r.state = RS_FAILED;
          r.err = FDE_EDEVICE;
          ++completed;
          continue;
        }
        ++r.cycles;
        int fin = 0;
        fde_stats st{};
        const int rc = group_step_result(r.h, g.hst[s], r.cycles, &fin, &st);
        if (!fin && rc == FDE_OK) continue;
        ++completed;
        r.iters += st.iters;
        if (rc == FDE_ENOCONV) {
          ++r.noconv;
        } else if (rc != FDE_OK) {
          r.state = RS_FAILED;
          r.err = rc;
          (void)mark_idle(g, s);
          continue;
        }
        const int nxt = 1 - r.cur;
        if (hipMemcpyAsync(r.u[nxt], async_result(r.h), r.N * sizeof(double), hipMemcpyDeviceToDevice, g.stream) !=
            hipSuccess) {
          r.state = RS_FAILED;
          r.err = FDE_EDEVICE;
          continue;
        }
        r.cur = nxt;
        ++r.steps_done;
        r.state = (r.steps_done >= r.nsteps) ? RS_DONE : RS_START;
        if (r.state == RS_DONE) (void)mark_idle(g, s);
      }
    }
    // start the steps of members that wait for one, then issue a cycle over the members that solve
    std::vector<int> run;
    for (int s = 0; s < g.nslots; ++s) {
      if (g.member[s] < 0) continue;
      Request& r = b->reqs.at(g.member[s]);
      if (r.state == RS_START) {
        const double t = r.t0 + (r.steps_done + 0.5) * r.p.tau;
        double phi[kMaxSrc];
        for (int k = 0; k < r.nsrc; ++k) phi[k] = r.coef[k] * std::exp(r.rate[k] * t);
        const int rc = group_step_start(r.h, r.u[r.cur], r.nsrc, phi, r.S);
        if (rc != FDE_OK) {
          r.state = RS_FAILED;
          r.err = rc;
          (void)mark_idle(g, s);
          ++completed;
          continue;
        }
        r.state = RS_RUNNING;
        r.cycles = 0;
      }
      if (r.state == RS_RUNNING) run.push_back(s);
    }
    if (run.empty()) continue;
    g.cyc = run;
    if (set_table(g, run) != hipSuccess || launch_piece(g, 0) != hipSuccess) {
      for (int s = 0; s < g.nslots; ++s) {
        if (g.member[s] < 0) continue;
        Request& r = b->reqs.at(g.member[s]);
        if (r.state == RS_RUNNING) {
          r.state = RS_FAILED;
          r.err = FDE_EDEVICE;
          ++completed;
        }
      }
      continue;
    }
    g.inflight = true;
    ++*active;
  }
  return completed;
}

}  // namespace

namespace {

// Starts the next CN step of an ungrouped request (its first cycle held with defer); false on error.
bool start_step(Request& r, bool defer) {
  // source amplitudes at the half step t^(m-1/2), m = steps_done + 1
  const double t = r.t0 + (r.steps_done + 0.5) * r.p.tau;
  double phi[kMaxSrc];
  for (int k = 0; k < r.nsrc; ++k) phi[k] = r.coef[k] * std::exp(r.rate[k] * t);
  const int rc = async_step_start(r.h, r.u[r.cur], r.nsrc, phi, r.S, defer);
  if (rc != FDE_OK) {
    r.state = RS_FAILED;
    r.err = rc;
    return false;
  }
  r.state = RS_RUNNING;
  return true;
}

// Work left in a request, for the shortest-remaining-work order: unknowns times remaining steps.
double remaining_work(const Request& r) { return (double)r.N * (double)(r.nsteps - r.steps_done); }

}  // namespace

extern "C" {

int fde_batch_step(fde_batch* b) {
  if (!b) return FDE_EINVAL;
  int completed = 0;
  const bool capped = b->max_running > 0 || b->busy_running >= 0 || !b->lanes.empty();
  while (true) {
    int active = 0;
    completed += step_groups(b, &active);
    if (!capped) {
      for (auto& kv : b->reqs) {
        Request& r = kv.second;
        if (r.group < 0 && r.state == RS_START && !start_step(r, false)) ++completed;
      }
    }
    for (auto& kv : b->reqs) {
      Request& r = kv.second;
      if (r.group >= 0) continue;
      if (r.state != RS_RUNNING) continue;
      ++active;
      int fin = 0;
      fde_stats st{};
      const int rc = async_poll(r.h, &fin, &st, capped);
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
    if (capped) {
      // at most max_running requests with a piece in flight (busy_running while a group has work);
      // the others wait at a piece boundary, and the next pieces go to the requests with the least
      // work left
      int limit = b->max_running > 0 ? b->max_running : INT_MAX;
      if (b->busy_running >= 0) {
        for (const Group& g : b->groups) {
          if (!g.arena) continue;
          bool busy = g.inflight;
          for (int s = 0; s < g.nslots && !busy; ++s)
            if (g.member[s] >= 0) {
              const int st = b->reqs.at(g.member[s]).state;
              busy = st == RS_START || st == RS_RUNNING;
            }
          if (busy) {
            limit = std::min(limit, b->busy_running);
            break;
          }
        }
      }
      int inflight = 0;
      int lane_busy[16] = {};
      std::vector<std::pair<double, Request*>> wait;
      for (auto& kv : b->reqs) {
        Request& r = kv.second;
        if (r.group >= 0) continue;
        if (r.state == RS_RUNNING && !async_held(r.h)) {
          ++inflight;
          if (r.lane >= 0) ++lane_busy[r.lane];
        } else if (r.state == RS_START || r.state == RS_RUNNING) {
          wait.emplace_back(remaining_work(r), &r);
        }
      }
      std::stable_sort(wait.begin(), wait.end(),
                       [](const std::pair<double, Request*>& a, const std::pair<double, Request*>& c) {
                         return a.first < c.first;
                       });
      for (auto& w : wait) {
        if (inflight >= limit) break;
        Request& r = *w.second;
        if (r.lane >= 0 && lane_busy[r.lane] > 0) continue;  // one piece in flight per lane
        if (r.state == RS_START) {
          if (!start_step(r, false)) {
            ++completed;
            continue;
          }
        } else if (async_issue(r.h) != FDE_OK) {
          r.state = RS_FAILED;
          r.err = FDE_EDEVICE;
          ++completed;
          continue;
        }
        ++inflight;
        ++active;
        if (r.lane >= 0) ++lane_busy[r.lane];
      }
    }
    if (completed > 0 || active == 0) break;
    std::this_thread::yield();
  }
  int running = 0;
  for (auto& kv : b->reqs)
    if (kv.second.state == RS_START || kv.second.state == RS_RUNNING) ++running;
  return running;
}

}  // extern "C"

namespace {
// Frees the request's slot: it is marked idle (ordered after the group's work) before the handle goes.
// A cycle still counted in flight is read out by the next fde_batch_step for the other members.
void leave_group(fde_batch* b, Request& r) {
  if (r.group < 0) return;
  Group& g = b->groups[r.group];
  (void)mark_idle(g, r.slot);
  if (g.stream) (void)hipStreamSynchronize(g.stream);
  g.member[r.slot] = -1;
}
}  // namespace

extern "C" {

int fde_batch_poll(fde_batch* b, int id, double* u_out, int64_t* iters_out) {
  if (!b) return FDE_EINVAL;
  auto it = b->reqs.find(id);
  if (it == b->reqs.end()) return FDE_EINVAL;
  Request& r = it->second;
  if (iters_out) *iters_out = r.iters;
  if (r.state == RS_FAILED) {
    const int e = r.err;
    b->used -= r.bytes;
    leave_group(b, r);
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
    leave_group(b, r);
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
  leave_group(b, it->second);
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
