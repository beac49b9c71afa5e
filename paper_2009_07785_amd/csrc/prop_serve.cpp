// prop_serve.cpp -- serving engine: propagation requests over resident
// problems with continuous batching into each problem's node slots.
//
// Per problem ("instance") the server keeps the batched-node layout of
// prop_run_batch_device: slots in groups of 8, each group a [n][8] block of
// start-of-round and candidate bound pairs, reached through a device table
// of group pointers so that groups can be allocated and released one by one.
// A request is packed into a free slot and started (its own round counter
// and round limit) between two rounds; from then on every round advances
// it.  A step is a few rounds of every instance with running slots, one
// launch per phase for all of them (the step table lists the instances and
// where each one's work items start); the end-of-round kernel reports the
// slots that finished in the step's completion list, which the host reads
// back with the step.  A finished slot is unpacked into its staging area,
// copied to the host, and freed once that copy has landed.
//
// Kernels and the step tables go on the server's stream; the copies of
// request bounds in and results out go on a second stream, ordered against
// the kernels with events (a slot's input copy before its pack kernel, its
// unpack kernel before the result copy), so that they overlap the rounds
// of other slots.  The host staging of a slot, and a step's host copy, are
// only rewritten after the device work that used them has completed
// (observed through an event).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <cstddef>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "prop.h"
#include "prop_handle.h"
#include "prop_launch.h"
#include "prop_layout.h"

using namespace prop;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kStepRing = 2;  // round steps in flight

enum ReqState { kQueued, kRunning, kDraining, kDone, kFailed };

struct Request {
  int64_t ticket = 0;
  int32_t inst = 0;
  int32_t max_rounds = 0;
  std::vector<double> lb, ub;  // the input, then the result
  prop_result res{};
  int state = kQueued;
  int err = 0;
  int32_t slot = -1;
  Clock::time_point t_submit;
};

struct SlotGroup {
  double2* A = nullptr;   // [n][8] start-of-round pairs
  double2* B = nullptr;   // [n][8] candidate targets
  double* d_io = nullptr; // [8][2][n] device staging: lb then ub of each slot
  double* h_io = nullptr; // pinned host staging, same layout
  hipEvent_t drain[kNodeGroup] = {};
  int used = 0;           // occupied slots
};

struct Instance {
  prop_problem* h = nullptr;
  int32_t id = 0;
  int32_t n = 0;
  Problem P{};            // the problem's matrix with the server's control block
  Batch bt{};             // per-slot state; gA/gB point to the device table
  int32_t cap = 0;        // slots
  void* d_state = nullptr;            // per-slot arrays, partials, tables, control
  std::vector<SlotGroup> groups;      // cap / 8 entries; A == nullptr when absent
  double2** h_table = nullptr;        // pinned host copy of the group tables (gA then gB)
  double2** d_table = nullptr;
  std::vector<Request*> slot_req;     // cap entries
  int running = 0;                    // requests in slots not yet reported finished
  std::deque<Request*> pending;
  int64_t fixed_bytes = 0;
  int32_t hi_groups = 0;              // 1 + highest allocated group
};

int64_t group_bytes(int32_t n) {
  return (int64_t)kNodeGroup * 48 * (int64_t)(n > 0 ? n : 1) + (int64_t)touch_bytes(n);
}

bool bound_ok(double l, double u) {
  const double huge = std::ldexp(1.0, 200);
  if (std::isnan(l) || std::isnan(u)) return false;
  if (l == INFINITY || u == -INFINITY) return false;
  if (std::isfinite(l) && std::fabs(l) > huge) return false;
  if (std::isfinite(u) && std::fabs(u) > huge) return false;
  return true;
}

}  // namespace

struct prop_server {
  prop_srv_config cfg{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work;   // new submissions / stop
  std::condition_variable cv_done;   // a request finished
  bool stop = false;
  int broken = 0;                    // error code once the device path failed
  std::string broken_msg;
  std::vector<std::unique_ptr<Instance>> insts;  // grows under mu
  std::vector<Instance*> live;                    // the scheduler's copy of insts
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  std::vector<Request*> incoming;
  int64_t next_ticket = 1;
  int64_t held = 0;                  // requests not yet read back by the caller
  int64_t device_bytes = 0, peak_bytes = 0;
  int64_t fixed_bytes = 0;           // server and per-instance state, never released
  // statistics (under mu)
  int64_t n_submitted = 0, n_completed = 0, n_queued = 0, n_running = 0, n_steps = 0;
  std::vector<double> lat_ms;
  bool have_first = false;
  Clock::time_point t_first, t_last;
  std::thread worker;
  // device side, created with the first instance
  hipStream_t stream = nullptr;
  hipStream_t copy = nullptr;         // request bounds in, results out
  hipEvent_t ev_in = nullptr;         // an input copy, for the pack kernel to wait on
  hipEvent_t ev_out = nullptr;        // an unpack kernel, for the result copy to wait on
  SrvInst* d_insts = nullptr;         // kSrvMaxInstances descriptors
  SrvStep* d_step[kStepRing] = {};
  SrvStep* h_step[kStepRing] = {};    // pinned: the step table up, completions down
  hipEvent_t step_ev[kStepRing] = {};
  uint64_t steps_queued = 0, steps_done = 0;

  void loop();
  bool poll_steps();
  bool poll_drains(Instance& I);
  int queue_step();
  int admit(Instance& I);
  int alloc_group(Instance& I, int g);
  void free_group(Instance& I, int g);
  bool reclaim(const Instance& need);
  void finish(Request* r, int state, int err);
  void fail_all(int code, const char* what);
  void charge(int64_t bytes) {
    std::lock_guard<std::mutex> lk(mu);
    device_bytes += bytes;
    peak_bytes = std::max(peak_bytes, device_bytes);
  }
};

namespace {

#define SRV_TRY(expr)                                                  \
  do {                                                                 \
    hipError_t e_ = (expr);                                            \
    if (e_ != hipSuccess) {                                            \
      fail(PROP_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));      \
      return PROP_EDEVICE;                                             \
    }                                                                  \
  } while (0)

}  // namespace

void prop_server::finish(Request* r, int state, int err) {
  std::lock_guard<std::mutex> lk(mu);
  r->state = state;
  r->err = err;
  if (state == kDone) {
    const auto now = Clock::now();
    lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
    t_last = now;
    ++n_completed;
  }
  --n_running;
  cv_done.notify_all();
}

void prop_server::fail_all(int code, const char* what) {
  std::lock_guard<std::mutex> lk(mu);
  broken = code;
  broken_msg = what;
  for (auto& kv : reqs) {
    Request* r = kv.second.get();
    if (r->state == kQueued || r->state == kRunning || r->state == kDraining) {
      r->state = kFailed;
      r->err = code;
    }
  }
  for (auto& I : insts) I->pending.clear();
  incoming.clear();
  n_queued = n_running = 0;
  cv_done.notify_all();
}

int prop_server::alloc_group(Instance& I, int g) {
  SlotGroup& G = I.groups[g];
  const size_t pairs = (size_t)kNodeGroup * (size_t)(I.n > 0 ? I.n : 1);
  SRV_TRY(hipMalloc((void**)&G.A, pairs * sizeof(double2)));
  // B is followed by its touch bytes, zero to start (stream order puts the
  // clear before any kernel that reads the group)
  SRV_TRY(hipMalloc((void**)&G.B, pairs * sizeof(double2) + touch_bytes(I.n)));
  SRV_TRY(hipMemsetAsync(G.B + pairs, 0, touch_bytes(I.n), stream));
  SRV_TRY(hipMalloc((void**)&G.d_io, 2 * pairs * sizeof(double)));
  SRV_TRY(hipHostMalloc((void**)&G.h_io, 2 * pairs * sizeof(double), hipHostMallocDefault));
  for (auto& e : G.drain) SRV_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  G.used = 0;
  charge(group_bytes(I.n));
  // The table entries reach the device in stream order, before any slot of
  // the group is packed; kernels already queued read only the entries of
  // groups with active slots.  The pinned source entries change again only
  // in free_group, after the stream has drained.
  const int32_t G8 = I.cap / kNodeGroup;
  I.h_table[g] = G.A;
  I.h_table[G8 + g] = G.B;
  SRV_TRY(hipMemcpyAsync(I.d_table + g, &I.h_table[g], sizeof(double2*), hipMemcpyHostToDevice,
                         stream));
  SRV_TRY(hipMemcpyAsync(I.d_table + G8 + g, &I.h_table[G8 + g], sizeof(double2*),
                         hipMemcpyHostToDevice, stream));
  I.hi_groups = std::max(I.hi_groups, g + 1);
  return PROP_OK;
}

// Releases an empty group.  Its slots are inactive, so no queued kernel
// touches its memory; hipFree waits for the device before releasing.
void release_group(SlotGroup& G) {
  if (G.A) hipFree(G.A);
  if (G.B) hipFree(G.B);
  if (G.d_io) hipFree(G.d_io);
  if (G.h_io) hipHostFree(G.h_io);
  for (auto& e : G.drain)
    if (e) hipEventDestroy(e);
  G = SlotGroup{};
}

void prop_server::free_group(Instance& I, int g) {
  hipStreamSynchronize(stream);
  hipStreamSynchronize(copy);
  release_group(I.groups[g]);
  const int32_t G8 = I.cap / kNodeGroup;
  I.h_table[g] = nullptr;
  I.h_table[G8 + g] = nullptr;
  while (I.hi_groups > 0 && I.groups[I.hi_groups - 1].A == nullptr) --I.hi_groups;
  charge(-group_bytes(I.n));
}

// Frees idle groups of other instances until `need` could allocate one.
bool prop_server::reclaim(const Instance& need) {
  const int64_t want = group_bytes(need.n);
  for (Instance* ip : live) {
    Instance& I = *ip;
    if (&I == &need || !I.pending.empty()) continue;
    for (int g = I.hi_groups - 1; g >= 0; --g) {
      if (I.groups[g].A == nullptr || I.groups[g].used != 0) continue;
      free_group(I, g);
      std::lock_guard<std::mutex> lk(mu);
      if (device_bytes + want <= cfg.budget_bytes) return true;
    }
  }
  std::lock_guard<std::mutex> lk(mu);
  return device_bytes + want <= cfg.budget_bytes;
}

// Admits queued requests of I into free slots; returns the number admitted,
// or a negative code on a device error.
int prop_server::admit(Instance& I) {
  int admitted = 0;
  const size_t n = (size_t)I.n;
  while (!I.pending.empty()) {
    int slot = -1;
    for (int g = 0; g < I.hi_groups && slot < 0; ++g) {
      if (I.groups[g].A == nullptr || I.groups[g].used == kNodeGroup) continue;
      for (int t = 0; t < kNodeGroup; ++t)
        if (!I.slot_req[g * kNodeGroup + t]) {
          slot = g * kNodeGroup + t;
          break;
        }
    }
    if (slot < 0) {
      int g = 0;
      while (g < I.cap / kNodeGroup && I.groups[g].A) ++g;
      if (g == I.cap / kNodeGroup) break;  // every slot of the instance is taken
      bool room;
      {
        std::lock_guard<std::mutex> lk(mu);
        room = device_bytes + group_bytes(I.n) <= cfg.budget_bytes;
      }
      if (!room && !reclaim(I)) break;  // wait for slots to drain
      int rc = alloc_group(I, g);
      if (rc) return rc;
      slot = g * kNodeGroup;
    }
    Request* r = I.pending.front();
    I.pending.pop_front();
    const int g = slot / kNodeGroup, t = slot % kNodeGroup;
    SlotGroup& G = I.groups[g];
    double* h = G.h_io + (size_t)t * 2 * n;
    double* d = G.d_io + (size_t)t * 2 * n;
    if (n) {
      std::memcpy(h, r->lb.data(), n * sizeof(double));
      std::memcpy(h + n, r->ub.data(), n * sizeof(double));
      SRV_TRY(hipMemcpyAsync(d, h, 2 * n * sizeof(double), hipMemcpyHostToDevice, copy));
      SRV_TRY(hipEventRecord(ev_in, copy));
      SRV_TRY(hipStreamWaitEvent(stream, ev_in, 0));
    }
    Batch bt = I.bt;
    bt.groups = I.hi_groups;
    bt.nodes = I.hi_groups * kNodeGroup;
    SRV_TRY(launch_pack_batch(I.P, bt, d, d + n, slot, 1, stream));
    SRV_TRY(launch_start_batch(I.P, bt, r->max_rounds, slot, 1, false, stream));
    r->slot = slot;
    I.slot_req[slot] = r;
    ++G.used;
    ++I.running;
    {
      std::lock_guard<std::mutex> lk(mu);
      r->state = kRunning;
      --n_queued;
      ++n_running;
    }
    ++admitted;
  }
  return admitted;
}

// Queues one step: the step table of every instance with running slots,
// rounds_per_step rounds of all of them, and the step's completions back.
int prop_server::queue_step() {
  const int ring = (int)(steps_queued % kStepRing);
  SrvStep& H = *h_step[ring];
  H.n = 0;
  H.n_done = 0;
  int64_t rw = 0, lw = 0, cb = 0, mb = 0;
  for (Instance* ip : live) {
    Instance& I = *ip;
    if (I.running == 0 || I.hi_groups == 0) continue;
    SrvEntry& E = H.e[H.n++];
    E.inst = I.id;
    E.groups = I.hi_groups;
    E.round_base = rw;
    E.long_base = lw;
    E.commit_base = cb;
    E.commit_blocks = (int32_t)std::min<int64_t>(256, ((int64_t)I.n * kNodeGroup + kBlock - 1) / kBlock);
    if (E.commit_blocks < 1) E.commit_blocks = 1;
    E.mark_base = mb;
    E.mark_blocks = I.bt.row_mark ? (int32_t)std::min<int64_t>(
                                        256, std::max<int64_t>(1, (I.P.n_pieces + kBlock - 1) / kBlock))
                                  : 0;
    rw += (int64_t)(I.P.n_chunks + I.P.n_segs) * E.groups;
    lw += (int64_t)I.P.n_segs * E.groups * kNodeGroup;
    cb += (int64_t)E.commit_blocks * E.groups;
    mb += (int64_t)E.mark_blocks * E.groups;
  }
  H.round_total = rw;
  H.long_total = lw;
  H.commit_total = cb;
  H.mark_total = mb;
  if (H.n == 0) return PROP_OK;
  SRV_TRY(hipMemcpyAsync(d_step[ring], &H, offsetof(SrvStep, e) + (size_t)H.n * sizeof(SrvEntry),
                         hipMemcpyHostToDevice, stream));
  for (int k = 0; k < cfg.rounds_per_step; ++k)
    SRV_TRY(launch_srv_round(d_insts, d_step[ring], H, stream));
  SRV_TRY(hipMemcpyAsync(&H, d_step[ring], offsetof(SrvStep, e), hipMemcpyDeviceToHost, stream));
  SRV_TRY(hipEventRecord(step_ev[ring], stream));
  ++steps_queued;
  std::lock_guard<std::mutex> lk(mu);
  ++n_steps;
  return PROP_OK;
}

// Finished steps: every reported slot is unpacked and copied out.
bool prop_server::poll_steps() {
  bool moved = false;
  while (steps_done < steps_queued) {
    const int ring = (int)(steps_done % kStepRing);
    hipError_t q = hipEventQuery(step_ev[ring]);
    if (q == hipErrorNotReady) break;
    if (q != hipSuccess) {
      fail_all(PROP_EDEVICE, hipGetErrorString(q));
      return false;
    }
    const SrvStep& H = *h_step[ring];
    const uint32_t nd = std::min<uint32_t>(H.n_done, (uint32_t)kSrvStepDone);
    for (uint32_t i = 0; i < nd; ++i) {
      const SrvDone& D = H.done[i];
      if (D.inst < 0 || D.inst >= (int32_t)live.size()) continue;
      Instance& I = *live[D.inst];
      if (D.slot < 0 || D.slot >= I.cap) continue;
      Request* r = I.slot_req[D.slot];
      if (!r || r->state != kRunning) continue;
      r->res.status = D.status;
      r->res.rounds = D.rounds;
      const size_t n = (size_t)I.n;
      const int g = D.slot / kNodeGroup, t = D.slot % kNodeGroup;
      SlotGroup& G = I.groups[g];
      double* d = G.d_io + (size_t)t * 2 * n;
      Batch bt = I.bt;
      bt.groups = I.hi_groups;
      bt.nodes = I.hi_groups * kNodeGroup;
      hipError_t e = launch_unpack_batch(I.P, bt, d, d + n, D.slot, 1, stream);
      if (e == hipSuccess) e = hipEventRecord(ev_out, stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(copy, ev_out, 0);
      if (e == hipSuccess && n)
        e = hipMemcpyAsync(G.h_io + (size_t)t * 2 * n, d, 2 * n * sizeof(double),
                           hipMemcpyDeviceToHost, copy);
      if (e == hipSuccess) e = hipEventRecord(G.drain[t], copy);
      if (e != hipSuccess) {
        fail_all(PROP_EDEVICE, hipGetErrorString(e));
        return false;
      }
      r->state = kDraining;
      --I.running;
    }
    ++steps_done;
    moved = true;
  }
  return moved;
}

// Drained slots: results to the request, slot freed.
bool prop_server::poll_drains(Instance& I) {
  bool moved = false;
  const size_t n = (size_t)I.n;
  for (int slot = 0; slot < I.hi_groups * kNodeGroup; ++slot) {
    Request* r = I.slot_req[slot];
    if (!r || r->state != kDraining) continue;
    const int g = slot / kNodeGroup, t = slot % kNodeGroup;
    SlotGroup& G = I.groups[g];
    hipError_t q = hipEventQuery(G.drain[t]);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) {
      fail_all(PROP_EDEVICE, hipGetErrorString(q));
      return false;
    }
    const double* h = G.h_io + (size_t)t * 2 * n;
    int state = kDone, err = 0;
    if (r->res.status == kInvalidInput) {  // screened at submission; kept as a guard
      state = kFailed;
      err = PROP_EINVAL;
    } else if (n) {
      std::memcpy(r->lb.data(), h, n * sizeof(double));
      std::memcpy(r->ub.data(), h + n, n * sizeof(double));
    }
    I.slot_req[slot] = nullptr;
    --G.used;
    finish(r, state, err);
    moved = true;
  }
  return moved;
}

void prop_server::loop() {
  bool device_set = false;
  std::unique_lock<std::mutex> lk(mu);
  while (!stop) {
    for (Request* r : incoming) insts[r->inst]->pending.push_back(r);
    incoming.clear();
    while (live.size() < insts.size()) live.push_back(insts[live.size()].get());
    lk.unlock();
    if (!device_set && !live.empty()) {
      // the thread touches the device only once a problem has been added
      if (hipSetDevice(live[0]->h->device) != hipSuccess)
        fail_all(PROP_EDEVICE, "hipSetDevice failed in the scheduler");
      device_set = true;
    }
    bool moved = false;
    bool busy = false;
    if (!broken) {
      moved |= poll_steps();
      for (Instance* ip : live) {
        if (broken) break;
        Instance& I = *ip;
        moved |= poll_drains(I);
        if (broken) break;
        const int a = admit(I);
        if (a < 0) {
          fail_all(a, g_error.c_str());
          break;
        }
        moved |= a > 0;
      }
      bool running = false;
      for (Instance* ip : live) {
        running |= ip->running > 0;
        busy |= ip->running > 0 || !ip->pending.empty();
        for (Request* r : ip->slot_req) busy |= r && r->state == kDraining;
      }
      busy |= steps_done < steps_queued;
      if (!broken && running && steps_queued - steps_done < (uint64_t)kStepRing) {
        if (queue_step()) fail_all(PROP_EDEVICE, g_error.c_str());
        moved = true;
      }
    }
    lk.lock();
    if (!moved && incoming.empty() && !stop) {
      if (busy)
        cv_work.wait_for(lk, std::chrono::microseconds(20));
      else
        cv_work.wait(lk, [&] { return stop || !incoming.empty(); });
    }
  }
}

extern "C" {

int prop_srv_create(const prop_srv_config* cfg, prop_server** out) {
  if (!cfg || !out) return fail(PROP_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->budget_bytes <= 0) return fail(PROP_EINVAL, "budget_bytes must be > 0");
  if (cfg->max_slots < 0 || cfg->max_slots % kNodeGroup != 0 || cfg->max_slots > (1 << 16))
    return fail(PROP_EINVAL, "max_slots must be a multiple of 8 in [0, 65536]");
  if (cfg->rounds_per_step < 0 || cfg->rounds_per_step > 64)
    return fail(PROP_EINVAL, "rounds_per_step must be in [0, 64]");
  if (cfg->max_pending < 0) return fail(PROP_EINVAL, "max_pending < 0");
  prop_server* s = new (std::nothrow) prop_server();
  if (!s) return fail(PROP_ENOMEM, "host allocation failed");
  s->cfg = *cfg;
  if (!s->cfg.max_slots) s->cfg.max_slots = 256;
  if (!s->cfg.rounds_per_step) s->cfg.rounds_per_step = 1;
  if (!s->cfg.max_pending) s->cfg.max_pending = 1 << 20;
  if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
  try {
    s->worker = std::thread([s] { s->loop(); });
  } catch (...) {
    delete s;
    return fail(PROP_ENOMEM, "cannot start the scheduler thread");
  }
  *out = s;
  g_error.clear();
  return PROP_OK;
}

// Device-wide state of the server, created with its first instance.
static int srv_device_init(prop_server* s) {
  if (s->stream) return PROP_OK;
  const int64_t bytes = kSrvMaxInstances * sizeof(SrvInst) + kStepRing * sizeof(SrvStep);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->device_bytes + bytes > s->cfg.budget_bytes)
      return fail(PROP_ENOMEM, "server state (%lld bytes) exceeds the budget", (long long)bytes);
  }
  HIP_TRY(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&s->ev_out, hipEventDisableTiming));
  HIP_TRY(hipMalloc((void**)&s->d_insts, kSrvMaxInstances * sizeof(SrvInst)));
  for (int i = 0; i < kStepRing; ++i) {
    HIP_TRY(hipMalloc((void**)&s->d_step[i], sizeof(SrvStep)));
    HIP_TRY(hipHostMalloc((void**)&s->h_step[i], sizeof(SrvStep), hipHostMallocDefault));
    std::memset(s->h_step[i], 0, sizeof(SrvStep));
    HIP_TRY(hipEventCreateWithFlags(&s->step_ev[i], hipEventDisableTiming));
  }
  std::lock_guard<std::mutex> lk(s->mu);
  s->device_bytes += bytes;
  s->fixed_bytes += bytes;
  s->peak_bytes = std::max(s->peak_bytes, s->device_bytes);
  return PROP_OK;
}

int prop_srv_add_instance(prop_server* s, prop_problem* p, int32_t* id) {
  if (!s || !p || !id) return fail(PROP_EINVAL, "NULL argument");
  if (p->P.nnz_split) return fail(PROP_EINVAL, "the nnz-split layout runs single bound vectors only");
  if (p->P.store32) return fail(PROP_EINVAL, "the single-precision store runs single bound vectors only");
  HIP_TRY(hipSetDevice(p->device));
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->broken) return fail(s->broken, "server failed: %s", s->broken_msg.c_str());
    if ((int)s->insts.size() >= kSrvMaxInstances)
      return fail(PROP_EINVAL, "a server holds at most %d instances", kSrvMaxInstances);
    if (!s->insts.empty() && s->insts[0]->h->device != p->device)
      return fail(PROP_EINVAL, "every instance of a server must live on one device");
  }
  int rc = srv_device_init(s);
  if (rc) return rc;
  auto I = std::make_unique<Instance>();
  I->h = p;
  I->n = p->n;
  I->cap = s->cfg.max_slots;
  const int32_t cap = I->cap, G8 = cap / kNodeGroup;
  const int32_t segs = p->P.n_segs;
  const bool marks = s->cfg.marking != 0;
  if (marks) {
    // the rows of every variable, uploaded once per problem (its own memory)
    const int rc2 = ensure_mark_data(p);
    if (rc2) return rc2;
  }
  // one allocation: 9 per-slot arrays, partials, the two group tables,
  // control, and with marked rounds the row stamps, changed-variable bitmaps
  // and two flags per group
  const size_t slot_arrays = 9 * (size_t)cap * sizeof(int32_t);
  const size_t part_off = (slot_arrays + 255) & ~(size_t)255;
  const size_t part_bytes = (size_t)(segs > 0 ? segs : 1) * cap * sizeof(SegPartial);
  const size_t table_off = (part_off + part_bytes + 255) & ~(size_t)255;
  const size_t ctrl_off = (table_off + 2 * (size_t)G8 * sizeof(double2*) + 255) & ~(size_t)255;
  const size_t words = ((size_t)(p->n > 0 ? p->n : 1) + kWave - 1) / kWave;
  const size_t rows = (size_t)(p->P.n_rows > 0 ? p->P.n_rows : 1);
  const size_t mark_off = (ctrl_off + sizeof(Ctrl) + 255) & ~(size_t)255;
  const size_t chg_off = (mark_off + (marks ? (size_t)G8 * rows * sizeof(int32_t) : 0) + 255) &
                         ~(size_t)255;
  const size_t flag_off = (chg_off + (marks ? (size_t)G8 * words * sizeof(uint64_t) : 0) + 255) &
                          ~(size_t)255;
  const size_t total = flag_off + (marks ? 2 * (size_t)G8 * sizeof(uint32_t) : 0);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->device_bytes + (int64_t)total > s->cfg.budget_bytes)
      return fail(PROP_ENOMEM, "instance state (%zu bytes) exceeds the remaining budget", total);
  }
  auto cleanup = [&]() {
    if (I->d_state) hipFree(I->d_state);
    if (I->h_table) hipHostFree(I->h_table);
  };
  if (hipMalloc(&I->d_state, total) != hipSuccess) {
    cleanup();
    return fail(PROP_ENOMEM, "hipMalloc(%zu) for instance state failed", total);
  }
  char* base = static_cast<char*>(I->d_state);
  if (hipMemset(base, 0, total) != hipSuccess) {
    cleanup();
    return fail(PROP_EDEVICE, "hipMemset of instance state failed");
  }
  int32_t* arr = reinterpret_cast<int32_t*>(base);
  Batch& bt = I->bt;
  bt.active = reinterpret_cast<uint32_t*>(arr);
  bt.status = arr + cap;
  bt.rounds = arr + 2 * cap;
  bt.changed = reinterpret_cast<uint32_t*>(arr + 3 * cap);
  bt.infeasible = reinterpret_cast<uint32_t*>(arr + 4 * cap);
  bt.invalid = reinterpret_cast<uint32_t*>(arr + 5 * cap);
  bt.maxr = arr + 6 * cap;
  bt.live = reinterpret_cast<uint32_t*>(arr + 7 * cap);
  bt.tiny = reinterpret_cast<uint32_t*>(arr + 8 * cap);
  bt.partials = reinterpret_cast<SegPartial*>(base + part_off);
  I->d_table = reinterpret_cast<double2**>(base + table_off);
  bt.gA = I->d_table;
  bt.gB = I->d_table + G8;
  bt.nodes = cap;
  bt.groups = G8;
  if (marks) {
    bt.row_mark = reinterpret_cast<int32_t*>(base + mark_off);
    bt.chg = reinterpret_cast<uint64_t*>(base + chg_off);
    bt.gall = reinterpret_cast<uint32_t*>(base + flag_off);
    bt.gcnt = bt.gall + G8;
  }
  I->P = p->P;
  I->P.ctrl = reinterpret_cast<Ctrl*>(base + ctrl_off);
  I->groups.resize(G8);
  I->slot_req.assign(cap, nullptr);
  I->fixed_bytes = (int64_t)total;
  if (hipHostMalloc((void**)&I->h_table, 2 * (size_t)G8 * sizeof(double2*),
                    hipHostMallocDefault) != hipSuccess) {
    cleanup();
    return fail(PROP_ENOMEM, "pinned host allocation failed");
  }
  std::memset(I->h_table, 0, 2 * (size_t)G8 * sizeof(double2*));
  std::lock_guard<std::mutex> lk(s->mu);
  I->id = (int32_t)s->insts.size();
  // the descriptor the serving kernels read; written before the instance is
  // visible to the scheduler, so no queued kernel can read this entry yet
  SrvInst desc;
  desc.P = I->P;
  desc.bt = I->bt;
  if (hipMemcpy(s->d_insts + I->id, &desc, sizeof(SrvInst), hipMemcpyHostToDevice) != hipSuccess) {
    cleanup();
    return fail(PROP_EDEVICE, "upload of the instance descriptor failed");
  }
  s->device_bytes += (int64_t)total;
  s->fixed_bytes += (int64_t)total;
  s->peak_bytes = std::max(s->peak_bytes, s->device_bytes);
  *id = I->id;
  s->insts.push_back(std::move(I));
  g_error.clear();
  return PROP_OK;
}

int prop_srv_submit(prop_server* s, int32_t id, const double* lb, const double* ub,
                    int32_t max_rounds, int64_t* ticket) {
  if (!s || !ticket) return fail(PROP_EINVAL, "NULL argument");
  if (max_rounds < 0) return fail(PROP_EINVAL, "max_rounds < 0");
  int32_t n;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (id < 0 || id >= (int32_t)s->insts.size()) return fail(PROP_EINVAL, "unknown instance %d", id);
    n = s->insts[id]->n;
    // the state of the server and of every instance is never released: a
    // group must fit beside it, or the request could never be admitted
    if (group_bytes(n) + s->fixed_bytes > s->cfg.budget_bytes)
      return fail(PROP_ENOMEM,
                  "one slot group of instance %d (%lld bytes) does not fit the budget beside "
                  "the server's fixed state (%lld bytes)",
                  id, (long long)group_bytes(n), (long long)s->fixed_bytes);
    // refuse before validating and copying the bounds (checked again below)
    if (s->held >= s->cfg.max_pending)
      return fail(PROP_EBUSY, "%lld requests held", (long long)s->held);
  }
  if (n > 0 && (!lb || !ub)) return fail(PROP_EINVAL, "bound arrays are NULL");
  for (int32_t j = 0; j < n; ++j)
    if (!bound_ok(lb[j], ub[j]))
      return fail(PROP_EINVAL,
                  "variable %d: a bound is NaN, +inf as lower, -inf as upper, or beyond 2^200", j);
  auto r = std::make_unique<Request>();
  r->inst = id;
  r->max_rounds = max_rounds;
  r->lb.assign(lb, lb + n);
  r->ub.assign(ub, ub + n);
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->broken) return fail(s->broken, "server failed: %s", s->broken_msg.c_str());
  if (s->held >= s->cfg.max_pending) return fail(PROP_EBUSY, "%lld requests held", (long long)s->held);
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  if (!s->have_first) {
    s->have_first = true;
    s->t_first = r->t_submit;
  }
  ++s->held;
  ++s->n_submitted;
  ++s->n_queued;
  s->incoming.push_back(r.get());
  s->reqs.emplace(r->ticket, std::move(r));
  s->cv_work.notify_one();
  g_error.clear();
  return PROP_OK;
}

static int take_result(prop_server* s, std::unordered_map<int64_t, std::unique_ptr<Request>>::iterator it,
                       prop_result* out, double* lb, double* ub) {
  Request* r = it->second.get();
  int rc = 1;
  if (r->state == kFailed) {
    rc = fail(r->err ? r->err : PROP_EDEVICE, "request %lld failed%s%s", (long long)r->ticket,
              s->broken ? ": " : "", s->broken ? s->broken_msg.c_str() : "");
  } else {
    if (out) *out = r->res;
    if (lb) std::memcpy(lb, r->lb.data(), r->lb.size() * sizeof(double));
    if (ub) std::memcpy(ub, r->ub.data(), r->ub.size() * sizeof(double));
    g_error.clear();
  }
  s->reqs.erase(it);
  --s->held;
  return rc;
}

int prop_srv_poll(prop_server* s, int64_t ticket, prop_result* out, double* lb, double* ub) {
  if (!s) return fail(PROP_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(PROP_EINVAL, "unknown ticket %lld", (long long)ticket);
  const int st = it->second->state;
  if (st != kDone && st != kFailed) return 0;
  return take_result(s, it, out, lb, ub);
}

int prop_srv_wait(prop_server* s, int64_t ticket, int32_t timeout_ms, prop_result* out, double* lb,
                  double* ub) {
  if (!s) return fail(PROP_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(PROP_EINVAL, "unknown ticket %lld", (long long)ticket);
  Request* r = it->second.get();
  auto ready = [&] { return r->state == kDone || r->state == kFailed; };
  if (timeout_ms < 0)
    s->cv_done.wait(lk, ready);
  else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
    return 0;
  return take_result(s, it, out, lb, ub);
}

int prop_srv_get_stats(prop_server* s, prop_srv_stats* out) {
  if (!s || !out) return fail(PROP_EINVAL, "NULL argument");
  std::vector<double> lat;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    *out = prop_srv_stats{};
    out->submitted = s->n_submitted;
    out->completed = s->n_completed;
    out->queued = s->n_queued;
    out->running = s->n_running;
    out->device_bytes = s->device_bytes;
    out->peak_device_bytes = s->peak_bytes;
    out->steps = s->n_steps;
    lat = s->lat_ms;
    if (s->have_first && s->n_completed > 0)
      out->wall_s = std::chrono::duration<double>(s->t_last - s->t_first).count();
  }
  if (!lat.empty()) {
    std::sort(lat.begin(), lat.end());
    // nearest-rank percentiles
    auto pct = [&](double q) {
      size_t k = (size_t)std::ceil(q * lat.size());
      return lat[k > 0 ? k - 1 : 0];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    double sum = 0;
    for (double v : lat) sum += v;
    out->mean_ms = sum / lat.size();
    out->max_ms = lat.back();
  }
  out->req_per_s = out->wall_s > 0 ? out->completed / out->wall_s : 0.0;
  return PROP_OK;
}

int prop_srv_reset_stats(prop_server* s) {
  if (!s) return fail(PROP_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  s->n_submitted = s->n_completed = s->n_steps = 0;
  s->lat_ms.clear();
  s->have_first = false;
  s->peak_bytes = s->device_bytes;
  return PROP_OK;
}

void prop_srv_destroy(prop_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  if (!s->insts.empty()) hipSetDevice(s->insts[0]->h->device);
  if (s->stream) hipStreamSynchronize(s->stream);
  if (s->copy) hipStreamSynchronize(s->copy);
  for (auto& up : s->insts) {
    Instance& I = *up;
    for (auto& G : I.groups) release_group(G);
    if (I.d_state) hipFree(I.d_state);
    if (I.h_table) hipHostFree(I.h_table);
  }
  if (s->d_insts) hipFree(s->d_insts);
  for (int i = 0; i < kStepRing; ++i) {
    if (s->d_step[i]) hipFree(s->d_step[i]);
    if (s->h_step[i]) hipHostFree(s->h_step[i]);
    if (s->step_ev[i]) hipEventDestroy(s->step_ev[i]);
  }
  if (s->ev_in) hipEventDestroy(s->ev_in);
  if (s->ev_out) hipEventDestroy(s->ev_out);
  if (s->copy) hipStreamDestroy(s->copy);
  if (s->stream) hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"
