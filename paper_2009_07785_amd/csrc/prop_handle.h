// prop_handle.h -- the library's internal view of a problem handle, shared
// by the single-run / batch runtime and the serving engine.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "prop.h"
#include "prop_layout.h"

namespace prop {

// Sets the calling thread's error message and returns `code`.
int fail(int code, const char* fmt, ...);
extern thread_local std::string g_error;

}  // namespace prop

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return prop::fail(e_ == hipErrorOutOfMemory ? PROP_ENOMEM : PROP_EDEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                   \
  } while (0)

// Uploads the rows of every variable for marked rounds (once per problem).
int ensure_mark_data(prop_problem* p);

struct prop_problem {
  int device = 0;
  int32_t m = 0, n = 0;
  int64_t nnz = 0, nnz_stored = 0;
  int32_t n_long_rows = 0;
  int grid = 0;
  int loop_mode = PROP_LOOP_STREAM;
  bool instance_infeasible = false;
  prop_params params{1e-6, 1e-6, 1e-6, 0, 0};
  int32_t steps = prop::kMaxSteps;  // layout: entries per lane of a short row
  prop::Problem P{};
  // device allocations
  std::vector<void*> allocs;
  int64_t device_bytes = 0;
  double* d_stage_lb = nullptr;  // staging for prop_run (host arrays)
  double* d_stage_ub = nullptr;
  prop::Ctrl* h_ctrl = nullptr;        // pinned host copy of the control block
  uint32_t* h_done = nullptr;    // pinned done flags of the stream driver's batches
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_batch[2] = {nullptr, nullptr};
  int batch_rounds = 4;          // rounds queued per batch by the stream driver
  bool kernel_timing = false;    // events around every round-kernel launch
  std::vector<hipEvent_t> kev;   // kev[2r], kev[2r+1] bracket round r's matrix kernel
  int kev_used = 0;              // rounds bracketed in the last run
  double last_kernel_ms = 0.0;
  float last_loop_ms = 0.f, last_total_ms = 0.f;
  // batch workspace (grown on demand, kept until destroy)
  prop::Batch bt{};
  int32_t batch_capacity = 0;
  std::vector<void*> batch_allocs;
  int32_t* h_bstatus = nullptr;  // pinned copies of per-node status / rounds
  int32_t* h_brounds = nullptr;
  int2* d_bret = nullptr;        // batch compaction: (slot, node) lists to unpack
  int2* d_bmove = nullptr;       // and (from slot, to slot) moves, batch capacity each
  int32_t* d_long_first = nullptr;  // first segment of each long row (batch row states)
  int32_t n_long = 0;
  // staging for prop_run_batch (host arrays), grown on demand
  double* d_bstage_lb = nullptr;
  double* d_bstage_ub = nullptr;
  int32_t bstage_capacity = 0;
  // marked rounds: rows of each variable (internal orders), uploaded on the
  // first prop_set_marking(p, 1)
  bool marking = false;
  bool mark_ready = false;
  double2* d_parent = nullptr;   // prop_set_parent's copy (P.parent points here when set)
  // marked batches: per-group row stamps, bitmaps and flags, for
  // mark_groups groups (grown on demand, kept until destroy)
  int32_t mark_groups = 0;
  std::vector<void*> mark_allocs;
  int32_t* mark_rows = nullptr;  // [mark_groups][n_rows]
  uint64_t* mark_chg = nullptr;  // [mark_groups][ceil(n / 64) + 1]
  uint32_t* mark_gall = nullptr; // [mark_groups]
  uint32_t* mark_gcnt = nullptr; // [mark_groups]
  int32_t bgraph_marking = -1;
  // graph driver: one captured batch of rounds per done-flag slot
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;
  int32_t graph_marking = -1;
  hipGraphExec_t bgexec[2] = {nullptr, nullptr};  // batches: rounds of `bgraph_nodes` nodes
  int32_t bgraph_nodes = -1;
  std::vector<int64_t> h_var_ptr;
  std::vector<int32_t> h_var_rows;
};
