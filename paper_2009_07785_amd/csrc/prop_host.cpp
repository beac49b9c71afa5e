// prop_host.cpp -- host runtime of the propagation library: input checks,
// the device layout (row chunks, long-row segments, variable relabelling),
// device memory, and the round-loop drivers behind the C ABI in prop.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "prop.h"
#include "prop_handle.h"
#include "prop_launch.h"
#include "prop_layout.h"
#include "prop_layout_host.h"

using namespace prop;

namespace prop {

thread_local std::string g_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

}  // namespace prop

namespace {

const double kHugeValue = std::ldexp(1.0, 200);
const double kCoefMin = std::ldexp(1.0, -64);
const double kCoefMax = std::ldexp(1.0, 64);

bool side_ok(double x, bool is_lhs) {
  if (std::isnan(x)) return false;
  if (std::isinf(x)) return is_lhs ? x < 0 : x > 0;
  return std::fabs(x) <= kHugeValue;
}

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
};

}  // namespace

namespace {

template <typename T>
int dev_alloc(prop_problem* p, T** out, size_t count) {
  size_t bytes = sizeof(T) * (count > 0 ? count : 1);
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, bytes);
  if (e != hipSuccess)
    return fail(PROP_ENOMEM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
  p->allocs.push_back(ptr);
  p->device_bytes += (int64_t)bytes;
  *out = static_cast<T*>(ptr);
  return PROP_OK;
}

template <typename T>
int dev_upload(prop_problem* p, T** out, const std::vector<T>& host) {
  int rc = dev_alloc(p, out, host.size());
  if (rc) return rc;
  if (!host.empty()) HIP_TRY(hipMemcpy(*out, host.data(), sizeof(T) * host.size(), hipMemcpyHostToDevice));
  return PROP_OK;
}

// Destroys the graph driver's captured rounds (single runs and batches).
void drop_batch_graphs(prop_problem* p) {
  for (auto& g : p->bgexec)
    if (g) hipGraphExecDestroy(g);
  p->bgexec[0] = p->bgexec[1] = nullptr;
  p->bgraph_nodes = -1;
}

void drop_graphs(prop_problem* p) {
  for (auto& g : p->gexec)
    if (g) hipGraphExecDestroy(g);
  p->gexec[0] = p->gexec[1] = nullptr;
  drop_batch_graphs(p);
}

void release(prop_problem* p) {
  if (!p) return;
  for (void* a : p->allocs) hipFree(a);
  p->allocs.clear();
  if (p->h_ctrl) hipHostFree(p->h_ctrl);
  if (p->h_done) hipHostFree(p->h_done);
  for (auto& e : p->ev)
    if (e) hipEventDestroy(e);
  for (auto& e : p->ev_batch)
    if (e) hipEventDestroy(e);
  for (auto& e : p->kev)
    if (e) hipEventDestroy(e);
  for (void* a : p->batch_allocs) hipFree(a);
  for (void* a : p->mark_allocs) hipFree(a);
  if (p->h_bstatus) hipHostFree(p->h_bstatus);
  if (p->h_brounds) hipHostFree(p->h_brounds);
  if (p->d_bstage_lb) hipFree(p->d_bstage_lb);
  if (p->d_bstage_ub) hipFree(p->d_bstage_ub);
  drop_graphs(p);
  if (p->cap_stream) hipStreamDestroy(p->cap_stream);
  delete p;
}

int validate(const prop_csr* A, const double* lhs, const double* rhs, const uint8_t* vartype,
             const prop_params* prm) {
  if (!A) return fail(PROP_EINVAL, "matrix is NULL");
  if (A->m < 0 || A->n < 0) return fail(PROP_EINVAL, "negative dimension");
  if (A->m > 0 && (!A->row_ptr || !lhs || !rhs))
    return fail(PROP_EINVAL, "row arrays are NULL");
  if (A->n > 0 && !vartype) return fail(PROP_EINVAL, "vartype is NULL");
  if (A->m == 0 && A->row_ptr == nullptr) {
    if (A->nnz != 0) return fail(PROP_EINVAL, "nnz without rows");
  } else {
    if (A->row_ptr[0] != 0) return fail(PROP_EINVAL, "row_ptr[0] != 0");
    for (int32_t i = 0; i < A->m; ++i)
      if (A->row_ptr[i + 1] < A->row_ptr[i]) return fail(PROP_EINVAL, "row_ptr decreases at row %d", i);
    if (A->row_ptr[A->m] != A->nnz) return fail(PROP_EINVAL, "row_ptr[m] != nnz");
  }
  if (A->nnz > 0 && (!A->col_idx || !A->vals)) return fail(PROP_EINVAL, "entry arrays are NULL");
  std::vector<int32_t> last(A->n > 0 ? A->n : 1, -1);
  for (int32_t i = 0; i < A->m; ++i) {
    for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) {
      const int32_t j = A->col_idx[k];
      if (j < 0 || j >= A->n) return fail(PROP_EINVAL, "column %d out of range in row %d", j, i);
      if (last[j] == i) return fail(PROP_EINVAL, "column %d repeated in row %d", j, i);
      last[j] = i;
      const double a = A->vals[k];
      if (!std::isfinite(a)) return fail(PROP_EINVAL, "non-finite coefficient in row %d", i);
      if (a != 0.0 && (std::fabs(a) < kCoefMin || std::fabs(a) > kCoefMax))
        return fail(PROP_EINVAL, "coefficient magnitude outside [2^-64, 2^64] in row %d", i);
    }
    if (!side_ok(lhs[i], true)) return fail(PROP_EINVAL, "invalid lhs in row %d", i);
    if (!side_ok(rhs[i], false)) return fail(PROP_EINVAL, "invalid rhs in row %d", i);
  }
  for (int32_t j = 0; j < A->n; ++j)
    if (vartype[j] > 1) return fail(PROP_EINVAL, "vartype[%d] is neither 0 nor 1", j);
  if (prm) {
    if (!(prm->eps_int >= 0.0 && prm->eps_int < 0.5))
      return fail(PROP_EINVAL, "eps_int must lie in [0, 0.5)");
    if (!(prm->cont_rel_tol >= 0.0 && std::isfinite(prm->cont_rel_tol)))
      return fail(PROP_EINVAL, "cont_rel_tol must be finite and >= 0");
    if (prm->steps != 0 && prm->steps != 4 && prm->steps != 8 && prm->steps != 16)
      return fail(PROP_EINVAL, "params.steps must be 0, 4, 8 or 16");
    if (prm->layout != 0 && prm->layout != 1) return fail(PROP_EINVAL, "params.layout must be 0 or 1");
    if (!(prm->feas_tol >= 0.0 && std::isfinite(prm->feas_tol)))
      return fail(PROP_EINVAL, "feas_tol must be finite and >= 0");
  }
  return PROP_OK;
}

// Builds the device layout (prop_layout_host.cpp) and uploads it.
int build_layout(prop_problem* p, const prop_csr* A, const double* lhs, const double* rhs,
                 const uint8_t* vartype) {
  const int32_t n = A->n;
  HostLayout L;
  std::string err;
  if (!layout_build(A, lhs, rhs, vartype, p->steps, &L, &err, p->params.layout))
    return fail(PROP_EINVAL, "%s", err.c_str());
  p->nnz = L.nnz;
  p->nnz_stored = L.stored;
  p->instance_infeasible = L.instance_infeasible;
  p->n_long_rows = L.n_long_rows;
  p->h_var_ptr = std::move(L.var_ptr);
  p->h_var_rows = std::move(L.var_rows);
  const std::vector<double>& h_vals = L.vals;
  const std::vector<int32_t>& h_cols = L.cols;
  const std::vector<ChunkDesc>& h_chunks = L.chunks;
  const std::vector<SegDesc>& h_segs = L.segs;
  const std::vector<double>& h_lhs = L.lhs;
  const std::vector<double>& h_rhs = L.rhs;
  const std::vector<uint8_t>& vtype = L.vtype;
  const std::vector<int32_t>& perm = L.perm;
  const int64_t n_rows_internal = L.n_rows;
  Problem& P = p->P;
  int rc;
  double* d_vals;
  int32_t* d_cols;
  ChunkDesc* d_chunks;
  SegDesc* d_segs;
  double *d_lhs, *d_rhs;
  uint8_t* d_vtype;
  int32_t* d_perm;
  if ((rc = dev_upload(p, &d_vals, h_vals))) return rc;
  if ((rc = dev_upload(p, &d_cols, h_cols))) return rc;
  if ((rc = dev_upload(p, &d_chunks, h_chunks))) return rc;
  if ((rc = dev_upload(p, &d_segs, h_segs))) return rc;
  {
    std::vector<int32_t> firsts;
    for (size_t q = 0; q < h_segs.size(); ++q)
      if (h_segs[q].first == (int32_t)q) firsts.push_back((int32_t)q);
    if (!firsts.empty() && (rc = dev_upload(p, &p->d_long_first, firsts))) return rc;
    p->n_long = (int32_t)firsts.size();
  }
  if ((rc = dev_upload(p, &d_lhs, h_lhs))) return rc;
  if ((rc = dev_upload(p, &d_rhs, h_rhs))) return rc;
  if ((rc = dev_upload(p, &d_vtype, vtype))) return rc;
  if ((rc = dev_upload(p, &d_perm, perm))) return rc;
  uint8_t* d_wflags = nullptr;
  if (p->params.layout == 1 && (rc = dev_upload(p, &d_wflags, L.wave_flags))) return rc;
  SegPartial* d_part;
  if ((rc = dev_alloc(p, &d_part, h_segs.size()))) return rc;
  double2 *b0, *b1;
  if ((rc = dev_alloc(p, &b0, (size_t)n))) return rc;
  // the candidate target is followed by its touch bytes, zero to start
  const size_t b1_pairs = (size_t)(n > 0 ? n : 1);
  if ((rc = dev_alloc(p, &b1, b1_pairs + touch_bytes(n) / sizeof(double2)))) return rc;
  HIP_TRY(hipMemset(b1 + b1_pairs, 0, touch_bytes(n)));
  uint16_t* codes;
  if ((rc = dev_alloc(p, &codes, (size_t)(n > 0 ? n : 1)))) return rc;
  const int32_t n_hot = L.n_hot;
  double2* stripes;
  if ((rc = dev_alloc(p, &stripes, (size_t)kStripes * (n_hot > 0 ? n_hot : 1)))) return rc;
  Ctrl* d_ctrl;
  if ((rc = dev_alloc(p, &d_ctrl, 1))) return rc;
  HIP_TRY(hipMemset(d_ctrl, 0, sizeof(Ctrl)));
  uint64_t* d_grp;
  if ((rc = dev_alloc(p, &d_grp, (size_t)kCommitGroups * kGroupWordStride))) return rc;
  HIP_TRY(hipMemset(d_grp, 0, sizeof(uint64_t) * kCommitGroups * kGroupWordStride));
  if ((rc = dev_alloc(p, &p->d_stage_lb, (size_t)n))) return rc;
  if ((rc = dev_alloc(p, &p->d_stage_ub, (size_t)n))) return rc;

  P.vals = d_vals;
  P.n_rows = (int32_t)n_rows_internal;
  P.marking = 0;
  P.cols = d_cols;
  P.chunks = d_chunks;
  P.segs = d_segs;
  P.partials = d_part;
  P.lhs = d_lhs;
  P.rhs = d_rhs;
  P.vtype = d_vtype;
  P.perm = d_perm;
  P.n_chunks = (int32_t)h_chunks.size();
  P.n_segs = (int32_t)h_segs.size();
  P.n = n;
  P.instance_infeasible = p->instance_infeasible ? 1 : 0;
  P.nnz_split = p->params.layout == 1 ? 1 : 0;
  P.wave_flags = d_wflags;
  P.bnd[0] = b0;
  P.bnd[1] = b1;
  P.codes = codes;
  P.b32 = nullptr;  // allocated by the first prop_set_store(p, 32)
  P.store32 = 0;
  P.stripes = stripes;
  P.n_hot = n_hot;
  P.ctrl = d_ctrl;
  P.commit_grp = d_grp;
  P.eps_int = p->params.eps_int;
  P.cont_rel_tol = p->params.cont_rel_tol;
  P.feas_tol = p->params.feas_tol;
  return PROP_OK;
}

// Queues round r, bracketing its matrix kernel with events when asked to.
int queue_round(prop_problem* p, int r, int32_t max_rounds, hipStream_t s) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (p->kernel_timing) {
    const size_t need = 2 * (size_t)r;
    while (p->kev.size() < need) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      p->kev.push_back(e);
    }
    e0 = p->kev[2 * (r - 1)];
    e1 = p->kev[2 * (r - 1) + 1];
    p->kev_used = r;
  }
  HIP_TRY(launch_round(p->P, s, e0, e1));
  return PROP_OK;
}

// Graph driver: batch_rounds rounds plus the copy of the done flag into
// h_done[slot], captured once per slot and replayed.  The launches carry
// the problem by value, so a change of the marking switch recaptures.
int ensure_graphs(prop_problem* p) {
  if (p->gexec[0] && p->graph_marking == p->P.marking) return PROP_OK;
  drop_graphs(p);
  if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  for (int slot = 0; slot < 2; ++slot) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < p->batch_rounds && e == hipSuccess; ++k)
      e = launch_round(p->P, p->cap_stream, nullptr, nullptr);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&p->h_done[slot], &p->P.ctrl->done, sizeof(uint32_t),
                         hipMemcpyDeviceToHost, p->cap_stream);
    const hipError_t e2 = hipStreamEndCapture(p->cap_stream, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->gexec[slot], g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    if (e != hipSuccess) {
      drop_graphs(p);
      return fail(PROP_EDEVICE, "round graph capture failed: %s", hipGetErrorString(e));
    }
  }
  p->graph_marking = p->P.marking;
  return PROP_OK;
}

// The same for batches of `bt.nodes` nodes (the batch kernels carry the
// workspace by value: a new workspace or node count recaptures).
int ensure_batch_graphs(prop_problem* p, const Batch& bt) {
  const int32_t marking = bt.row_mark ? 1 : 0;
  if (p->bgexec[0] && p->bgraph_nodes == bt.nodes && p->bgraph_marking == marking) return PROP_OK;
  drop_batch_graphs(p);
  if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  for (int slot = 0; slot < 2; ++slot) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < p->batch_rounds && e == hipSuccess; ++k)
      e = launch_round_batch(p->P, bt, p->cap_stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&p->h_done[slot], &p->P.ctrl->done, sizeof(uint32_t),
                         hipMemcpyDeviceToHost, p->cap_stream);
    const hipError_t e2 = hipStreamEndCapture(p->cap_stream, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->bgexec[slot], g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    if (e != hipSuccess) {
      drop_batch_graphs(p);
      return fail(PROP_EDEVICE, "batch round graph capture failed: %s", hipGetErrorString(e));
    }
  }
  p->bgraph_nodes = bt.nodes;
  p->bgraph_marking = marking;
  return PROP_OK;
}

int run_loop(prop_problem* p, int32_t max_rounds, hipStream_t s) {
  const Problem& P = p->P;
  p->kev_used = 0;
  hipError_t e;
  switch (p->loop_mode) {
    case PROP_LOOP_PERSISTENT: {
      // no more blocks than the work needs: one wave per chunk or segment
      // and about four variables per commit thread; every block takes part
      // in every grid barrier, so idle blocks only add to their cost
      const int64_t items = (int64_t)P.n_chunks + P.n_segs;
      const int64_t want =
          std::max<int64_t>({(items + kWavesPerBlock - 1) / kWavesPerBlock,
                             ((int64_t)P.n + 4 * kBlock - 1) / (4 * kBlock), (int64_t)1});
      const int grid = (int)std::min<int64_t>(p->grid, want);
      e = launch_persistent(P, max_rounds, grid, s);
      if (e != hipSuccess)
        return fail(PROP_EDEVICE, "cooperative launch failed: %s", hipGetErrorString(e));
      return PROP_OK;
    }
    case PROP_LOOP_STREAM: {
      // Rounds are queued in batches; after each batch the device's done
      // flag is copied to pinned memory behind an event.  The host waits for
      // batch i only after batch i+1 is queued, so the GPU never idles on
      // the host, and at most two batches of early-exit launches follow
      // convergence.
      HIP_TRY(launch_start(P, max_rounds, s));
      if (P.marking && P.parent) HIP_TRY(launch_seed(P, s));
      int slot = 0;
      bool pending[2] = {false, false};
      for (int r = 1; r <= max_rounds;) {
        const int last = std::min(max_rounds, r + p->batch_rounds - 1);
        for (; r <= last; ++r) {
          const int rc = queue_round(p, r, max_rounds, s);
          if (rc) return rc;
        }
        HIP_TRY(hipMemcpyAsync(&p->h_done[slot], &P.ctrl->done, sizeof(uint32_t),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(p->ev_batch[slot], s));
        pending[slot] = true;
        slot ^= 1;
        if (pending[slot]) {
          HIP_TRY(hipEventSynchronize(p->ev_batch[slot]));
          pending[slot] = false;
          if (p->h_done[slot] == 1) break;
        }
      }
      return PROP_OK;
    }
    case PROP_LOOP_GRAPH_ALL: {
      // every replay the round limit may need, queued before any wait: the
      // round loop runs without the host (rounds after the end exit at once)
      HIP_TRY(launch_start(P, max_rounds, s));
      if (P.marking && P.parent) HIP_TRY(launch_seed(P, s));
      const int rc = ensure_graphs(p);
      if (rc) return rc;
      for (int r = 1, slot = 0; r <= max_rounds; r += p->batch_rounds, slot ^= 1)
        HIP_TRY(hipGraphLaunch(p->gexec[slot], s));
      return PROP_OK;
    }
    case PROP_LOOP_GRAPH: {
      // as the stream driver, with each batch one replay of a captured graph
      // (rounds past the limit find the done flag set and exit at once)
      HIP_TRY(launch_start(P, max_rounds, s));
      if (P.marking && P.parent) HIP_TRY(launch_seed(P, s));
      const int rc = ensure_graphs(p);
      if (rc) return rc;
      int slot = 0;
      bool pending[2] = {false, false};
      for (int r = 1; r <= max_rounds; r += p->batch_rounds) {
        HIP_TRY(hipGraphLaunch(p->gexec[slot], s));
        HIP_TRY(hipEventRecord(p->ev_batch[slot], s));
        pending[slot] = true;
        slot ^= 1;
        if (pending[slot]) {
          HIP_TRY(hipEventSynchronize(p->ev_batch[slot]));
          pending[slot] = false;
          if (p->h_done[slot] == 1) break;
        }
      }
      return PROP_OK;
    }
    default:
      HIP_TRY(launch_start(P, max_rounds, s));
      if (P.marking && P.parent) HIP_TRY(launch_seed(P, s));
      for (int r = 1; r <= max_rounds; ++r) {
        const int rc = queue_round(p, r, max_rounds, s);
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(&p->h_ctrl->done, &P.ctrl->done, sizeof(uint32_t),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (p->h_ctrl->done == 1) break;
      }
      return PROP_OK;
  }
}

// Makes the batch workspace hold at least `nodes` nodes.
int ensure_batch(prop_problem* p, int32_t nodes) {
  if (nodes <= p->batch_capacity) return PROP_OK;
  drop_batch_graphs(p);
  for (void* a : p->batch_allocs) hipFree(a);
  p->batch_allocs.clear();
  if (p->h_bstatus) hipHostFree(p->h_bstatus);
  if (p->h_brounds) hipHostFree(p->h_brounds);
  p->h_bstatus = p->h_brounds = nullptr;
  p->batch_capacity = 0;
  const int32_t groups = (nodes + kNodeGroup - 1) / kNodeGroup;
  const size_t pairs = (size_t)groups * kNodeGroup * (size_t)(p->n > 0 ? p->n : 1);
  auto alloc = [&](void** ptr, size_t bytes) -> int {
    hipError_t e = hipMalloc(ptr, bytes > 0 ? bytes : 1);
    if (e != hipSuccess)
      return fail(PROP_ENOMEM, "batch workspace hipMalloc(%zu bytes): %s", bytes,
                  hipGetErrorString(e));
    p->batch_allocs.push_back(*ptr);
    return PROP_OK;
  };
  Batch b{};
  int rc;
  double2 *A = nullptr, *B = nullptr;
  double2** tables = nullptr;
  // group g's [n][8] block of B is followed by its touch bytes
  const size_t per_group = (size_t)kNodeGroup * (size_t)(p->n > 0 ? p->n : 1);
  const size_t per_group_b = per_group + touch_bytes(p->n) / sizeof(double2);
  if ((rc = alloc((void**)&A, pairs * sizeof(double2)))) return rc;
  if ((rc = alloc((void**)&B, (size_t)groups * per_group_b * sizeof(double2)))) return rc;
  HIP_TRY(hipMemset(B, 0, (size_t)groups * per_group_b * sizeof(double2)));
  if ((rc = alloc((void**)&tables, 2 * (size_t)groups * sizeof(double2*)))) return rc;
  {
    std::vector<double2*> h((size_t)2 * groups);
    for (int32_t g = 0; g < groups; ++g) {
      h[g] = A + g * per_group;
      h[groups + g] = B + g * per_group_b;
    }
    HIP_TRY(hipMemcpy(tables, h.data(), h.size() * sizeof(double2*), hipMemcpyHostToDevice));
    b.gA = tables;
    b.gB = tables + groups;
  }
  if ((rc = alloc((void**)&b.partials,
                  (size_t)(p->P.n_segs > 0 ? p->P.n_segs : 1) * nodes * sizeof(SegPartial))))
    return rc;
  if (p->P.n_segs > 0 &&
      (rc = alloc((void**)&b.row_state, (size_t)p->P.n_segs * nodes * kRowStateBytes)))
    return rc;
  b.long_first = p->d_long_first;
  b.n_long = p->n_long;
  if ((rc = alloc((void**)&b.active, nodes * sizeof(uint32_t)))) return rc;
  if ((rc = alloc((void**)&b.status, nodes * sizeof(int32_t)))) return rc;
  if ((rc = alloc((void**)&b.rounds, nodes * sizeof(int32_t)))) return rc;
  if ((rc = alloc((void**)&b.changed, nodes * sizeof(uint32_t)))) return rc;
  if ((rc = alloc((void**)&b.infeasible, nodes * sizeof(uint32_t)))) return rc;
  if ((rc = alloc((void**)&b.invalid, nodes * sizeof(uint32_t)))) return rc;
  if ((rc = alloc((void**)&b.maxr, nodes * sizeof(int32_t)))) return rc;
  if ((rc = alloc((void**)&b.tiny, nodes * sizeof(uint32_t)))) return rc;
  if ((rc = alloc((void**)&p->d_bret, nodes * sizeof(int2)))) return rc;
  if ((rc = alloc((void**)&p->d_bmove, nodes * sizeof(int2)))) return rc;
  HIP_TRY(hipMemset(b.invalid, 0, nodes * sizeof(uint32_t)));
  HIP_TRY(hipMemset(b.infeasible, 0, nodes * sizeof(uint32_t)));
  HIP_TRY(hipMemset(b.tiny, 0, nodes * sizeof(uint32_t)));
  if (hipHostMalloc((void**)&p->h_bstatus, nodes * sizeof(int32_t), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&p->h_brounds, nodes * sizeof(int32_t), hipHostMallocDefault) !=
          hipSuccess)
    return fail(PROP_ENOMEM, "pinned host allocation failed");
  p->bt = b;
  p->batch_capacity = nodes;
  return PROP_OK;
}

// Marked batches: row stamps, changed-variable bitmaps and flags for
// `groups` groups, grown on demand (the previous arrays are dropped).
int ensure_batch_marks(prop_problem* p, int32_t groups) {
  if (groups <= p->mark_groups) return PROP_OK;
  drop_batch_graphs(p);
  for (void* a : p->mark_allocs) hipFree(a);
  p->mark_allocs.clear();
  p->mark_groups = 0;
  auto alloc = [&](void** ptr, size_t bytes) -> int {
    hipError_t e = hipMalloc(ptr, bytes > 0 ? bytes : 1);
    if (e != hipSuccess)
      return fail(PROP_ENOMEM, "batch marking hipMalloc(%zu bytes): %s", bytes,
                  hipGetErrorString(e));
    p->mark_allocs.push_back(*ptr);
    return PROP_OK;
  };
  const size_t rows = (size_t)(p->P.n_rows > 0 ? p->P.n_rows : 1);
  const size_t words = (size_t)(p->n + kWave - 1) / kWave + 1;
  int rc;
  void *marks, *chg, *gall, *gcnt;
  if ((rc = alloc(&marks, (size_t)groups * rows * sizeof(int32_t)))) return rc;
  if ((rc = alloc(&chg, (size_t)groups * words * sizeof(uint64_t)))) return rc;
  if ((rc = alloc(&gall, (size_t)groups * sizeof(uint32_t)))) return rc;
  if ((rc = alloc(&gcnt, (size_t)groups * sizeof(uint32_t)))) return rc;
  HIP_TRY(hipMemset(marks, 0, (size_t)groups * rows * sizeof(int32_t)));
  p->mark_groups = groups;
  p->mark_rows = static_cast<int32_t*>(marks);
  p->mark_chg = static_cast<uint64_t*>(chg);
  p->mark_gall = static_cast<uint32_t*>(gall);
  p->mark_gcnt = static_cast<uint32_t*>(gcnt);
  return PROP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// tuning cache: layout steps per matrix shape signature
// ---------------------------------------------------------------------------
namespace {

std::mutex g_tune_mu;
std::map<uint64_t, int32_t> g_tune;  // signature -> steps
bool g_tune_loaded = false;

// FNV-1a over m, n, nnz and the counts of rows per power-of-two length.
uint64_t shape_signature(const prop_csr* A) {
  int64_t hist[40] = {0};
  int64_t nnz = 0;
  for (int32_t i = 0; i < A->m; ++i) {
    int64_t len = 0;
    for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) len += A->vals[k] != 0.0;
    nnz += len;
    int b = 0;
    while (b < 39 && (1ll << b) <= len) ++b;
    ++hist[b];
  }
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t x) {
    for (int q = 0; q < 8; ++q) {
      h ^= (uint64_t)((x >> (8 * q)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  mix(A->m);
  mix(A->n);
  mix(nnz);
  for (int64_t c : hist) mix(c);
  return h;
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("PROP_TUNE_CACHE");
  if (!path || !*path) return;
  std::FILE* f = std::fopen(path, "r");
  if (!f) return;
  unsigned long long sig;
  int steps;
  while (std::fscanf(f, "%llx %d", &sig, &steps) == 2)
    if (steps == 4 || steps == 8 || steps == 16) g_tune[(uint64_t)sig] = steps;
  std::fclose(f);
}

int32_t tune_lookup(uint64_t sig) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(sig);
  return it == g_tune.end() ? 0 : it->second;
}

void tune_store(uint64_t sig, int32_t steps) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tune[sig] = steps;
  const char* path = std::getenv("PROP_TUNE_CACHE");
  if (!path || !*path) return;
  if (std::FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "%016llx %d\n", (unsigned long long)sig, (int)steps);
    std::fclose(f);
  }
}

}  // namespace

// Uploads what marked rounds need (the rows of every variable in pieces for
// the mark kernels, the row stamps, the changed-variable bitmap), once.
int ensure_mark_data(prop_problem* p) {
  if (!p->mark_ready) {
    HIP_TRY(hipSetDevice(p->device));
    Problem& P = p->P;
    int64_t *vp, *poff;
    int32_t *vr, *marks, *pvar;
    uint64_t* bits;
    int rc;
    // pieces of <= kMarkPiece rows of one variable, one mark-kernel thread each
    std::vector<int32_t> h_pvar;
    std::vector<int64_t> h_poff;
    for (int32_t v = 0; v < p->n; ++v)
      for (int64_t q = p->h_var_ptr[v]; q < p->h_var_ptr[(size_t)v + 1]; q += kMarkPiece) {
        h_pvar.push_back(v);
        h_poff.push_back(q);
      }
    if ((rc = dev_upload(p, &vp, p->h_var_ptr))) return rc;
    if ((rc = dev_upload(p, &vr, p->h_var_rows))) return rc;
    if ((rc = dev_upload(p, &pvar, h_pvar))) return rc;
    if ((rc = dev_upload(p, &poff, h_poff))) return rc;
    if ((rc = dev_alloc(p, &marks, (size_t)(P.n_rows > 0 ? P.n_rows : 1)))) return rc;
    HIP_TRY(hipMemset(marks, 0, sizeof(int32_t) * (size_t)(P.n_rows > 0 ? P.n_rows : 1)));
    if ((rc = dev_alloc(p, &bits, (size_t)(p->n + kWave - 1) / kWave + 1))) return rc;
    P.var_ptr = vp;
    P.var_rows = vr;
    P.row_mark = marks;
    P.chg_bits = bits;
    P.piece_var = pvar;
    P.piece_off = poff;
    P.n_pieces = (int64_t)h_pvar.size();
    std::vector<int64_t>().swap(p->h_var_ptr);
    std::vector<int32_t>().swap(p->h_var_rows);
    p->mark_ready = true;
  }
  return PROP_OK;
}

extern "C" {

int prop_create(const prop_csr* A, const double* lhs, const double* rhs, const uint8_t* vartype,
                const prop_params* params, prop_problem** out) {
  if (!out) return fail(PROP_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(A, lhs, rhs, vartype, params);
  if (rc) return rc;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0)
    return fail(PROP_EDEVICE, "no HIP device available (%s)", hipGetErrorString(e));
  prop_problem* p = new (std::nothrow) prop_problem();
  if (!p) return fail(PROP_ENOMEM, "host allocation failed");
  if (params) p->params = *params;
  p->steps = p->params.steps ? p->params.steps : tune_lookup(shape_signature(A));
  if (!p->steps) {
    // untuned shapes: by size, as the autotuner chose on the instances it was
    // measured on (smaller matrices gain from shorter chains per lane)
    const int64_t nnz = A->m > 0 ? A->row_ptr[A->m] : 0;
    p->steps = nnz <= 100000 ? 4 : nnz <= 5000000 ? 8 : kMaxSteps;
  }
  p->m = A->m;
  p->n = A->n;
  if (hipGetDevice(&p->device) != hipSuccess) {
    release(p);
    return fail(PROP_EDEVICE, "hipGetDevice failed");
  }
  rc = build_layout(p, A, lhs, rhs, vartype);
  if (rc) {
    release(p);
    return rc;
  }
  int coop = 0, cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, p->device) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess ||
      persistent_occupancy(&per_cu, p->params.layout == 1) != hipSuccess || cus <= 0 || per_cu <= 0) {
    release(p);
    return fail(PROP_EDEVICE, "device attribute / occupancy query failed");
  }
  p->grid = cus * per_cu;
  if (!coop) p->loop_mode = PROP_LOOP_STREAM;
  if (hipHostMalloc((void**)&p->h_ctrl, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&p->h_done, 4 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
    release(p);
    return fail(PROP_ENOMEM, "pinned host allocation failed");
  }
  for (auto& ev : p->ev)
    if (hipEventCreate(&ev) != hipSuccess) {
      release(p);
      return fail(PROP_EDEVICE, "hipEventCreate failed");
    }
  for (auto& ev : p->ev_batch)
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      release(p);
      return fail(PROP_EDEVICE, "hipEventCreate failed");
    }
  *out = p;
  g_error.clear();
  return PROP_OK;
}

int prop_run_device(prop_problem* p, double* d_lb, double* d_ub, int32_t max_rounds, void* stream,
                    prop_result* out) {
  if (!p || !out) return fail(PROP_EINVAL, "NULL argument");
  if (max_rounds < 0) return fail(PROP_EINVAL, "max_rounds < 0");
  if (p->n > 0 && (!d_lb || !d_ub)) return fail(PROP_EINVAL, "bound arrays are NULL");
  HIP_TRY(hipSetDevice(p->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  // marked rounds need the per-round kernel sequence of the stream / host drivers
  p->P.marking = (p->marking && p->loop_mode != PROP_LOOP_PERSISTENT) ? 1 : 0;
  const Problem& P = p->P;
  HIP_TRY(hipEventRecord(p->ev[0], s));
  HIP_TRY(launch_init(P, s));
  HIP_TRY(launch_pack(P, d_lb, d_ub, s));
  HIP_TRY(hipEventRecord(p->ev[1], s));
  int rc = run_loop(p, max_rounds, s);
  if (rc) {
    hipStreamSynchronize(s);
    return rc;
  }
  HIP_TRY(hipEventRecord(p->ev[2], s));
  HIP_TRY(launch_unpack(P, d_lb, d_ub, s));
  HIP_TRY(hipMemcpyAsync(p->h_ctrl, P.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipEventRecord(p->ev[3], s));
  HIP_TRY(hipStreamSynchronize(s));
  hipEventElapsedTime(&p->last_loop_ms, p->ev[1], p->ev[2]);
  hipEventElapsedTime(&p->last_total_ms, p->ev[0], p->ev[3]);
  p->last_kernel_ms = 0.0;
  // launches queued after the last executed round exit at once; leave them out
  if (p->kev_used > p->h_ctrl->rounds) p->kev_used = p->h_ctrl->rounds;
  for (int r = 0; r < p->kev_used; ++r) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->kev[2 * r], p->kev[2 * r + 1]) == hipSuccess)
      p->last_kernel_ms += ms;
  }
  const Ctrl& C = *p->h_ctrl;
  if (C.invalid) return fail(PROP_EINVAL, "a bound is NaN, +inf as lower, -inf as upper, or beyond 2^200");
  if (C.abort) return fail(PROP_EDEVICE, "grid barrier wait timed out");
  if (C.done != 1) return fail(PROP_EDEVICE, "round loop did not finish (done=%u)", C.done);
  out->status = C.status;
  out->rounds = C.rounds;
  g_error.clear();
  return PROP_OK;
}

int prop_run(prop_problem* p, double* lb, double* ub, int32_t max_rounds, prop_result* out) {
  if (!p || !out) return fail(PROP_EINVAL, "NULL argument");
  if (p->n > 0 && (!lb || !ub)) return fail(PROP_EINVAL, "bound arrays are NULL");
  HIP_TRY(hipSetDevice(p->device));
  const size_t bytes = sizeof(double) * (size_t)p->n;
  if (bytes) {
    HIP_TRY(hipMemcpy(p->d_stage_lb, lb, bytes, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->d_stage_ub, ub, bytes, hipMemcpyHostToDevice));
  }
  int rc = prop_run_device(p, p->d_stage_lb, p->d_stage_ub, max_rounds, nullptr, out);
  if (rc) return rc;
  if (bytes) {
    HIP_TRY(hipMemcpy(lb, p->d_stage_lb, bytes, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ub, p->d_stage_ub, bytes, hipMemcpyDeviceToHost));
  }
  return PROP_OK;
}

namespace {

// Compaction of a running batch, at a point where all queued rounds are
// done: every slot whose node has finished is unpacked into the caller's
// row of that node (its result kept in `res`), and the active nodes of
// slots at or above A (the number of active nodes) move into the free slots
// below A, so the next rounds run over ceil(A / 8) groups instead of all.
// A node's arithmetic does not depend on its slot, so its results do not
// change.  slot_node[k] is the caller's node in slot k, -1 for none.
int compact_batch(prop_problem* p, Batch& bt, std::vector<int32_t>& slot_node,
                  std::vector<prop_result>& res, double* d_lb, double* d_ub, hipStream_t s) {
  const Problem& P = p->P;
  const int S = bt.nodes;
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<uint32_t> active(S);
  std::vector<int32_t> status(S), rounds(S);
  HIP_TRY(hipMemcpy(active.data(), bt.active, S * sizeof(uint32_t), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(status.data(), bt.status, S * sizeof(int32_t), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(rounds.data(), bt.rounds, S * sizeof(int32_t), hipMemcpyDeviceToHost));
  std::vector<int2> ret, mv;
  int A = 0;
  for (int k = 0; k < S; ++k) {
    if (slot_node[k] < 0) continue;
    if (active[k]) {
      ++A;
      continue;
    }
    res[slot_node[k]] = prop_result{status[k], rounds[k]};
    ret.push_back(make_int2(k, slot_node[k]));
    slot_node[k] = -1;
  }
  int src = S - 1;
  for (int h = 0; h < A; ++h) {
    if (slot_node[h] >= 0) continue;
    while (slot_node[src] < 0) --src;  // an active slot >= A exists for every hole < A
    mv.push_back(make_int2(src, h));
    slot_node[h] = slot_node[src];
    slot_node[src] = -1;
    --src;
  }
  if (!ret.empty()) {
    HIP_TRY(hipMemcpy(p->d_bret, ret.data(), ret.size() * sizeof(int2), hipMemcpyHostToDevice));
    HIP_TRY(launch_unpack_slots(P, bt, d_lb, d_ub, p->d_bret, (int)ret.size(), s));
  }
  if (!mv.empty()) {
    HIP_TRY(hipMemcpy(p->d_bmove, mv.data(), mv.size() * sizeof(int2), hipMemcpyHostToDevice));
    HIP_TRY(launch_move_batch(P, bt, p->d_bmove, (int)mv.size(), s));
  }
  bt.nodes = A;
  bt.groups = (A + kNodeGroup - 1) / kNodeGroup;
  return PROP_OK;
}

// The end of a batch run: the rows of the nodes still in slots are
// unpacked, every node's status and rounds are read, the stream is
// synchronised and *out filled.
int finish_batch(prop_problem* p, const Batch& bt, int32_t nodes, double* d_lb, double* d_ub,
                 const std::vector<int32_t>& slot_node, std::vector<prop_result>& res,
                 bool compacted, hipStream_t s, prop_result* out) {
  const Problem& P = p->P;
  HIP_TRY(hipEventRecord(p->ev[2], s));
  if (!compacted) {
    HIP_TRY(launch_unpack_batch(P, bt, d_lb, d_ub, 0, nodes, s));
  } else if (bt.nodes > 0) {
    std::vector<int2> fin;
    for (int k = 0; k < bt.nodes; ++k)
      if (slot_node[k] >= 0) fin.push_back(make_int2(k, slot_node[k]));
    // the stream may still run a compaction's unpack of d_bret
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(p->d_bret, fin.data(), fin.size() * sizeof(int2), hipMemcpyHostToDevice));
    HIP_TRY(launch_unpack_slots(P, bt, d_lb, d_ub, p->d_bret, (int)fin.size(), s));
  }
  if (bt.nodes > 0) {
    HIP_TRY(hipMemcpyAsync(p->h_bstatus, bt.status, bt.nodes * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(p->h_brounds, bt.rounds, bt.nodes * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipEventRecord(p->ev[3], s));
  HIP_TRY(hipStreamSynchronize(s));
  hipEventElapsedTime(&p->last_loop_ms, p->ev[1], p->ev[2]);
  hipEventElapsedTime(&p->last_total_ms, p->ev[0], p->ev[3]);
  p->kev_used = 0;
  p->last_kernel_ms = 0.0;
  for (int k = 0; k < bt.nodes; ++k)
    if (slot_node[k] >= 0) res[slot_node[k]] = prop_result{p->h_bstatus[k], p->h_brounds[k]};
  for (int32_t k = 0; k < nodes; ++k)
    if (res[k].status == kInvalidInput)
      return fail(PROP_EINVAL, "node %d: a bound is NaN, +inf as lower, -inf as upper, or beyond 2^200", k);
  for (int32_t k = 0; k < nodes; ++k) out[k] = res[k];
  g_error.clear();
  return PROP_OK;
}

}  // namespace

int prop_run_batch_device(prop_problem* p, int32_t nodes, double* d_lb, double* d_ub,
                          int32_t max_rounds, void* stream, prop_result* out) {
  if (!p || !out) return fail(PROP_EINVAL, "NULL argument");
  if (nodes < 1) return fail(PROP_EINVAL, "nodes < 1");
  if (max_rounds < 0) return fail(PROP_EINVAL, "max_rounds < 0");
  if (p->n > 0 && (!d_lb || !d_ub)) return fail(PROP_EINVAL, "bound arrays are NULL");
  if (p->P.nnz_split) return fail(PROP_EINVAL, "the nnz-split layout runs single bound vectors only");
  if (p->P.store32) return fail(PROP_EINVAL, "the single-precision store runs single bound vectors only");
  HIP_TRY(hipSetDevice(p->device));
  int rc = ensure_batch(p, nodes);
  if (rc) return rc;
  const int32_t groups = (nodes + kNodeGroup - 1) / kNodeGroup;
  if (p->marking) {
    if ((rc = ensure_mark_data(p))) return rc;
    if ((rc = ensure_batch_marks(p, groups))) return rc;
  }
  p->P.marking = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Problem& P = p->P;
  Batch bt = p->bt;
  bt.nodes = nodes;
  bt.groups = groups;
  if (p->marking) {
    // marked rounds per group (rows of variables changed in any of the
    // group's nodes); with a parent, round 1 is marked too
    bt.row_mark = p->mark_rows;
    bt.chg = p->mark_chg;
    bt.gall = p->mark_gall;
    bt.gcnt = p->mark_gcnt;
  }
  HIP_TRY(hipEventRecord(p->ev[0], s));
  HIP_TRY(launch_init(P, s));
  HIP_TRY(hipMemsetAsync(bt.invalid, 0, nodes * sizeof(uint32_t), s));
  HIP_TRY(hipMemsetAsync(bt.infeasible, 0, nodes * sizeof(uint32_t), s));
  HIP_TRY(launch_pack_batch(P, bt, d_lb, d_ub, 0, nodes, s));
  HIP_TRY(launch_start_batch(P, bt, max_rounds, 0, nodes, true, s));
  if (bt.row_mark && P.parent) HIP_TRY(launch_seed_batch(P, bt, s));
  HIP_TRY(hipEventRecord(p->ev[1], s));
  std::vector<int32_t> slot_node(nodes);
  std::iota(slot_node.begin(), slot_node.end(), 0);
  std::vector<prop_result> res(nodes, prop_result{kInvalidInput, 0});
  bool compacted = false;
  if (p->loop_mode == PROP_LOOP_GRAPH_ALL) {
    // every replay the round limit may need, queued before any wait: no
    // host read and no compaction (finished nodes leave their groups, which
    // keep running with the rest)
    rc = ensure_batch_graphs(p, bt);
    if (rc) return rc;
    for (int r = 1, slot = 0; r <= max_rounds; r += p->batch_rounds, slot ^= 1)
      HIP_TRY(hipGraphLaunch(p->bgexec[slot], s));
    return finish_batch(p, bt, nodes, d_lb, d_ub, slot_node, res, compacted, s, out);
  }
  // rounds in batches; the done flag and the active-node count are read one
  // batch behind (see the stream driver of single runs).  When the active
  // nodes would fit in fewer groups, the batch is compacted.
  bool graph = p->loop_mode == PROP_LOOP_GRAPH;
  if (graph) {
    rc = ensure_batch_graphs(p, bt);
    if (rc) return rc;
  }
  int r = 1;
  if (bt.groups > 1 && max_rounds >= 1) {
    // round 1 on its own: nodes whose input domains or first round make
    // them infeasible leave at once, and the batch is compacted before the
    // remaining rounds instead of a batch of rounds later
    HIP_TRY(launch_round_batch(P, bt, s));
    HIP_TRY(hipMemcpyAsync(&p->h_done[0], &P.ctrl->done, sizeof(uint32_t), hipMemcpyDeviceToHost,
                           s));
    HIP_TRY(hipMemcpyAsync(&p->h_done[2], &P.ctrl->active_nodes, sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    r = 2;
    const uint32_t act = p->h_done[2];
    if (p->h_done[0] == 1) {
      r = max_rounds + 1;  // every node has finished
    } else if (act > 0 && (act + kNodeGroup - 1) / kNodeGroup < (uint32_t)bt.groups) {
      rc = compact_batch(p, bt, slot_node, res, d_lb, d_ub, s);
      if (rc) return rc;
      compacted = true;
      graph = false;
      if (bt.nodes == 0) r = max_rounds + 1;
    }
  }
  int slot = 0;
  bool pending[2] = {false, false};
  for (; r <= max_rounds;) {
    const int last = std::min(max_rounds, r + p->batch_rounds - 1);
    if (graph) {
      // one replay: batch_rounds rounds (past the limit they exit at once)
      HIP_TRY(hipGraphLaunch(p->bgexec[slot], s));
      r = last + 1;
    } else {
      for (; r <= last; ++r) HIP_TRY(launch_round_batch(P, bt, s));
      HIP_TRY(hipMemcpyAsync(&p->h_done[slot], &P.ctrl->done, sizeof(uint32_t),
                             hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipMemcpyAsync(&p->h_done[2 + slot], &P.ctrl->active_nodes, sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(p->ev_batch[slot], s));
    pending[slot] = true;
    slot ^= 1;
    if (pending[slot]) {
      HIP_TRY(hipEventSynchronize(p->ev_batch[slot]));
      pending[slot] = false;
      if (p->h_done[slot] == 1) break;
      const uint32_t act = p->h_done[2 + slot];
      if (r <= max_rounds && act > 0 &&
          (act + kNodeGroup - 1) / kNodeGroup < (uint32_t)bt.groups) {
        rc = compact_batch(p, bt, slot_node, res, d_lb, d_ub, s);
        if (rc) return rc;
        compacted = true;
        graph = false;  // the captured rounds are for the old group count
        pending[0] = pending[1] = false;
        if (bt.nodes == 0) break;
      }
    }
  }
  return finish_batch(p, bt, nodes, d_lb, d_ub, slot_node, res, compacted, s, out);
}


int prop_run_batch(prop_problem* p, int32_t nodes, double* lb, double* ub, int32_t max_rounds,
                   prop_result* out) {
  if (!p || !out) return fail(PROP_EINVAL, "NULL argument");
  if (nodes < 1) return fail(PROP_EINVAL, "nodes < 1");
  if (p->n > 0 && (!lb || !ub)) return fail(PROP_EINVAL, "bound arrays are NULL");
  if (p->P.store32) return fail(PROP_EINVAL, "the single-precision store runs single bound vectors only");
  HIP_TRY(hipSetDevice(p->device));
  const size_t bytes = sizeof(double) * (size_t)p->n * (size_t)nodes;
  if (nodes > p->bstage_capacity && bytes) {
    if (p->d_bstage_lb) hipFree(p->d_bstage_lb);
    if (p->d_bstage_ub) hipFree(p->d_bstage_ub);
    p->d_bstage_lb = p->d_bstage_ub = nullptr;
    p->bstage_capacity = 0;
    if (hipMalloc((void**)&p->d_bstage_lb, bytes) != hipSuccess ||
        hipMalloc((void**)&p->d_bstage_ub, bytes) != hipSuccess)
      return fail(PROP_ENOMEM, "staging for %d nodes (2 x %zu bytes) failed", nodes, bytes);
    p->bstage_capacity = nodes;
  }
  if (bytes) {
    HIP_TRY(hipMemcpy(p->d_bstage_lb, lb, bytes, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->d_bstage_ub, ub, bytes, hipMemcpyHostToDevice));
  }
  int rc = prop_run_batch_device(p, nodes, p->d_bstage_lb, p->d_bstage_ub, max_rounds, nullptr,
                                 out);
  if (rc) return rc;
  if (bytes) {
    HIP_TRY(hipMemcpy(lb, p->d_bstage_lb, bytes, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ub, p->d_bstage_ub, bytes, hipMemcpyDeviceToHost));
  }
  return PROP_OK;
}

int prop_autotune(const prop_csr* A, const double* lhs, const double* rhs, const uint8_t* vartype,
                  const prop_params* params, const double* lb, const double* ub,
                  int32_t max_rounds, int32_t* steps_out) {
  if (!steps_out) return fail(PROP_EINVAL, "steps_out is NULL");
  if (max_rounds < 0) return fail(PROP_EINVAL, "max_rounds < 0");
  int rc = validate(A, lhs, rhs, vartype, params);
  if (rc) return rc;
  if (A->n > 0 && (!lb || !ub)) return fail(PROP_EINVAL, "bound arrays are NULL");
  const size_t bytes = sizeof(double) * (size_t)A->n;
  double *d_lb = nullptr, *d_ub = nullptr;
  if (bytes) {
    HIP_TRY(hipMalloc((void**)&d_lb, bytes));
    if (hipMalloc((void**)&d_ub, bytes) != hipSuccess) {
      hipFree(d_lb);
      return fail(PROP_ENOMEM, "hipMalloc for the tuning bounds failed");
    }
  }
  prop_params prm = params ? *params : prop_params{1e-6, 1e-6, 1e-6, 0, 0};
  int32_t best = 0;
  double best_ms = 0.0;
  for (int32_t steps : {16, 8, 4}) {
    prm.steps = steps;
    prop_problem* p = nullptr;
    rc = prop_create(A, lhs, rhs, vartype, &prm, &p);
    if (rc) break;
    double t[4];
    for (int k = 0; k < 4 && !rc; ++k) {  // one warm-up run, three timed
      if (bytes) {
        if (hipMemcpy(d_lb, lb, bytes, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d_ub, ub, bytes, hipMemcpyHostToDevice) != hipSuccess)
          rc = fail(PROP_EDEVICE, "copy of the tuning bounds failed");
      }
      prop_result res;
      if (!rc) rc = prop_run_device(p, d_lb, d_ub, max_rounds, nullptr, &res);
      t[k] = p->last_loop_ms;
    }
    prop_destroy(p);
    if (rc) break;
    std::sort(t + 1, t + 4);
    if (!best || t[2] < best_ms) {
      best = steps;
      best_ms = t[2];
    }
  }
  if (d_lb) hipFree(d_lb);
  if (d_ub) hipFree(d_ub);
  if (rc) return rc;
  tune_store(shape_signature(A), best);
  *steps_out = best;
  g_error.clear();
  return PROP_OK;
}

int prop_set_loop(prop_problem* p, int32_t mode) {
  if (!p) return fail(PROP_EINVAL, "NULL problem");
  if (mode != PROP_LOOP_PERSISTENT && mode != PROP_LOOP_STREAM && mode != PROP_LOOP_HOST &&
      mode != PROP_LOOP_GRAPH && mode != PROP_LOOP_GRAPH_ALL)
    return fail(PROP_EINVAL, "unknown loop mode %d", mode);
  p->loop_mode = mode;
  return PROP_OK;
}

int prop_set_marking(prop_problem* p, int32_t enable) {
  if (!p) return fail(PROP_EINVAL, "NULL problem");
  if (enable) {
    const int rc = ensure_mark_data(p);
    if (rc) return rc;
  }
  p->marking = enable != 0;
  return PROP_OK;
}

int prop_set_store(prop_problem* p, int32_t bits) {
  if (!p) return fail(PROP_EINVAL, "NULL problem");
  if (bits != PROP_STORE_F64 && bits != PROP_STORE_F32)
    return fail(PROP_EINVAL, "bound store of %d bits: 64 or 32", bits);
  const int32_t want = bits == PROP_STORE_F32 ? 1 : 0;
  if (want && p->P.nnz_split)
    return fail(PROP_EINVAL, "the single-precision store runs on the layout of length classes");
  if (want == p->P.store32) return PROP_OK;
  HIP_TRY(hipSetDevice(p->device));
  if (want && !p->P.b32) {
    float2* b32 = nullptr;
    const int rc = dev_alloc(p, &b32, (size_t)(p->n > 0 ? p->n : 1));
    if (rc) return rc;
    p->P.b32 = b32;
  }
  // captured rounds hold the old store's kernels; a parent was rounded for
  // the old store
  drop_graphs(p);
  p->P.parent = nullptr;
  p->P.store32 = want;
  return PROP_OK;
}

int prop_set_parent(prop_problem* p, const double* d_lb, const double* d_ub, void* stream) {
  if (!p) return fail(PROP_EINVAL, "NULL problem");
  if (!d_lb && !d_ub) {
    p->P.parent = nullptr;
    return PROP_OK;
  }
  if (p->n > 0 && (!d_lb || !d_ub)) return fail(PROP_EINVAL, "one parent bound array is NULL");
  HIP_TRY(hipSetDevice(p->device));
  int rc = ensure_mark_data(p);
  if (rc) return rc;
  if (!p->d_parent && (rc = dev_alloc(p, &p->d_parent, (size_t)(p->n > 0 ? p->n : 1)))) return rc;
  p->P.parent = nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  p->h_ctrl->invalid = 0;
  HIP_TRY(hipMemcpyAsync(&p->P.ctrl->invalid, &p->h_ctrl->invalid, sizeof(uint32_t),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(launch_set_parent(p->P, p->d_parent, d_lb, d_ub, s));
  HIP_TRY(hipMemcpyAsync(&p->h_ctrl->invalid, &p->P.ctrl->invalid, sizeof(uint32_t),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (p->h_ctrl->invalid)
    return fail(PROP_EINVAL, "parent: a bound is NaN, +inf as lower, -inf as upper, or beyond 2^200");
  p->P.parent = p->d_parent;
  return PROP_OK;
}

int prop_get_info(const prop_problem* p, prop_info* out) {
  if (!p || !out) return fail(PROP_EINVAL, "NULL argument");
  out->m = p->m;
  out->n = p->n;
  out->nnz = p->nnz;
  out->nnz_stored = p->nnz_stored;
  out->n_chunks = p->P.n_chunks;
  out->n_long_rows = p->n_long_rows;
  out->n_segments = p->P.n_segs;
  out->grid_blocks = p->grid;
  out->device_bytes = p->device_bytes;
  out->alg_bytes_round = 12 * p->nnz + 20 * (int64_t)p->m + 33 * (int64_t)p->n + 4;
  out->steps = p->steps;
  out->layout = p->params.layout;
  return PROP_OK;
}

int prop_last_timing(const prop_problem* p, double* loop_ms, double* total_ms) {
  if (!p) return fail(PROP_EINVAL, "NULL problem");
  if (loop_ms) *loop_ms = p->last_loop_ms;
  if (total_ms) *total_ms = p->last_total_ms;
  return PROP_OK;
}

int prop_set_kernel_timing(prop_problem* p, int32_t enable) {
  if (!p) return fail(PROP_EINVAL, "NULL problem");
  p->kernel_timing = enable != 0;
  return PROP_OK;
}

int prop_last_kernel_timing(const prop_problem* p, double* ms, int32_t* launches) {
  if (!p) return fail(PROP_EINVAL, "NULL problem");
  if (ms) *ms = p->last_kernel_ms;
  if (launches) *launches = p->kev_used;
  return PROP_OK;
}

void prop_destroy(prop_problem* p) {
  if (!p) return;
  hipSetDevice(p->device);
  hipDeviceSynchronize();
  release(p);
}

const char* prop_last_error(void) { return g_error.c_str(); }

}  // extern "C"
