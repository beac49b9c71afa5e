// prop_static.hip -- prop_run_batch_device_static: batched branch-and-bound
// nodes (the rounds of prop_run_batch_device) for callers that cannot
// allocate device memory.  The batch workspace lives in `scratch`, a fixed
// device array of the library, instead of memory the call allocates.
//
// In host code `scratch` names a host-side stand-in, not the device array:
// its device address comes from hipGetSymbolAddress, taken once per device
// (each device holds its own copy of the array at its own address) and
// kept in g_scratch; only that address is passed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "prop_device.h"
#include "prop_handle.h"
#include "prop_launch.h"
#include "prop_layout.h"

namespace prop {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device).
int scratch_address(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(PROP_EDEVICE, "device %d out of range", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(PROP_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch[device] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch[device];
  return PROP_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of the workspace regions inside the array.
struct StaticLayout {
  size_t pairs_a, pairs_b, tables, partials, nodes32, results, total;
};

StaticLayout static_layout(int32_t n, int32_t n_segs, int32_t nodes) {
  const size_t groups = (size_t)(nodes + kNodeGroup - 1) / kNodeGroup;
  const size_t pair_bytes = groups * kNodeGroup * (size_t)(n > 0 ? n : 1) * sizeof(double2);
  StaticLayout L;
  size_t off = 0;
  L.pairs_a = off;
  off = align256(off + pair_bytes);
  L.pairs_b = off;  // each group's block followed by its touch bytes
  off = align256(off + pair_bytes + groups * touch_bytes(n));
  L.tables = off;
  off = align256(off + 2 * groups * sizeof(double2*));
  L.partials = off;
  off = align256(off + (size_t)(n_segs > 0 ? n_segs : 1) * nodes * sizeof(SegPartial));
  L.nodes32 = off;  // eight per-node 32-bit arrays
  off = align256(off + 8 * (size_t)nodes * sizeof(uint32_t));
  L.results = off;  // (status, rounds) per node for the copy to the caller
  off = align256(off + (size_t)nodes * sizeof(int2));
  L.total = off;
  return L;
}

}  // namespace

// Group tables (group g's [n][8] block in each pair array) and the per-node
// flags that the pack kernel only ever sets: invalid, infeasible, tiny.
// The array keeps whatever the last call left, so they are cleared here
// (a kernel, not a memset, so the clear also works inside captured work).
// The touch bytes after each group's B block are left as they are: a stale
// set byte only makes the first commit compare pairs that are equal.
__global__ __launch_bounds__(kBlock) void k_static_setup(double2** tables, double2* A, double2* B,
                                                         int groups, size_t per_group,
                                                         size_t per_group_b, uint32_t* flags,
                                                         int flag_words) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < groups) {
    tables[i] = A + (size_t)i * per_group;
    tables[groups + i] = B + (size_t)i * per_group_b;
  }
  for (int q = i; q < flag_words; q += gridDim.x * blockDim.x) flags[q] = 0;
}

// (status, rounds) per node, in the layout of prop_result.
__global__ __launch_bounds__(kBlock) void k_static_results(const int32_t* status,
                                                           const int32_t* rounds, int2* out,
                                                           int nodes) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nodes; k += gridDim.x * blockDim.x)
    out[k] = make_int2(status[k], rounds[k]);
}

}  // namespace prop

using namespace prop;

extern "C" int prop_run_batch_device_static(prop_problem* p, int32_t nodes, double* d_lb,
                                            double* d_ub, int32_t max_rounds, void* stream,
                                            prop_result* out) {
  static_assert(sizeof(prop_result) == sizeof(int2), "prop_result is two int32 words");
  if (!p || !out) return fail(PROP_EINVAL, "NULL argument");
  if (nodes < 1) return fail(PROP_EINVAL, "nodes < 1");
  if (max_rounds < 0) return fail(PROP_EINVAL, "max_rounds < 0");
  if (p->n > 0 && (!d_lb || !d_ub)) return fail(PROP_EINVAL, "bound arrays are NULL");
  if (p->P.nnz_split) return fail(PROP_EINVAL, "the nnz-split layout runs single bound vectors only");
  if (p->P.store32) return fail(PROP_EINVAL, "the single-precision store runs single bound vectors only");
  const StaticLayout L = static_layout(p->n, p->P.n_segs, nodes);
  if (L.total > kScratchBytes)
    return fail(PROP_EINVAL,
                "%d nodes of %d variables need %zu bytes of workspace; the fixed array holds %zu",
                nodes, p->n, L.total, kScratchBytes);
  HIP_TRY(hipSetDevice(p->device));
  unsigned char* base = nullptr;
  int rc = scratch_address(p->device, &base);
  if (rc) return rc;
  p->P.marking = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Problem& P = p->P;
  const int32_t groups = (nodes + kNodeGroup - 1) / kNodeGroup;
  const size_t per_group = (size_t)kNodeGroup * (size_t)(p->n > 0 ? p->n : 1);
  double2* A = reinterpret_cast<double2*>(base + L.pairs_a);
  double2* B = reinterpret_cast<double2*>(base + L.pairs_b);
  double2** tables = reinterpret_cast<double2**>(base + L.tables);
  uint32_t* n32 = reinterpret_cast<uint32_t*>(base + L.nodes32);
  int2* results = reinterpret_cast<int2*>(base + L.results);
  Batch bt{};
  bt.gA = tables;
  bt.gB = tables + groups;
  bt.partials = reinterpret_cast<SegPartial*>(base + L.partials);
  bt.invalid = n32;
  bt.infeasible = n32 + nodes;
  bt.tiny = n32 + 2 * (size_t)nodes;
  bt.active = n32 + 3 * (size_t)nodes;
  bt.status = reinterpret_cast<int32_t*>(n32 + 4 * (size_t)nodes);
  bt.rounds = reinterpret_cast<int32_t*>(n32 + 5 * (size_t)nodes);
  bt.changed = n32 + 6 * (size_t)nodes;
  bt.maxr = reinterpret_cast<int32_t*>(n32 + 7 * (size_t)nodes);
  bt.live = nullptr;
  bt.nodes = nodes;
  bt.groups = groups;

  HIP_TRY(hipEventRecord(p->ev[0], s));
  const int setup_blocks = (3 * nodes + kBlock - 1) / kBlock > (groups + kBlock - 1) / kBlock
                               ? (3 * nodes + kBlock - 1) / kBlock
                               : (groups + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_static_setup, dim3(setup_blocks < 1024 ? setup_blocks : 1024), dim3(kBlock),
                     0, s, tables, A, B, groups, per_group,
                     per_group + touch_bytes(p->n) / sizeof(double2), n32, 3 * nodes);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_init(P, s));
  HIP_TRY(launch_pack_batch(P, bt, d_lb, d_ub, 0, nodes, s));
  HIP_TRY(launch_start_batch(P, bt, max_rounds, 0, nodes, true, s));
  HIP_TRY(hipEventRecord(p->ev[1], s));
  // every group runs until all nodes have finished (no compaction, which
  // needs host-side lists); the done flag is read one batch of rounds
  // behind, as by the stream driver
  int slot = 0;
  bool pending[2] = {false, false};
  for (int r = 1; r <= max_rounds;) {
    const int last = max_rounds < r + p->batch_rounds - 1 ? max_rounds : r + p->batch_rounds - 1;
    for (; r <= last; ++r) HIP_TRY(launch_round_batch(P, bt, s));
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
  HIP_TRY(hipEventRecord(p->ev[2], s));
  HIP_TRY(launch_unpack_batch(P, bt, d_lb, d_ub, 0, nodes, s));
  hipLaunchKernelGGL(k_static_results, dim3((nodes + kBlock - 1) / kBlock < 64
                                                ? (nodes + kBlock - 1) / kBlock
                                                : 64),
                     dim3(kBlock), 0, s, bt.status, bt.rounds, results, nodes);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out, results, (size_t)nodes * sizeof(int2), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipEventRecord(p->ev[3], s));
  HIP_TRY(hipStreamSynchronize(s));
  hipEventElapsedTime(&p->last_loop_ms, p->ev[1], p->ev[2]);
  hipEventElapsedTime(&p->last_total_ms, p->ev[0], p->ev[3]);
  p->kev_used = 0;
  p->last_kernel_ms = 0.0;
  for (int32_t k = 0; k < nodes; ++k)
    if (out[k].status == kInvalidInput)
      return fail(PROP_EINVAL,
                  "node %d: a bound is NaN, +inf as lower, -inf as upper, or beyond 2^200", k);
  g_error.clear();
  return PROP_OK;
}
