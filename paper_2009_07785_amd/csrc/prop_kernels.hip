// prop_kernels.hip -- gfx950 kernels of one synchronous propagation round on
// a single bound vector (Sofranac, Gleixner, Pokutta, arXiv 2009.07785,
// Algorithms 2 and 3), the round-loop drivers, and their launchers.  The
// device functions they share with the batched kernels, and the derivation
// of the candidate skip filter, are in prop_device.h.
#include <hip/hip_runtime.h>

#include "prop_device.h"
#include "prop_launch.h"
#include "prop_layout.h"

#pragma clang fp contract(off)

namespace prop {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void k_init(Problem P) {
  if (blockIdx.x == 0 && threadIdx.x < kCommitGroups)
    P.commit_grp[threadIdx.x * kGroupWordStride] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctrl* C = P.ctrl;
    C->commit_word = 0;
    C->infeasible = 0;
    C->invalid = 0;
    C->status = kMaxRounds;
    C->rounds = 0;
    C->done = 0;
    C->round = 1;
    C->tiny = 0;
    C->bar_gen = 0;
    C->abort = 0;
    C->mark_all = 1;
  }
}

// Validate, integer-round and relabel the caller's bounds into both arrays.
__global__ __launch_bounds__(kBlock) void k_pack(Problem P, const double* __restrict__ ulb,
                                                 const double* __restrict__ uub) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)P.n; v += stride) {
    double l = ulb[v], u = uub[v];
    const bool bad = __builtin_isnan(l) || __builtin_isnan(u) || l == __builtin_inf() ||
                     u == -__builtin_inf() ||
                     (!is_inf(l) && __builtin_fabs(l) > PROP_HUGE) ||
                     (!is_inf(u) && __builtin_fabs(u) > PROP_HUGE);
    if (bad) __hip_atomic_store(&P.ctrl->invalid, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t j = P.perm[v];
    const bool is_int = P.vtype[j] != 0;
    if (is_int) {
      l = __builtin_ceil(l - P.eps_int);
      u = __builtin_floor(u + P.eps_int);
    }
    l = l + 0.0;
    u = u + 0.0;
    if (P.store32) {
      const float2 s32 = make_float2(store_down32(l), store_up32(u));
      P.b32[j] = s32;
      l = (double)s32.x;
      u = (double)s32.y;
    }
    const double2 b = make_double2(l, u);
    P.bnd[0][j] = b;
    P.bnd[1][j] = b;
    P.codes[j] = bound_code(is_int, l, u);
    if (tiny_bound(l) || tiny_bound(u))
      __hip_atomic_store(&P.ctrl->tiny, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (domain_empty(is_int, l, u, P.feas_tol))
      __hip_atomic_store(&P.ctrl->infeasible, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(kBlock) void k_reset_stripes(Problem P) {
  const size_t total = (size_t)kStripes * P.n_hot;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
    P.stripes[i] = make_double2(-__builtin_inf(), __builtin_inf());
}

__global__ __launch_bounds__(kBlock) void k_unpack(Problem P, double* __restrict__ ulb,
                                                   double* __restrict__ uub) {
  const double2* src = P.bnd[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)P.n; v += stride) {
    const double2 b = src[P.perm[v]];
    ulb[v] = b.x;
    uub[v] = b.y;
  }
}

// ---- persistent driver: every round inside one cooperative launch -------
// kMode: 0 chunks, 1 nnz-split waves, 2 chunks with the single-precision
// store's copies as the gather source.
template <int kMode>
__global__ __launch_bounds__(kBlock) void k_persistent(Problem P, int max_rounds) {
  constexpr bool kNz = kMode == 1;
  constexpr int kSrc = kMode == 2 ? kSrcCodes32 : kSrcCodes;
  Ctrl* C = P.ctrl;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gwave = blockIdx.x * kWavesPerBlock + wave;
  const int nwaves = gridDim.x * kWavesPerBlock;
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nthreads = gridDim.x * blockDim.x;
  const double2* A = P.bnd[0];
  double2* B = P.bnd[1];

  if (!grid_barrier(P, kActStart, 0, max_rounds)) return;
  if (u32_load(&C->done)) return;

  const int items = P.n_segs + P.n_chunks;
  for (int r = 1; r <= max_rounds; ++r) {
    const uint32_t exact = u32_load(&C->tiny) ? 1u : 0u;
    // long rows' first phase and the chunks in one pass, segments first (as
    // the per-round kernel numbers its waves), so that no wave is left with
    // segments after the others have run out of chunks
    for (int it = gwave; it < items; it += nwaves) {
      if (it < P.n_segs) seg_phase1<kSrc>(P, it, A, 1, 1, P.partials, 1, 0);
      else if (kNz) nz_wave_round(P, it - P.n_segs, A, B, exact != 0);
      else chunk_dispatch<kSrc>(P, it - P.n_segs, A, B, 1, 1, exact);
    }
    if (P.n_segs) {
      if (!grid_barrier(P, kActNone, r, max_rounds)) return;
      for (int s = gwave; s < P.n_segs; s += nwaves)
        seg_phase2<true, kSrc>(P, s, A, B, 1, 0, P.partials, 1, 0, exact != 0);
    }
    if (!grid_barrier(P, kActNone, r, max_rounds)) return;
    uint32_t changed = 0, infeasible = 0;
    commit_range<false>(P, tid, nthreads, changed, infeasible);
    block_sum2(changed, infeasible);
    const uint64_t add = (uint64_t)changed | (infeasible ? kCommitInf : 0ull);
    if (!grid_barrier(P, kActEndRound, r, max_rounds, add)) return;
    if (u32_load(&C->done)) return;
  }
}

// ---- stream / host drivers: one launch per phase, early exit when done ----
__global__ void k_start(Problem P, int max_rounds) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    P.ctrl->max_rounds = max_rounds;
    start_status(P, max_rounds);
  }
}

// The per-round kernels take the round number and the round limit from the
// control block (the commit of round r sets the next round number), so one
// captured sequence of rounds can be replayed for every batch of a run.
__device__ __forceinline__ int round_of(const Problem& P) {
  return __hip_atomic_load(&P.ctrl->round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Marked rounds: whether round r skips unstamped rows (read once per wave).
__device__ __forceinline__ bool marked_round(const Problem& P) {
  return P.marking && !u32_load(&P.ctrl->mark_all);
}

// Six waves per SIMD (at most 84 VGPRs; the kernel fits in 78 without
// spills): the round is bound by the gathers of the activity pass, and
// resident waves hide their latency.  Eight waves (64 VGPRs) spill and run
// twice as long.  kSrc: kSrcCodes, or kSrcCodes32 with the single-precision
// store.
template <int kSrc>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_round(
    Problem P) {
  if (u32_load(&P.ctrl->done)) return;
  const int r = round_of(P);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int item = blockIdx.x * kWavesPerBlock + wave;
  const bool marked = marked_round(P);
  if (item < P.n_segs)
    seg_phase1<kSrc>(P, item, P.bnd[0], 1, 1, P.partials, 1, 0, marked, r, P.row_mark);
  else if (item - P.n_segs < P.n_chunks)
    chunk_dispatch<kSrc>(P, item - P.n_segs, P.bnd[0], P.bnd[1], 1, 1,
                         u32_load(&P.ctrl->tiny) ? 1u : 0u, marked, r, P.row_mark);
}

// The same round for the nnz-split layout (a kernel of its own, so that
// neither layout's registers limit the other's occupancy).  Its waves
// process every row, marked or not (processing a row is always exact).
__global__ __launch_bounds__(kBlock) void k_round_nz(Problem P) {
  if (u32_load(&P.ctrl->done)) return;
  const int r = round_of(P);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int item = blockIdx.x * kWavesPerBlock + wave;
  if (item < P.n_segs)
    seg_phase1<kSrcCodes>(P, item, P.bnd[0], 1, 1, P.partials, 1, 0, marked_round(P), r,
                          P.row_mark);
  else if (item - P.n_segs < P.n_chunks)
    nz_wave_round(P, item - P.n_segs, P.bnd[0], P.bnd[1], u32_load(&P.ctrl->tiny) != 0);
}

template <int kSrc>
__global__ __launch_bounds__(kBlock) void k_round_long(Problem P) {
  if (u32_load(&P.ctrl->done)) return;
  const int r = round_of(P);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int s = blockIdx.x * kWavesPerBlock + wave;
  if (s < P.n_segs)
    seg_phase2<true, kSrc>(P, s, P.bnd[0], P.bnd[1], 1, 0, P.partials, 1, 0,
                     u32_load(&P.ctrl->tiny) != 0, marked_round(P), r, P.row_mark);
}

// Marked rounds, after the commit of round r: stamps the rows of every
// changed variable with r + 1, the round the commit has set as the next one
// (a thread per piece of <= kMarkPiece rows of one variable), unless that
// round runs over every row anyway.
__global__ __launch_bounds__(kBlock) void k_mark(Problem P) {
  const Ctrl* C = P.ctrl;
  if (u32_load(&C->done) || u32_load(&C->mark_all)) return;
  const int next = round_of(P);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < P.n_pieces; q += stride) {
    const int32_t v = P.piece_var[q];
    if (!((P.chg_bits[v / kWave] >> (v % kWave)) & 1ull)) continue;
    const int64_t start = P.piece_off[q];
    const int64_t stop = P.var_ptr[v + 1] < start + kMarkPiece ? P.var_ptr[v + 1] : start + kMarkPiece;
    for (int64_t i = start; i < stop; ++i) P.row_mark[P.var_rows[i]] = next;
  }
}

// Marked runs from a parent fixed point, after the start kernel: bit v of
// the changed-variable bitmap is set when variable v's start bounds differ
// from the parent's, and round 1 becomes a marked round; k_mark then stamps
// the rows of those variables with round 1.  Every other row would compute
// the candidates the parent's last round computed from the same bounds, and
// none of those counted (the parent is a fixed point).
__global__ __launch_bounds__(kBlock) void k_seed(Problem P) {
  Ctrl* C = P.ctrl;
  if (u32_load(&C->done)) return;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t words = ((uint32_t)P.n + kWave - 1) / kWave;
  const uint32_t nw = gridDim.x * kWavesPerBlock;
  for (uint32_t w = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); w < words; w += nw) {
    const uint32_t v = w * kWave + lane;
    bool diff = false;
    if (v < (uint32_t)P.n) {
      const double2 a = P.bnd[0][v];
      const double2 b = P.parent[v];
      diff = a.x != b.x || a.y != b.y;
    }
    const uint64_t bits = __ballot(diff);
    if (lane == 0) P.chg_bits[w] = bits;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) C->mark_all = 0;
}

// The parent's bounds, validated and integer-rounded as the pack kernel
// does, into internal order.
__global__ __launch_bounds__(kBlock) void k_set_parent(Problem P, double2* __restrict__ parent,
                                                       const double* __restrict__ ulb,
                                                       const double* __restrict__ uub) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)P.n; v += stride) {
    double l = ulb[v], u = uub[v];
    const bool bad = __builtin_isnan(l) || __builtin_isnan(u) || l == __builtin_inf() ||
                     u == -__builtin_inf() ||
                     (!is_inf(l) && __builtin_fabs(l) > PROP_HUGE) ||
                     (!is_inf(u) && __builtin_fabs(u) > PROP_HUGE);
    if (bad) __hip_atomic_store(&P.ctrl->invalid, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t j = P.perm[v];
    if (P.vtype[j] != 0) {
      l = __builtin_ceil(l - P.eps_int);
      u = __builtin_floor(u + P.eps_int);
    }
    l = l + 0.0;
    u = u + 0.0;
    if (P.store32) {
      l = (double)store_down32(l);
      u = (double)store_up32(u);
    }
    parent[j] = make_double2(l, u);
  }
}

// Commit of round r; the last block to finish decides the status.
__global__ __launch_bounds__(kBlock) void k_commit(Problem P) {
  Ctrl* C = P.ctrl;
  if (u32_load(&C->done)) return;
  // read before the last block's end_of_round advances them: every other
  // block has finished by then
  const int r = round_of(P);
  const int max_rounds = C->max_rounds;
  uint32_t changed = 0, infeasible = 0;
  commit_range<true>(P, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, changed,
               infeasible);
  block_sum2(changed, infeasible);
  if (threadIdx.x == 0) {
    const uint64_t add = kCommitBlock | (uint64_t)changed | (infeasible ? kCommitInf : 0ull);
    const uint32_t grp = blockIdx.x / kCommitGroup;
    const uint32_t in_grp = min((uint32_t)kCommitGroup, gridDim.x - grp * kCommitGroup);
    uint64_t* gw = P.commit_grp + (size_t)grp * kGroupWordStride;
    const uint64_t gold = __hip_atomic_fetch_add(gw, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((gold >> 48) == in_grp - 1u) {
      // last block of its group: every other block of the group has added
      const uint64_t gtot = gold + add;
      __hip_atomic_store(gw, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint64_t old =
          __hip_atomic_fetch_add(&C->commit_word, gtot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint64_t tot = old + gtot;
      if ((tot >> 48) == gridDim.x) {
        end_of_round(P, r, max_rounds, (uint32_t)tot, (uint32_t)((tot >> 32) & 0xffff));
        __hip_atomic_store(&C->commit_word, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}


// ---------------------------------------------------------------------------
// launchers (host side)
// ---------------------------------------------------------------------------

hipError_t launch_init(const Problem& P, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_pack(const Problem& P, const double* lb, const double* ub, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(blocks_for(P.n, kBlock, 4096)), dim3(kBlock), 0, s, P, lb, ub);
  if (P.n_hot)
    hipLaunchKernelGGL(k_reset_stripes, dim3(blocks_for((int64_t)kStripes * P.n_hot, kBlock, 1024)),
                       dim3(kBlock), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_unpack(const Problem& P, double* lb, double* ub, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack, dim3(blocks_for(P.n, kBlock, 4096)), dim3(kBlock), 0, s, P, lb,
                     ub);
  return hipGetLastError();
}

// Blocks per CU of the persistent kernel; for the chunk layout the smaller
// figure of its two store variants, so one grid fits either.
hipError_t persistent_occupancy(int* blocks_per_cu, bool nnz_split) {
  if (nnz_split)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_persistent<1>, kBlock, 0);
  int a = 0, b = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_persistent<0>, kBlock, 0);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_persistent<2>, kBlock, 0);
  *blocks_per_cu = a < b ? a : b;
  return e;
}

hipError_t launch_persistent(const Problem& P, int max_rounds, int grid, hipStream_t s) {
  Problem p = P;
  void* args[] = {(void*)&p, (void*)&max_rounds};
  const void* fn = P.nnz_split ? (const void*)k_persistent<1>
                   : P.store32 ? (const void*)k_persistent<2>
                               : (const void*)k_persistent<0>;
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBlock), args, 0, s);
}

hipError_t launch_seed(const Problem& P, hipStream_t s) {
  hipLaunchKernelGGL(k_seed, dim3(blocks_for(((int64_t)P.n + kWave - 1) / kWave, kWavesPerBlock, 4096)),
                     dim3(kBlock), 0, s, P);
  hipLaunchKernelGGL(k_mark, dim3(1024), dim3(kBlock), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_set_parent(const Problem& P, double2* parent, const double* lb,
                             const double* ub, hipStream_t s) {
  hipLaunchKernelGGL(k_set_parent, dim3(blocks_for(P.n, kBlock, 4096)), dim3(kBlock), 0, s, P,
                     parent, lb, ub);
  return hipGetLastError();
}

hipError_t launch_start(const Problem& P, int max_rounds, hipStream_t s) {
  hipLaunchKernelGGL(k_start, dim3(1), dim3(64), 0, s, P, max_rounds);
  return hipGetLastError();
}

hipError_t launch_round(const Problem& P, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const int items = P.n_chunks + P.n_segs;
  if (e0) hipEventRecord(e0, s);
  if (P.nnz_split)
    hipLaunchKernelGGL(k_round_nz, dim3(blocks_for(items, kWavesPerBlock, 1 << 30)), dim3(kBlock),
                       0, s, P);
  else if (P.store32)
    hipLaunchKernelGGL(k_round<kSrcCodes32>, dim3(blocks_for(items, kWavesPerBlock, 1 << 30)),
                       dim3(kBlock), 0, s, P);
  else
    hipLaunchKernelGGL(k_round<kSrcCodes>, dim3(blocks_for(items, kWavesPerBlock, 1 << 30)),
                       dim3(kBlock), 0, s, P);
  if (e1) hipEventRecord(e1, s);
  if (P.n_segs && P.store32)
    hipLaunchKernelGGL(k_round_long<kSrcCodes32>, dim3(blocks_for(P.n_segs, kWavesPerBlock, 1 << 30)),
                       dim3(kBlock), 0, s, P);
  else if (P.n_segs)
    hipLaunchKernelGGL(k_round_long<kSrcCodes>, dim3(blocks_for(P.n_segs, kWavesPerBlock, 1 << 30)),
                       dim3(kBlock), 0, s, P);
  // at most 65535 blocks: the packed commit counter keeps 16 bits per field
  hipLaunchKernelGGL(k_commit, dim3(blocks_for((int64_t)P.n / 4 + 2 * (int64_t)P.n_hot, kBlock,
                                                kCommitMaxBlocks)),
                     dim3(kBlock), 0, s, P);
  if (P.marking) hipLaunchKernelGGL(k_mark, dim3(1024), dim3(kBlock), 0, s, P);
  return hipGetLastError();
}

}  // namespace prop
