// Sliced streaming update: the replica axis of every row is cut into kReplicaSlices slices, and
// slice s of every row is updated by workgroups on XCD s.  The coupling product gathers,
// for each edge, only the neighbour's slice, so the rows an XCD gathers from are 1/kReplicaSlices
// of P_in and stay in that XCD's L2 instead of being fetched again from the fabric.
//
// The replica statistics mu_i, sigma_i need all S replicas of a row, so one update is two
// launches:
//   row_stats_kernel   (mu_i, cg_i = -alpha_c / sigma_i) of every row of P_in, computed
//                      with the row's lane layout and the same butterfly as the whole-row
//                      kernel;
//   slice_step_kernel  the coupling gathers (plain edge order, or the split rows' partial
//                      sums), the gradient, AdamW, noise and clamp for one slice of one row.
// Every element therefore sees the same operations in the same order as in step_kernel,
// and the result is bitwise identical to it.
//
// Workgroup-to-XCD placement: consecutive workgroup ids of a launch are dispatched to
// consecutive XCDs, round robin, so workgroup b runs on XCD b mod 8.  Slice = b mod kReplicaSlices.
#include "qqa_device.h"

namespace qqa {

template <int LPR, int QPL, bool FULL>
__global__ __launch_bounds__(kBlock) void row_stats_kernel(StepParams a, float2* __restrict__ stats) {
  int row = (int)(((long long)blockIdx.x * kBlock + threadIdx.x) / LPR);
  if (LPR == 64) row = __builtin_amdgcn_readfirstlane(row);
  if (row >= a.n) return;  // whole lane groups leave together
  const int gl = threadIdx.x & (LPR - 1);
  const int nq = FULL ? LPR * QPL : (a.S + 3) >> 2;
  float4 p[QPL];
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int q = gl + LPR * k;
    p[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (FULL || q < nq) p[k] = *reinterpret_cast<const float4*>(a.P_in + (size_t)row * a.stride + 4 * q);
  }
  float mu, cg;
  row_stats<LPR, QPL, FULL>(a, gl, p, mu, cg);
  if (gl == 0) stats[row] = make_float2(mu, cg);
}

// LS lanes x QS quads serve one slice of one row.  Slice s holds quads
// [s nq / kReplicaSlices, (s + 1) nq / kReplicaSlices) of the row's nq quads (at most LS * QS of them).
template <int LS, int QS, bool FULL, bool SUMS>
__global__ __launch_bounds__(kBlock) void slice_step_kernel(StepParams a, const float2* __restrict__ stats) {
  const int slice = (int)(blockIdx.x % kReplicaSlices);
  const int row = (int)(blockIdx.x / kReplicaSlices) * (kBlock / LS) + (int)(threadIdx.x / LS);
  if (row >= a.n) return;  // whole lane groups leave together
  const int gl = threadIdx.x & (LS - 1);
  const int nq = (a.S + 3) >> 2;
  const int q0 = slice * nq / kReplicaSlices, q1 = (slice + 1) * nq / kReplicaSlices;
  const size_t off = 4 * (size_t)q0;
  // the slice as a row of its own: pointers at its first replica, S = its valid replicas
  StepParams b = a;
  b.P_in = a.P_in + off;
  b.P_out = a.P_out + off;
  b.m = a.m ? a.m + off : nullptr;
  b.v = a.v ? a.v + off : nullptr;
  b.coupling = a.coupling ? a.coupling + off : nullptr;
  b.hub_partial = a.hub_partial ? a.hub_partial + off : nullptr;
  b.colsum = a.colsum ? a.colsum + off : nullptr;
  b.S = min(a.S, 4 * q1) - 4 * q0;
  float4 p[QS], mm[QS], vv[QS], acc[QS], po[QS], mo[QS], vo[QS];
  load_row<LS, QS, FULL>(b, b.P_in, row, gl, p, mm, vv);
  row_coupling<LS, QS, FULL, false, false>(b, row, gl, acc);
  const float2 st = stats[row];
  finish_elems<LS, QS, FULL, SUMS>(b, row, gl, q0, st.x, st.y, p, mm, vv, acc, po, mo, vo);
  store_row<LS, QS, FULL>(b, b.P_out, row, gl, po, mo, vo, true);
}

static unsigned blocks_of(long long threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

SliceShape slice_shape(int S) {
  SliceShape r{0, 0, 0};
  const int nq = (S + 3) / 4;
  const int sq = (nq + kReplicaSlices - 1) / kReplicaSlices;  // the largest slice
  // every slice holds at least two quads (32 bytes)
  if (S <= 0 || S > kMaxReplicas || nq < 2 * kReplicaSlices) return r;
  int ls = 2;
  while (ls < sq && ls < 64) ls *= 2;
  r.sq = sq;
  r.ls = ls;
  r.qs = (sq + ls - 1) / ls;
  int qs = 1;
  while (qs < r.qs) qs *= 2;
  r.qs = qs;
  return r;
}

template <int LPR, int QPL>
static void launch_stats_t(const StepParams& p, float2* stats, hipStream_t st) {
  const dim3 grid(blocks_of((long long)p.n * LPR)), block(kBlock);
  if (p.S == 4 * LPR * QPL)
    hipLaunchKernelGGL((row_stats_kernel<LPR, QPL, true>), grid, block, 0, st, p, stats);
  else
    hipLaunchKernelGGL((row_stats_kernel<LPR, QPL, false>), grid, block, 0, st, p, stats);
}

template <int LS, int QS>
static void launch_slice_t(const StepParams& p, const float2* stats, hipStream_t st) {
  const dim3 grid((unsigned)kReplicaSlices * blocks_of((long long)p.n * LS)), block(kBlock);
  const bool full = p.S == 4 * kReplicaSlices * LS * QS;  // equal slices, every lane's quads valid
  const bool sums = p.problem == kMAXCLIQUE;
  if (sums) {
    if (full) hipLaunchKernelGGL((slice_step_kernel<LS, QS, true, true>), grid, block, 0, st, p, stats);
    else hipLaunchKernelGGL((slice_step_kernel<LS, QS, false, true>), grid, block, 0, st, p, stats);
  } else {
    if (full) hipLaunchKernelGGL((slice_step_kernel<LS, QS, true, false>), grid, block, 0, st, p, stats);
    else hipLaunchKernelGGL((slice_step_kernel<LS, QS, false, false>), grid, block, 0, st, p, stats);
  }
}

hipError_t launch_row_stats(const StepParams& p, float2* stats, hipStream_t st) {
  if (p.n == 0) return hipSuccess;
  const ReplicaShape r = replica_shape(p.S, p.lanes_per_row);
#define X(L, Q)                       \
  if (r.lpr == L && r.qpl == Q) {     \
    launch_stats_t<L, Q>(p, stats, st); \
    return hipGetLastError();         \
  }
  QQA_FOR_EACH_LAYOUT(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_slice_step(const StepParams& p, const float2* stats, hipStream_t st) {
  if (p.n == 0) return hipSuccess;
  const SliceShape s = slice_shape(p.S);
  if (s.sq == 0) return hipErrorInvalidValue;
#define X(L, Q)                                   \
  if (s.ls == L && s.qs == Q) {                   \
    launch_slice_t<L, Q>(p, stats, st);           \
    return hipGetLastError();                     \
  }
  X(2, 1) X(4, 1) X(8, 1) X(16, 1) X(32, 1) X(64, 1) X(64, 2)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace qqa
