// Sliced streaming update: the replica axis of every row is cut into kReplicaSlices slices,
// and slice s of every row is updated by workgroups on XCD s.  The coupling product
// gathers, for each edge, only the neighbour's slice, so the rows an XCD gathers from are
// 1/kReplicaSlices of P_in and mostly stay in that XCD's L2 instead of crossing the fabric.
// Where an eighth of a row would be narrower than a 128-byte line, the row is cut into four
// slices instead, and slice s is served by the XCD pair 2s, 2s + 1, each taking every other
// block of rows.
//
// The replica statistics mu_i, sigma_i (Eq. 10) need all S replicas of a row.  Each slice
// kernel therefore also writes, for the next update, its slice's partial statistics of the
// new values: {mean_s, M2_s}, with M2_s the sum of squared deviations from the slice mean.
// The next update combines a row's kReplicaSlices partials into mu and sigma (the pairwise
// combination of Chan, Golub and LeVeque, 1979) in a fixed order, with no division:
//   mu = (sum_s n_s mean_s) / S,   M2 = sum_s (M2_s + n_s (mean_s - mu)^2),   sigma = sqrt(M2 / S).
// One launch per update; the first update's partials come from slice_stats_kernel, which
// forms them from P with the same lanes and the same arithmetic.  The coupling sums run in
// plain edge order (or as the split rows' chunk sums), as in step_kernel; only mu and sigma
// are rounded differently from the whole-row kernels.
//
// Workgroup-to-XCD placement: consecutive workgroup ids of a launch are dispatched to
// consecutive XCDs, round robin, so workgroup b runs on XCD b mod 8.  Slice = b mod 8 (eight
// slices) or (b mod 8) / 2 (four).
#include "qqa_device.h"

namespace qqa {

// The slice of `row` served by this workgroup, as a row of its own: pointers at the slice's
// first replica, S = its valid replicas.  Slice s of NSL holds quads [s nq / NSL,
// (s + 1) nq / NSL) of the row's nq quads.
// SM (slice-major state, equal slices, no sums or dense product): P, m and v hold slice
// s's rows contiguously, [slice][row][its 4 (q1 - q0) replicas], so the row of the view is
// 4 (q1 - q0) floats apart; the split rows' chunk partials likewise, [slice][chunk][width]
// (nchunks chunks).
template <int NSL, bool SM = false>
__device__ __forceinline__ StepParams slice_view(const StepParams& a, const int slice, int* q0_out,
                                                 const int nchunks = 0) {
  const int nq = (a.S + 3) >> 2;
  const int q0 = slice * nq / NSL, q1 = (slice + 1) * nq / NSL;
  const size_t off = 4 * (size_t)q0;
  StepParams b = a;
  const size_t soff = SM ? (size_t)slice * a.n * 4 * (size_t)(q1 - q0) : off;
  if (SM) b.stride = 4 * (q1 - q0);
  b.P_in = a.P_in + soff;
  b.P_out = a.P_out + soff;
  b.m = a.m ? a.m + soff : nullptr;
  b.v = a.v ? a.v + soff : nullptr;
  b.coupling = a.coupling ? a.coupling + off : nullptr;
  const size_t hoff = SM ? (size_t)slice * nchunks * 4 * (size_t)(q1 - q0) : off;
  b.hub_partial = a.hub_partial ? a.hub_partial + hoff : nullptr;
  b.colsum = a.colsum ? a.colsum + off : nullptr;
  b.S = min(a.S, 4 * q1) - 4 * q0;
  *q0_out = q0;
  return b;
}

// A slice row's own values, as load_row reads them, with the AdamW moments read
// non-temporally: they are read and written once per update, so they need not take L2 lines
// from the slice of P_in the XCD gathers from (measured at S = 256, ER n = 20,000: 28.0
// against 28.8 us; the same for the moment stores: 32.6, slower).
template <int LS, int QS, bool FULL>
__device__ __forceinline__ void slice_load_row(const StepParams& b, const int row, const int gl, float4 (&p)[QS],
                                               float4 (&mm)[QS], float4 (&vv)[QS]) {
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  const int nq = FULL ? LS * QS : (b.S + 3) >> 2;
  const size_t base = (size_t)row * b.stride;
  const bool adam = b.rule == kADAMW;
#pragma unroll
  for (int k = 0; k < QS; ++k) {
    const int q = gl + LS * k;
    const size_t off = base + 4 * (size_t)((FULL || q < nq) ? q : nq - 1);
    p[k] = *reinterpret_cast<const float4*>(b.P_in + off);
    const f32x4 xm = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>((adam ? b.m : b.P_in) + off));
    const f32x4 xv = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>((adam ? b.v : b.P_in) + off));
    mm[k] = make_float4(xm.x, xm.y, xm.z, xm.w);
    vv[k] = make_float4(xv.x, xv.y, xv.z, xv.w);
  }
}

// {mean, M2} of one slice's valid values v (lane gl's quads of the slice), over the LS lanes.
template <int LS, int QS, bool FULL>
__device__ __forceinline__ float2 slice_partial(const StepParams& b, const int gl, const float4 (&v)[QS]) {
  float sum = 0.f;
#pragma unroll
  for (int k = 0; k < QS; ++k) {
    const int q = gl + LS * k;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (FULL || 4 * q + c < b.S) sum += comp(v[k], c);
  }
  sum = group_sum<LS>(sum);
  const float mean = sum * __builtin_amdgcn_rcpf((float)b.S);
  float m2 = 0.f;
#pragma unroll
  for (int k = 0; k < QS; ++k) {
    const int q = gl + LS * k;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (FULL || 4 * q + c < b.S) {
        const float d = comp(v[k], c) - mean;
        m2 = fmaf(d, d, m2);
      }
  }
  m2 = group_sum<LS>(m2);
  return make_float2(mean, m2);
}

// mu and the communication coefficient cg = -alpha_c / sigma (0 when sigma = 0) of `row`
// from its slices' partials.  Partials are stored slice-major (part[slice * n + row]): each
// XCD writes one contiguous array.  Lane gl of the LS-lane group reads slices gl, gl + LS,
// ... (one load for the group when LS >= kReplicaSlices) and adds them in that order; a
// butterfly over the group then adds the lanes (a fixed tree, the same bits in every lane).
template <int LS, int NSL>
__device__ __forceinline__ void combine_partials(const StepParams& a, const float2* __restrict__ part, const int row,
                                                 const int gl, float& mu, float& cg) {
  constexpr int PER = LS >= NSL ? 1 : NSL / LS;  // slices per lane
  const int nq = (a.S + 3) >> 2;
  float2 ps[PER];
  float ns[PER];  // valid replicas of each slice; 0 for lanes past the last slice
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int sl = gl + LS * j;
    const bool ok = sl < NSL;
    const int sc = ok ? sl : NSL - 1;  // unconditional load, no join
    const float2 x = part[(size_t)sc * a.n + row];
    ps[j] = ok ? x : make_float2(0.f, 0.f);
    ns[j] = ok ? (float)(min(a.S, 4 * ((sc + 1) * nq / NSL)) - 4 * (sc * nq / NSL)) : 0.f;
  }
  float sum = 0.f;
#pragma unroll
  for (int j = 0; j < PER; ++j) sum = fmaf(ns[j], ps[j].x, sum);
  sum = group_sum<LS>(sum);
  mu = sum * a.inv_S;
  float m2 = 0.f;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const float d = ps[j].x - mu;
    m2 += ps[j].y + ns[j] * (d * d);
  }
  m2 = group_sum<LS>(m2);
  const float sigma = __builtin_amdgcn_sqrtf(m2 * a.inv_S);
  cg = sigma > 0.f ? -a.comm_alpha * __builtin_amdgcn_rcpf(sigma) : 0.f;
}

// The slice and the first row of workgroup b.  Eight slices: slice b mod 8 (its XCD), row
// block b / 8.  Four slices: XCDs 2s and 2s + 1 serve slice s, each every other row block.
template <int NSL>
__device__ __forceinline__ void slice_of_block(const int b, int* slice, int* row_block) {
  const int xcd = b % kReplicaSlices;
  if (NSL == kReplicaSlices) {
    *slice = xcd;
    *row_block = b / kReplicaSlices;
  } else {  // NSL == kReplicaSlices / 2
    *slice = xcd >> 1;
    *row_block = (b / kReplicaSlices) * 2 + (xcd & 1);
  }
}

// Partials of P (= a.P_in) for every (row, slice): the first update's statistics.
template <int LS, int QS, bool FULL, int NSL, bool SM>
__global__ __launch_bounds__(kBlock) void slice_stats_kernel(StepParams a, float2* __restrict__ part) {
  int slice, rb;
  slice_of_block<NSL>((int)blockIdx.x, &slice, &rb);
  const int row = rb * (kBlock / LS) + (int)(threadIdx.x / LS);
  if (row >= a.n) return;  // whole lane groups leave together
  const int gl = threadIdx.x & (LS - 1);
  int q0;
  const StepParams b = slice_view<NSL, SM>(a, slice, &q0);
  float4 p[QS], mm[QS], vv[QS];
  load_row<LS, QS, FULL>(b, b.P_in, row, gl, p, mm, vv);
  const float2 pt = slice_partial<LS, QS, FULL>(b, gl, p);
  if (gl == 0) part[(size_t)slice * a.n + row] = pt;
}

// One update of one slice of one row, LS lanes x QS quads; reads the row's partials of
// P_in from part_in and writes this slice's partial of P_out to part_out.
// One quad per lane: eight waves per SIMD, the register budget held to 64 (at most 62 used, no
// spills; 80 unbounded, six waves).  Measured: 30.3 against 30.7 us at S = 256, 29.2 against
// 30.4 at S = 512.  Two quads per lane would spill under that budget and keep theirs.
template <int LS, int QS, bool FULL, bool SUMS, int NSL, bool SM, int SPEC = 0>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(QS == 1 ? 8 : 1, 8))) void slice_step_kernel(StepParams a, const float2* __restrict__ part_in,
                                                            float2* __restrict__ part_out, int nchunks) {
  int slice, rb;
  slice_of_block<NSL>((int)blockIdx.x, &slice, &rb);
  const int row = rb * (kBlock / LS) + (int)(threadIdx.x / LS);
  if (row >= a.n) return;  // whole lane groups leave together
  const int gl = threadIdx.x & (LS - 1);
  int q0;
  const StepParams b = slice_view<NSL, SM>(a, slice, &q0, nchunks);
  float4 p[QS], mm[QS], vv[QS], acc[QS], po[QS], mo[QS], vo[QS];
  const RowMeta rm = row_meta(b, row);
  float mu, cg;
  combine_partials<LS, NSL>(a, part_in, row, gl, mu, cg);
  slice_load_row<LS, QS, FULL>(b, row, gl, p, mm, vv);
  // gather batches of 6 edges at up to 8 lanes per slice row (one quad each): most rows of a
  // sparse graph take one memory round trip (measured: 30.7 against 31.9 us with 4 at S = 256,
  // ER n = 20,000, mean degree 5).  Wider slices keep 4-quad batches, which measured best there.
  // The batch size changes no result: the edge order of the sums is the same.
  constexpr int kSliceGatherQuads = LS <= 8 ? 6 : 4;
  row_coupling<LS, QS, FULL, false, false, false, kSliceGatherQuads, SPEC>(b, row, rm, gl, acc);
  finish_elems<LS, QS, FULL, SUMS, false, SPEC>(b, row, gl, q0, mu, cg, p, mm, vv, acc, po, mo, vo);
  store_row<LS, QS, FULL>(b, b.P_out, row, gl, po, mo, vo, true);
  const float2 pt = slice_partial<LS, QS, FULL>(b, gl, po);
  if (gl == 0) part_out[(size_t)slice * a.n + row] = pt;
}

// Split rows with slice-major state: the partial coupling sum of one chunk over one slice
// of the replicas, in the chunk's edge order (the same sums, bit for bit, as the whole-row
// chunk kernel's), written [slice][chunk][width].  Workgroup b serves slice b mod 8 (XCD
// pairs with four slices), as the update does.
template <int LS, int QS, int NSL>
__global__ __launch_bounds__(kBlock) void slice_hub_partial_kernel(StepParams a, const HubChunk* __restrict__ chunks,
                                                                   int nchunks) {
  int slice, rb;
  slice_of_block<NSL>((int)blockIdx.x, &slice, &rb);
  const int c = rb * (kBlock / LS) + (int)(threadIdx.x / LS);
  if (c >= nchunks) return;  // whole lane groups leave together
  const int gl = threadIdx.x & (LS - 1);
  int q0;
  const StepParams b = slice_view<NSL, true>(a, slice, &q0, nchunks);
  const HubChunk ch = chunks[c];
  const int e_end = min(ch.e0 + kHubChunk, a.row_ptr[ch.row + 1]);
  float4 acc[QS];
#pragma unroll
  for (int k = 0; k < QS; ++k) acc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
  gather_coupling<LS, QS, true, false, false>(b, ch.e0, e_end, gl, LS * QS, a.problem == kMAXCUT, acc);
  float* out = const_cast<float*>(b.hub_partial) + (size_t)c * b.stride;
#pragma unroll
  for (int k = 0; k < QS; ++k) *reinterpret_cast<float4*>(out + 4 * (gl + LS * k)) = acc[k];
}

static unsigned blocks_of(long long threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

SliceShape slice_shape(int S) {
  SliceShape r{0, 0, 0, 0};
  const int nq = (S + 3) / 4;
  if (S <= 0 || S > kMaxReplicas) return r;
  // eight slices (one XCD each) when each is at least a 128-byte line; else four (an XCD pair
  // each) when those are; else eight of at least two quads (32 bytes)
  int nsl = 0;
  if (nq >= 8 * kReplicaSlices) nsl = kReplicaSlices;
  else if (nq >= 8 * (kReplicaSlices / 2)) nsl = kReplicaSlices / 2;
  else if (nq >= 2 * kReplicaSlices) nsl = kReplicaSlices;
  if (!nsl) return r;
  const int sq = (nq + nsl - 1) / nsl;  // the largest slice
  int ls = 2;
  while (ls < sq && ls < 64) ls *= 2;
  r.nsl = nsl;
  r.sq = sq;
  r.ls = ls;
  r.qs = (sq + ls - 1) / ls;
  int qs = 1;
  while (qs < r.qs) qs *= 2;
  r.qs = qs;
  return r;
}

// workgroups of a launch: every slice covers all row blocks, eight slices one XCD each,
// four slices an XCD pair each (every other row block per XCD)
static dim3 slice_grid(int n, int LS, int nsl) {
  const unsigned rb = blocks_of((long long)n * LS);
  return dim3(nsl == kReplicaSlices ? kReplicaSlices * rb : kReplicaSlices * ((rb + 1) / 2));
}

template <int LS, int QS, int NSL>
static void launch_slice_stats_t(const StepParams& p, float2* part, bool sm, hipStream_t st) {
  const dim3 grid = slice_grid(p.n, LS, NSL), block(kBlock);
  if (sm)
    hipLaunchKernelGGL((slice_stats_kernel<LS, QS, true, NSL, true>), grid, block, 0, st, p, part);
  else if (p.S == 4 * NSL * LS * QS)  // equal slices, every lane's quads valid
    hipLaunchKernelGGL((slice_stats_kernel<LS, QS, true, NSL, false>), grid, block, 0, st, p, part);
  else
    hipLaunchKernelGGL((slice_stats_kernel<LS, QS, false, NSL, false>), grid, block, 0, st, p, part);
}

template <int LS, int QS, int NSL>
static void launch_slice_t(const StepParams& p, const float2* part_in, float2* part_out, bool sm, int nchunks,
                           hipStream_t st) {
  const dim3 grid = slice_grid(p.n, LS, NSL), block(kBlock);
  const bool full = p.S == 4 * NSL * LS * QS;  // equal slices, every lane's quads valid
  const bool sums = p.problem == kMAXCLIQUE;
#define L(FU, SU, M) \
  hipLaunchKernelGGL((slice_step_kernel<LS, QS, FU, SU, NSL, M>), grid, block, 0, st, p, part_in, part_out, nchunks)
#define LSPEC(PROBLEM)                                                                                       \
  hipLaunchKernelGGL((slice_step_kernel<LS, QS, true, false, NSL, true, spec_of(PROBLEM, kADAMW, 4)>), grid, block, 0, \
                     st, p, part_in, part_out, nchunks)
  // the default schedules (AdamW, entropy alpha 4) of MIS and max-cut with slice-major state
  // run with those facts fixed at compile time
  const bool spec = p.rule == kADAMW && p.alpha_e == 4;
  if (sm && spec && p.problem == kMIS) LSPEC(kMIS);
  else if (sm && spec && p.problem == kMAXCUT) LSPEC(kMAXCUT);
  else if (sm) L(true, false, true);
  else if (sums) {
    if (full) L(true, true, false);
    else L(false, true, false);
  } else {
    if (full) L(true, false, false);
    else L(false, false, false);
  }
#undef LSPEC
#undef L
}

bool slice_major_ok(const StepParams& p) {
  const SliceShape s = slice_shape(p.S);
  return s.sq != 0 && p.S == 4 * s.nsl * s.ls * s.qs && p.stride == p.S && !p.colsum && !p.coupling &&
         p.problem != kMAXCLIQUE;
}

template <int LS, int QS, int NSL>
static void launch_slice_hub_t(const StepParams& p, const HubChunk* chunks, int nchunks, hipStream_t st) {
  hipLaunchKernelGGL((slice_hub_partial_kernel<LS, QS, NSL>), slice_grid(nchunks, LS, NSL), dim3(kBlock), 0, st, p,
                     chunks, nchunks);
}

__global__ void slice_permute_kernel(const float4* __restrict__ src, float4* __restrict__ dst, int n, int nsl,
                                     int wq, bool to_slice_major) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;  // quad index, row-major
  const long long total = (long long)n * nsl * wq;
  if (i >= total) return;
  const long long row = i / ((long long)nsl * wq);
  const int rest = (int)(i - row * nsl * wq), slice = rest / wq, k = rest - slice * wq;
  const long long j = ((long long)slice * n + row) * wq + k;  // its quad index, slice-major
  if (to_slice_major) dst[j] = src[i];
  else dst[i] = src[j];
}

hipError_t launch_slice_permute(const float* src, float* dst, int n, int S, bool to_slice_major, hipStream_t st) {
  const SliceShape s = slice_shape(S);
  if (s.sq == 0 || S != 4 * s.nsl * s.ls * s.qs) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  const int wq = S / 4 / s.nsl;
  hipLaunchKernelGGL(slice_permute_kernel, dim3(blocks_of((long long)n * s.nsl * wq)), dim3(kBlock), 0, st,
                     reinterpret_cast<const float4*>(src), reinterpret_cast<float4*>(dst), n, s.nsl, wq,
                     to_slice_major);
  return hipGetLastError();
}

// (lanes, quads per lane, slices) of the kernels built: four slices serve 8 to 15 quads each
#define QQA_FOR_EACH_SLICE_LAYOUT(X) \
  X(2, 1, 8) X(4, 1, 8) X(8, 1, 8) X(16, 1, 8) X(32, 1, 8) X(64, 1, 8) X(64, 2, 8) X(8, 1, 4) X(16, 1, 4)

hipError_t launch_slice_stats(const StepParams& p, float2* part, hipStream_t st, bool slice_major) {
  if (p.n == 0) return hipSuccess;
  const SliceShape s = slice_shape(p.S);
  if (s.sq == 0) return hipErrorInvalidValue;
  if (slice_major && !slice_major_ok(p)) return hipErrorInvalidValue;
#define X(L, Q, N)                                     \
  if (s.ls == L && s.qs == Q && s.nsl == N) {          \
    launch_slice_stats_t<L, Q, N>(p, part, slice_major, st); \
    return hipGetLastError();                  \
  }
  QQA_FOR_EACH_SLICE_LAYOUT(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_slice_step(const StepParams& p, const float2* part_in, float2* part_out, hipStream_t st,
                             bool slice_major, int nchunks) {
  if (p.n == 0) return hipSuccess;
  const SliceShape s = slice_shape(p.S);
  if (s.sq == 0) return hipErrorInvalidValue;
  if (slice_major && !slice_major_ok(p)) return hipErrorInvalidValue;
#define X(L, Q, N)                                       \
  if (s.ls == L && s.qs == Q && s.nsl == N) {            \
    launch_slice_t<L, Q, N>(p, part_in, part_out, slice_major, nchunks, st); \
    return hipGetLastError();                            \
  }
  QQA_FOR_EACH_SLICE_LAYOUT(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_slice_hub_partials(const StepParams& p, const HubChunk* chunks, int nchunks, hipStream_t st) {
  if (nchunks == 0) return hipSuccess;
  if (!slice_major_ok(p)) return hipErrorInvalidValue;
  const SliceShape s = slice_shape(p.S);
#define X(L, Q, N)                                       \
  if (s.ls == L && s.qs == Q && s.nsl == N) {            \
    launch_slice_hub_t<L, Q, N>(p, chunks, nchunks, st); \
    return hipGetLastError();                            \
  }
  QQA_FOR_EACH_SLICE_LAYOUT(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace qqa
