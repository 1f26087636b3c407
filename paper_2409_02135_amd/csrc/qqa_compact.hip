// Compact engine for one replica per variable (S = 1, the paper's scaling study of large
// random regular graphs).  The replica layout pads every row to a float4 quad, so at S = 1
// P, m and v would take 16 B per variable and the neighbour gathers would fetch from a P
// four times the size of its values.  Here P, m and v are n floats each: one lane per
// variable's state, gathers of single floats from a P a quarter the size.  A variable's
// edges are shared by the context's lanes per row (the edge split of the whole-row layout for
// one quad), and the arithmetic is the whole-row kernel's through the same device functions
// (row statistics, gradient, AdamW, noise, clamp); the coupling sum is split and ordered as
// there, with 16-edge chunk sums added in chunk order for split rows.  So the results are
// bitwise those of step_kernel at the same layout.
#include "qqa_device.h"

namespace qqa {

// Neighbour values loaded per batch and lane: all issued before the first is used.
constexpr int kCompactBatch = 8;

// sum over the edges of [e0, e1) that lane gl of LPR takes (e0 + gl, e0 + gl + LPR, ...) of
// w_e f(p_col(e)), in that order from zero; then a butterfly over the LPR lanes (offsets
// LPR/2 .. 1) adds the lanes' sums.  The same edge split and order as the whole-row kernel's
// gather at LPR lanes per row for one quad, so the same bits.
template <int LPR>
__device__ __forceinline__ float compact_gather(const StepParams& a, const float* __restrict__ P, const int e0,
                                                const int e1, const int gl, const bool maxcut) {
  float acc = 0.f;
  for (int b = e0 + gl; b < e1; b += kCompactBatch * LPR) {
    float x[kCompactBatch], w[kCompactBatch];
    bool ok[kCompactBatch];
#pragma unroll
    for (int u = 0; u < kCompactBatch; ++u) {
      const int e = b + u * LPR;
      ok[u] = e < e1;
      const int ec = ok[u] ? e : e1 - 1;  // a valid edge of this range: unconditional loads
      x[u] = P[a.col[ec]];
      w[u] = a.w ? a.w[ec] : 1.f;
    }
#pragma unroll
    for (int u = 0; u < kCompactBatch; ++u) {
      const float f = maxcut ? 2.f * x[u] - 1.f : x[u];
      const float r = fmaf(w[u], f, acc);
      acc = ok[u] ? r : acc;
    }
  }
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
  return acc;
}

// Split rows: the sum over 16-edge chunks of [e0, e1), each chunk's sum formed exactly as
// compact_gather forms it (the LPR lane slices, then the butterfly), the chunk sums added in
// chunk order.  kHubGroup chunks at a time have all their loads issued before any is used, so
// a row of many chunks does not wait for one chunk's loads before issuing the next's.
constexpr int kHubGroup = 4;

template <int LPR>
__device__ __forceinline__ float compact_hub_sum(const StepParams& a, const float* __restrict__ P, const int e0,
                                                 const int e1, const int gl, const bool maxcut) {
  constexpr int U = (kHubChunk + LPR - 1) / LPR;  // edges per lane and chunk
  float C = 0.f;
  for (int g0 = e0; g0 < e1; g0 += kHubGroup * kHubChunk) {
    float x[kHubGroup][U], w[kHubGroup][U];
    bool ok[kHubGroup][U];
#pragma unroll
    for (int c = 0; c < kHubGroup; ++c) {
      const int c0 = g0 + c * kHubChunk, c1 = min(c0 + kHubChunk, e1);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = c0 + gl + u * LPR;
        ok[c][u] = e < c1;
        const int ec = ok[c][u] ? e : e1 - 1;  // a valid edge of the row: unconditional loads
        x[c][u] = P[a.col[ec]];
        w[c][u] = a.w ? a.w[ec] : 1.f;
      }
    }
#pragma unroll
    for (int c = 0; c < kHubGroup; ++c) {
      float acc = 0.f;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float f = maxcut ? 2.f * x[c][u] - 1.f : x[c][u];
        const float r = fmaf(w[c][u], f, acc);
        acc = ok[c][u] ? r : acc;
      }
#pragma unroll
      for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
      if (g0 + c * kHubChunk < e1) C += acc;  // chunks past the row's end add nothing
    }
  }
  return C;
}

// One update of every variable: Pc_in -> Pc_out, m and v in place (n floats each).  LPR
// lanes share a variable's edges; every lane forms the same update and lane 0 stores it.
template <int LPR>
__global__ __launch_bounds__(kBlock) void compact_step_kernel(StepParams a, const float* __restrict__ Pc_in,
                                                              float* __restrict__ Pc_out, float* __restrict__ mc,
                                                              float* __restrict__ vc) {
  int row = (int)(((long long)blockIdx.x * kBlock + threadIdx.x) / LPR);
  if (LPR == 64) row = __builtin_amdgcn_readfirstlane(row);
  if (row >= a.n) return;  // whole lane groups leave together
  const int gl = threadIdx.x & (LPR - 1);
  const bool maxcut = a.problem == kMAXCUT;
  const bool adam = a.rule == kADAMW;
  const RowMeta rm = row_meta(a, row);
  float4 p[1], mm[1], vv[1], acc[1], po[1], mo[1], vo[1];
  p[0] = make_float4(Pc_in[row], 0.f, 0.f, 0.f);
  mm[0] = make_float4(adam ? mc[row] : 0.f, 0.f, 0.f, 0.f);
  vv[0] = make_float4(adam ? vc[row] : 0.f, 0.f, 0.f, 0.f);
  float C = 0.f;
  if (rm.hub >= 0) {
    C = compact_hub_sum<LPR>(a, Pc_in, rm.e0, rm.e1, gl, maxcut);
  } else {
    C = compact_gather<LPR>(a, Pc_in, rm.e0, rm.e1, gl, maxcut);
  }
  acc[0] = make_float4(C, 0.f, 0.f, 0.f);
  float mu, cg;
  row_stats<1, 1, false>(a, 0, p, mu, cg);
  finish_elems<1, 1, false, false>(a, row, 0, 0, mu, cg, p, mm, vv, acc, po, mo, vo);
  if (gl == 0) {
    Pc_out[row] = po[0].x;
    if (adam) {
      mc[row] = mo[0].x;
      vc[row] = vo[0].x;
    }
  }
}

// replica 0 of every row of a padded n x stride array <-> n compact floats
__global__ __launch_bounds__(kBlock) void compact_pack_kernel(const float* __restrict__ src, int stride, int n,
                                                              float* __restrict__ dst) {
  const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (i < n) dst[i] = src[(size_t)i * stride];
}
__global__ __launch_bounds__(kBlock) void compact_unpack_kernel(const float* __restrict__ src, int n, int stride,
                                                                float* __restrict__ dst) {
  const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (i >= n) return;
  float4 x = make_float4(src[i], 0.f, 0.f, 0.f);  // padding replicas stay 0
  *reinterpret_cast<float4*>(dst + (size_t)i * stride) = x;
}

static unsigned blocks_n(int n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_compact_step(const StepParams& p, const float* Pc_in, float* Pc_out, float* mc, float* vc,
                               hipStream_t st) {
  if (p.n == 0) return hipSuccess;
  if (p.S != 1 || p.coupling || p.problem == kMAXCLIQUE) return hipErrorInvalidValue;
  // lanes per variable: the context's replica layout for S = 1
  const int lpr = replica_shape(1, p.lanes_per_row).lpr;
#define X(L)                                                                                          \
  if (lpr == L) {                                                                                     \
    hipLaunchKernelGGL((compact_step_kernel<L>), dim3((unsigned)(((long long)p.n * L + kBlock - 1) / kBlock)), \
                       dim3(kBlock), 0, st, p, Pc_in, Pc_out, mc, vc);                                \
    return hipGetLastError();                                                                         \
  }
  X(1) X(2) X(4) X(8) X(16) X(32) X(64)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_compact_pack(const float* src, int stride, int n, float* dst, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(compact_pack_kernel, dim3(blocks_n(n)), dim3(kBlock), 0, st, src, stride, n, dst);
  return hipGetLastError();
}

hipError_t launch_compact_unpack(const float* src, int n, int stride, float* dst, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (stride != 4) return hipErrorInvalidValue;
  hipLaunchKernelGGL(compact_unpack_kernel, dim3(blocks_n(n)), dim3(kBlock), 0, st, src, n, stride, dst);
  return hipGetLastError();
}

}  // namespace qqa
