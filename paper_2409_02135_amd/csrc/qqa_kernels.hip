// HIP kernels (gfx950) of the PQQA replica update: counter-based noise, initial state,
// the fused sparse update, and exact rounding/evaluation.
//
// Data layout: replica state is row-major n x stride float32 with the replica index
// contiguous, so the S values of one variable are one contiguous row.  A row is served
// by `lpr` adjacent lanes of one wavefront (lpr = 64 for S >= 256, several rows per
// wavefront for smaller S); each lane owns float4 quads of replicas, which makes every
// neighbour-row gather a coalesced, 16-byte-per-lane load and gives one Philox call
// (4 normals) per lane and quad.
#include <algorithm>

#include "qqa_device.h"

namespace qqa {

__global__ void philox_kernel(uint32_t k0, uint32_t k1, int n, int nquads, uint32_t k, uint32_t sid, uint32_t* out) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * nquads) return;
  const int i = (int)(idx / nquads), q = (int)(idx % nquads);
  const U4 r = philox4x32_10((uint32_t)i, (uint32_t)q, k, sid, k0, k1);
  reinterpret_cast<uint4*>(out)[idx] = make_uint4(r.x, r.y, r.z, r.w);
}

__global__ void noise_kernel(uint32_t k0, uint32_t k1, int n, int nquads, int S, uint32_t k, float* xi) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * nquads) return;
  const int i = (int)(idx / nquads), q = (int)(idx % nquads);
  float4 z = normals4(philox4x32_10((uint32_t)i, (uint32_t)q, k, kStreamNoise, k0, k1));
  const int s0 = 4 * q;
  if (s0 + 1 >= S) z.y = 0.f;
  if (s0 + 2 >= S) z.z = 0.f;
  if (s0 + 3 >= S) z.w = 0.f;
  reinterpret_cast<float4*>(xi)[idx] = z;
}

__global__ void init_kernel(uint32_t k0, uint32_t k1, int n, int nquads, int S, float* P, float* m, float* v) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * nquads) return;
  const int i = (int)(idx / nquads), q = (int)(idx % nquads);
  const U4 r = philox4x32_10((uint32_t)i, (uint32_t)q, 0u, kStreamInit, k0, k1);
  const int s0 = 4 * q;
  float4 p = make_float4(u01(r.x), s0 + 1 < S ? u01(r.y) : 0.f, s0 + 2 < S ? u01(r.z) : 0.f,
                         s0 + 3 < S ? u01(r.w) : 0.f);
  reinterpret_cast<float4*>(P)[idx] = p;
  if (m) reinterpret_cast<float4*>(m)[idx] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (v) reinterpret_cast<float4*>(v)[idx] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Partial coupling sum of one chunk of a split row.
template <int LPR, int QPL, bool FULL>
__global__ __launch_bounds__(kBlock) void hub_partial_kernel(StepParams a, const HubChunk* chunks, int nchunks) {
  int c = (int)(((long long)blockIdx.x * kBlock + threadIdx.x) / LPR);
  if (LPR == 64) c = __builtin_amdgcn_readfirstlane(c);
  if (c >= nchunks) return;
  const int gl = threadIdx.x & (LPR - 1);
  const int nq = FULL ? LPR * QPL : (a.S + 3) >> 2;
  const HubChunk ch = chunks[c];
  const int e_end = min(ch.e0 + kHubChunk, a.row_ptr[ch.row + 1]);
  float4 acc[QPL];
#pragma unroll
  for (int k = 0; k < QPL; ++k) acc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
  gather_coupling<LPR, QPL, FULL>(a, ch.e0, e_end, gl, nq, a.problem == kMAXCUT, acc);
  float* out = const_cast<float*>(a.hub_partial) + (size_t)c * a.stride;
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int q = gl + LPR * k;
    if (FULL || q < nq) *reinterpret_cast<float4*>(out + 4 * q) = acc[k];
  }
}

// SUMS: the max-clique instance (reads the per-replica sums); the others do not carry it.
// DENSE: the coupling product comes from a.coupling (dense graphs, any problem).
template <int LPR, int QPL, bool FULL, bool SUMS, bool DENSE = false>
__global__ __launch_bounds__(kBlock) void step_kernel(StepParams a) {
  int row = (int)(((long long)blockIdx.x * kBlock + threadIdx.x) / LPR);
  // a whole wavefront serves one row when LPR = 64: make that explicit so the CSR reads
  // become scalar loads and neighbour addresses a scalar base plus the lane offset
  if (LPR == 64) row = __builtin_amdgcn_readfirstlane(row);
  if (row >= a.n) return;  // whole LPR-lane groups leave together
  update_row<LPR, QPL, FULL, SUMS, DENSE>(a, row, threadIdx.x & (LPR - 1));
}

// ---------------------------------------------------------------------------------------
// Exact rounding + evaluation.  Each lane keeps int64 partial counts for the replicas it
// owns over a grid-stride of rows, the block folds them in LDS, then one atomic per
// replica per block; integer addition makes the result independent of order.
// ---------------------------------------------------------------------------------------
template <int LPR, int QPL>
__global__ __launch_bounds__(kBlock) void eval_kernel(EvalParams a) {
  extern __shared__ unsigned long long sh[];  // [2][stride]
  const int nq = (a.S + 3) >> 2;
  for (int s = threadIdx.x; s < 2 * a.stride; s += kBlock) sh[s] = 0ull;
  __syncthreads();
  const int gpb = kBlock / LPR;
  const int gl = threadIdx.x & (LPR - 1);
  const bool maxcut = a.problem == kMAXCUT;
  long long ca[QPL][4], cb[QPL][4];
#pragma unroll
  for (int k = 0; k < QPL; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) ca[k][c] = cb[k][c] = 0;

  for (int row = blockIdx.x * gpb + threadIdx.x / LPR; row < a.n; row += gridDim.x * gpb) {
    bool xi[QPL][4];
#pragma unroll
    for (int k = 0; k < QPL; ++k) {
      const int q = gl + LPR * k;
      float4 pv = make_float4(0.f, 0.f, 0.f, 0.f);
      if (q < nq) pv = *reinterpret_cast<const float4*>(a.P + (size_t)row * a.stride + 4 * q);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        xi[k][c] = comp(pv, c) > 0.5f;
        if (!maxcut) ca[k][c] += xi[k][c];
      }
    }
    const int deg = a.dense ? a.n : a.row_ptr[row + 1] - a.row_ptr[row];
    for (int u = 0; u < deg; ++u) {
      int j;
      float w;
      if (a.dense) {
        j = u;
        w = a.dense[(size_t)row * a.n + u];
      } else {
        const int e = a.row_ptr[row] + u;
        j = a.col[e];
        w = a.w ? a.w[e] : 1.f;
      }
      if (j <= row || w == 0.f) continue;  // each undirected edge once
      const long long qw = maxcut ? (long long)(w * 65536.0f) : 0;
#pragma unroll
      for (int k = 0; k < QPL; ++k) {
        const int q = gl + LPR * k;
        if (q >= nq) continue;
        const float4 pj = *reinterpret_cast<const float4*>(a.P + (size_t)j * a.stride + 4 * q);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const bool xj = comp(pj, c) > 0.5f;
          if (maxcut) ca[k][c] += (xi[k][c] != xj) ? qw : 0;
          else cb[k][c] += (xi[k][c] && xj);
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int q = gl + LPR * k;
    if (q >= nq) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int s = 4 * q + c;
      if (s >= a.S) continue;
      if (ca[k][c]) atomicAdd(&sh[s], (unsigned long long)ca[k][c]);
      if (cb[k][c]) atomicAdd(&sh[a.stride + s], (unsigned long long)cb[k][c]);
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < a.S; s += kBlock) {
    if (sh[s]) atomicAdd(&a.acc[s], sh[s]);
    if (sh[a.stride + s]) atomicAdd(&a.acc[a.stride + s], sh[a.stride + s]);
  }
}

// Violations and objective of replica s from the counts: MIS counts selected adjacent
// pairs; max clique turns the count of selected adjacent pairs into the selected pairs
// that are not adjacent, size (size - 1) / 2 - count; max-cut has none.
__device__ __forceinline__ void derive(const EvalParams& a, int s, long long* A, long long* B, long long* o) {
  *A = (long long)a.acc[s];
  if (a.problem == kCOLORING) {  // cost = violations = edges whose ends share a colour
    *B = *A;
    *o = *A;
    return;
  }
  const long long cnt = (long long)a.acc[a.stride + s];
  *B = a.problem == kMAXCLIQUE ? *A * (*A - 1) / 2 - cnt : cnt;
  *o = a.problem == kMAXCUT ? -*A : -*A + a.lambda * *B;
}

// objectives and the lexicographic best replica (violations > 0, l, index)
__global__ __launch_bounds__(kBlock) void finalize_kernel(EvalParams a) {
  __shared__ int best_s[kBlock];
  int mine = -1;
  bool mi = false;
  long long mo = 0;
  for (int s = threadIdx.x; s < a.S; s += kBlock) {
    long long A, B, o;
    derive(a, s, &A, &B, &o);
    a.size_or_cut[s] = A;
    a.viol[s] = B;
    a.obj[s] = o;
    const bool inf = B > 0;
    if (mine < 0 || (inf < mi) || (inf == mi && o < mo)) {
      mine = s;
      mi = inf;
      mo = o;
    }
  }
  best_s[threadIdx.x] = mine;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const int x = best_s[threadIdx.x], y = best_s[threadIdx.x + off];
      if (y >= 0) {
        bool take = x < 0;
        if (!take) {
          long long Ax, Bx, ox, Ay, By, oy;
          derive(a, x, &Ax, &Bx, &ox);
          derive(a, y, &Ay, &By, &oy);
          const bool ix = Bx > 0, iy = By > 0;
          take = (iy < ix) || (iy == ix && (oy < ox || (oy == ox && y < x)));
        }
        if (take) best_s[threadIdx.x] = y;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) a.best[0] = best_s[0];
}

__global__ void extract_kernel(const float* P, int n, int stride, const int32_t* best, uint8_t* x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = P[(size_t)i * stride + best[0]] > 0.5f ? 1 : 0;
}

// ---------------------------------------------------------------------------------------
// Per-replica sums of P (max clique).  Block b sums rows [b * rows, (b + 1) * rows): each
// thread takes one quad of replicas and every lanes-th row of the band, in 2^-32 fixed
// point (p in [0, 1] times 2^32 is exact in double, then rounded once), so the block's
// partial and the final total are exact integers whatever order the additions run in.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void colsum_kernel(const float* __restrict__ P, int n, int stride, int rows,
                                                        unsigned long long* __restrict__ T) {
  extern __shared__ unsigned long long colsum_sh[];  // [stride]
  for (int c = threadIdx.x; c < stride; c += kBlock) colsum_sh[c] = 0ull;
  __syncthreads();
  const int nq = stride >> 2;
  const int lanes = nq >= kBlock ? 1 : kBlock / nq;  // row lanes per quad
  const int r0 = blockIdx.x * rows, r1 = min(n, r0 + rows);
  for (int slot = threadIdx.x; slot < lanes * nq; slot += kBlock) {
    const int q = slot % nq, rl = slot / nq;
    unsigned long long acc[4] = {0ull, 0ull, 0ull, 0ull};
    for (int r = r0 + rl; r < r1; r += lanes) {
      const float4 v = *reinterpret_cast<const float4*>(P + (size_t)r * stride + 4 * q);
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] += (unsigned long long)__double2ull_rn((double)comp(v, c) * 0x1p32);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (acc[c]) atomicAdd(&colsum_sh[4 * q + c], acc[c]);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < stride; c += kBlock)
    if (colsum_sh[c]) atomicAdd(&T[c], colsum_sh[c]);
}

__global__ void fill_u64_kernel(unsigned long long* p, size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
}

// ---------------------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------------------
ReplicaShape replica_shape(int S) { return replica_shape(S, 0); }

// lanes_per_row = 0: the default layout (fewest quads per lane, at most one wavefront per
// row); otherwise the requested power of two, with enough quads per lane to cover S.
ReplicaShape replica_shape(int S, int lanes_per_row) {
  ReplicaShape r;
  r.nquads = (S + 3) / 4;
  r.stride = 4 * r.nquads;
  int lpr = 1;
  if (lanes_per_row > 0) {
    while (lpr < lanes_per_row && lpr < 64) lpr <<= 1;
    // a group wider than the row's quads splits the row's edges between lane slices, which
    // needs the quad count to divide the group; otherwise no wider than the row needs
    const bool pow2 = (r.nquads & (r.nquads - 1)) == 0;
    if (!pow2)
      while (lpr > 1 && lpr / 2 >= r.nquads) lpr >>= 1;
  } else {
    while (lpr < r.nquads && lpr < 64) lpr <<= 1;
  }
  r.lpr = lpr;
  int qpl = 1;
  while (lpr * qpl < r.nquads) qpl <<= 1;
  r.qpl = qpl;
  return r;
}


bool layout_supported(int S, int lanes_per_row) {
  const ReplicaShape r = replica_shape(S, lanes_per_row);
#define X(L, Q) \
  if (r.lpr == L && r.qpl == Q) return true;
  QQA_FOR_EACH_LAYOUT(X)
#undef X
  return false;
}


static unsigned grid_for(long long threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

hipError_t launch_philox(uint64_t seed, int n, int nquads, uint32_t k, uint32_t sid, uint32_t* out, hipStream_t st) {
  const long long work = (long long)n * nquads;
  if (work == 0) return hipSuccess;
  hipLaunchKernelGGL(philox_kernel, dim3(grid_for(work)), dim3(kBlock), 0, st, (uint32_t)seed,
                     (uint32_t)(seed >> 32), n, nquads, k, sid, out);
  return hipGetLastError();
}

hipError_t launch_noise(uint64_t seed, int n, int S, uint32_t k, float* xi, hipStream_t st) {
  const int nq = (S + 3) / 4;
  const long long work = (long long)n * nq;
  if (work == 0) return hipSuccess;
  hipLaunchKernelGGL(noise_kernel, dim3(grid_for(work)), dim3(kBlock), 0, st, (uint32_t)seed, (uint32_t)(seed >> 32),
                     n, nq, S, k, xi);
  return hipGetLastError();
}

hipError_t launch_init(uint64_t seed, int n, int S, float* P, float* m, float* v, hipStream_t st) {
  const int nq = (S + 3) / 4;
  const long long work = (long long)n * nq;
  if (work == 0) return hipSuccess;
  hipLaunchKernelGGL(init_kernel, dim3(grid_for(work)), dim3(kBlock), 0, st, (uint32_t)seed, (uint32_t)(seed >> 32),
                     n, nq, S, P, m, v);
  return hipGetLastError();
}

template <int LPR, int QPL>
static void launch_step_t(const StepParams& p, hipStream_t st) {
  const dim3 grid(grid_for((long long)p.n * LPR)), block(kBlock);
  const bool full = p.S == 4 * LPR * QPL;
  if (p.coupling) {
    if (full) hipLaunchKernelGGL((step_kernel<LPR, QPL, true, true, true>), grid, block, 0, st, p);
    else hipLaunchKernelGGL((step_kernel<LPR, QPL, false, true, true>), grid, block, 0, st, p);
  } else if (p.problem == kMAXCLIQUE) {
    if (full) hipLaunchKernelGGL((step_kernel<LPR, QPL, true, true>), grid, block, 0, st, p);
    else hipLaunchKernelGGL((step_kernel<LPR, QPL, false, true>), grid, block, 0, st, p);
  } else {
    if (full) hipLaunchKernelGGL((step_kernel<LPR, QPL, true, false>), grid, block, 0, st, p);
    else hipLaunchKernelGGL((step_kernel<LPR, QPL, false, false>), grid, block, 0, st, p);
  }
}

template <int LPR, int QPL>
static void launch_hub_t(const StepParams& p, const HubChunk* chunks, int nchunks, hipStream_t st) {
  const dim3 grid(grid_for((long long)nchunks * LPR)), block(kBlock);
  if (p.S == 4 * LPR * QPL)
    hipLaunchKernelGGL((hub_partial_kernel<LPR, QPL, true>), grid, block, 0, st, p, chunks, nchunks);
  else
    hipLaunchKernelGGL((hub_partial_kernel<LPR, QPL, false>), grid, block, 0, st, p, chunks, nchunks);
}

hipError_t launch_hub_partials(const StepParams& p, const HubChunk* chunks, int nchunks, hipStream_t st) {
  if (nchunks == 0) return hipSuccess;
  const ReplicaShape r = replica_shape(p.S, p.lanes_per_row);
#define X(L, Q)                                 \
  if (r.lpr == L && r.qpl == Q) {               \
    launch_hub_t<L, Q>(p, chunks, nchunks, st); \
    return hipGetLastError();                   \
  }
  QQA_FOR_EACH_LAYOUT(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_step(const StepParams& p, hipStream_t st) {
  if (p.n == 0) return hipSuccess;
  const ReplicaShape r = replica_shape(p.S, p.lanes_per_row);
#define X(L, Q)                   \
  if (r.lpr == L && r.qpl == Q) { \
    launch_step_t<L, Q>(p, st);   \
    return hipGetLastError();     \
  }
  QQA_FOR_EACH_LAYOUT(X)
#undef X
  return hipErrorInvalidValue;
}


hipError_t launch_colsum(const float* P, int n, int stride, unsigned long long* T, hipStream_t st) {
  hipError_t e = launch_fill_u64(T, (size_t)stride, st);
  if (e != hipSuccess || n == 0) return e;
  // a few hundred blocks: enough loads in flight to stream P, few integer atomics per column
  const int blocks = std::max(1, std::min(256, (n + 7) / 8));
  const int rows = (n + blocks - 1) / blocks;
  hipLaunchKernelGGL(colsum_kernel, dim3((n + rows - 1) / rows), dim3(kBlock), (size_t)stride * sizeof(unsigned long long),
                     st, P, n, stride, rows, T);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, size_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for((long long)count)), dim3(kBlock), 0, st, p, count);
  return hipGetLastError();
}

template <int LPR, int QPL>
static void launch_eval_t(const EvalParams& p, hipStream_t st) {
  const int gpb = kBlock / LPR;
  int blocks = (p.n + gpb - 1) / gpb;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  const size_t shmem = 2 * (size_t)p.stride * sizeof(unsigned long long);
  hipLaunchKernelGGL((eval_kernel<LPR, QPL>), dim3(blocks), dim3(kBlock), shmem, st, p);
}

hipError_t launch_eval(const EvalParams& p, hipStream_t st) {
  hipError_t e = launch_fill_u64(p.acc, 2 * (size_t)p.stride, st);
  if (e != hipSuccess) return e;
  const ReplicaShape r = replica_shape(p.S);
  if (p.n > 0) {
    bool launched = false;
#define X(L, Q)                         \
    if (!launched && r.lpr == L && r.qpl == Q) { \
      launch_eval_t<L, Q>(p, st);       \
      launched = true;                  \
    }
    QQA_FOR_EACH_LAYOUT(X)
#undef X
    if (!launched) return hipErrorInvalidValue;
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return launch_finalize(p, st);
}

hipError_t launch_finalize(const EvalParams& p, hipStream_t st) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kBlock), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_extract(const float* P, int n, int stride, const int32_t* best, uint8_t* x, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(extract_kernel, dim3(grid_for(n)), dim3(kBlock), 0, st, P, n, stride, best, x);
  return hipGetLastError();
}

}  // namespace qqa
