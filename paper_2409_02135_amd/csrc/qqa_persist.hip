// Persistent engines: one launch runs every update of an instance with its replica state
// (p, m, v) resident in registers (multi-block, grid barrier between updates) or, for an
// instance small enough, P resident in the LDS of a single workgroup.  Rows use the same
// device functions as the streaming kernels (qqa_device.h), so every engine produces the
// same bits.
#include "qqa_device.h"

namespace qqa {

namespace {

constexpr unsigned kSpinLimit = 1u << 22;  // about seconds of polling: a barrier that never fills aborts
constexpr int kLdsBlock = 1024;

// Grid-wide barrier: every block arrives once per update; `target` counts arrivals since
// the launch.  The state other blocks read (P) is written and read with device-coherent
// accesses, so the barrier only has to order completion: each wave waits for its stores
// to complete before the workgroup arrives.  Returns false when the barrier aborted.
__device__ __forceinline__ bool grid_sync(unsigned* bar, unsigned target) {
  __shared__ int ok;
  __builtin_amdgcn_s_waitcnt(0);  // this wave's coherent stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    int good = 1;
    atomicAdd(&bar[0], 1u);
    unsigned spins = 0;
    while (__hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++spins > kSpinLimit) {
        atomicOr(&bar[1], 1u);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

__device__ __forceinline__ void per_update(const PersistParams& pp, int t, StepParams* a) {
  const float4 tb = pp.table[t];
  a->ce = tb.x;
  a->inv_bc1 = tb.y;
  a->inv_bc2 = tb.z;
  a->k = (uint32_t)t + 1u;
}

template <int LPR, int RPG, bool COHERENT>
__device__ __forceinline__ void run_rows(StepParams& a, const int row0, const int gl, float4 (&p)[RPG][1],
                                         float4 (&mm)[RPG][1], float4 (&vv)[RPG][1]) {
#pragma unroll
  for (int r = 0; r < RPG; ++r) {
    const int row = row0 + r;
    if (row >= a.n) continue;
    float4 acc[1], po[1], mo[1], vo[1];
    // one edge per batch: the register-resident engine needs the registers, and the LDS engine
    // gathers from LDS, where batches only add loads past the row's end (measured on the
    // LDS engine: 3.5 against 4.4 us per update at 8 edges, RRG n = 256, S = 16)
    row_coupling<LPR, 1, true, COHERENT, true, false, 1>(a, row, row_meta(a, row), gl, acc);
    finish_row<LPR, 1, true, false>(a, row, gl, p[r], mm[r], vv[r], acc, po, mo, vo);  // never max clique
    store_row<LPR, 1, true, COHERENT>(a, a.P_out, row, gl, po, mo, vo, false);
    p[r][0] = po[0];
    mm[r][0] = mo[0];
    vv[r][0] = vo[0];
  }
}

template <int LPR, int RPG>
__device__ __forceinline__ void store_moments(const StepParams& a, const int row0, const int gl,
                                              const float4 (&mm)[RPG][1], const float4 (&vv)[RPG][1]) {
  if (a.rule != kADAMW) return;
#pragma unroll
  for (int r = 0; r < RPG; ++r) {
    const int row = row0 + r;
    if (row >= a.n) continue;
    const size_t off = (size_t)row * a.stride + 4 * gl;
    *reinterpret_cast<float4*>(a.m + off) = mm[r][0];
    *reinterpret_cast<float4*>(a.v + off) = vv[r][0];
  }
}

}  // namespace

template <int LPR, int RPG>
__global__ __launch_bounds__(kBlock) void persistent_kernel(PersistParams pp) {
  int group = (int)(((long long)blockIdx.x * kBlock + threadIdx.x) / LPR);
  if (LPR == 64) group = __builtin_amdgcn_readfirstlane(group);
  const int gl = threadIdx.x & (LPR - 1);
  const int row0 = group * RPG;
  StepParams a = pp.a;
  float4 p[RPG][1], mm[RPG][1], vv[RPG][1];
#pragma unroll
  for (int r = 0; r < RPG; ++r)
    if (row0 + r < a.n) load_row<LPR, 1, true>(a, pp.P[pp.t0 & 1], row0 + r, gl, p[r], mm[r], vv[r]);
  for (int t = pp.t0; t < pp.t1; ++t) {
    a.P_in = pp.P[t & 1];
    a.P_out = pp.P[(t + 1) & 1];
    per_update(pp, t, &a);
    run_rows<LPR, RPG, true>(a, row0, gl, p, mm, vv);
    if (!grid_sync(pp.bar, (unsigned)(t - pp.t0 + 1) * gridDim.x)) return;
  }
  store_moments<LPR, RPG>(a, row0, gl, mm, vv);
}

// Single workgroup: P ping-pongs between two LDS buffers, updates are separated by
// workgroup barriers only.  The update loop reads no global memory but the per-update
// scalars and the normals, which the whole GPU forms beforehand (pp.noise): one workgroup
// cannot hide the generator's dependent chain behind other rows.  Both are loaded one
// update ahead (the loop is unrolled by two, so the loaded registers are never copied, which
// would wait for the loads), and the rows' CSR ranges stay in registers.  CSR: where the
// column indices (1), and the weights (2), sit: 0 global memory, else copied into LDS after
// the two P buffers, so that the gathers wait on LDS alone.
template <int LPR, int RPG, int CSR, int SPEC>
__device__ __forceinline__ void lds_update(const StepParams& a0, float4* lds, const int* lcol,
                                           const float* lw, const int in_q, const int out_q, const int t,
                                           const float4 tb, const int row0, const int gl, const int (&e0)[RPG],
                                           const int (&e1)[RPG], float4 (&p)[RPG][1], float4 (&mm)[RPG][1],
                                           float4 (&vv)[RPG][1], const float4 (&xi)[RPG]) {
  StepParams a = a0;
  a.ce = tb.x;
  a.inv_bc1 = tb.y;
  a.inv_bc2 = tb.z;
  a.k = (uint32_t)t + 1u;
  const bool maxcut = SPEC ? spec_problem(SPEC) == kMAXCUT : a.problem == kMAXCUT;
  // a lane group past the last row updates that row too (its registers hold it) and stores
  // nothing: no branch around the update, across which the loads in flight would be waited for
#pragma unroll
  for (int r = 0; r < RPG; ++r) {
    const int row = min(row0 + r, a.n - 1);
    // the coupling sum in CSR order, as gather_coupling forms it
    float4 acc[1] = {make_float4(0.f, 0.f, 0.f, 0.f)};
    for (int e = e0[r]; e < e1[r]; ++e) {
      const int j = CSR ? lcol[e] : a.col[e];
      const float w = CSR == 2 ? lw[e] : (CSR == 0 && a.w ? a.w[e] : 1.f);
      const float4 x = lds[in_q + j * LPR + gl];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float xc = comp(x, c);
        const float f = maxcut ? 2.f * xc - 1.f : xc;
        set_comp(acc[0], c, fmaf(w, f, comp(acc[0], c)));
      }
    }
    float mu, cg;
    row_stats<LPR, 1, true>(a, gl, p[r], mu, cg);
    float4 po[1], mo[1], vo[1];
    const float4 x[1] = {xi[r]};
    finish_elems<LPR, 1, true, false, true, SPEC>(a, row, gl, 0, mu, cg, p[r], mm[r], vv[r], acc, po, mo, vo, x);
    if (row0 + r < a.n) lds[out_q + row * LPR + gl] = po[0];
    p[r][0] = po[0];
    mm[r][0] = mo[0];
    vv[r][0] = vo[0];
  }
}

template <int LPR, int RPG, int CSR, int SPEC>
__global__ __launch_bounds__(kLdsBlock) void lds_block_kernel(PersistParams pp) {
  extern __shared__ float4 lds[];
  const StepParams a = pp.a;
  const int n = a.n;
  const int quads = n * LPR;  // float4 per P buffer (S = 4 LPR, so the stride is 4 LPR)
  const int t0 = pp.t0, t1 = pp.t1;
  {
    const float4* src = reinterpret_cast<const float4*>(pp.P[t0 & 1]);
    const int b = (t0 & 1) * quads;
    for (int i = threadIdx.x; i < quads; i += kLdsBlock) lds[b + i] = src[i];
  }
  int* lcol = reinterpret_cast<int*>(lds + 2 * quads);
  float* lw = reinterpret_cast<float*>(lcol + pp.nnz);
  if (CSR)
    for (int i = threadIdx.x; i < pp.nnz; i += kLdsBlock) {
      lcol[i] = a.col[i];
      if (CSR == 2) lw[i] = a.w[i];
    }
  const int group = (int)threadIdx.x / LPR;
  const int gl = threadIdx.x & (LPR - 1);
  const int row0 = group * RPG;
  float4 p[RPG][1], mm[RPG][1], vv[RPG][1];
  int e0[RPG], e1[RPG];
#pragma unroll
  for (int r = 0; r < RPG; ++r) {
    const int row = min(row0 + r, n - 1);
    load_row<LPR, 1, true>(a, pp.P[t0 & 1], row, gl, p[r], mm[r], vv[r]);
    e0[r] = a.row_ptr[row];
    e1[r] = a.row_ptr[row + 1];
  }
  __syncthreads();
  // normals of update t, row i, lane quad gl at noise[((t - t0) n + i) LPR + gl]
  const size_t per_update = (size_t)n * LPR;
  float4 xa[RPG], xb[RPG], ta, tb;
  auto fetch = [&](int t, float4(&x)[RPG], float4& tv) {
    t = min(t, t1 - 1);
    tv = pp.table[t];
#pragma unroll
    for (int r = 0; r < RPG; ++r)
      x[r] = pp.noise[(size_t)(t - t0) * per_update + (size_t)min(row0 + r, n - 1) * LPR + gl];
  };
  if (t0 < t1) fetch(t0, xa, ta);
  for (int t = t0; t < t1;) {
    fetch(t + 1, xb, tb);
    lds_update<LPR, RPG, CSR, SPEC>(a, lds, lcol, lw, (t & 1) * quads, ((t + 1) & 1) * quads, t, ta, row0, gl, e0,
                              e1, p, mm, vv, xa);
    __syncthreads();
    if (++t >= t1) break;
    fetch(t + 1, xa, ta);
    lds_update<LPR, RPG, CSR, SPEC>(a, lds, lcol, lw, (t & 1) * quads, ((t + 1) & 1) * quads, t, tb, row0, gl, e0,
                              e1, p, mm, vv, xb);
    __syncthreads();
    ++t;
  }
  float4* out = reinterpret_cast<float4*>(pp.P[t1 & 1]);
  const int b = (t1 & 1) * quads;
  for (int i = threadIdx.x; i < quads; i += kLdsBlock) out[i] = lds[b + i];
  store_moments<LPR, RPG>(a, row0, gl, mm, vv);
}

// ---- planning and launch -------------------------------------------------------------------
#define QQA_LDS_LAYOUTS(X) X(1) X(2) X(4) X(8) X(16) X(32) X(64)

template <int LPR, int RPG>
static int coresident_blocks() {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<LPR, RPG>, kBlock, 0) != hipSuccess)
    return 0;
  return per_cu * prop.multiProcessorCount;
}

static size_t lds_limit() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  return prop.sharedMemPerBlock;
}

// rows per lane group the multi-block engine is built for, per lanes-per-row (chosen so
// that the resident state fits the register file without spills)
#define QQA_PERSIST_RPG_64(X) X(64, 2) X(64, 4) X(64, 6) X(64, 8) X(64, 10)
#define QQA_PERSIST_RPG_32(X) X(32, 2) X(32, 4) X(32, 6) X(32, 8)
#define QQA_PERSIST_RPG_16(X) X(16, 2) X(16, 4) X(16, 6) X(16, 8)
#define QQA_PERSIST_ALL(X) QQA_PERSIST_RPG_64(X) QQA_PERSIST_RPG_32(X) QQA_PERSIST_RPG_16(X)

int persistent_plan(const StepParams& a, bool has_hubs, int allow, int* rows_per_group, int* grid) {
  if (!allow || has_hubs || a.coupling || a.n <= 0) return kEngineStream;
  const ReplicaShape r = replica_shape(a.S, a.lanes_per_row);
  if (r.qpl != 1 || a.S != 4 * r.lpr) return kEngineStream;
  // one workgroup with P in LDS
  const size_t lds = 2 * (size_t)a.n * a.stride * sizeof(float);
  const int groups_lds = kLdsBlock / r.lpr;
  if ((allow & 1) && lds <= lds_limit()) {
    for (int rpg = 1; rpg <= 4; rpg *= 2)
      if ((long long)groups_lds * rpg >= a.n) {
        *rows_per_group = rpg;
        *grid = 1;
        return kEngineLdsBlock;
      }
  }
  if (!(allow & 2)) return kEngineStream;
  // many workgroups, state in registers: the fewest rows per group whose grid is co-resident
#define X(L, R)                                                        \
  if (r.lpr == L) {                                                    \
    const long long groups = (a.n + R - 1) / R;                        \
    const long long blocks = (groups * L + kBlock - 1) / kBlock;       \
    if (blocks <= coresident_blocks<L, R>()) {                         \
      *rows_per_group = R;                                             \
      *grid = (int)blocks;                                             \
      return kEnginePersistent;                                        \
    }                                                                  \
  }
  QQA_PERSIST_ALL(X)
#undef X
  return kEngineStream;
}

template <int LPR, int RPG>
static hipError_t launch_coop(const PersistParams& pp, int grid, hipStream_t st) {
  PersistParams arg = pp;
  void* args[] = {&arg};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(persistent_kernel<LPR, RPG>), dim3(grid),
                                    dim3(kBlock), args, 0, st);
}

hipError_t launch_persistent(const PersistParams& pp, int engine, int rpg, int grid, hipStream_t st) {
  const ReplicaShape r = replica_shape(pp.a.S, pp.a.lanes_per_row);
  if (engine == kEngineLdsBlock) {
    if (!pp.noise || pp.t0 > pp.t1) return hipErrorInvalidValue;
    if (pp.t0 == pp.t1) return hipSuccess;
    // the CSR arrays join P in LDS when they fit
    const size_t lds_p = 2 * (size_t)pp.a.n * pp.a.stride * sizeof(float);
    const size_t lds_csr = (size_t)pp.nnz * sizeof(int32_t) * (pp.a.w ? 2 : 1);
    const int csr = pp.nnz > 0 && lds_p + lds_csr <= lds_limit() ? (pp.a.w ? 2 : 1) : 0;
    const size_t lds = lds_p + (csr ? lds_csr : 0);
    // the default schedule (AdamW, entropy alpha 4) of unweighted MIS and weighted max-cut with
    // the CSR in LDS runs with those facts fixed at compile time
    const bool dflt = pp.a.rule == kADAMW && pp.a.alpha_e == 4;
    const bool mis1 = dflt && csr == 1 && pp.a.problem == kMIS, cut2 = dflt && csr == 2 && pp.a.problem == kMAXCUT;
#define K(L, R, C, SP) hipLaunchKernelGGL((lds_block_kernel<L, R, C, SP>), dim3(1), dim3(kLdsBlock), lds, st, pp)
#define RPG_CASE(L, N)                                          \
  case N:                                                       \
    if (cut2) K(L, N, 2, spec_of(kMAXCUT, kADAMW, 4));          \
    else if (mis1) K(L, N, 1, spec_of(kMIS, kADAMW, 4));        \
    else if (csr == 2) K(L, N, 2, 0);                           \
    else if (csr == 1) K(L, N, 1, 0);                           \
    else K(L, N, 0, 0);                                         \
    break;
#define X(L)                                  \
  if (r.lpr == L) {                           \
    switch (rpg) {                            \
      RPG_CASE(L, 1) RPG_CASE(L, 2) RPG_CASE(L, 4) \
      default: return hipErrorInvalidValue;   \
    }                                         \
    return hipGetLastError();                 \
  }
    QQA_LDS_LAYOUTS(X)
#undef X
#undef RPG_CASE
#undef K
    return hipErrorInvalidValue;
  }
  if (engine == kEnginePersistent) {
#define X(L, R) \
  if (r.lpr == L && rpg == R) return launch_coop<L, R>(pp, grid, st);
    QQA_PERSIST_ALL(X)
#undef X
  }
  return hipErrorInvalidValue;
}

// The noise table of an LDS-block solve: thread i forms the normals of quad q of row `row`
// at update t, exactly as finish_elems does in the update kernels.
__global__ __launch_bounds__(kBlock) void noise_table_kernel(StepParams a, int t0, int t1, int nq,
                                                             float4* __restrict__ xi) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long per = (long long)a.n * nq;
  if (i >= per * (t1 - t0)) return;
  const int dt = (int)(i / per);
  const long long rq = i - (long long)dt * per;
  const int row = (int)(rq / nq), q = (int)(rq - (long long)row * nq);
  xi[i] = normals4(philox4x32_10((uint32_t)row, (uint32_t)q, (uint32_t)(t0 + dt) + 1u, kStreamNoise, a.key0, a.key1));
}

hipError_t launch_noise_table(const StepParams& a, int t0, int t1, float4* xi, hipStream_t st) {
  if (a.n <= 0 || t1 <= t0) return hipSuccess;
  const int nq = a.stride / 4;
  const long long total = (long long)a.n * nq * (t1 - t0);
  hipLaunchKernelGGL(noise_table_kernel, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, a, t0,
                     t1, nq, xi);
  return hipGetLastError();
}

}  // namespace qqa
