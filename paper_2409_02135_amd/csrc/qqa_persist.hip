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
// workgroup barriers only.
template <int LPR, int RPG>
__global__ __launch_bounds__(kLdsBlock) void lds_block_kernel(PersistParams pp) {
  extern __shared__ float4 lds[];
  StepParams a = pp.a;
  const size_t words = (size_t)a.n * a.stride;
  float* sP[2] = {reinterpret_cast<float*>(lds), reinterpret_cast<float*>(lds) + words};
  const float4* src = reinterpret_cast<const float4*>(pp.P[pp.t0 & 1]);
  float4* dst0 = reinterpret_cast<float4*>(sP[pp.t0 & 1]);
  for (size_t i = threadIdx.x; i < words / 4; i += kLdsBlock) dst0[i] = src[i];
  __syncthreads();
  const int group = (int)threadIdx.x / LPR;
  const int gl = threadIdx.x & (LPR - 1);
  const int row0 = group * RPG;
  float4 p[RPG][1], mm[RPG][1], vv[RPG][1];
#pragma unroll
  for (int r = 0; r < RPG; ++r)
    if (row0 + r < a.n) load_row<LPR, 1, true>(a, sP[pp.t0 & 1], row0 + r, gl, p[r], mm[r], vv[r]);
  for (int t = pp.t0; t < pp.t1; ++t) {
    a.P_in = sP[t & 1];
    a.P_out = sP[(t + 1) & 1];
    per_update(pp, t, &a);
    run_rows<LPR, RPG, false>(a, row0, gl, p, mm, vv);
    __syncthreads();
  }
  const float4* fin = reinterpret_cast<const float4*>(sP[pp.t1 & 1]);
  float4* out = reinterpret_cast<float4*>(pp.P[pp.t1 & 1]);
  for (size_t i = threadIdx.x; i < words / 4; i += kLdsBlock) out[i] = fin[i];
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
    const size_t lds = 2 * (size_t)pp.a.n * pp.a.stride * sizeof(float);
#define X(L)                                                                                                \
  if (r.lpr == L) {                                                                                         \
    switch (rpg) {                                                                                          \
      case 1: hipLaunchKernelGGL((lds_block_kernel<L, 1>), dim3(1), dim3(kLdsBlock), lds, st, pp); break; \
      case 2: hipLaunchKernelGGL((lds_block_kernel<L, 2>), dim3(1), dim3(kLdsBlock), lds, st, pp); break; \
      case 4: hipLaunchKernelGGL((lds_block_kernel<L, 4>), dim3(1), dim3(kLdsBlock), lds, st, pp); break; \
      default: return hipErrorInvalidValue;                                                                 \
    }                                                                                                       \
    return hipGetLastError();                                                                               \
  }
    QQA_LDS_LAYOUTS(X)
#undef X
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

}  // namespace qqa
