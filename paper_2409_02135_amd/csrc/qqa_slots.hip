// Multi-instance ("slot") kernels: a work list of (slot, row block) items lets one launch
// advance many instances of different sizes -- a ragged batch or the server's admitted
// requests -- each at its own update index.  Every row goes through the same device
// functions as a single solve (qqa_device.h).
#include "qqa_device.h"

namespace qqa {

namespace {

__device__ __forceinline__ bool slot_update_index(const SlotDesc& sd, const int32_t* clock, int t_arg, int* t) {
  *t = *clock + t_arg - sd.start;
  return sd.active && *t >= 0 && *t < sd.K;
}

__device__ __forceinline__ void slot_params(const SlotDesc& sd, int t, StepParams* a) {
  *a = sd.p;
  a->P_in = sd.P[t & 1];
  a->P_out = sd.P[(t + 1) & 1];
  const float4 tb = sd.table[t];
  a->ce = tb.x;
  a->inv_bc1 = tb.y;
  a->inv_bc2 = tb.z;
  a->k = (uint32_t)t + 1u;
}

}  // namespace

template <int LPR>
__global__ __launch_bounds__(kBlock) void slot_init_kernel(const SlotDesc* slots, const WorkItem* items, int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem w = items[it];
    const SlotDesc& sd = slots[w.slot];
    if (!sd.active) continue;
    const int row = w.row0 + (int)threadIdx.x / LPR;
    if (row >= sd.p.n) continue;
    const int nq = (sd.p.S + 3) >> 2;
    for (int q = threadIdx.x & (LPR - 1); q < nq; q += LPR) {
      const U4 r = philox4x32_10((uint32_t)row, (uint32_t)q, 0u, kStreamInit, (uint32_t)sd.seed, (uint32_t)(sd.seed >> 32));
      const int s0 = 4 * q;
      const float4 p = make_float4(u01(r.x), s0 + 1 < sd.p.S ? u01(r.y) : 0.f, s0 + 2 < sd.p.S ? u01(r.z) : 0.f,
                                   s0 + 3 < sd.p.S ? u01(r.w) : 0.f);
      const size_t off = (size_t)row * sd.p.stride + 4 * q;
      *reinterpret_cast<float4*>(sd.P[0] + off) = p;
      if (sd.p.rule == kADAMW) {
        *reinterpret_cast<float4*>(sd.p.m + off) = make_float4(0.f, 0.f, 0.f, 0.f);
        *reinterpret_cast<float4*>(sd.p.v + off) = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  }
}

template <int LPR, int QPL, bool FULL, int SPEC>
__global__ __launch_bounds__(kBlock) void slot_step_kernel(const SlotDesc* slots, const WorkItem* items, int nitems,
                                                           const int32_t* clock, int t_arg) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem w = items[it];
    const SlotDesc& sd = slots[w.slot];
    int t;
    if (!slot_update_index(sd, clock, t_arg, &t)) continue;
    StepParams a;
    slot_params(sd, t, &a);
    int row = w.row0 + (int)threadIdx.x / LPR;
    if (LPR == 64) row = __builtin_amdgcn_readfirstlane(row);
    if (row >= a.n) continue;  // whole lane groups
    update_row<LPR, QPL, FULL, false, false, SPEC>(a, row, threadIdx.x & (LPR - 1));  // never max clique
  }
}

template <int LPR, int QPL, bool FULL>
__global__ __launch_bounds__(kBlock) void slot_hub_kernel(const SlotDesc* slots, const HubItem* items, int nitems,
                                                          const int32_t* clock, int t_arg) {
  const int gpb = kBlock / LPR;
  for (int base = blockIdx.x * gpb; base < nitems; base += gridDim.x * gpb) {
    const int it = base + (int)threadIdx.x / LPR;
    if (it >= nitems) continue;
    const HubItem h = items[it];
    const SlotDesc& sd = slots[h.slot];
    int t;
    if (!slot_update_index(sd, clock, t_arg, &t)) continue;
    StepParams a;
    slot_params(sd, t, &a);
    const int gl = threadIdx.x & (LPR - 1);
    const int nq = FULL ? LPR * QPL : (a.S + 3) >> 2;
    const HubChunk ch = sd.chunks[h.chunk];
    const int e_end = min(ch.e0 + kHubChunk, a.row_ptr[ch.row + 1]);
    float4 acc[QPL];
#pragma unroll
    for (int k = 0; k < QPL; ++k) acc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    gather_coupling<LPR, QPL, FULL>(a, ch.e0, e_end, gl, nq, a.problem == kMAXCUT, acc);
    float* out = const_cast<float*>(a.hub_partial) + (size_t)h.chunk * a.stride;
#pragma unroll
    for (int k = 0; k < QPL; ++k) {
      const int q = gl + LPR * k;
      if (FULL || q < nq) *reinterpret_cast<float4*>(out + 4 * q) = acc[k];
    }
  }
}

__global__ void clock_advance_kernel(int32_t* clock, int by) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *clock += by;
}

// ---- evaluation ---------------------------------------------------------------------------
__global__ void slot_zero_acc_kernel(const SlotDesc* slots, const int32_t* ids, int nslots) {
  for (int i = blockIdx.x; i < nslots; i += gridDim.x) {
    const SlotDesc& sd = slots[ids[i]];
    for (int s = threadIdx.x; s < 2 * sd.p.stride; s += blockDim.x) sd.acc[s] = 0ull;
  }
}

// The rounded state after the last update is P[K & 1].
template <int LPR>
__global__ __launch_bounds__(kBlock) void slot_eval_kernel(const SlotDesc* slots, const WorkItem* items, int nitems) {
  extern __shared__ unsigned long long sh[];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem w = items[it];
    const SlotDesc& sd = slots[w.slot];
    if (!sd.active) continue;  // uniform per block
    const int S = sd.p.S, stride = sd.p.stride, nq = (S + 3) >> 2;
    for (int s = threadIdx.x; s < 2 * stride; s += kBlock) sh[s] = 0ull;
    __syncthreads();
    const float* P = sd.P[sd.K & 1];
    const int row = w.row0 + (int)threadIdx.x / LPR;
    const bool maxcut = sd.p.problem == kMAXCUT;
    if (row < sd.p.n) {
      for (int q = threadIdx.x & (LPR - 1); q < nq; q += LPR) {
        const float4 pv = *reinterpret_cast<const float4*>(P + (size_t)row * stride + 4 * q);
        bool xi[4];
        long long ca[4] = {0, 0, 0, 0}, cb[4] = {0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          xi[c] = comp(pv, c) > 0.5f;
          if (!maxcut) ca[c] += xi[c];
        }
        for (int e = sd.p.row_ptr[row]; e < sd.p.row_ptr[row + 1]; ++e) {
          const int j = sd.p.col[e];
          const float wgt = sd.p.w ? sd.p.w[e] : 1.f;
          if (j <= row || wgt == 0.f) continue;
          const long long qw = maxcut ? (long long)(wgt * 65536.0f) : 0;
          const float4 pj = *reinterpret_cast<const float4*>(P + (size_t)j * stride + 4 * q);
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const bool xj = comp(pj, c) > 0.5f;
            if (maxcut) ca[c] += (xi[c] != xj) ? qw : 0;
            else cb[c] += (xi[c] && xj);
          }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (4 * q + c >= S) continue;
          if (ca[c]) atomicAdd(&sh[4 * q + c], (unsigned long long)ca[c]);
          if (cb[c]) atomicAdd(&sh[stride + 4 * q + c], (unsigned long long)cb[c]);
        }
      }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < S; s += kBlock) {
      if (sh[s]) atomicAdd(&sd.acc[s], sh[s]);
      if (sh[stride + s]) atomicAdd(&sd.acc[stride + s], sh[stride + s]);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void slot_finalize_kernel(const SlotDesc* slots, const int32_t* ids, int nslots) {
  __shared__ int best_s[kBlock];
  for (int i = blockIdx.x; i < nslots; i += gridDim.x) {
    const SlotDesc& sd = slots[ids[i]];
    const int S = sd.p.S, stride = sd.p.stride;
    const bool maxcut = sd.p.problem == kMAXCUT;
    int mine = -1;
    bool mi = false;
    long long mo = 0;
    for (int s = threadIdx.x; s < S; s += kBlock) {
      const long long A = (long long)sd.acc[s], B = (long long)sd.acc[stride + s];
      const long long o = maxcut ? -A : -A + sd.lambda64 * B;
      sd.size_or_cut[s] = A;
      sd.viol[s] = B;
      sd.obj[s] = o;
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
            const long long Ax = (long long)sd.acc[x], Bx = (long long)sd.acc[stride + x];
            const long long Ay = (long long)sd.acc[y], By = (long long)sd.acc[stride + y];
            const long long ox = maxcut ? -Ax : -Ax + sd.lambda64 * Bx;
            const long long oy = maxcut ? -Ay : -Ay + sd.lambda64 * By;
            const bool ix = Bx > 0, iy = By > 0;
            take = (iy < ix) || (iy == ix && (oy < ox || (oy == ox && y < x)));
          }
          if (take) best_s[threadIdx.x] = y;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) sd.best[0] = best_s[0];
    __syncthreads();
  }
}

template <int LPR>
__global__ __launch_bounds__(kBlock) void slot_extract_kernel(const SlotDesc* slots, const WorkItem* items, int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem w = items[it];
    const SlotDesc& sd = slots[w.slot];
    if (!sd.active) continue;
    const int row = w.row0 + (int)threadIdx.x / LPR;
    if (row >= sd.p.n || (threadIdx.x & (LPR - 1)) != 0) continue;
    sd.x[row] = sd.P[sd.K & 1][(size_t)row * sd.p.stride + sd.best[0]] > 0.5f ? 1 : 0;
  }
}

// ---- launchers ------------------------------------------------------------------------------
static unsigned slot_grid(int nitems) { return (unsigned)(nitems < 8192 ? (nitems > 0 ? nitems : 1) : 8192); }

#define QQA_SLOT_LAYOUTS(X)                                                                       \
  X(1, 1) X(1, 2) X(1, 4) X(1, 8) X(2, 1) X(2, 2) X(2, 4) X(2, 8) X(4, 1) X(4, 2) X(4, 4) X(4, 8)   \
  X(8, 1) X(8, 2) X(8, 4) X(8, 8) X(16, 1) X(16, 2) X(16, 4) X(16, 8) X(32, 1) X(32, 2) X(32, 4)  \
  X(32, 8) X(64, 1) X(64, 2) X(64, 4) X(64, 8) X(64, 16)

hipError_t launch_slot_init(const SlotDesc* slots, const WorkItem* items, int nitems, int lanes_per_row,
                            hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  switch (lanes_per_row) {
#define L(N)                                                                                              \
  case N:                                                                                                 \
    hipLaunchKernelGGL(slot_init_kernel<N>, dim3(slot_grid(nitems)), dim3(kBlock), 0, st, slots, items, nitems); \
    break;
    L(1) L(2) L(4) L(8) L(16) L(32) L(64)
#undef L
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_slot_step(const SlotDesc* slots, const WorkItem* items, int nitems, int S, int lanes_per_row,
                            int spec, const int32_t* clock, int t_arg, hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  const ReplicaShape r = replica_shape(S, lanes_per_row);
  const bool full = S == 4 * r.lpr * r.qpl;
#define K(LL, QQ, FU, SP) \
  hipLaunchKernelGGL((slot_step_kernel<LL, QQ, FU, SP>), dim3(slot_grid(nitems)), dim3(kBlock), 0, st, slots, items, \
                     nitems, clock, t_arg)
#define X(LL, QQ)                                                             \
  if (r.lpr == LL && r.qpl == QQ) {                                           \
    if (full && spec == spec_of(kMIS, kADAMW, 4)) K(LL, QQ, true, spec_of(kMIS, kADAMW, 4));          \
    else if (full && spec == spec_of(kMAXCUT, kADAMW, 4)) K(LL, QQ, true, spec_of(kMAXCUT, kADAMW, 4)); \
    else if (full) K(LL, QQ, true, 0);                                        \
    else K(LL, QQ, false, 0);                                                 \
    return hipGetLastError();                                                 \
  }
  QQA_SLOT_LAYOUTS(X)
#undef X
#undef K
  return hipErrorInvalidValue;
}

hipError_t launch_slot_hubs(const SlotDesc* slots, const HubItem* items, int nitems, int S, int lanes_per_row,
                            const int32_t* clock, int t_arg, hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  const ReplicaShape r = replica_shape(S, lanes_per_row);
  const bool full = S == 4 * r.lpr * r.qpl;
  const int gpb = kBlock / r.lpr;
  const int blocks = (nitems + gpb - 1) / gpb;
  const unsigned grid = (unsigned)(blocks < 8192 ? blocks : 8192);
#define X(LL, QQ)                                                                                           \
  if (r.lpr == LL && r.qpl == QQ) {                                                                         \
    if (full)                                                                                               \
      hipLaunchKernelGGL((slot_hub_kernel<LL, QQ, true>), dim3(grid), dim3(kBlock), 0, st, slots, items,    \
                         nitems, clock, t_arg);                                                             \
    else                                                                                                    \
      hipLaunchKernelGGL((slot_hub_kernel<LL, QQ, false>), dim3(grid), dim3(kBlock), 0, st, slots, items,   \
                         nitems, clock, t_arg);                                                             \
    return hipGetLastError();                                                                               \
  }
  QQA_SLOT_LAYOUTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_clock_advance(int32_t* clock, int by, hipStream_t st) {
  hipLaunchKernelGGL(clock_advance_kernel, dim3(1), dim3(64), 0, st, clock, by);
  return hipGetLastError();
}

hipError_t launch_slot_eval(const SlotDesc* slots, const int32_t* slot_ids, int nslots, const WorkItem* items,
                            int nitems, int S, int lanes_per_row, hipStream_t st) {
  if (nslots == 0) return hipSuccess;
  hipLaunchKernelGGL(slot_zero_acc_kernel, dim3(nslots < 1024 ? nslots : 1024), dim3(kBlock), 0, st, slots, slot_ids,
                     nslots);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t shmem = 2 * (size_t)replica_shape(S).stride * sizeof(unsigned long long);
  switch (lanes_per_row) {
#define L(N)                                                                                                     \
  case N:                                                                                                        \
    if (nitems)                                                                                                  \
      hipLaunchKernelGGL(slot_eval_kernel<N>, dim3(slot_grid(nitems)), dim3(kBlock), shmem, st, slots, items, nitems); \
    break;
    L(1) L(2) L(4) L(8) L(16) L(32) L(64)
#undef L
    default: return hipErrorInvalidValue;
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(slot_finalize_kernel, dim3(nslots < 1024 ? nslots : 1024), dim3(kBlock), 0, st, slots, slot_ids,
                     nslots);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (lanes_per_row) {
#define L(N)                                                                                                        \
  case N:                                                                                                           \
    if (nitems)                                                                                                     \
      hipLaunchKernelGGL(slot_extract_kernel<N>, dim3(slot_grid(nitems)), dim3(kBlock), 0, st, slots, items, nitems); \
    break;
    L(1) L(2) L(4) L(8) L(16) L(32) L(64)
#undef L
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace qqa
