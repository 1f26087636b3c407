// Resident batch engine: one cooperative launch runs every update of a ragged batch of
// independent instances.  Each instance is a job, run by a team of workgroups that all sit
// on one XCD.  The team's lane groups keep their rows' p, m, v in registers for the whole
// schedule; the new p of every update goes to memory, where the neighbour rows are read,
// and the team meets at a barrier between updates.  Because a team never leaves its XCD,
// P is shared through that XCD's L2: a member's row stores reach L2 before it raises its
// barrier flag, and neighbour rows are read with non-temporal loads, which do not return
// the stale copies a CU's L1 may hold from earlier updates.  (Measured on the 512-instance
// batch: plain loads after a group-scope L1 invalidate, and loads with the group-coherence
// bit, read stale rows; non-temporal loads, agent-scope loads and agent-scope invalidates
// read correct ones, non-temporal loads the fastest.)  Nothing else crosses the fabric
// while a job runs, and an instance's P ping-pong (256 B per row at 32 replicas) stays in
// L2.
//
// The host splits the jobs over the XCDs (longest processing time first) and orders each
// XCD's jobs in rounds whose teams fill its workgroups (first-fit decreasing).  On each XCD,
// workgroups claim team places in job order from a counter and read which XCD they run on
// from the hardware, so a team forms from whichever workgroups of that XCD free up first.
// Every job's team fits the XCD's resident workgroups, so the lowest job with unclaimed
// places always completes its team: the claiming order cannot deadlock.  A barrier that
// waits longer than the host's time limit raises the abort flag and every workgroup returns.
//
// Rows go through the same device functions as the streaming kernels (qqa_device.h), with
// edges summed in CSR order, so every instance ends with the bits of the same solve alone.
// The work of an update that needs no neighbour row (the normals, mu and sigma) is done
// while the team barrier waits, for the next update.
#include "qqa_device.h"

namespace qqa {

namespace {

// the XCD this workgroup runs on (hardware register XCC_ID, its low bits)
__device__ __forceinline__ int xcd_id() {
  const unsigned v = __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 20);
  return (int)(v & 0xfu) % kResidentXcds;
}

// Team barrier of one job.  Every member but the first publishes the number of updates it
// has finished in its own flag (one 64-byte line, an agent-scope store issued once its row
// stores have reached L2).  The first member's first wavefront polls those flags at once, one
// lane per member; when all show `epoch` it publishes `epoch` in its own flag, the one line
// the other members poll.  No counter is shared, so the arrivals do not serialise on one
// address, and a poll reads one line except at the first member.  (Measured on the
// 512-instance batch: 8% less time per update than every member polling every flag.)
// Split in two: team_arrive publishes this member's arrival, team_wait waits for the release;
// between them the member's waves do the work of the next update that needs no other row.
__device__ __forceinline__ void team_arrive(unsigned* flags, const int member, const unsigned epoch) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's row stores have reached L2
  __syncthreads();
  if (threadIdx.x == 0 && member != 0)
    __hip_atomic_store(flags + (size_t)member * kFlagWords, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool team_wait(const ResidentParams& rp, unsigned* flags, const int member, const int team,
                                          const unsigned epoch) {
  __shared__ int ok;
  if (threadIdx.x < 64) {
    const long long t0 = wall_clock64();
    int good = 1;
    for (;;) {
      bool mine = true;
      if (member == 0) {  // lane l watches members l and l + 64
        for (int m = (int)threadIdx.x; m < team; m += 64)
          mine = mine && (m == 0 || __hip_atomic_load(flags + (size_t)m * kFlagWords, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT) >= epoch);
      } else {
        mine = __hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch;
      }
      if (__all(mine)) {
        if (member == 0 && threadIdx.x == 0)
          __hip_atomic_store(flags, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // release the team
        break;
      }
      if (__hip_atomic_load(rp.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          wall_clock64() - t0 > rp.timeout_ticks) {
        if (threadIdx.x == 0) atomicOr(rp.abort, 1u);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (threadIdx.x == 0) ok = good;
  }
  __syncthreads();
  return ok != 0;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// A neighbour quad: a non-temporal load, which does not return stale L1 contents, so rows
// that other team members rewrote since this CU last read them come from L2.
__device__ __forceinline__ float4 load_shared(const float* p) {
  const f32x4 x = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
  return make_float4(x.x, x.y, x.z, x.w);
}

// The coupling sum of one row for lane gl's quad (one quad per lane, every quad valid), U
// edges per batch: the same operations in the same edge order as the streaming kernels'.
template <int LPR, int U, int SPEC>
__device__ __forceinline__ float4 res_coupling(const StepParams& a, const int row, const int gl) {
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  const int e_begin = a.row_ptr[row], e_end = a.row_ptr[row + 1];
  const bool maxcut = SPEC ? spec_problem(SPEC) == kMAXCUT : a.problem == kMAXCUT;
  for (int e0 = e_begin; e0 < e_end; e0 += U) {
    const float* src[U];
    float w[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u;
      ok[u] = e < e_end;
      const int ec = ok[u] ? e : e_end - 1;
      src[u] = a.P_in + (size_t)a.col[ec] * a.stride + 4 * gl;
      w[u] = a.w ? a.w[ec] : 1.f;
    }
    float4 x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = load_shared(src[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float xc = comp(x[u], c);
        const float f = maxcut ? 2.f * xc - 1.f : xc;
        const float r = fmaf(w[u], f, comp(acc, c));
        set_comp(acc, c, ok[u] ? r : comp(acc, c));
      }
  }
  return acc;
}

template <int LPR, int RPG, int QUADS, int SPEC>
__device__ __forceinline__ bool run_job(const ResidentParams& rp, const int job, const int member) {
  constexpr int kGroups = kBlock / LPR;
  const ResidentJob jb = rp.jobs[job];
  const SlotDesc& sd = rp.slots[jb.slot];
  StepParams a = sd.p;
  const int gl = threadIdx.x & (LPR - 1);
  int grp = (int)threadIdx.x / LPR;
  if (LPR == 64) grp = __builtin_amdgcn_readfirstlane(grp);
  // rows member * kGroups * RPG + r * kGroups + grp: a wavefront's lane groups take
  // consecutive rows, so its stores of new rows are contiguous
  const int row0 = member * kGroups * RPG + grp;
  float4 p[RPG][1], mm[RPG][1], vv[RPG][1];
#pragma unroll
  for (int r = 0; r < RPG; ++r)
    if (row0 + r * kGroups < a.n) {
      load_row<LPR, 1, true>(a, sd.P[0], row0 + r * kGroups, gl, p[r], mm[r], vv[r]);
      p[r][0] = load_shared(sd.P[0] + (size_t)(row0 + r * kGroups) * a.stride + 4 * gl);  // as the gathers read it
    }
  unsigned* flags = rp.flags + (size_t)jb.flag_base * kFlagWords;
  // The parts of the coming update that need only the lane's own rows: each row quad's
  // normals (the generator and counters of finish_elems) and each row's mu and sigma term
  // (row_stats of the new p), formed while the member waits for its team.  They wait in LDS,
  // each thread's own slots: in registers they would spill (measured on the 512-instance
  // batch, us per update: 270 as part of the update, 263 with the normals in registers and
  // 4 registers spilled, 346 with the statistics too and 16 spilled, 255-258 in LDS).
  __shared__ float4 xi_lds[RPG][kBlock];
  __shared__ float2 st_lds[RPG][kBlock];
  auto normals = [&](const uint32_t k) {
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
      xi_lds[r][threadIdx.x] =
          normals4(philox4x32_10((uint32_t)(row0 + r * kGroups), (uint32_t)gl, k, kStreamNoise, a.key0, a.key1));
      float mu, cg;
      row_stats<LPR, 1, true>(a, gl, p[r], mu, cg);
      st_lds[r][threadIdx.x] = make_float2(mu, cg);
    }
  };
  normals(1u);
  for (int t = 0; t < sd.K; ++t) {
    a.P_in = sd.P[t & 1];
    a.P_out = sd.P[(t + 1) & 1];
    const float4 tb = sd.table[t];
    a.ce = tb.x;
    a.inv_bc1 = tb.y;
    a.inv_bc2 = tb.z;
    a.k = (uint32_t)t + 1u;
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
      const int row = row0 + r * kGroups;
      if (row >= a.n) continue;  // whole lane groups
      float4 acc[1], po[1], mo[1], vo[1];
      acc[0] = res_coupling<LPR, QUADS, SPEC>(a, row, gl);
      const float2 st = st_lds[r][threadIdx.x];
      const float4 x[1] = {xi_lds[r][threadIdx.x]};
      finish_elems<LPR, 1, true, false, true, SPEC>(a, row, gl, 0, st.x, st.y, p[r], mm[r], vv[r], acc, po, mo, vo,
                                                    x);
      store_row<LPR, 1, true, false>(a, a.P_out, row, gl, po, mo, vo, false);
      p[r][0] = po[0];
      mm[r][0] = mo[0];
      vv[r][0] = vo[0];
    }
    team_arrive(flags, member, (unsigned)t + 1u);
    if (t + 1 < sd.K) normals((uint32_t)t + 2u);
    if (!team_wait(rp, flags, member, jb.team, (unsigned)t + 1u)) return false;
  }
  if (member == 0 && threadIdx.x == 0) atomicAdd(rp.done, 1u);
  return true;
}

}  // namespace

template <int LPR, int RPG, int QUADS, int SPEC>
// Held to four waves per SIMD (at most 128 registers, none spilled at three rows per lane
// group).  Measured on the 512-instance batch, µs per update: three rows at four waves 298-305,
// four rows at three waves 333-335, two rows at five waves (spilling) 326, five rows at three
// waves 394.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void resident_kernel(ResidentParams rp) {
  __shared__ int sh_job, sh_member;
  const int x = xcd_id();
  for (;;) {
    if (threadIdx.x == 0) {
      int job = -1, member = 0;
      if (__hip_atomic_load(rp.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
        const unsigned place = atomicAdd(&rp.claim[x], 1u);
        if (place < (unsigned)rp.xcd_places[x]) {
          // the job whose places contain `place` (first places ascend within an XCD)
          int lo = rp.xcd_jobs[x], hi = rp.xcd_jobs[x + 1] - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((unsigned)rp.jobs[mid].first_place <= place) lo = mid;
            else hi = mid - 1;
          }
          job = lo;
          member = (int)place - rp.jobs[lo].first_place;
        }
      }
      sh_job = job;
      sh_member = member;
    }
    __syncthreads();
    // uniform across the workgroup: the job's descriptors are then read with scalar loads
    const int job = __builtin_amdgcn_readfirstlane(sh_job), member = __builtin_amdgcn_readfirstlane(sh_member);
    __syncthreads();  // every wave has read the claim before thread 0 makes the next
    if (job < 0) return;
    if (!run_job<LPR, RPG, QUADS, SPEC>(rp, job, member)) return;
  }
}

// After the launch: each slot's result record carries the outcome in its barrier word
// (1: a barrier timed out or a job never ran; the evaluation then describes no solve).
__global__ void resident_flags_kernel(ResidentParams rp, int nslots, int njobs) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  const SlotDesc& sd = rp.slots[s];
  unsigned* bar = reinterpret_cast<unsigned*>(reinterpret_cast<char*>(sd.size_or_cut) + 3 * (size_t)sd.p.S * 8 + 8);
  bar[0] = 0u;
  bar[1] = (*rp.abort != 0u || *rp.done != (unsigned)njobs) ? 1u : 0u;
}

// ---- planning and launch -------------------------------------------------------------------
// (lanes per row, rows per lane group) pairs the engine is built for: one quad per lane
#define QQA_RESIDENT_SHAPES(X) \
  X(4, 3) X(8, 3) X(16, 3) X(32, 3) X(64, 3)
constexpr int kResidentQuads = 4;

// SPEC: a batch whose instances all run the default schedule of one problem (AdamW, entropy
// alpha 4, MIS or max-cut) runs the kernel with those facts fixed (default_spec), else 0
#define QQA_RESIDENT_SPEC(L, R, F)                                    \
  F(L, R, 0) F(L, R, spec_of(kMIS, kADAMW, 4)) F(L, R, spec_of(kMAXCUT, kADAMW, 4))

int resident_workgroups(int lanes_per_row, int rows_per_group, int spec) {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
#define F(L, R, SP)                                                                                             \
  if (lanes_per_row == L && rows_per_group == R && spec == SP) {                                                \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, resident_kernel<L, R, kResidentQuads, SP>, kBlock, \
                                                     0) != hipSuccess)                                             \
      return 0;                                                                                                 \
    return per_cu * prop.multiProcessorCount;                                                                   \
  }
#define X(L, R) QQA_RESIDENT_SPEC(L, R, F)
  QQA_RESIDENT_SHAPES(X)
#undef X
#undef F
  return 0;
}

hipError_t launch_resident(const ResidentParams& rp, int lanes_per_row, int rows_per_group, int spec, int grid,
                           int nslots, int njobs, hipStream_t st) {
  ResidentParams arg = rp;
  void* args[] = {&arg};
  hipError_t e = hipErrorInvalidValue;
#define F(L, R, SP)                                                                                              \
  if (lanes_per_row == L && rows_per_group == R && spec == SP)                                                   \
    e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(resident_kernel<L, R, kResidentQuads, SP>),       \
                                   dim3(grid), dim3(kBlock), args, 0, st);
#define X(L, R) QQA_RESIDENT_SPEC(L, R, F)
  QQA_RESIDENT_SHAPES(X)
#undef X
#undef F
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(resident_flags_kernel, dim3((nslots + kBlock - 1) / kBlock), dim3(kBlock), 0, st, rp, nslots,
                     njobs);
  return hipGetLastError();
}

}  // namespace qqa
