// Internal interface between the HIP kernels (qqa_kernels.hip) and the host runtime
// (qqa_runtime.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qqa {

enum : int32_t { kMIS = 0, kMAXCUT = 1, kMAXCLIQUE = 2, kCOLORING = 3 };
enum : int32_t { kADAMW = 0, kLANGEVIN = 1 };

// Facts about a solve that a kernel may fix at compile time, so that the uniform branches and
// selects on them leave its instruction stream: 0 (none: every fact read from the
// parameters) or spec_of(problem, step rule, entropy alpha).  A fixed fact changes no
// arithmetic: the same operations run in the same order.
constexpr int spec_of(int problem, int rule, int alpha_e) { return 1 + problem + 4 * rule + 8 * alpha_e; }
constexpr int spec_problem(int s) { return (s - 1) % 4; }
constexpr int spec_rule(int s) { return ((s - 1) / 4) % 2; }
constexpr int spec_alpha(int s) { return (s - 1) / 8; }
// the fixed facts of a default schedule (AdamW, entropy alpha 4) of MIS or max-cut, else 0
constexpr int default_spec(int problem, int rule, int alpha_e) {
  return rule == kADAMW && alpha_e == 4 && (problem == kMIS || problem == kMAXCUT) ? spec_of(problem, rule, alpha_e) : 0;
}
enum : uint32_t { kStreamInit = 0, kStreamNoise = 1 };

constexpr int kMaxReplicas = 4096;
constexpr int kBlock = 256;
// Rows with more than kHubDegree neighbours are split into chunks of kHubChunk edges whose
// partial coupling sums are computed by their own lane groups (hub_partial_kernel).
constexpr int kHubDegree = 64;
constexpr int kHubChunk = 16;

// How the S replicas of one variable map onto lanes: a row is served by `lpr` adjacent
// lanes (a power of two, at most one wavefront), each lane owns `qpl` float4 quads.
struct ReplicaShape {
  int lpr;     // lanes per row
  int qpl;     // quads per lane
  int nquads;  // ceil(S / 4)
  int stride;  // floats per row = 4 * nquads
};
ReplicaShape replica_shape(int S);
ReplicaShape replica_shape(int S, int lanes_per_row);
bool layout_supported(int S, int lanes_per_row);

// Chunks of split rows: {row, first edge}; the chunk ends at min(first + kHubChunk, row end).
struct HubChunk {
  int32_t row;
  int32_t e0;
};

// Everything one launch of the fused update needs for one instance at one update index.
// Per-update scalars (gamma_t, bias corrections) are computed on the host in double
// precision and rounded once.
struct StepParams {
  const int32_t* row_ptr;  // sparse CSR (device), or nullptr when `coupling` is given
  const int32_t* col;
  const float* w;          // nullptr: unweighted
  const float* coupling;   // dense path: precomputed coupling product, n x stride, or nullptr
  int32_t coupling_parts;  // dense path: coupling holds this many partial products (n x stride
                           // each, consecutive), added in part order; 0 or 1: one product
  const int32_t* hub_first;  // per row: first chunk of a split row, -1 otherwise (nullptr: no hubs)
  const float* hub_partial;  // per chunk: partial coupling sums, nchunks x stride
  // max clique: per-replica sums 1^T p of P_in in 2^-32 fixed point ([stride]), else nullptr
  const unsigned long long* colsum;
  const float* P_in;
  float* P_out;
  float* m;
  float* v;
  int32_t n, S, stride, problem, rule, alpha_e;
  int32_t lanes_per_row;   // replica layout (0 = default); selects the kernel instance
  float lambda;            // MIS / max-clique penalty
  float lr, wd_factor;     // wd_factor = 1 - lr * weight_decay
  float comm_alpha;
  float beta1, omb1, beta2, omb2, eps;
  float noise_scale;       // sqrt(2 lr T)
  float ce;                // -2 alpha_e gamma_t
  float inv_S;             // 1 / S
  float inv_bc1, inv_bc2;  // 1 / (1 - beta^k)
  uint32_t key0, key1;     // Philox key = seed
  uint32_t k;              // update count t + 1 (Philox counter word 2)
};

struct EvalParams {
  const int32_t* row_ptr;
  const int32_t* col;
  const float* w;
  const float* dense;      // n x n or nullptr
  const float* P;
  int32_t n, S, stride, problem;
  int64_t lambda;
  unsigned long long* acc; // [2][stride]: size_or_cut, violations (zeroed by launch_eval)
  int64_t* size_or_cut;    // [S] outputs
  int64_t* viol;
  int64_t* obj;
  int32_t* best;           // [1]
};

// ---- multi-instance slots ------------------------------------------------------------
// One slot per instance in a batch or in the server.  A launch over a work list advances
// every active slot by one update; the update index of a slot is t = clock + t_arg - start,
// so a captured sequence of launches (t_arg = 0..R-1) can be replayed after the clock
// moves on.  Per-update scalars come from the slot's table, computed on the host exactly
// as for a single solve, so a slot follows the same arithmetic as a solve run alone.
struct SlotDesc {
  StepParams p;                 // static fields; P_in / P_out / per-update fields set per launch
  float* P[2];                  // ping-pong state
  const float4* table;          // per update t: {ce, inv_bc1, inv_bc2, 0}
  const HubChunk* chunks;       // split plan of the slot's graph
  int32_t nchunks;
  int32_t K;                    // updates
  int32_t start;                // clock value of the slot's first update
  int32_t active;               // 0: skipped by every kernel
  uint64_t seed;
  int64_t lambda64;             // MIS penalty for the exact evaluation
  unsigned long long* acc;      // [2][stride] evaluation accumulators
  int64_t* size_or_cut;         // [S] outputs
  int64_t* viol;
  int64_t* obj;
  int32_t* best;
  uint8_t* x;                   // [n]
};

struct WorkItem {
  int32_t slot;
  int32_t row0;                 // first row; a block covers kBlock / lanes_per_row rows
};
struct HubItem {
  int32_t slot;
  int32_t chunk;
};

// Launches over a work list of one replica layout.  `clock` is a device int.  spec: the
// default_spec every slot of the step's list shares, else 0.
hipError_t launch_slot_init(const SlotDesc* slots, const WorkItem* items, int nitems, int lanes_per_row, hipStream_t st);
hipError_t launch_slot_step(const SlotDesc* slots, const WorkItem* items, int nitems, int S, int lanes_per_row,
                            int spec, const int32_t* clock, int t_arg, hipStream_t st);
hipError_t launch_slot_hubs(const SlotDesc* slots, const HubItem* items, int nitems, int S, int lanes_per_row,
                            const int32_t* clock, int t_arg, hipStream_t st);
hipError_t launch_clock_advance(int32_t* clock, int by, hipStream_t st);
// Evaluation of slots whose update loop is complete: zero accumulators, accumulate,
// finalize (objectives + best replica), extract x of the best replica.
hipError_t launch_slot_eval(const SlotDesc* slots, const int32_t* slot_ids, int nslots, const WorkItem* items,
                            int nitems, int S, int lanes_per_row, hipStream_t st);

// ---- persistent engines ----------------------------------------------------------------
// One launch runs updates [t0, t1) of one instance.  Every lane group owns rows_per_group
// consecutive rows for the whole launch and keeps their p, m, v in registers; only the new
// p of each update goes to memory, for the neighbours to read.  The multi-block engine
// separates updates with a grid barrier (cooperative launch, bounded spin: on time-out it
// raises bar[1] and every block returns); the single-block engine keeps P itself in LDS.
struct PersistParams {
  StepParams a;                 // static fields; per-update fields come from `table`
  float* P[2];                  // P[t0 & 1] holds the state before update t0
  const float4* table;          // per update t: {ce, inv_bc1, inv_bc2, 0}
  int32_t t0, t1;
  unsigned* bar;                // [0] arrivals (zero before the launch), [1] abort flag
  // LDS engine (required there): the normals of update t, row i, quad q at
  // noise[((t - t0) n + i) nq + q] (nq = stride / 4), formed by launch_noise_table
  const float4* noise;
  int32_t nnz;                  // LDS engine: the graph's edges (CSR entries); 0 keeps them in global memory
};
// The normals of updates [t0, t1) of every row and replica quad of `a`, as the update
// kernels generate them (the same counters and keys), into xi ((t1 - t0) n nq quads).
hipError_t launch_noise_table(const StepParams& a, int t0, int t1, float4* xi, hipStream_t st);
// the largest noise table an LDS-block solve holds (longer solves run in chunks of updates)
constexpr size_t kNoiseTableMaxBytes = (size_t)64 << 20;
enum PersistEngine {
  kEngineStream = 0, kEnginePersistent = 1, kEngineLdsBlock = 2, kEngineBatch = 3, kEngineSliced = 4, kEngineCompact = 5,
  kEngineResident = 6
};
// Which engine can run this instance (FULL layouts with one quad per lane, no split
// rows); `allow` is a mask (1: one workgroup with P in LDS, 2: many workgroups with state
// in registers).  Fills rows per group and the grid for the chosen one.
int persistent_plan(const StepParams& a, bool has_hubs, int allow, int* rows_per_group, int* grid);
hipError_t launch_persistent(const PersistParams& pp, int engine, int rows_per_group, int grid, hipStream_t st);

// ---- resident batch engine -----------------------------------------------------------------
// One cooperative launch runs every update of a batch whose instances all use one layout
// with one quad per lane and have no split rows.  Each instance (job) is run by a team of
// `team` workgroups on one XCD, p, m, v in registers, P shared through that XCD's L2; the
// team meets at a barrier between updates (bounded by timeout_ticks of the 100 MHz wall
// clock; on time-out *abort is raised and every workgroup returns).
constexpr int kResidentXcds = 8;
// rows whose state each lane group holds (three rows fit four waves per SIMD without spills)
constexpr int kResidentRowsPerGroup = 3;
struct ResidentJob {
  int32_t slot;         // slot descriptor of the instance
  int32_t team;         // workgroups that run it (at most 128)
  int32_t first_place;  // its first team place among the places of its XCD
  int32_t flag_base;    // its members' barrier flags: flags[(flag_base + member) * kFlagWords]
};
constexpr int kFlagWords = 16;  // one 64-byte line per barrier flag
constexpr int kResidentMaxTeam = 128;
struct ResidentParams {
  const SlotDesc* slots;
  const ResidentJob* jobs;    // grouped by XCD, in claim order
  const int32_t* xcd_jobs;    // [kResidentXcds + 1]: XCD x runs jobs [xcd_jobs[x], xcd_jobs[x + 1])
  const int32_t* xcd_places;  // [kResidentXcds]: team places of XCD x (its jobs' teams summed)
  unsigned* claim;            // [kResidentXcds] places claimed (zero before the launch)
  unsigned* flags;            // barrier flags, kFlagWords per team member (zero before the launch)
  unsigned* abort;            // [1] raised when a barrier times out (zero before the launch)
  unsigned* done;             // [1] jobs completed (zero before the launch)
  long long timeout_ticks;    // longest wait at one barrier, in wall-clock ticks
};
// Co-resident workgroups of the kernel for a (lanes per row, rows per lane group) shape and
// the batch's fixed facts (spec: default_spec of its instances' common schedule, else 0),
// 0 if the shape is not built.
int resident_workgroups(int lanes_per_row, int rows_per_group, int spec);
// The launch, then a kernel that writes each slot's outcome into its result record's
// barrier word [1] (0: every job ran to completion).
hipError_t launch_resident(const ResidentParams& rp, int lanes_per_row, int rows_per_group, int spec, int grid,
                           int nslots, int njobs, hipStream_t st);

// Dense coupling product C = W f(P) on the matrix cores (W symmetric n x n, P and C
// n x stride; f(p) = 2p - 1 for max-cut, p for MIS).
// every (lanes per row, quads per lane) pair the kernels are built for
#define QQA_FOR_EACH_LAYOUT(X)                                                                   \
  X(1, 1) X(1, 2) X(1, 4) X(1, 8) X(2, 1) X(2, 2) X(2, 4) X(2, 8) X(4, 1) X(4, 2) X(4, 4) X(4, 8)   \
  X(8, 1) X(8, 2) X(8, 4) X(8, 8) X(16, 1) X(16, 2) X(16, 4) X(16, 8) X(32, 1) X(32, 2) X(32, 4)  \
  X(32, 8) X(64, 1) X(64, 2) X(64, 4) X(64, 8) X(64, 16)

// Per-replica sums T[s] = sum_i P[i][s] (max clique), accumulated exactly in 2^-32 fixed
// point: each p is rounded once to a multiple of 2^-32, and the integer sums are independent
// of the order of addition.  T (stride entries) is cleared by the launcher.
hipError_t launch_colsum(const float* P, int n, int stride, unsigned long long* T, hipStream_t st);

// Graph coloring (categorical K-state variant): rows i*K + k of the replica layout.
// sigma = Clamp-normalised rows of V; G = dR/dsigma over N*K rows (p.n = N*K, p.P_in = sigma,
// p.ce = -gamma c alpha K); the update over N variables (p.n = N, p.P_in / P_out = V) also
// rewrites sigma for the new V; evaluation writes colours X (n x stride bytes) and the
// conflict count per replica into acc[0..S).
hipError_t launch_cat_sigma(const float* V, float* sig, int n, int K, int stride, int S, hipStream_t st);
hipError_t launch_cat_grad(const StepParams& p, int K, float* G, hipStream_t st);
hipError_t launch_cat_update(const StepParams& p, int K, const float* G, float* sig, hipStream_t st);
// Gradient and update in one launch (p as for launch_cat_update, ce the gradient's entropy
// coefficient), reading sigma from sig_in and writing the new sigma to sig_out; for shapes
// where cat_fused_shape holds (K <= 8 colours, a power-of-two number of replica quads served
// one per lane by the layout, K rounded up to a power of two times the quads <= 64).  Bitwise
// the same as launch_cat_grad followed by launch_cat_update.  nnz (the graph's edge count)
// sets how many neighbour loads each lane keeps in flight.
bool cat_fused_shape(int S, int lanes_per_row, int K);
hipError_t launch_cat_fused(const StepParams& p, int K, float ce, const float* sig_in, float* sig_out, int64_t nnz,
                            hipStream_t st);
hipError_t launch_cat_eval(const int32_t* row_ptr, const int32_t* col, const float* V, uint8_t* X, int n, int K,
                           int stride, int S, unsigned long long* acc, hipStream_t st);
hipError_t launch_cat_extract(const uint8_t* X, int n, int stride, const int32_t* best, uint8_t* x, hipStream_t st);
hipError_t launch_finalize(const EvalParams& p, hipStream_t st);

// `work` holds dense_workspace_bytes(n, stride) bytes of split-K partial products (none
// needed when that is 0); C must not overlap it.  launch_dense_parts writes the
// dense_splits(n, stride) partial products to `parts` (n x stride each, consecutive)
// without adding them: an update kernel with coupling_parts = dense_splits adds them.
int dense_splits(int n, int stride);
size_t dense_workspace_bytes(int n, int stride);
hipError_t launch_dense_coupling(const float* W, const float* P, float* C, int n, int stride, int problem,
                                 float* work, hipStream_t st);
hipError_t launch_dense_parts(const float* W, const float* P, float* parts, int n, int stride, int problem,
                              hipStream_t st);

hipError_t launch_philox(uint64_t seed, int n, int nquads, uint32_t k, uint32_t stream_id, uint32_t* out,
                         hipStream_t st);
hipError_t launch_noise(uint64_t seed, int n, int S, uint32_t k, float* xi, hipStream_t st);
hipError_t launch_init(uint64_t seed, int n, int S, float* P, float* m, float* v, hipStream_t st);
hipError_t launch_step(const StepParams& p, hipStream_t st);

// Sliced streaming update: the replica axis is cut into nsl slices of at most sq quads
// (sizes differ by at most one), each served by ls lanes x qs quads: kReplicaSlices slices,
// one per XCD, or half as many, one per XCD pair, when only that makes each slice a whole
// 128-byte line (sq == 0: S is not sliceable, i.e. fewer than 2 quads per slice of eight).
// Partial statistics {mean, M2} per (slice, row), nsl x n entries, ping-pong between updates:
// launch_slice_stats forms them from p.P_in before the first update; each launch_slice_step
// reads part_in (of P_in) and writes part_out (of P_out).  Same arithmetic per element as
// launch_step, except that mu and sigma are combined from the slices' partials.
constexpr int kReplicaSlices = 8;
// The automatic engine policy slices sparse streaming solves when every slice is at least
// one 128-byte line of a row (S >= 256) and one XCD's slice of P fits in its 4 MiB L2 with
// room to spare (P at most 24 MiB).  Narrower slices waste fetched lines; larger P leaves
// the gathers missing L2 anyway.  Where the state can be kept slice-major (a context's
// solve with equal slices, not max clique), each XCD streams its slice as one region and the
// sliced engine wins further: from S = 128 (four slices of a line each below 256) with P up
// to 64 MiB.  (Measured, 500 updates, stream against slice-major sliced, us per update: ER
// mean degree 5, S = 256, n = 50,000 / 60,000 / 100,000: 80.4 / 73.8, 96.4 / 89.9,
// 159.4 / 161.6; S = 128, n = 20,000 / 50,000 / 100,000 / 130,000: 19.7 / 18.4,
// 41.8 / 39.4, 80.7 / 79.3, 101.8 / 104.7; BA m = 4 with split hub rows, S = 128,
// n = 50,000 / 100,000: 50.9 / 45.8, 99.4 / 94.7; S = 256, n = 50,000: 99.0 / 83.2.)
constexpr int kSliceAutoMinReplicas = 256;
constexpr size_t kSliceAutoMaxBytes = (size_t)24 << 20;
constexpr size_t kSliceMajorAutoMaxBytes = (size_t)64 << 20;
inline bool slice_by_default(int n, int S, bool slice_major) {
  const size_t stride = 4 * (size_t)((S + 3) / 4);
  const size_t bytes = (size_t)n * stride * sizeof(float);
  if (slice_major && S >= 128 && bytes <= kSliceMajorAutoMaxBytes) return true;
  return S >= kSliceAutoMinReplicas && bytes <= kSliceAutoMaxBytes;
}
struct SliceShape {
  int sq, ls, qs;
  int nsl;  // slices: kReplicaSlices, or kReplicaSlices / 2 (XCD pairs) when that makes each a whole line
};
SliceShape slice_shape(int S);
// slice_major: P (both buffers), m and v hold the state slice-major, [slice][row][slice
// width], and the split rows' chunk partials [slice][chunk][slice width], written by
// launch_slice_hub_partials (equal slices, stride == S, no max clique or dense product:
// slice_major_ok); launch_slice_permute converts between that and the row-major n x stride.
hipError_t launch_slice_stats(const StepParams& p, float2* part, hipStream_t st, bool slice_major = false);
bool slice_major_ok(const StepParams& p);
hipError_t launch_slice_hub_partials(const StepParams& p, const HubChunk* chunks, int nchunks, hipStream_t st);
hipError_t launch_slice_permute(const float* src, float* dst, int n, int S, bool to_slice_major, hipStream_t st);

// Compact engine (S = 1, sparse MIS or max-cut): P, m, v as n floats each.  pack takes
// replica 0 of every row of a padded n x stride array; unpack writes rows {x, 0, 0, 0}
// (stride 4).  The step is bitwise step_kernel's at one lane per row.
hipError_t launch_compact_step(const StepParams& p, const float* Pc_in, float* Pc_out, float* mc, float* vc,
                               hipStream_t st);
hipError_t launch_compact_pack(const float* src, int stride, int n, float* dst, hipStream_t st);
hipError_t launch_compact_unpack(const float* src, int n, int stride, float* dst, hipStream_t st);
hipError_t launch_slice_step(const StepParams& p, const float2* part_in, float2* part_out, hipStream_t st,
                             bool slice_major = false, int nchunks = 0);

// Partial coupling sums of every chunk into p.hub_partial (reads P_in, row_ptr, col, w).
hipError_t launch_hub_partials(const StepParams& p, const HubChunk* chunks, int nchunks, hipStream_t st);
hipError_t launch_eval(const EvalParams& p, hipStream_t st);
hipError_t launch_extract(const float* P, int n, int stride, const int32_t* best, uint8_t* x, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, size_t count, hipStream_t st);
// the evaluation's fixed device scratch on the current device: address and size in words
hipError_t eval_scratch(unsigned long long** out, size_t* words);

}  // namespace qqa
