// Ragged multi-instance batches (qqa_solve_batch) and the continuous-batching server.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "qqa.h"
#include "qqa_batch.h"
#include "qqa_ctx.h"

using namespace qqa;
using Clock = std::chrono::steady_clock;

namespace qqa {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

std::vector<float4> schedule_table(const qqa_schedule& s, int K) {
  std::vector<float4> t((size_t)K);
  StepParams p{};
  for (int i = 0; i < K; ++i) {
    fill_step_scalars(p, s, i, K);
    t[i] = make_float4(p.ce, p.inv_bc1, p.inv_bc2, 0.f);
  }
  return t;
}

SlotLayout slot_layout(int n, int S, int rule, int nchunks) {
  const size_t stride = (size_t)replica_shape(S).stride;
  const size_t state = align256((size_t)n * stride * sizeof(float));
  SlotLayout L{};
  size_t o = 0;
  L.P0 = o;
  o += state;
  L.P1 = o;
  o += state;
  L.m = o;
  if (rule == QQA_STEP_ADAMW) o += state;
  L.v = o;
  if (rule == QQA_STEP_ADAMW) o += state;
  L.hub = o;
  o += align256((size_t)nchunks * stride * sizeof(float));
  L.acc = o;
  o += align256(2 * stride * sizeof(unsigned long long));
  L.bytes = o;
  L.out_size = out_bytes(n, S);
  return L;
}

SlotDesc make_slot(const DevGraph& g, int problem, const qqa_schedule& sched, int S, int K, uint64_t seed,
                   int lanes_per_row, char* arena, const SlotLayout& L, char* out, const float4* table, int start) {
  SlotDesc d{};
  StepParams& p = d.p;
  p.row_ptr = g.row_ptr;
  p.col = g.col;
  p.w = problem == QQA_MAXCUT ? g.w : nullptr;
  p.coupling = nullptr;
  p.hub_first = g.hub_first;
  p.hub_partial = g.nchunks ? reinterpret_cast<float*>(arena + L.hub) : nullptr;
  p.m = sched.rule == QQA_STEP_ADAMW ? reinterpret_cast<float*>(arena + L.m) : nullptr;
  p.v = sched.rule == QQA_STEP_ADAMW ? reinterpret_cast<float*>(arena + L.v) : nullptr;
  p.n = g.n;
  fill_static_scalars(p, sched, problem, S, seed);
  p.lanes_per_row = lanes_per_row;
  d.P[0] = reinterpret_cast<float*>(arena + L.P0);
  d.P[1] = reinterpret_cast<float*>(arena + L.P1);
  d.table = table;
  d.chunks = g.chunks;
  d.nchunks = g.nchunks;
  d.K = K;
  d.start = start;
  d.active = 1;
  d.seed = seed;
  d.lambda64 = sched.penalty_lambda;
  d.acc = reinterpret_cast<unsigned long long*>(arena + L.acc);
  int64_t *a, *b, *o;
  int32_t* best;
  uint8_t* x;
  out_views(out, g.n, S, &a, &b, &o, &best, &x);
  d.size_or_cut = a;
  d.viol = b;
  d.obj = o;
  d.best = best;
  d.x = x;
  return d;
}

void append_items(int slot, const DevGraph& g, int lanes_per_row, std::vector<WorkItem>* items,
                  std::vector<HubItem>* hubs) {
  const int rows_per_block = kBlock / lanes_per_row;
  for (int r = 0; r < g.n; r += rows_per_block) items->push_back(WorkItem{slot, r});
  for (int c = 0; c < g.nchunks; ++c) hubs->push_back(HubItem{slot, c});
}

BatchRun::~BatchRun() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (c) {
    c->dpool.put(arena, arena_bytes);
    c->hpool.put(host_out, host_out_bytes);
    c->in_use -= footprint;
  }
}

}  // namespace qqa

namespace {

// One replica layout class of a batch: its slots' row blocks and split-row chunks.
struct LayoutClass {
  int S = 0, lanes = 0;
  int spec = -1;  // the default_spec its instances share (0: none), -1 before the first
  std::vector<WorkItem> items;
  std::vector<HubItem> hubs;
  std::vector<int32_t> ids;
  size_t off_items = 0, off_hubs = 0, off_ids = 0;
};

}  // namespace

extern "C" {

int qqa_solve_batch(qqa_ctx* c, int32_t count, const qqa_graph_id* graphs, const qqa_problem* problems,
                    const qqa_schedule* sched, const int32_t* S, const int32_t* steps, const uint64_t* seeds,
                    qqa_req* out_ids) {
  if (!c) return QQA_E_ARG;
  if (count <= 0 || !graphs || !problems || !S || !steps || !seeds || !out_ids)
    return set_err(c, QQA_E_ARG, "batch arguments missing");
  (void)hipSetDevice(c->device);
  struct Inst {
    const DevGraph* g;
    int64_t gid;
    int problem, S, K, lanes, table;
    uint64_t seed;
    qqa_schedule s;
    SlotLayout L;
    size_t off, out_off;
  };
  std::vector<Inst> inst((size_t)count);
  std::vector<std::vector<float4>> tables;
  std::map<std::string, int> table_of;
  int maxK = 0;
  size_t arena = 0, out_total = 0;
  for (int i = 0; i < count; ++i) {
    Inst& I = inst[i];
    auto git = c->graphs.find(graphs[i]);
    if (git == c->graphs.end() || git->second.release_pending) return set_err(c, QQA_E_ARG, "unknown graph id in batch");
    I.g = &git->second;
    I.gid = graphs[i];
    I.problem = problems[i];
    if (!known_problem(I.problem)) return set_err(c, QQA_E_ARG, "unknown problem");
    if (I.problem == QQA_MAXCLIQUE || I.problem == QQA_COLORING) return set_err(c, QQA_E_ARG, "max clique and coloring are solved one at a time");
    if (I.g->problem != I.problem) return set_err(c, QQA_E_ARG, "graph was uploaded for another problem type");
    if (I.g->dense) return set_err(c, QQA_E_ARG, "dense graphs are solved one at a time");
    I.S = S[i];
    I.K = steps[i];
    if (I.S <= 0 || I.S > kMaxReplicas || I.K <= 0) return set_err(c, QQA_E_ARG, "need 1 <= S <= 4096 and steps > 0");
    I.seed = seeds[i];
    if (sched) I.s = sched[i]; else qqa_schedule_default(&I.s, (qqa_problem)I.problem, I.g->n);
    std::string why;
    if (!schedule_valid(I.s, &why)) return set_err(c, QQA_E_ARG, why);
    I.lanes = replica_shape(I.S, c->layout_for(I.S)).lpr;
    I.L = slot_layout(I.g->n, I.S, I.s.rule, I.g->nchunks);
    I.off = arena;
    arena += I.L.bytes;
    I.out_off = out_total;
    out_total += align256(I.L.out_size);
    std::string key(reinterpret_cast<const char*>(&I.s), sizeof(qqa_schedule));
    key += std::to_string(I.K);
    auto it = table_of.find(key);
    if (it == table_of.end()) {
      it = table_of.emplace(key, (int)tables.size()).first;
      tables.push_back(schedule_table(I.s, I.K));
    }
    I.table = it->second;
    maxK = std::max(maxK, I.K);
  }
  // layout classes
  std::map<std::pair<int, int>, LayoutClass> classes;
  for (int i = 0; i < count; ++i) {
    LayoutClass& lc = classes[{inst[i].S, inst[i].lanes}];
    lc.S = inst[i].S;
    lc.lanes = inst[i].lanes;
    const int sp = default_spec(inst[i].problem, inst[i].s.rule, inst[i].s.entropy_alpha);
    lc.spec = lc.spec < 0 || lc.spec == sp ? sp : 0;
    append_items(i, *inst[i].g, inst[i].lanes, &lc.items, &lc.hubs);
    lc.ids.push_back(i);
  }
  // The resident engine runs the batch when every instance shares one layout with one quad
  // per lane, none has split rows, and each instance's team fits the workgroups one XCD
  // holds; the automatic policy uses it then, QQA_ENGINE_STREAM keeps the slot launches.
  bool resident = c->engine_policy < 0 && classes.size() == 1;
  if (resident) {
    auto pref = c->batch_resident.find(classes.begin()->second.S);
    resident = pref == c->batch_resident.end() || pref->second != 0;
  }
  int res_lanes = 0, res_grid = 0, rows_per_wg = 0;
  // the facts every instance shares (the default schedule of one problem), fixed in the kernel
  int res_spec = default_spec(inst[0].problem, inst[0].s.rule, inst[0].s.entropy_alpha);
  for (int i = 1; i < count && res_spec; ++i)
    if (default_spec(inst[i].problem, inst[i].s.rule, inst[i].s.entropy_alpha) != res_spec) res_spec = 0;
  if (resident) {
    const LayoutClass& lc = classes.begin()->second;
    const ReplicaShape sh = replica_shape(lc.S, lc.lanes);
    res_lanes = sh.lpr;
    resident = sh.qpl == 1 && lc.S == 4 * sh.lpr;
    for (int i = 0; i < count && resident; ++i) resident = inst[i].g->nchunks == 0;
    if (resident) {
      res_grid = resident_workgroups(res_lanes, kResidentRowsPerGroup, res_spec);
      rows_per_wg = (kBlock / res_lanes) * kResidentRowsPerGroup;
      int max_team = 0;
      for (int i = 0; i < count; ++i) max_team = std::max(max_team, (inst[i].g->n + rows_per_wg - 1) / rows_per_wg);
      resident = res_grid >= kResidentXcds && max_team <= std::min(kResidentMaxTeam, res_grid / kResidentXcds);
    }
  }
  std::vector<ResidentJob> jobs;
  std::vector<int32_t> xcd_jobs(kResidentXcds + 1, 0), xcd_places(kResidentXcds, 0);
  double longest_xcd_updates = 0.0;
  if (resident) {
    // longest processing time first: each instance, largest cost first, goes to the XCD with
    // the least cost so far
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    auto team_of = [&](int i) { return (inst[i].g->n + rows_per_wg - 1) / rows_per_wg; };
    // cost of a job: its team x updates x (8 + mean degree), the row work of an update
    // growing with the gathers (measured on the 512-instance batch: 268-270 against 279 us per
    // update with team x updates alone; 8 was the best of 0.5, 3, 8 and 16, the others no
    // better than team x updates)
    auto cost_of = [&](int i) {
      const double deg = inst[i].g->n ? (double)inst[i].g->nnz / inst[i].g->n : 0.0;
      return (double)team_of(i) * inst[i].K * (8.0 + deg);
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost_of(a) > cost_of(b); });
    std::vector<std::vector<int>> per(kResidentXcds);
    std::vector<double> load(kResidentXcds, 0);
    std::vector<double> updates(kResidentXcds, 0.0);
    for (int i : order) {
      const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      per[x].push_back(i);
      load[x] += cost_of(i);
      updates[x] += inst[i].K;
    }
    // within an XCD: first-fit decreasing into rounds whose teams fill the XCD's workgroups,
    // claimed round after round, so that the jobs running together leave few workgroups
    // waiting for an incomplete team (measured on the 512-instance batch: 280 against 301 us
    // per update in plain decreasing order)
    const int per_xcd = res_grid / kResidentXcds;
    for (int x = 0; x < kResidentXcds; ++x) {
      std::vector<std::vector<int>> bins;
      std::vector<int> room;
      for (int i : per[x]) {
        size_t b = 0;
        while (b < bins.size() && room[b] < team_of(i)) ++b;
        if (b == bins.size()) {
          bins.emplace_back();
          room.push_back(per_xcd);
        }
        bins[b].push_back(i);
        room[b] -= team_of(i);
      }
      per[x].clear();
      for (const auto& bn : bins) per[x].insert(per[x].end(), bn.begin(), bn.end());
    }
    int32_t flag = 0;
    for (int x = 0; x < kResidentXcds; ++x) {
      xcd_jobs[x] = (int32_t)jobs.size();
      int32_t place = 0;
      for (int i : per[x]) {
        jobs.push_back(ResidentJob{i, team_of(i), place, flag});
        place += team_of(i);
        flag += team_of(i);
      }
      xcd_places[x] = place;
      longest_xcd_updates = std::max(longest_xcd_updates, updates[x]);
    }
    xcd_jobs[kResidentXcds] = (int32_t)jobs.size();
  }

  // arena tail: tables, slot descriptors, work lists, clock, then the result records
  std::vector<size_t> table_off(tables.size());
  for (size_t k = 0; k < tables.size(); ++k) {
    table_off[k] = arena;
    arena += align256(tables[k].size() * sizeof(float4));
  }
  const size_t off_slots = arena;
  arena += align256((size_t)count * sizeof(SlotDesc));
  for (auto& kv : classes) {
    LayoutClass& lc = kv.second;
    lc.off_items = arena;
    arena += align256(lc.items.size() * sizeof(WorkItem));
    lc.off_hubs = arena;
    arena += align256(lc.hubs.size() * sizeof(HubItem));
    lc.off_ids = arena;
    arena += align256(lc.ids.size() * sizeof(int32_t));
  }
  const size_t off_clock = arena;
  arena += 256;
  // resident engine tables and counters (zero in the uploaded image)
  const size_t off_jobs = arena;
  arena += align256(jobs.size() * sizeof(ResidentJob));
  const size_t off_xcd = arena;
  arena += align256((2 * kResidentXcds + 1) * sizeof(int32_t));
  size_t flag_count = 0;
  for (const ResidentJob& j : jobs) flag_count += (size_t)j.team;
  const size_t off_counters = arena;
  arena += align256((kResidentXcds + 2) * sizeof(unsigned));
  const size_t off_flags = arena;
  arena += align256(flag_count * kFlagWords * sizeof(unsigned));
  const size_t off_out = arena;
  arena += out_total;

  auto run = std::make_shared<BatchRun>();
  run->footprint = arena;
  hipError_t e = hipSuccess;
  if (arena > c->budget) return set_err(c, QQA_E_ADMISSION, "batch footprint exceeds the HBM budget");
  if (!budget_fits(c, arena)) return set_err(c, QQA_E_NOMEM, "HBM budget held by earlier requests");
  e = c->dpool.get(arena, (void**)&run->arena);
  if (e == hipSuccess) {
    run->arena_bytes = arena;
    e = c->hpool.get(out_total, (void**)&run->host_out);
  }
  if (e == hipSuccess) run->host_out_bytes = out_total;
  for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&run->ev[i]);
  run->c = c;  // from here on the destructor returns what was taken
  c->in_use += arena;
  if (e != hipSuccess) return set_err(c, e == hipErrorOutOfMemory ? QQA_E_NOMEM : QQA_E_DEVICE, hipGetErrorString(e));

  // host image of everything up to the result records, uploaded in one copy
  std::vector<char> image(off_out, 0);
  char* A = run->arena;
  for (size_t k = 0; k < tables.size(); ++k)
    std::memcpy(image.data() + table_off[k], tables[k].data(), tables[k].size() * sizeof(float4));
  for (int i = 0; i < count; ++i) {
    const Inst& I = inst[i];
    SlotDesc d = make_slot(*I.g, I.problem, I.s, I.S, I.K, I.seed, I.lanes, A + I.off, I.L, A + off_out + I.out_off,
                           reinterpret_cast<const float4*>(A + table_off[I.table]), 0);
    std::memcpy(image.data() + off_slots + (size_t)i * sizeof(SlotDesc), &d, sizeof(SlotDesc));
  }
  for (auto& kv : classes) {
    const LayoutClass& lc = kv.second;
    std::memcpy(image.data() + lc.off_items, lc.items.data(), lc.items.size() * sizeof(WorkItem));
    std::memcpy(image.data() + lc.off_hubs, lc.hubs.data(), lc.hubs.size() * sizeof(HubItem));
    std::memcpy(image.data() + lc.off_ids, lc.ids.data(), lc.ids.size() * sizeof(int32_t));
  }
  if (resident) {
    std::memcpy(image.data() + off_jobs, jobs.data(), jobs.size() * sizeof(ResidentJob));
    std::memcpy(image.data() + off_xcd, xcd_jobs.data(), xcd_jobs.size() * sizeof(int32_t));
    std::memcpy(image.data() + off_xcd + xcd_jobs.size() * sizeof(int32_t), xcd_places.data(),
                xcd_places.size() * sizeof(int32_t));
  }
  const SlotDesc* d_slots = reinterpret_cast<const SlotDesc*>(A + off_slots);
  int32_t* d_clock = reinterpret_cast<int32_t*>(A + off_clock);
  hipStream_t st = c->stream;
  // the state buffers are written by the init kernel; upload tables onwards
  const size_t up0 = tables.empty() ? off_slots : table_off[0];
  e = hipMemcpyAsync(A + up0, image.data() + up0, off_out - up0, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host image goes out of scope

  const auto t_submit = Clock::now();
  if (e == hipSuccess) e = hipEventRecord(run->ev[0], st);
  for (auto& kv : classes) {
    const LayoutClass& lc = kv.second;
    if (e == hipSuccess)
      e = launch_slot_init(d_slots, reinterpret_cast<const WorkItem*>(A + lc.off_items), (int)lc.items.size(), lc.lanes,
                           st);
  }
  // the update loop: R launches per layout class and a clock advance, captured once and
  // replayed until the longest instance has run all of its updates; or one resident launch.
  // Its start event is recorded once the graph is built, so the loop's device time does not
  // include the host's capture.
  const int R = std::min(maxK, 64);
  if (resident && e == hipSuccess) {
    ResidentParams rp{};
    rp.slots = d_slots;
    rp.jobs = reinterpret_cast<const ResidentJob*>(A + off_jobs);
    rp.xcd_jobs = reinterpret_cast<const int32_t*>(A + off_xcd);
    rp.xcd_places = rp.xcd_jobs + kResidentXcds + 1;
    unsigned* counters = reinterpret_cast<unsigned*>(A + off_counters);
    rp.claim = counters;
    rp.abort = counters + kResidentXcds;
    rp.done = counters + kResidentXcds + 1;
    rp.flags = reinterpret_cast<unsigned*>(A + off_flags);
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) != hipSuccess || khz <= 0)
      khz = 100000;
    // a barrier may wait for the XCD's earlier jobs to free workgroups: allow 10 s plus
    // 100 us for every update those jobs run
    rp.timeout_ticks = (long long)((10.0 + 1e-4 * longest_xcd_updates) * 1e3 * khz);
    e = hipEventRecord(run->ev[1], st);
    if (e == hipSuccess) e = launch_resident(rp, res_lanes, kResidentRowsPerGroup, res_spec, res_grid, count, count, st);
  } else if (e == hipSuccess) e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (!resident && e == hipSuccess) {
    hipError_t ce = hipSuccess;
    for (int r = 0; r < R && ce == hipSuccess; ++r)
      for (auto& kv : classes) {
        const LayoutClass& lc = kv.second;
        if (ce == hipSuccess && !lc.hubs.empty())
          ce = launch_slot_hubs(d_slots, reinterpret_cast<const HubItem*>(A + lc.off_hubs), (int)lc.hubs.size(), lc.S,
                                lc.lanes, d_clock, r, st);
        if (ce == hipSuccess)
          ce = launch_slot_step(d_slots, reinterpret_cast<const WorkItem*>(A + lc.off_items), (int)lc.items.size(),
                                lc.S, lc.lanes, std::max(lc.spec, 0), d_clock, r, st);
      }
    if (ce == hipSuccess) ce = launch_clock_advance(d_clock, R, st);
    e = hipStreamEndCapture(st, &run->graph);
    if (e == hipSuccess) e = ce;
  }
  if (!resident && e == hipSuccess) e = hipGraphInstantiate(&run->exec, run->graph, nullptr, nullptr, 0);
  if (!resident && e == hipSuccess) e = hipEventRecord(run->ev[1], st);
  for (int done = 0; !resident && done < maxK && e == hipSuccess; done += R) e = hipGraphLaunch(run->exec, st);
  if (e == hipSuccess) e = hipEventRecord(run->ev[2], st);
  for (auto& kv : classes) {
    const LayoutClass& lc = kv.second;
    if (e == hipSuccess)
      e = launch_slot_eval(d_slots, reinterpret_cast<const int32_t*>(A + lc.off_ids), (int)lc.ids.size(),
                           reinterpret_cast<const WorkItem*>(A + lc.off_items), (int)lc.items.size(), lc.S, lc.lanes,
                           st);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(run->host_out, A + off_out, out_total, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipEventRecord(run->ev[3], st);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(st);
    return set_err(c, QQA_E_DEVICE, std::string("batch enqueue: ") + hipGetErrorString(e));
  }
  for (int i = 0; i < count; ++i) {
    const Inst& I = inst[i];
    auto r = std::make_unique<Request>();
    r->id = c->next_req++;
    r->graph = I.gid;
    r->problem = I.problem;
    r->sched = I.s;
    r->S = I.S;
    r->K = I.K;
    r->n = I.g->n;
    r->seed = I.seed;
    r->shape = replica_shape(I.S);
    r->lanes_per_row = I.lanes;
    r->engine = resident ? kEngineResident : kEngineBatch;
    r->out_host = run->host_out + I.out_off;
    r->out_size = I.L.out_size;
    for (int k = 0; k < 4; ++k) r->ev[k] = run->ev[k];
    r->owner = run;
    r->t_submit = t_submit;
    r->state = Request::kRunning;
    c->graphs[I.gid].refs++;
    out_ids[i] = r->id;
    c->reqs.emplace(r->id, std::move(r));
  }
  return QQA_OK;
}

// Device time of one batch's update loop per update of its longest instance, and the engine
// that ran it.  Seeds 1..count; results are discarded.
static int time_batch(qqa_ctx* c, const std::vector<qqa_graph_id>& g, const std::vector<qqa_problem>& prob,
                      const std::vector<qqa_schedule>& sched, const std::vector<int32_t>& S,
                      const std::vector<int32_t>& K, double* us, int* engine) {
  const int count = (int)g.size();
  std::vector<uint64_t> seeds((size_t)count);
  for (int i = 0; i < count; ++i) seeds[i] = (uint64_t)i + 1;
  std::vector<qqa_req> ids((size_t)count);
  int rc = qqa_solve_batch(c, count, g.data(), prob.data(), sched.empty() ? nullptr : sched.data(), S.data(), K.data(),
                           seeds.data(), ids.data());
  if (rc) return rc;
  qqa_result first{};
  for (int i = 0; i < count; ++i) {
    qqa_result r{};
    const int prc = qqa_poll(c, ids[i], &r, -1);
    if (prc != QQA_OK && rc == QQA_OK) rc = prc;
    if (i == 0) first = r;
  }
  if (rc) return rc;
  *us = first.step_loop_ms * 1e3 / *std::max_element(K.begin(), K.end());
  *engine = first.engine;
  return QQA_OK;
}

int qqa_autotune_batch(qqa_ctx* c, int32_t count, const qqa_graph_id* graphs, const qqa_problem* problems,
                       const qqa_schedule* sched, const int32_t* S, const int32_t* steps, int32_t* lanes_out,
                       int32_t* resident_out) {
  if (!c) return QQA_E_ARG;
  if (count <= 0 || !graphs || !problems || !S || !steps) return set_err(c, QQA_E_ARG, "batch arguments missing");
  if (c->engine_policy >= 0 && c->engine_policy != QQA_ENGINE_STREAM)
    return set_err(c, QQA_E_ARG, "the batch autotuner runs under the automatic or STREAM policy");
  int maxK = 0;
  for (int i = 0; i < count; ++i) {
    if (S[i] <= 0 || S[i] > kMaxReplicas || steps[i] <= 0)
      return set_err(c, QQA_E_ARG, "need 1 <= S <= 4096 and steps > 0");
    maxK = std::max(maxK, steps[i]);
  }
  // a shortened copy of the batch: the longest instance runs kProbe updates, the others
  // keep their share of it, so that the work of the resident engine's teams keeps its mix
  constexpr int kProbe = 64, kRepeats = 2;
  std::map<int, std::vector<int>> by_S;
  for (int i = 0; i < count; ++i) by_S[S[i]].push_back(i);
  const auto saved_layout = c->layout;
  const auto saved_resident = c->batch_resident;
  const int saved_policy = c->engine_policy;
  auto sub = [&](const std::vector<int>& idx, std::vector<qqa_graph_id>* g, std::vector<qqa_problem>* pr,
                 std::vector<qqa_schedule>* sc, std::vector<int32_t>* s, std::vector<int32_t>* k) {
    for (int i : idx) {
      g->push_back(graphs[i]);
      pr->push_back(problems[i]);
      if (sched) sc->push_back(sched[i]);
      s->push_back(S[i]);
      k->push_back(std::max(2, (int)(((int64_t)steps[i] * kProbe + maxK - 1) / maxK)));
    }
  };
  auto best_of = [&](const std::vector<qqa_graph_id>& g, const std::vector<qqa_problem>& pr,
                     const std::vector<qqa_schedule>& sc, const std::vector<int32_t>& s, const std::vector<int32_t>& k,
                     double* us, int* engine) {
    *us = 1e300;
    for (int rep = 0; rep < kRepeats; ++rep) {  // the first run also loads the kernels
      double t = 0.0;
      const int rc = time_batch(c, g, pr, sc, s, k, &t, engine);
      if (rc) return rc;
      *us = std::min(*us, t);
    }
    return (int)QQA_OK;
  };
  auto fail = [&](int rc) {
    const std::string why = c->err;
    c->layout = saved_layout;
    c->batch_resident = saved_resident;
    c->engine_policy = saved_policy;
    return set_err(c, rc, "batch autotune: " + why);
  };
  // each S: every replica layout on the slot launches, over that S's instances alone (the
  // layout classes of a batch run one after another, so their times add)
  c->engine_policy = QQA_ENGINE_STREAM;
  std::map<int, std::pair<int, double>> best;  // S -> (lanes per row, us per update)
  for (const auto& kv : by_S) {
    std::vector<qqa_graph_id> g;
    std::vector<qqa_problem> pr;
    std::vector<qqa_schedule> sc;
    std::vector<int32_t> s, k;
    sub(kv.second, &g, &pr, &sc, &s, &k);
    std::pair<int, double> b{0, 1e300};
    int last = -1;
    for (int want = 1; want <= 64; want <<= 1) {
      const ReplicaShape sh = replica_shape(kv.first, want);
      if (sh.lpr == last || !layout_supported(kv.first, want)) continue;
      last = sh.lpr;
      c->layout[kv.first] = sh.lpr;
      double us = 0.0;
      int engine = 0;
      const int rc = best_of(g, pr, sc, s, k, &us, &engine);
      if (rc) return fail(rc);
      if (us < b.second) b = {sh.lpr, us};
    }
    best[kv.first] = b;
    c->layout[kv.first] = b.first;
  }
  c->engine_policy = saved_policy;
  // one layout class under the automatic policy: the resident engine at the default layout
  int resident = 0;
  if (saved_policy < 0 && by_S.size() == 1) {
    const int s0 = by_S.begin()->first;
    std::vector<qqa_graph_id> g;
    std::vector<qqa_problem> pr;
    std::vector<qqa_schedule> sc;
    std::vector<int32_t> s, k;
    sub(by_S.begin()->second, &g, &pr, &sc, &s, &k);
    c->layout.erase(s0);
    c->batch_resident.erase(s0);
    double us = 0.0;
    int engine = 0;
    const int rc = best_of(g, pr, sc, s, k, &us, &engine);
    if (rc) return fail(rc);
    resident = engine == QQA_ENGINE_BATCH_RESIDENT && us < best[s0].second;
    c->batch_resident[s0] = resident;
    if (!resident) c->layout[s0] = best[s0].first;
  }
  if (lanes_out)
    for (int i = 0; i < count; ++i) lanes_out[i] = replica_shape(S[i], c->layout_for(S[i])).lpr;
  if (resident_out) *resident_out = resident;
  return QQA_OK;
}

}  // extern "C"
