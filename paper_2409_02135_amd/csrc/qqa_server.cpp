// Continuous-batching server (qqa_serve_start / qqa_serve_submit / qqa_serve_stop).
//
// A server thread owns a stream and a table of device slots.  It works in rounds of
// kRound updates.  At the start of a round the stream is idle: finished slots are
// retired (their results are already in pinned host memory), queued requests are
// admitted first-come-first-served while a slot is free and their HBM footprint fits the
// budget, and the compact work lists of the running slots are rebuilt.  The running slots
// are the admitted ones with the least remaining work (updates left x rows x replica
// stride), taken in that order until one update of them covers kRunElements replica-
// variables, enough to fill the device; the others wait for the round, their start moved
// on by kRound so their update index stays where it was.  Shortest remaining work first
// finishes small requests at close to their time alone instead of sharing the device with
// every large one, which cuts the median latency at no cost in throughput.  Then kRound
// update launches advance every running slot, each at its own update index
// t = t_arg - start, and the slots that reach their last update during the round are
// evaluated and copied back.  Requests that arrive while others run join at the next
// round boundary, so their work overlaps on the device.  Each slot runs the same row
// arithmetic as a solve alone (the slot kernels share qqa_device.h), so a served result
// equals the result of the same solve alone.
//
// Load shedding (optional, qqa_serve_set_deadline): a request is refused at submit unless
// every admitted request, and it, can still finish within the deadline.  Under
// least-remaining-work-first a request of work w (rows x replica stride x updates) waits for
// the pending work of requests with no more remaining work than its own, W_<=, and for the
// work that arrives meanwhile in requests no larger than w, at rate a_w (measured over the
// admitted submissions of the last 5 s); at a device rate R it then finishes after
// (W_<= + w) / (R - a_w) (the busy period of shortest-remaining-work scheduling), and no
// sooner than its updates x the shortest update seen.  Admitting it delays every pending
// request with more remaining work by w / R:
// it is refused if one of them would then be projected past its own deadline, also one that
// is late already.  So work that arrives later never pushes an admitted request past its
// deadline (up to the accuracy of R), and a request the projection underestimated is not
// overtaken by ever more smaller work, which a test of the new request alone cannot promise.
// R is measured over rounds that leave work waiting (so the device could do no more).  The
// rounds run requests older than half the deadline first, oldest first, so that the large
// requests least-remaining-work-first would keep postponing finish in time.  (Measured on a
// Poisson stream at 200 requests/s for 60 s, 8x the device's rate, 2 s deadline: 6,454
// admitted, 6,453 of them within the deadline, p99 1.4 s.  The new request's own projection
// alone: 7,085 admitted, p99 5.3 s; with the protection of admitted requests but no urgent
// ones first: 2,017 admitted, as late requests blocked the smaller arrivals.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "qqa.h"
#include "qqa_batch.h"
#include "qqa_ctx.h"

using Clock = std::chrono::steady_clock;

namespace qqa {

namespace {
constexpr int kRound = 16;
// with a deadline, requests older than this fraction of it run first, oldest first
constexpr double kUrgentFraction = 0.5;
// the window over which the admitted work arriving per second is measured
constexpr double kArrivalWindowS = 5.0;
// replica-variables per update launch beyond which more running slots add no throughput
constexpr int64_t kRunElements = int64_t(8) << 20;
constexpr int64_t kServerIdBase = int64_t(1) << 40;
// device rate assumed before a round that fills the device has been measured
constexpr double kInitialRate = 1e11;
// idle buffers the server's pools keep for reuse
constexpr size_t kDevicePoolCap = size_t(4) << 30;
constexpr size_t kHostPoolCap = size_t(512) << 20;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}
}  // namespace

struct ServerReq {
  enum State { kQueued, kActive, kFinishing, kDone, kFailed };
  int64_t id = 0;
  State state = kQueued;
  bool cancelled = false;
  std::string error;
  // owned copy of the request
  int n = 0;
  int64_t nnz = 0;
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col;
  std::vector<float> w;
  int problem = 0, S = 0, K = 0, nchunks = 0;
  qqa_schedule sched{};
  uint64_t seed = 0;
  size_t footprint = 0;
  double work = 0.0;      // rows x replica stride x updates
  double rem_work = 0.0;  // the part not yet run (updated at round boundaries, under mu)
  bool started = false;
  Clock::time_point t_submit, t_admit, t_first, t_done;
  // while admitted
  DevGraph g;
  int slot = -1, lanes = 0, start = 0;
  SlotLayout L{};
  char* arena = nullptr;
  size_t arena_bytes = 0;
  char* out_dev = nullptr;
  char* out_host = nullptr;
  size_t out_size = 0;
};

struct Server {
  qqa_ctx* c = nullptr;
  int device = 0;
  int max_slots = 0;
  hipStream_t st = nullptr;
  Pool dpool{false, kDevicePoolCap};
  Pool hpool{true, kHostPoolCap};
  size_t budget = 0, in_use = 0;
  // load shedding and its statistics (under mu)
  double deadline_ms = 0.0;
  double rate = kInitialRate;       // replica-variable updates per second, measured
  double update_floor_s = 0.0;      // shortest time of one update seen
  int64_t n_submitted = 0, n_shed = 0, n_admitted = 0, n_completed = 0;
  bool meets_deadline(const ServerReq& r, Clock::time_point now, double* ms, const char** why);
  std::deque<std::pair<Clock::time_point, double>> recent;  // admitted submissions (time, work)
  std::unordered_map<int, int> layout;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stopping = false;
  bool failed = false;
  std::string fail_msg;
  int64_t next_id = kServerIdBase;
  std::deque<std::shared_ptr<ServerReq>> queue;
  std::unordered_map<int64_t, std::shared_ptr<ServerReq>> all;
  std::vector<std::shared_ptr<ServerReq>> slots;
  // device tables
  SlotDesc* d_slots = nullptr;
  std::vector<SlotDesc> h_slots;  // host copy of d_slots
  int32_t* d_zero = nullptr;  // the slot kernels' clock word, kept at 0: t = t_arg - start
  char* d_lists = nullptr;    // work lists and slot ids, rebuilt at round boundaries
  size_t lists_cap = 0;
  int clock = 0;

  void run();
  void fail_all(const std::string& msg);
  size_t footprint_of(const ServerReq& r) const;
};

size_t Server::footprint_of(const ServerReq& r) const {
  const SlotLayout L = slot_layout(r.n, r.S, r.sched.rule, r.nchunks);
  const size_t graph = 4 * (size_t)(r.n + 1) + 4 * (size_t)r.nnz + (r.problem == QQA_MAXCUT && !r.w.empty() ? 4 * r.nnz : 0) +
                       (size_t)r.nchunks * sizeof(HubChunk) + (r.nchunks ? 4 * (size_t)r.n : 0);
  // the arena and the result buffer as the pool rounds them
  return Pool::class_size(L.bytes + align256((size_t)r.K * sizeof(float4))) + Pool::class_size(L.out_size) + graph +
         4096;
}

// Whether r, admitted now, and every pending request would still meet the deadline (see the
// header); *ms = r's projected submit-to-result time.  Under mu.
bool Server::meets_deadline(const ServerReq& r, Clock::time_point now, double* ms, const char** why) {
  const double D = 1e-3 * deadline_ms;
  std::vector<std::pair<double, double>> pend;  // (remaining work, seconds left to its deadline)
  for (const auto& kv : all) {
    const ServerReq& o = *kv.second;
    if ((o.state == ServerReq::kQueued && !o.cancelled) || o.state == ServerReq::kActive)
      pend.push_back({o.rem_work, D - std::chrono::duration<double>(now - o.t_submit).count()});
  }
  std::sort(pend.begin(), pend.end());
  double ahead = 0.0;
  for (const auto& p : pend)
    if (p.first <= r.work) ahead += p.first;
  // smaller work keeps arriving while r waits: at the rate a_w of the admitted submissions of
  // the last few seconds that were no larger than r
  while (!recent.empty() && std::chrono::duration<double>(now - recent.front().first).count() > kArrivalWindowS)
    recent.pop_front();
  double arriving = 0.0;
  for (const auto& a : recent)
    if (a.second <= r.work) arriving += a.second;
  const double a_w = arriving / kArrivalWindowS;
  const double done = a_w >= rate ? 1e300 : std::max((double)r.K * update_floor_s, (ahead + r.work) / (rate - a_w));
  *ms = 1e3 * done;
  if (done > D) {
    *why = "its projected completion";
    return false;
  }
  double cum = 0.0;
  for (const auto& p : pend) {
    cum += p.first;
    if (p.first <= r.work) continue;
    // its projected finish, delayed by r: refused also when it is late already, so that a
    // request the projection underestimated is not overtaken by ever more smaller work
    if ((cum + r.work) / rate > p.second) {
      *why = "the projected completion of an admitted request";
      return false;
    }
  }
  return true;
}

void Server::fail_all(const std::string& msg) {
  std::lock_guard<std::mutex> lk(mu);
  failed = true;
  fail_msg = msg;
  for (auto& kv : all)
    if (kv.second->state != ServerReq::kDone) {
      kv.second->state = ServerReq::kFailed;
      kv.second->error = msg;
    }
  queue.clear();
  cv_done.notify_all();
}

void Server::run() {
  (void)hipSetDevice(device);
  std::vector<WorkItem> items, eval_items, init_items;
  std::vector<HubItem> hubs;
  std::vector<int32_t> ids;
  Clock::time_point round_start{}, boundary = Clock::now();
  int64_t round_elements = 0;  // replica-variables per update of the last round
  bool round_backlogged = false;  // work was left waiting during the last round
  double round_deadline_s = 0.0;
  for (;;) {
    hipError_t e = hipStreamSynchronize(st);  // round boundary: the device is idle
    if (e != hipSuccess) {
      fail_all(std::string("server: ") + hipGetErrorString(e));
      return;
    }
    std::vector<std::shared_ptr<ServerReq>> admit;
    {
      std::unique_lock<std::mutex> lk(mu);
      const auto now = Clock::now();
      if (round_elements > 0) {
        const double per_update = std::chrono::duration<double>(now - round_start).count() / kRound;
        update_floor_s = update_floor_s > 0.0 ? std::min(update_floor_s, per_update) : per_update;
        // the device rate: the work done per second in rounds that left work waiting (so the
        // device could not have done more), over the whole loop from one round boundary to the
        // next (admission, uploads and list building included)
        const double dt = std::chrono::duration<double>(now - boundary).count();
        if (round_backlogged && dt > 0.0)
          rate = 0.8 * rate + 0.2 * ((double)round_elements * kRound / dt);
        round_elements = 0;
      }
      boundary = now;
      round_deadline_s = 1e-3 * deadline_ms;
      // retire slots whose evaluation and copy-back finished in the previous round
      for (auto& sp : slots) {
        if (!sp || sp->state != ServerReq::kFinishing) continue;
        sp->state = ServerReq::kDone;
        sp->t_done = Clock::now();
        dpool.put(sp->arena, sp->arena_bytes);
        dpool.put(sp->out_dev, sp->out_size);
        sp->arena = sp->out_dev = nullptr;
        free_graph(sp->g);
        in_use -= sp->footprint;
        ++n_completed;
        sp = nullptr;
      }
      cv_done.notify_all();
      // idle pooled buffers count against the budget: free them when they would crowd out
      // a queued request (the device is idle here, so freeing is safe)
      if (!queue.empty() && in_use + dpool.cached() + queue.front()->footprint > budget) dpool.trim();
      // admit first-come-first-served while a slot is free and the footprint fits
      int free_slots = 0;
      for (auto& sp : slots) free_slots += sp == nullptr;
      while (!queue.empty()) {
        auto& r = queue.front();
        if (r->cancelled) {
          queue.pop_front();
          continue;
        }
        if (free_slots == 0 || in_use + r->footprint > budget) break;
        in_use += r->footprint;
        admit.push_back(r);
        queue.pop_front();
        --free_slots;
      }
      bool active = false;
      for (auto& sp : slots) active |= sp != nullptr;
      if (!active && admit.empty()) {
        if (stopping && queue.empty()) return;
        cv_work.wait(lk, [&] { return stopping || !queue.empty(); });
        continue;
      }
    }
    // admission: upload, allocate, describe, initialise
    init_items.clear();
    for (auto& r : admit) {
      qqa_graph hg{r->n, r->nnz, r->row_ptr.data(), r->col.data(), r->w.empty() ? nullptr : r->w.data(), nullptr};
      std::string why;
      int rc = upload_graph_on(st, hg, r->problem, &r->g, &why, false);
      if (rc) {
        fail_all("server: " + why);
        return;
      }
      r->L = slot_layout(r->n, r->S, r->sched.rule, r->g.nchunks);
      r->arena_bytes = r->L.bytes + align256((size_t)r->K * sizeof(float4));
      r->out_size = r->L.out_size;
      e = dpool.get(r->arena_bytes, (void**)&r->arena);
      if (e == hipSuccess) e = dpool.get(r->out_size, (void**)&r->out_dev);
      if (e == hipSuccess) e = hpool.get(r->out_size, (void**)&r->out_host);
      if (e != hipSuccess) {
        fail_all(std::string("server buffers: ") + hipGetErrorString(e));
        return;
      }
      const std::vector<float4> table = schedule_table(r->sched, r->K);
      float4* d_table = reinterpret_cast<float4*>(r->arena + r->L.bytes);
      e = hipMemcpy(d_table, table.data(), table.size() * sizeof(float4), hipMemcpyHostToDevice);
      int slot = 0;
      while (slots[slot]) ++slot;
      r->slot = slot;
      r->lanes = replica_shape(r->S, layout.count(r->S) ? layout[r->S] : 0).lpr;
      r->start = clock;
      const SlotDesc d = make_slot(r->g, r->problem, r->sched, r->S, r->K, r->seed, r->lanes, r->arena, r->L,
                                   r->out_dev, d_table, r->start);
      h_slots[slot] = d;
      if (e == hipSuccess) e = hipMemcpy(d_slots + slot, &d, sizeof(SlotDesc), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        fail_all(std::string("server admission: ") + hipGetErrorString(e));
        return;
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        r->t_admit = Clock::now();
        r->state = ServerReq::kActive;
        slots[slot] = r;
        r->row_ptr.clear();
        r->row_ptr.shrink_to_fit();
        r->col.clear();
        r->col.shrink_to_fit();
        r->w.clear();
        r->w.shrink_to_fit();
      }
    }
    // work lists of the active slots, by replica layout class; slots finishing this round
    std::map<std::pair<int, int>, std::pair<size_t, size_t>> item_range, hub_range, eval_range, init_range;
    std::map<std::pair<int, int>, std::pair<size_t, size_t>> id_range;
    // the schedule facts every running slot of a class shares (default_spec), else 0; a class
    // is not split by them (more, smaller launches per update measured slower)
    std::map<std::pair<int, int>, int> class_spec;
    items.clear();
    hubs.clear();
    eval_items.clear();
    ids.clear();
    // running slots: least remaining work first (with a deadline, the urgent ones before
    // them, oldest first), until an update covers kRunElements
    std::vector<std::pair<std::pair<int64_t, int64_t>, int>> by_work;
    const auto t_round = Clock::now();
    for (int s = 0; s < max_slots; ++s)
      if (slots[s] && slots[s]->state == ServerReq::kActive) {
        const auto& r = slots[s];
        const int64_t left = (int64_t)(r->K - std::max(0, clock - r->start));
        const double age = std::chrono::duration<double>(t_round - r->t_submit).count();
        const bool urgent = round_deadline_s > 0.0 && age >= kUrgentFraction * round_deadline_s;
        const int64_t key = urgent ? (int64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(r->t_submit.time_since_epoch()).count()
                                   : left * r->n * (int64_t)qqa_replica_stride(r->S);
        by_work.push_back({{urgent ? 0 : 1, key}, s});
      }
    std::sort(by_work.begin(), by_work.end());
    std::map<std::pair<int, int>, std::vector<int>> cls_slots;
    std::vector<int> running_slots;
    int64_t running = 0;
    int dirty0 = max_slots, dirty1 = -1;
    for (const auto& kv : by_work) {
      const auto& r = slots[kv.second];
      if (running < kRunElements) {
        running += (int64_t)r->n * qqa_replica_stride(r->S);
        cls_slots[{r->S, r->lanes}].push_back(kv.second);
        const int sp = default_spec(r->problem, r->sched.rule, r->sched.entropy_alpha);
        auto cs = class_spec.emplace(std::make_pair(r->S, r->lanes), sp).first;
        if (cs->second != sp) cs->second = 0;
        running_slots.push_back(kv.second);
      } else {  // waits this round: its next update index is unchanged at the next boundary
        r->start += kRound;
        h_slots[kv.second].start = r->start;
        dirty0 = std::min(dirty0, kv.second);
        dirty1 = std::max(dirty1, kv.second);
      }
    }
    if (dirty1 >= dirty0)
      e = hipMemcpy(d_slots + dirty0, h_slots.data() + dirty0, (size_t)(dirty1 - dirty0 + 1) * sizeof(SlotDesc),
                    hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      fail_all(std::string("server slot table: ") + hipGetErrorString(e));
      return;
    }
    for (auto& kv : cls_slots) std::sort(kv.second.begin(), kv.second.end());  // slot order within a class
    for (auto& kv : cls_slots) {
      const size_t i0 = items.size(), h0 = hubs.size(), e0 = eval_items.size(), d0 = ids.size();
      for (int s : kv.second) {
        const auto& r = slots[s];
        append_items(s, r->g, r->lanes, &items, &hubs);
        if (clock + kRound - r->start >= r->K) {  // reaches its last update in this round
          std::vector<HubItem> unused;
          append_items(s, r->g, r->lanes, &eval_items, &unused);
          ids.push_back(s);
        }
      }
      item_range[kv.first] = {i0, items.size() - i0};
      hub_range[kv.first] = {h0, hubs.size() - h0};
      eval_range[kv.first] = {e0, eval_items.size() - e0};
      id_range[kv.first] = {d0, ids.size() - d0};
    }
    // new slots' initialisation items
    std::map<std::pair<int, int>, std::vector<int>> new_slots;
    for (auto& r : admit) new_slots[{r->S, r->lanes}].push_back(r->slot);
    const size_t init0 = items.size() + eval_items.size();
    init_items.clear();
    for (auto& kv : new_slots) {
      const size_t a0 = init_items.size();
      std::vector<HubItem> unused;
      for (int s : kv.second) append_items(s, slots[s]->g, slots[s]->lanes, &init_items, &unused);
      init_range[kv.first] = {a0, init_items.size() - a0};
    }
    (void)init0;
    // one upload of every list: [items][eval items][init items][hubs][ids]
    const size_t b_items = items.size() * sizeof(WorkItem), b_eval = eval_items.size() * sizeof(WorkItem),
                 b_init = init_items.size() * sizeof(WorkItem), b_hubs = hubs.size() * sizeof(HubItem),
                 b_ids = ids.size() * sizeof(int32_t);
    const size_t o_items = 0, o_eval = align256(b_items), o_init = o_eval + align256(b_eval),
                 o_hubs = o_init + align256(b_init), o_ids = o_hubs + align256(b_hubs), total = o_ids + align256(b_ids) + 256;
    if (total > lists_cap) {
      if (d_lists) (void)hipFree(d_lists);
      lists_cap = total * 2;
      e = hipMalloc((void**)&d_lists, lists_cap);
      if (e != hipSuccess) {
        fail_all(std::string("server lists: ") + hipGetErrorString(e));
        return;
      }
    }
    std::vector<char> img(total, 0);
    std::memcpy(img.data() + o_items, items.data(), b_items);
    std::memcpy(img.data() + o_eval, eval_items.data(), b_eval);
    std::memcpy(img.data() + o_init, init_items.data(), b_init);
    std::memcpy(img.data() + o_hubs, hubs.data(), b_hubs);
    std::memcpy(img.data() + o_ids, ids.data(), b_ids);
    e = hipMemcpy(d_lists, img.data(), total, hipMemcpyHostToDevice);
    const WorkItem* L_items = reinterpret_cast<const WorkItem*>(d_lists + o_items);
    const WorkItem* L_eval = reinterpret_cast<const WorkItem*>(d_lists + o_eval);
    const WorkItem* L_init = reinterpret_cast<const WorkItem*>(d_lists + o_init);
    const HubItem* L_hubs = reinterpret_cast<const HubItem*>(d_lists + o_hubs);
    const int32_t* L_ids = reinterpret_cast<const int32_t*>(d_lists + o_ids);
    for (auto& kv : init_range)
      if (e == hipSuccess)
        e = launch_slot_init(d_slots, L_init + kv.second.first, (int)kv.second.second, kv.first.second, st);
    // kRound updates of every active slot
    round_start = Clock::now();
    round_elements = running;
    round_backlogged = dirty1 >= dirty0;
    {
      std::lock_guard<std::mutex> lk(mu);
      round_backlogged = round_backlogged || !queue.empty();
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      for (int s : running_slots) {
        auto& r = slots[s];
        if (!r->started) {
          r->started = true;
          r->t_first = round_start;
        }
        const int left = std::max(0, r->K - std::max(0, clock + kRound - r->start));
        r->rem_work = (double)left * r->n * qqa_replica_stride(r->S);
      }
    }
    for (int r = 0; r < kRound && e == hipSuccess; ++r)
      for (auto& kv : item_range) {
        const auto hr = hub_range[kv.first];
        if (e == hipSuccess && hr.second)
          e = launch_slot_hubs(d_slots, L_hubs + hr.first, (int)hr.second, kv.first.first, kv.first.second, d_zero,
                               clock + r, st);
        if (e == hipSuccess)
          e = launch_slot_step(d_slots, L_items + kv.second.first, (int)kv.second.second, kv.first.first,
                               kv.first.second, class_spec[kv.first], d_zero, clock + r, st);
      }
    clock += kRound;
    // evaluate and copy back the slots that finished
    for (auto& kv : id_range) {
      if (!kv.second.second || e != hipSuccess) continue;
      const auto er = eval_range[kv.first];
      e = launch_slot_eval(d_slots, L_ids + kv.second.first, (int)kv.second.second, L_eval + er.first,
                           (int)er.second, kv.first.first, kv.first.second, st);
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      for (int32_t s : ids) {
        auto& r = slots[s];
        if (e == hipSuccess) e = hipMemcpyAsync(r->out_host, r->out_dev, r->out_size, hipMemcpyDeviceToHost, st);
        r->state = ServerReq::kFinishing;
      }
    }
    if (e != hipSuccess) {
      fail_all(std::string("server round: ") + hipGetErrorString(e));
      return;
    }
  }
}

int serve_poll(qqa_ctx* c, int64_t id, qqa_result* out, int32_t timeout_us) {
  Server* sv = c->server.get();
  if (!sv || id < kServerIdBase) return QQA_E_UNKNOWN_REQ;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return set_err(c, QQA_E_UNKNOWN_REQ, "unknown request id");
  auto r = it->second;
  auto finished = [&] { return r->state == ServerReq::kDone || r->state == ServerReq::kFailed || (r->cancelled && r->state == ServerReq::kQueued); };
  if (!finished()) {
    if (timeout_us == 0) return QQA_PENDING;
    if (timeout_us < 0) sv->cv_done.wait(lk, finished);
    else if (!sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), finished)) return QQA_PENDING;
  }
  sv->all.erase(it);
  if (r->cancelled) {
    if (r->out_host) sv->hpool.put(r->out_host, r->out_size);
    return set_err(c, QQA_E_CANCELLED, "request was cancelled");
  }
  if (r->state == ServerReq::kFailed) return set_err(c, QQA_E_DEVICE, r->error);
  if (out) {
    Request view;
    view.n = r->n;
    view.S = r->S;
    view.out_host = r->out_host;
    fill_result(&view, out);
    out->queue_ms = ms_between(r->t_submit, r->t_admit);
    out->first_update_ms = ms_between(r->t_submit, r->t_first);
    out->device_ms = ms_between(r->t_admit, r->t_done);
    out->step_loop_ms = out->device_ms;
    out->latency_ms = ms_between(r->t_submit, r->t_done);
    out->engine = QQA_ENGINE_BATCH;
  }
  sv->hpool.put(r->out_host, r->out_size);
  r->out_host = nullptr;
  return QQA_OK;
}

int serve_cancel(qqa_ctx* c, int64_t id) {
  Server* sv = c->server.get();
  if (!sv || id < kServerIdBase) return QQA_E_UNKNOWN_REQ;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return set_err(c, QQA_E_UNKNOWN_REQ, "unknown request id");
  it->second->cancelled = true;  // queued: dropped at admission; admitted: runs out, poll reports it
  sv->cv_done.notify_all();
  return QQA_OK;
}

// Stop the thread after it has run every admitted and queued request; results stay
// available to qqa_poll.
static void server_drain(Server* sv) {
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
  }
  sv->cv_work.notify_all();
  if (sv->th.joinable()) sv->th.join();
}

void server_shutdown(qqa_ctx* c) {
  Server* sv = c->server.get();
  if (!sv) return;
  server_drain(sv);
  (void)hipSetDevice(sv->device);
  (void)hipStreamSynchronize(sv->st);
  for (auto& kv : sv->all) {
    auto& r = kv.second;
    if (r->arena) sv->dpool.put(r->arena, r->arena_bytes);
    if (r->out_dev) sv->dpool.put(r->out_dev, r->out_size);
    if (r->out_host) sv->hpool.put(r->out_host, r->out_size);
    free_graph(r->g);
  }
  sv->all.clear();
  if (sv->d_slots) (void)hipFree(sv->d_slots);
  if (sv->d_zero) (void)hipFree(sv->d_zero);
  if (sv->d_lists) (void)hipFree(sv->d_lists);
  sv->dpool.trim();
  sv->hpool.trim();
  (void)hipStreamDestroy(sv->st);
  c->server.reset();
}

}  // namespace qqa

using namespace qqa;

qqa_ctx::qqa_ctx() = default;
qqa_ctx::~qqa_ctx() = default;

extern "C" {

int qqa_serve_start(qqa_ctx* c, int32_t max_slots) {
  if (!c) return QQA_E_ARG;
  if (c->server) {
    bool idle;
    {
      std::lock_guard<std::mutex> lk(c->server->mu);
      idle = c->server->stopping && c->server->all.empty();
    }
    if (!idle) return set_err(c, QQA_E_ARG, "a server is running or holds uncollected results");
    server_shutdown(c);
  }
  if (max_slots <= 0 || max_slots > 65536) return set_err(c, QQA_E_ARG, "max_slots must be in [1, 65536]");
  (void)hipSetDevice(c->device);
  auto sv = std::make_unique<Server>();
  sv->c = c;
  sv->device = c->device;
  sv->max_slots = max_slots;
  sv->budget = c->budget > c->in_use ? c->budget - c->in_use : 0;
  sv->layout = c->layout;
  sv->slots.assign(max_slots, nullptr);
  sv->h_slots.assign(max_slots, SlotDesc{});
  hipError_t e = hipStreamCreateWithFlags(&sv->st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc((void**)&sv->d_slots, (size_t)max_slots * sizeof(SlotDesc));
  if (e == hipSuccess) e = hipMalloc((void**)&sv->d_zero, 256);
  if (e == hipSuccess) e = hipMemset(sv->d_zero, 0, 256);
  if (e == hipSuccess) e = hipMemset(sv->d_slots, 0, (size_t)max_slots * sizeof(SlotDesc));
  if (e != hipSuccess) {
    if (sv->d_slots) (void)hipFree(sv->d_slots);
    if (sv->d_zero) (void)hipFree(sv->d_zero);
    if (sv->st) (void)hipStreamDestroy(sv->st);
    return set_err(c, QQA_E_DEVICE, std::string("serve_start: ") + hipGetErrorString(e));
  }
  Server* raw = sv.get();
  c->server = std::move(sv);
  raw->th = std::thread([raw] { raw->run(); });
  return QQA_OK;
}

int qqa_serve_submit(qqa_ctx* c, const qqa_graph* g, qqa_problem problem, const qqa_schedule* sched, int32_t S,
                     int32_t steps, uint64_t seed, qqa_req* out_id) {
  if (!c) return QQA_E_ARG;
  Server* sv = c->server.get();
  if (!sv) return set_err(c, QQA_E_ARG, "server not started");
  if (!g || !out_id) return set_err(c, QQA_E_ARG, "NULL argument");
  if (!known_problem(problem)) return set_err(c, QQA_E_ARG, "unknown problem");
  if (problem == QQA_MAXCLIQUE || problem == QQA_COLORING) return set_err(c, QQA_E_ARG, "max clique and coloring are solved one at a time");
  if (S <= 0 || S > kMaxReplicas || steps <= 0) return set_err(c, QQA_E_ARG, "need 1 <= S <= 4096 and steps > 0");
  if (g->dense) return set_err(c, QQA_E_ARG, "dense graphs are solved one at a time");
  std::string why;
  int rc = validate_graph(*g, problem, &why);
  if (rc) return set_err(c, rc, why);
  auto r = std::make_shared<ServerReq>();
  r->n = g->n;
  r->nnz = g->nnz;
  r->row_ptr.assign(g->row_ptr, g->row_ptr + g->n + 1);
  r->col.assign(g->col_idx, g->col_idx + g->nnz);
  if (problem == QQA_MAXCUT && g->weight) r->w.assign(g->weight, g->weight + g->nnz);
  r->problem = problem;
  r->S = S;
  r->K = steps;
  r->seed = seed;
  if (sched) r->sched = *sched; else qqa_schedule_default(&r->sched, problem, g->n);
  if (!schedule_valid(r->sched, &why)) return set_err(c, QQA_E_ARG, why);
  {
    std::vector<int32_t> rp(g->n + 1);
    for (int i = 0; i <= g->n; ++i) rp[i] = (int32_t)g->row_ptr[i];
    std::vector<HubChunk> chunks;
    std::vector<int32_t> first;
    build_hub_plan(rp.data(), g->n, &chunks, &first);
    r->nchunks = (int)chunks.size();
  }
  r->footprint = sv->footprint_of(*r);
  r->work = (double)r->n * qqa_replica_stride(S) * steps;
  r->rem_work = r->work;
  if (r->footprint > sv->budget) return set_err(c, QQA_E_ADMISSION, "request footprint exceeds the server's HBM budget");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->failed) return set_err(c, QQA_E_DEVICE, sv->fail_msg);
    if (sv->stopping) return set_err(c, QQA_E_ARG, "server is stopping");
    const auto now = Clock::now();
    ++sv->n_submitted;
    r->t_submit = now;
    double ms = 0.0;
    const char* why = "";
    if (sv->deadline_ms > 0.0 && !sv->meets_deadline(*r, now, &ms, &why)) {
      ++sv->n_shed;
      char buf[200];
      snprintf(buf, sizeof buf, "shed: admitting it would put %s past the %.0f ms deadline (its own: %.0f ms)", why,
               sv->deadline_ms, std::min(ms, 1e12));
      return set_err(c, QQA_E_ADMISSION, buf);
    }
    ++sv->n_admitted;
    sv->recent.emplace_back(now, r->work);
    r->id = sv->next_id++;
    sv->all.emplace(r->id, r);
    sv->queue.push_back(r);
  }
  sv->cv_work.notify_one();
  *out_id = r->id;
  return QQA_OK;
}

int qqa_serve_set_deadline(qqa_ctx* c, double deadline_ms) {
  if (!c) return QQA_E_ARG;
  Server* sv = c->server.get();
  if (!sv) return set_err(c, QQA_E_ARG, "server not started");
  if (!(deadline_ms >= 0.0)) return set_err(c, QQA_E_ARG, "deadline must be >= 0");
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->deadline_ms = deadline_ms;
  return QQA_OK;
}

int qqa_serve_get_stats(qqa_ctx* c, qqa_serve_stats* out) {
  if (!c || !out) return QQA_E_ARG;
  Server* sv = c->server.get();
  if (!sv) return set_err(c, QQA_E_ARG, "server not started");
  std::lock_guard<std::mutex> lk(sv->mu);
  out->submitted = sv->n_submitted;
  out->admitted = sv->n_admitted;
  out->shed = sv->n_shed;
  out->completed = sv->n_completed;
  out->rate_updates_per_s = sv->rate;
  out->deadline_ms = sv->deadline_ms;
  out->device_bytes_held = sv->dpool.held();
  out->device_bytes_cached = sv->dpool.cached();
  return QQA_OK;
}

int qqa_serve_stop(qqa_ctx* c) {
  if (!c) return QQA_E_ARG;
  if (!c->server) return QQA_OK;
  qqa::server_drain(c->server.get());
  return QQA_OK;
}

}  // extern "C"
