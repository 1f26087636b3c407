// Request-level API of include/qqa.h: contexts, resident graphs, plain solves, polling.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "qqa.h"
#include "qqa_ctx.h"
#include "qqa_internal.h"
#include "qqa_runtime.h"

using namespace qqa;
using Clock = std::chrono::steady_clock;

namespace qqa {

size_t request_footprint(int n, int S, int rule, int problem) {
  const size_t stride = (size_t)replica_shape(S).stride;
  // buffers as the pool rounds them
  const size_t state = Pool::class_size((size_t)n * stride * sizeof(float)) * (rule == QQA_STEP_ADAMW ? 4 : 2);
  const size_t sums = problem == QQA_MAXCLIQUE ? stride * sizeof(unsigned long long) : 0;
  return state + Pool::class_size(out_bytes(n, S)) + 2 * stride * sizeof(unsigned long long) + sums + 4096;
}

// result record: size_or_cut[S], viol[S], obj[S] (int64), best (int32) + pad, barrier
// words (2 x uint32), x[n] (uint8)
size_t out_bytes(int n, int S) { return 3 * (size_t)S * sizeof(int64_t) + 16 + (size_t)n; }

unsigned* out_bar(char* base, int S) { return reinterpret_cast<unsigned*>(base + 3 * (size_t)S * sizeof(int64_t) + 8); }

void out_views(char* base, int n, int S, int64_t** a, int64_t** b, int64_t** o, int32_t** best, uint8_t** x) {
  *a = reinterpret_cast<int64_t*>(base);
  *b = *a + S;
  *o = *b + S;
  *best = reinterpret_cast<int32_t*>(*o + S);
  *x = reinterpret_cast<uint8_t*>(base + 3 * (size_t)S * sizeof(int64_t) + 16);
  (void)n;
}

int upload_graph(qqa_ctx* c, const qqa_graph& g, int problem, DevGraph* out, std::string* why) {
  return upload_graph_on(c->stream, g, problem, out, why, true);
}

int upload_graph_on(hipStream_t stream, const qqa_graph& g, int problem, DevGraph* out, std::string* why,
                    bool validate) {
  if (validate) {
    int rc = validate_graph(g, problem, why);
    if (rc) return rc;
  }
  DevGraph d;
  d.n = g.n;
  d.problem = problem;
  auto dev_copy = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(dst, bytes ? bytes : 4);
    if (e != hipSuccess) return e;
    d.bytes += bytes;
    return bytes ? hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, stream) : hipSuccess;
  };
  hipError_t e = hipSuccess;
  if (g.dense) {
    d.nnz = (int64_t)g.n * g.n;
    e = dev_copy((void**)&d.dense, g.dense, (size_t)g.n * g.n * sizeof(float));
  } else {
    d.nnz = g.nnz;
    std::vector<int32_t> rp(g.n + 1);
    for (int i = 0; i <= g.n; ++i) rp[i] = (int32_t)g.row_ptr[i];
    e = dev_copy((void**)&d.row_ptr, rp.data(), rp.size() * sizeof(int32_t));
    if (e == hipSuccess) e = dev_copy((void**)&d.col, g.col_idx, (size_t)g.nnz * sizeof(int32_t));
    if (e == hipSuccess && problem == QQA_MAXCUT && g.weight)
      e = dev_copy((void**)&d.w, g.weight, (size_t)g.nnz * sizeof(float));
    std::vector<HubChunk> chunks;
    std::vector<int32_t> hub_first;
    build_hub_plan(rp.data(), g.n, &chunks, &hub_first);
    if (e == hipSuccess && !chunks.empty()) {
      d.nchunks = (int)chunks.size();
      e = dev_copy((void**)&d.chunks, chunks.data(), chunks.size() * sizeof(HubChunk));
      if (e == hipSuccess) e = dev_copy((void**)&d.hub_first, hub_first.data(), hub_first.size() * sizeof(int32_t));
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);  // host arrays may go away on return
  }
  if (e == hipSuccess && g.dense) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    free_graph(d);
    return fail(why, e == hipErrorOutOfMemory ? QQA_E_NOMEM : QQA_E_DEVICE,
                std::string("graph upload: ") + hipGetErrorString(e));
  }
  *out = d;
  return QQA_OK;
}

void free_graph(DevGraph& d) {
  if (d.row_ptr) (void)hipFree(d.row_ptr);
  if (d.col) (void)hipFree(d.col);
  if (d.w) (void)hipFree(d.w);
  if (d.dense) (void)hipFree(d.dense);
  if (d.chunks) (void)hipFree(d.chunks);
  if (d.hub_first) (void)hipFree(d.hub_first);
  d = DevGraph{};
}

void graph_unref(qqa_ctx* c, int64_t gid) {
  auto it = c->graphs.find(gid);
  if (it == c->graphs.end()) return;
  if (--it->second.refs <= 0 && it->second.release_pending) {
    c->in_use -= it->second.bytes;
    free_graph(it->second);
    c->graphs.erase(it);
  }
}

// Idle pooled buffers count against the budget: when they would crowd out a new request,
// they are freed first (hipFree waits for the device).
bool budget_fits(qqa_ctx* c, size_t bytes) {
  if (c->in_use + c->dpool.cached() + bytes > c->budget) c->dpool.trim();
  return c->in_use + bytes <= c->budget;
}

int alloc_request_buffers(qqa_ctx* c, Request* r, std::string* why, int nchunks) {
  const size_t state = (size_t)r->n * std::max(1, r->colors) * r->shape.stride * sizeof(float);
  const bool adam = r->sched.rule == QQA_STEP_ADAMW;
  hipError_t e = hipSuccess;
  auto get = [&](void** p, size_t b) {
    if (e == hipSuccess) e = c->dpool.get(b, p);
  };
  get((void**)&r->P[0], state);
  get((void**)&r->P[1], state);
  if (adam) {
    get((void**)&r->m, state);
    get((void**)&r->v, state);
  }
  get((void**)&r->acc, 2 * (size_t)r->shape.stride * sizeof(unsigned long long));
  r->hub_bytes = (size_t)nchunks * r->shape.stride * sizeof(float);
  if (nchunks) get((void**)&r->hub_partial, r->hub_bytes);
  if (r->problem == QQA_MAXCLIQUE) get((void**)&r->colsum, (size_t)r->shape.stride * sizeof(unsigned long long));
  if (r->engine == kEngineSliced) get((void**)&r->stats, 2 * (size_t)r->n * kReplicaSlices * sizeof(float2));
  if (r->engine == kEngineCompact) get((void**)&r->compact, 4 * (size_t)r->n * sizeof(float));
  if (r->colors > 0) {
    get((void**)&r->cat_sigma, state);
    get((void**)&r->cat_grad, state);
    get((void**)&r->cat_colors, (size_t)r->n * r->shape.stride);
  }
  r->coupling_bytes = 0;
  auto git = c->graphs.find(r->graph);
  if (git != c->graphs.end() && git->second.dense) {
    // the product's split-K parts (one part when the k range is not split)
    r->coupling_bytes = (size_t)dense_splits(r->n, r->shape.stride) * state;
    get((void**)&r->coupling, r->coupling_bytes);
  }
  r->out_size = out_bytes(r->n, r->S);
  get((void**)&r->out_dev, r->out_size);
  if (e == hipSuccess) e = c->hpool.get(r->out_size, (void**)&r->out_host);
  for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&r->ev[i]);
  if ((r->engine == kEngineStream || r->engine == kEngineSliced || r->engine == kEngineCompact) && r->K > 0) {
    // sampled updates t with t % every == every / 2, at most kProbes of them
    r->probe_every = std::max(1, (r->K + kProbes - 1) / kProbes);
    const int samples = (r->K - r->probe_every / 2 + r->probe_every - 1) / r->probe_every;
    r->probe.assign(2 * (size_t)samples, nullptr);
    for (size_t i = 0; i < r->probe.size() && e == hipSuccess; ++i) e = hipEventCreate(&r->probe[i]);
  }
  if (e != hipSuccess) {
    release_request_buffers(c, r);
    return fail(why, e == hipErrorOutOfMemory ? QQA_E_NOMEM : QQA_E_DEVICE,
                std::string("request buffers: ") + hipGetErrorString(e));
  }
  return QQA_OK;
}

void release_request_buffers(qqa_ctx* c, Request* r) {
  if (r->owner) {
    for (int i = 0; i < 4; ++i) r->ev[i] = nullptr;
    r->out_dev = r->out_host = nullptr;
    r->owner.reset();
    return;
  }
  const size_t state = (size_t)r->n * std::max(1, r->colors) * r->shape.stride * sizeof(float);
  c->dpool.put(r->P[0], state);
  c->dpool.put(r->P[1], state);
  c->dpool.put(r->m, state);
  c->dpool.put(r->v, state);
  c->dpool.put(r->acc, 2 * (size_t)r->shape.stride * sizeof(unsigned long long));
  c->dpool.put(r->hub_partial, r->hub_bytes);
  r->hub_partial = nullptr;
  c->dpool.put(r->coupling, r->coupling_bytes);
  r->coupling = nullptr;
  if (r->colsum) c->dpool.put(r->colsum, (size_t)r->shape.stride * sizeof(unsigned long long));
  r->colsum = nullptr;
  if (r->stats) c->dpool.put(r->stats, 2 * (size_t)r->n * kReplicaSlices * sizeof(float2));
  r->stats = nullptr;
  if (r->compact) c->dpool.put(r->compact, 4 * (size_t)r->n * sizeof(float));
  r->compact = nullptr;
  if (r->cat_sigma) c->dpool.put(r->cat_sigma, state);
  if (r->cat_grad) c->dpool.put(r->cat_grad, state);
  if (r->cat_colors) c->dpool.put(r->cat_colors, (size_t)r->n * r->shape.stride);
  r->cat_sigma = r->cat_grad = nullptr;
  r->cat_colors = nullptr;
  c->dpool.put(r->out_dev, r->out_size);
  c->hpool.put(r->out_host, r->out_size);
  c->dpool.put(r->table_dev, r->table_bytes);
  c->hpool.put(r->table_host, r->table_bytes);
  r->table_dev = nullptr;
  r->table_host = nullptr;
  c->dpool.put(r->noise_dev, r->noise_bytes);
  r->noise_dev = nullptr;
  r->P[0] = r->P[1] = r->m = r->v = nullptr;
  r->acc = nullptr;
  r->out_dev = r->out_host = nullptr;
  for (int i = 0; i < 4; ++i)
    if (r->ev[i]) {
      (void)hipEventDestroy(r->ev[i]);
      r->ev[i] = nullptr;
    }
  for (hipEvent_t& ev : r->probe)
    if (ev) (void)hipEventDestroy(ev);
  r->probe.clear();
}

StepParams request_step_params(const Request* r, const DevGraph& g) {
  StepParams p{};
  p.row_ptr = g.row_ptr;
  p.col = g.col;
  p.w = r->problem == QQA_MAXCUT ? g.w : nullptr;
  p.hub_first = g.hub_first;
  p.hub_partial = r->hub_partial;
  p.colsum = r->colsum;
  p.coupling = g.dense ? r->coupling : nullptr;
  p.coupling_parts = g.dense ? dense_splits(r->n, r->shape.stride) : 0;
  p.m = r->m;
  p.v = r->v;
  p.n = r->n;
  fill_static_scalars(p, r->sched, r->problem, r->S, r->seed);
  p.lanes_per_row = r->lanes_per_row;
  return p;
}

// Enqueue rounding, exact evaluation, best-x extraction and the copy of the result
// record into pinned host memory; `final_P` is the state after the last update.
hipError_t enqueue_finish(qqa_ctx* c, Request* r, const DevGraph& g, const float* final_P) {
  int64_t *a, *b, *o;
  int32_t* best;
  uint8_t* x;
  out_views(r->out_dev, r->n, r->S, &a, &b, &o, &best, &x);
  EvalParams ep{};
  ep.row_ptr = g.row_ptr;
  ep.col = g.col;
  ep.w = r->problem == QQA_MAXCUT ? g.w : nullptr;
  ep.dense = g.dense;
  ep.P = final_P;
  ep.n = r->n;
  ep.S = r->S;
  ep.stride = r->shape.stride;
  ep.problem = r->problem;
  ep.lambda = r->sched.penalty_lambda;
  ep.acc = r->acc;
  ep.size_or_cut = a;
  ep.viol = b;
  ep.obj = o;
  ep.best = best;
  hipError_t e = launch_eval(ep, c->stream);
  if (e == hipSuccess) e = launch_extract(final_P, r->n, r->shape.stride, best, x, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(r->out_host, r->out_dev, r->out_size, hipMemcpyDeviceToHost, c->stream);
  return e;
}

int set_err(qqa_ctx* c, int code, const std::string& msg) {
  c->err = msg;
  return code;
}

}  // namespace qqa

// ---------------------------------------------------------------------------------------
// plain solve: init, K update launches, finish -- all enqueued on the context stream
// ---------------------------------------------------------------------------------------
static int submit_plain(qqa_ctx* c, int64_t gid, bool temp, qqa_problem problem, const qqa_schedule* sched, int32_t S,
                        int32_t steps, uint64_t seed, qqa_req* out_id) {
  auto git = c->graphs.find(gid);
  if (git == c->graphs.end()) return set_err(c, QQA_E_ARG, "unknown graph id");
  DevGraph& g = git->second;
  if (g.problem != problem) return set_err(c, QQA_E_ARG, "graph was uploaded for another problem type");
  auto r = std::make_unique<Request>();
  r->id = c->next_req++;
  r->graph = gid;
  r->temp_graph = temp;
  r->problem = problem;
  if (sched) r->sched = *sched; else qqa_schedule_default(&r->sched, problem, g.n);
  std::string why;
  if (!schedule_valid(r->sched, &why)) return set_err(c, QQA_E_ARG, why);
  r->S = S;
  r->K = steps;
  r->seed = seed;
  r->n = g.n;
  r->shape = replica_shape(S);
  r->lanes_per_row = c->layout_for(S);
  r->footprint = request_footprint(g.n, S, r->sched.rule, problem) + (size_t)g.nchunks * r->shape.stride * sizeof(float) +
                 (g.dense ? (size_t)dense_splits(g.n, r->shape.stride) * g.n * r->shape.stride * sizeof(float) : 0);
  if (r->footprint + g.bytes > c->budget) return set_err(c, QQA_E_ADMISSION, "request footprint exceeds the HBM budget");
  {
    StepParams probe = request_step_params(r.get(), g);
    // auto: one workgroup with P in LDS when the instance fits, else one launch per update
    // (measured faster on this GPU than the register-resident engine for larger instances).
    // Dense graphs and max clique always stream: the coupling product (matrix cores) and
    // the per-replica sums are separate launches before every update, which no
    // persistent engine performs.
    const int allow = g.dense || problem == QQA_MAXCLIQUE ? 0 : c->engine_policy < 0 ? 1 : (c->engine_policy == QQA_ENGINE_LDS_BLOCK ? 1 :
                                                 (c->engine_policy == QQA_ENGINE_PERSISTENT ? 2 : 0));
    r->engine = allow ? persistent_plan(probe, g.nchunks > 0, allow, &r->rows_per_group, &r->grid) : kEngineStream;
    // one replica per variable: compact state (asked for, or by default)
    if (r->engine == kEngineStream && !g.dense && S == 1 && problem != QQA_MAXCLIQUE &&
        (c->engine_policy == QQA_ENGINE_COMPACT || c->engine_policy < 0)) {
      r->engine = kEngineCompact;
      r->footprint += 4 * (size_t)g.n * sizeof(float);
    }
    // a streaming sparse solve runs sliced when asked for, or by default when its slices
    // are whole cache lines and fit the XCDs' L2 (further when its state can be slice-major)
    StepParams shape{};
    shape.S = S;
    shape.stride = r->shape.stride;
    shape.problem = problem;
    const bool sm = slice_major_ok(shape);
    if (r->engine == kEngineStream && !g.dense && slice_shape(S).sq > 0 &&
        (c->engine_policy == QQA_ENGINE_SLICED || (c->engine_policy < 0 && slice_by_default(g.n, S, sm)))) {
      r->engine = kEngineSliced;
      r->footprint += 2 * (size_t)g.n * kReplicaSlices * sizeof(float2);
    }
    if (r->engine == kEnginePersistent || r->engine == kEngineLdsBlock) {
      r->table_bytes = (size_t)steps * sizeof(float4);
      r->footprint += r->table_bytes;
    }
    // one workgroup cannot hide the generator's dependent chain behind other rows: its
    // normals are formed beforehand by the whole GPU, a bounded chunk of updates at a time
    if (r->engine == kEngineLdsBlock && steps > 0) {
      const size_t per_update = (size_t)g.n * (r->shape.stride / 4) * sizeof(float4);
      r->noise_chunk = (int)std::min<size_t>((size_t)steps, std::max<size_t>(1, kNoiseTableMaxBytes / per_update));
      r->noise_bytes = per_update * (size_t)r->noise_chunk;
      r->footprint += r->noise_bytes;
    }
  }
  if (!budget_fits(c, r->footprint))
    return set_err(c, QQA_E_NOMEM, "HBM budget held by earlier requests; poll them first");
  int rc = alloc_request_buffers(c, r.get(), &c->err, g.nchunks);
  if (rc) return rc;
  hipError_t e = hipSuccess;
  if (r->table_bytes) {
    e = c->dpool.get(r->table_bytes, (void**)&r->table_dev);
    if (e == hipSuccess) e = c->hpool.get(r->table_bytes, (void**)&r->table_host);
    if (e == hipSuccess && r->noise_bytes) e = c->dpool.get(r->noise_bytes, (void**)&r->noise_dev);
    if (e != hipSuccess) {
      release_request_buffers(c, r.get());
      return set_err(c, QQA_E_NOMEM, std::string("request buffers: ") + hipGetErrorString(e));
    }
    StepParams q{};
    for (int t = 0; t < steps; ++t) {
      fill_step_scalars(q, r->sched, t, steps);
      r->table_host[t] = make_float4(q.ce, q.inv_bc1, q.inv_bc2, 0.f);
    }
  }
  c->in_use += r->footprint;
  g.refs++;
  r->t_submit = Clock::now();

  e = hipEventRecord(r->ev[0], c->stream);
  if (e == hipSuccess) e = launch_init(seed, g.n, S, r->P[0], r->m, r->v, c->stream);
  if (e == hipSuccess) e = hipEventRecord(r->ev[1], c->stream);
  StepParams p = request_step_params(r.get(), g);
  if (r->engine == kEngineCompact) {
    const size_t n = (size_t)g.n;
    float* Pc[2] = {r->compact, r->compact + n};
    float* mc = r->compact + 2 * n;
    float* vc = r->compact + 3 * n;
    const int stride = r->shape.stride;
    if (e == hipSuccess) e = launch_compact_pack(r->P[0], stride, g.n, Pc[0], c->stream);
    if (r->m && e == hipSuccess) e = launch_compact_pack(r->m, stride, g.n, mc, c->stream);  // AdamW only
    if (r->v && e == hipSuccess) e = launch_compact_pack(r->v, stride, g.n, vc, c->stream);
    const int every = r->probe_every;
    for (int t = 0; t < steps && e == hipSuccess; ++t) {
      fill_step_scalars(p, r->sched, t, steps);
      const size_t pi = 2 * (size_t)(t / every);
      const bool probe = t % every == every / 2 && pi + 1 < r->probe.size();
      if (probe) e = hipEventRecord(r->probe[pi], c->stream);
      if (e == hipSuccess) e = launch_compact_step(p, Pc[t & 1], Pc[(t + 1) & 1], mc, vc, c->stream);
      if (probe && e == hipSuccess) e = hipEventRecord(r->probe[pi + 1], c->stream);
    }
    // the final state in the padded layout, for the exact evaluation
    if (e == hipSuccess) e = launch_compact_unpack(Pc[steps & 1], g.n, stride, r->P[steps & 1], c->stream);
  } else if (r->engine == kEngineStream || r->engine == kEngineSliced) {
    const bool sliced = r->engine == kEngineSliced;
    float2* part[2] = {r->stats, r->stats + (size_t)g.n * kReplicaSlices};
    // the sliced engine keeps the state slice-major where it can (each XCD's slice of P, m and
    // v contiguous): P starts in P[1] and the loop's ping-pong begins there; m and v start at
    // zero, and only P is converted back, for the evaluation
    const bool sm = sliced && slice_major_ok(p);
    float* Ps[2] = {r->P[0], r->P[1]};
    if (sm) {
      std::swap(Ps[0], Ps[1]);
      if (e == hipSuccess) e = launch_slice_permute(r->P[0], Ps[0], g.n, S, true, c->stream);
    }
    if (sliced && e == hipSuccess) {
      p.P_in = Ps[0];
      e = launch_slice_stats(p, part[0], c->stream, sm);
    }
    const int every = r->probe_every;
    for (int t = 0; t < steps && e == hipSuccess; ++t) {
      p.P_in = Ps[t & 1];
      p.P_out = Ps[(t + 1) & 1];
      fill_step_scalars(p, r->sched, t, steps);
      if (r->colsum) {
        p.colsum = r->colsum;
        e = launch_colsum(p.P_in, g.n, p.stride, r->colsum, c->stream);
        if (e != hipSuccess) break;
      }
      const size_t pi = 2 * (size_t)(t / every);
      const bool probe = t % every == every / 2 && pi + 1 < r->probe.size();
      if (g.dense) {
        if (probe) e = hipEventRecord(r->probe[pi], c->stream);
        if (e == hipSuccess) e = launch_dense_parts(g.dense, p.P_in, r->coupling, g.n, p.stride, problem, c->stream);
        if (probe && e == hipSuccess) e = hipEventRecord(r->probe[pi + 1], c->stream);
      }
      if (g.nchunks && e == hipSuccess)
        e = sm ? launch_slice_hub_partials(p, g.chunks, g.nchunks, c->stream)
               : launch_hub_partials(p, g.chunks, g.nchunks, c->stream);
      if (!g.dense && probe && e == hipSuccess) e = hipEventRecord(r->probe[pi], c->stream);
      if (sliced) {
        if (e == hipSuccess) e = launch_slice_step(p, part[t & 1], part[(t + 1) & 1], c->stream, sm, g.nchunks);
      } else if (e == hipSuccess) {
        e = launch_step(p, c->stream);
      }
      if (!g.dense && probe && e == hipSuccess) e = hipEventRecord(r->probe[pi + 1], c->stream);
    }
    // the final P, row-major, in the buffer the evaluation reads (P[steps & 1])
    if (sm && e == hipSuccess) e = launch_slice_permute(Ps[steps & 1], r->P[steps & 1], g.n, S, false, c->stream);
  } else {
    unsigned* bar = out_bar(r->out_dev, S);
    if (e == hipSuccess)
      e = hipMemcpyAsync(r->table_dev, r->table_host, r->table_bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_fill_u64(reinterpret_cast<unsigned long long*>(bar), 1, c->stream);
    PersistParams pp{};
    pp.a = p;
    pp.P[0] = r->P[0];
    pp.P[1] = r->P[1];
    pp.table = r->table_dev;
    pp.t0 = 0;
    pp.t1 = steps;
    pp.bar = bar;
    if (r->engine == kEngineLdsBlock) {
      // LDS block: each chunk's normals, then the chunk's updates (P and the moments pass
      // through global memory between chunks)
      pp.noise = r->noise_dev;
      pp.nnz = g.nnz <= INT32_MAX ? (int32_t)g.nnz : 0;
      for (int t0 = 0; t0 < steps && e == hipSuccess; t0 += r->noise_chunk) {
        pp.t0 = t0;
        pp.t1 = std::min(steps, t0 + r->noise_chunk);
        e = launch_noise_table(p, pp.t0, pp.t1, r->noise_dev, c->stream);
        if (e == hipSuccess) e = launch_persistent(pp, r->engine, r->rows_per_group, r->grid, c->stream);
      }
    } else if (e == hipSuccess) {
      e = launch_persistent(pp, r->engine, r->rows_per_group, r->grid, c->stream);
    }
  }
  if (e == hipSuccess) e = hipEventRecord(r->ev[2], c->stream);
  if (e == hipSuccess) e = enqueue_finish(c, r.get(), g, r->P[steps & 1]);
  if (e == hipSuccess) e = hipEventRecord(r->ev[3], c->stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(c->stream);
    release_request_buffers(c, r.get());
    c->in_use -= r->footprint;
    graph_unref(c, gid);
    return set_err(c, QQA_E_DEVICE, std::string("enqueue: ") + hipGetErrorString(e));
  }
  r->state = Request::kRunning;
  *out_id = r->id;
  c->reqs.emplace(r->id, std::move(r));
  return QQA_OK;
}

// ---------------------------------------------------------------------------------------
// graph coloring (categorical K-state variant): init, sigma, K x (gradient, update), finish
// ---------------------------------------------------------------------------------------
static double gamma_at(const qqa_schedule& s, int t, int K) {
  if (K <= 1) return s.gamma_min;
  return (double)s.gamma_min + ((double)s.gamma_max - (double)s.gamma_min) * (double)t / (double)(K - 1);
}

static int submit_coloring(qqa_ctx* c, int64_t gid, bool temp, int32_t colors, const qqa_schedule* sched, int32_t S,
                           int32_t steps, uint64_t seed, qqa_req* out_id) {
  auto git = c->graphs.find(gid);
  if (git == c->graphs.end()) return set_err(c, QQA_E_ARG, "unknown graph id");
  DevGraph& g = git->second;
  if (g.problem != QQA_COLORING) return set_err(c, QQA_E_ARG, "graph was uploaded for another problem type");
  auto r = std::make_unique<Request>();
  r->id = c->next_req++;
  r->graph = gid;
  r->temp_graph = temp;
  r->problem = QQA_COLORING;
  r->colors = colors;
  if (sched) r->sched = *sched; else qqa_schedule_default(&r->sched, QQA_COLORING, g.n);
  std::string why;
  if (!schedule_valid(r->sched, &why)) return set_err(c, QQA_E_ARG, why);
  r->S = S;
  r->K = steps;
  r->seed = seed;
  r->n = g.n;
  r->shape = replica_shape(S);
  r->lanes_per_row = c->layout_for(S);
  r->engine = kEngineStream;
  const size_t stride = r->shape.stride;
  const size_t state = (size_t)g.n * colors * stride * sizeof(float);
  r->footprint = state * (r->sched.rule == QQA_STEP_ADAMW ? 6 : 4) + (size_t)g.n * stride + out_bytes(g.n, S) +
                 2 * stride * sizeof(unsigned long long) + 4096;
  if (r->footprint + g.bytes > c->budget) return set_err(c, QQA_E_ADMISSION, "request footprint exceeds the HBM budget");
  if (!budget_fits(c, r->footprint))
    return set_err(c, QQA_E_NOMEM, "HBM budget held by earlier requests; poll them first");
  int rc = alloc_request_buffers(c, r.get(), &c->err, 0);
  if (rc) return rc;
  c->in_use += r->footprint;
  g.refs++;
  r->t_submit = Clock::now();

  // the colour-k gradient uses the categorical entropy's coefficient c = 1/((K-1)((K-1)^(a-1)+1))
  const int a_e = r->sched.entropy_alpha;
  const double cK = 1.0 / ((double)(colors - 1) * (std::pow((double)(colors - 1), a_e - 1) + 1.0));
  StepParams base = request_step_params(r.get(), g);
  base.w = nullptr;
  hipError_t e = hipEventRecord(r->ev[0], c->stream);
  if (e == hipSuccess) e = launch_init(seed, g.n * colors, S, r->P[0], r->m, r->v, c->stream);
  if (e == hipSuccess) e = launch_cat_sigma(r->P[0], r->cat_sigma, g.n, colors, (int)stride, S, c->stream);
  if (e == hipSuccess) e = hipEventRecord(r->ev[1], c->stream);
  const int every = r->probe_every;
  // small shapes: gradient and update in one launch, sigma ping-ponging between the two
  // state-sized buffers (the gradient buffer is then not needed)
  const bool fused = c->engine_policy < 0 && cat_fused_shape(S, r->lanes_per_row, colors);
  float* sig[2] = {r->cat_sigma, r->cat_grad};
  for (int t = 0; t < steps && e == hipSuccess; ++t) {
    StepParams pg = base;
    pg.n = g.n * colors;
    pg.P_in = r->cat_sigma;
    pg.ce = (float)(-gamma_at(r->sched, t, steps) * cK * (double)a_e * (double)colors);
    StepParams pu = base;
    pu.P_in = r->P[t & 1];
    pu.P_out = r->P[(t + 1) & 1];
    fill_step_scalars(pu, r->sched, t, steps);
    const size_t pi = 2 * (size_t)(t / every);
    const bool probe = t % every == every / 2 && pi + 1 < r->probe.size();
    if (probe) e = hipEventRecord(r->probe[pi], c->stream);
    if (fused) {
      if (e == hipSuccess) e = launch_cat_fused(pu, colors, pg.ce, sig[t & 1], sig[(t + 1) & 1], g.nnz, c->stream);
      if (probe && e == hipSuccess) e = hipEventRecord(r->probe[pi + 1], c->stream);
      continue;
    }
    if (e == hipSuccess) e = launch_cat_grad(pg, colors, r->cat_grad, c->stream);
    if (probe && e == hipSuccess) e = hipEventRecord(r->probe[pi + 1], c->stream);
    if (e == hipSuccess) e = launch_cat_update(pu, colors, r->cat_grad, r->cat_sigma, c->stream);
  }
  if (e == hipSuccess) e = hipEventRecord(r->ev[2], c->stream);
  if (e == hipSuccess) {
    int64_t *a, *b, *o;
    int32_t* best;
    uint8_t* x;
    out_views(r->out_dev, r->n, r->S, &a, &b, &o, &best, &x);
    e = launch_cat_eval(g.row_ptr, g.col, r->P[steps & 1], r->cat_colors, g.n, colors, (int)stride, S, r->acc,
                        c->stream);
    EvalParams ep{};
    ep.n = g.n;
    ep.S = S;
    ep.stride = (int)stride;
    ep.problem = QQA_COLORING;
    ep.acc = r->acc;
    ep.size_or_cut = a;
    ep.viol = b;
    ep.obj = o;
    ep.best = best;
    if (e == hipSuccess) e = launch_finalize(ep, c->stream);
    if (e == hipSuccess) e = launch_cat_extract(r->cat_colors, g.n, (int)stride, best, x, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->out_host, r->out_dev, r->out_size, hipMemcpyDeviceToHost, c->stream);
  }
  if (e == hipSuccess) e = hipEventRecord(r->ev[3], c->stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(c->stream);
    release_request_buffers(c, r.get());
    c->in_use -= r->footprint;
    graph_unref(c, gid);
    return set_err(c, QQA_E_DEVICE, std::string("enqueue: ") + hipGetErrorString(e));
  }
  r->state = Request::kRunning;
  *out_id = r->id;
  c->reqs.emplace(r->id, std::move(r));
  return QQA_OK;
}

static int check_coloring_args(qqa_ctx* c, int32_t colors, int32_t S, int32_t steps, qqa_req* out_id) {
  if (!out_id) return set_err(c, QQA_E_ARG, "out_id is NULL");
  if (colors < 2 || colors > 255) return set_err(c, QQA_E_ARG, "colours must be in [2, 255]");
  if (S <= 0 || S > kMaxReplicas) return set_err(c, QQA_E_ARG, "S must be in [1, 4096]");
  if (steps <= 0) return set_err(c, QQA_E_ARG, "steps must be positive");
  return QQA_OK;
}

extern "C" {

int qqa_create(qqa_ctx** out, int device, size_t hbm_budget_bytes, void* hip_stream) {
  if (!out) return QQA_E_ARG;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return QQA_E_DEVICE;
  auto c = std::make_unique<qqa_ctx>();
  c->device = device;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
    c->own_stream = false;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return QQA_E_DEVICE;
    c->own_stream = true;
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return QQA_E_DEVICE;
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
  *out = c.release();
  return QQA_OK;
}

void qqa_destroy(qqa_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  server_shutdown(c);
  (void)hipStreamSynchronize(c->stream);
  for (auto& kv : c->reqs) release_request_buffers(c, kv.second.get());
  c->reqs.clear();
  for (auto& kv : c->graphs) free_graph(kv.second);
  c->graphs.clear();
  c->dpool.trim();
  c->hpool.trim();
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* qqa_last_error(const qqa_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

int qqa_graph_upload(qqa_ctx* c, const qqa_graph* g, qqa_problem problem, qqa_graph_id* out) {
  if (!c || !g || !out) return c ? set_err(c, QQA_E_ARG, "NULL argument") : QQA_E_ARG;
  if (!known_problem(problem)) return set_err(c, QQA_E_ARG, "unknown problem");
  (void)hipSetDevice(c->device);
  DevGraph d;
  int rc = upload_graph(c, *g, problem, &d, &c->err);
  if (rc) return rc;
  c->in_use += d.bytes;
  const int64_t id = c->next_graph++;
  c->graphs.emplace(id, d);
  *out = id;
  return QQA_OK;
}

int qqa_graph_release(qqa_ctx* c, qqa_graph_id id) {
  if (!c) return QQA_E_ARG;
  auto it = c->graphs.find(id);
  if (it == c->graphs.end() || it->second.release_pending) return set_err(c, QQA_E_ARG, "unknown graph id");
  it->second.release_pending = true;
  if (it->second.refs == 0) {
    c->in_use -= it->second.bytes;
    free_graph(it->second);
    c->graphs.erase(it);
  }
  return QQA_OK;
}

static int check_solve_args(qqa_ctx* c, qqa_problem problem, int32_t S, int32_t steps, qqa_req* out_id) {
  if (!out_id) return set_err(c, QQA_E_ARG, "out_id is NULL");
  if (!known_problem(problem)) return set_err(c, QQA_E_ARG, "unknown problem");
  if (problem == QQA_COLORING) return set_err(c, QQA_E_ARG, "graph coloring needs the colour count: qqa_solve_coloring");
  if (S <= 0 || S > kMaxReplicas) return set_err(c, QQA_E_ARG, "S must be in [1, 4096]");
  if (steps <= 0) return set_err(c, QQA_E_ARG, "steps must be positive");
  return QQA_OK;
}

int qqa_solve(qqa_ctx* c, const qqa_graph* g, qqa_problem problem, const qqa_schedule* sched, int32_t S, int32_t steps,
              uint64_t seed, qqa_req* out_id) {
  if (!c) return QQA_E_ARG;
  if (!g) return set_err(c, QQA_E_ARG, "graph is NULL");
  int rc = check_solve_args(c, problem, S, steps, out_id);
  if (rc) return rc;
  qqa_graph_id gid;
  rc = qqa_graph_upload(c, g, problem, &gid);
  if (rc) return rc;
  rc = submit_plain(c, gid, true, problem, sched, S, steps, seed, out_id);
  qqa_graph_release(c, gid);  // freed when the request is collected
  return rc;
}

int qqa_solve_coloring(qqa_ctx* c, const qqa_graph* g, int32_t colors, const qqa_schedule* sched, int32_t S,
                       int32_t steps, uint64_t seed, qqa_req* out_id) {
  if (!c) return QQA_E_ARG;
  if (!g) return set_err(c, QQA_E_ARG, "graph is NULL");
  int rc = check_coloring_args(c, colors, S, steps, out_id);
  if (rc) return rc;
  qqa_graph_id gid;
  rc = qqa_graph_upload(c, g, QQA_COLORING, &gid);
  if (rc) return rc;
  rc = submit_coloring(c, gid, true, colors, sched, S, steps, seed, out_id);
  qqa_graph_release(c, gid);  // freed when the request is collected
  return rc;
}

int qqa_solve_coloring_resident(qqa_ctx* c, qqa_graph_id g, int32_t colors, const qqa_schedule* sched, int32_t S,
                                int32_t steps, uint64_t seed, qqa_req* out_id) {
  if (!c) return QQA_E_ARG;
  int rc = check_coloring_args(c, colors, S, steps, out_id);
  if (rc) return rc;
  (void)hipSetDevice(c->device);
  return submit_coloring(c, g, false, colors, sched, S, steps, seed, out_id);
}

int qqa_solve_resident(qqa_ctx* c, qqa_graph_id g, qqa_problem problem, const qqa_schedule* sched, int32_t S,
                       int32_t steps, uint64_t seed, qqa_req* out_id) {
  if (!c) return QQA_E_ARG;
  int rc = check_solve_args(c, problem, S, steps, out_id);
  if (rc) return rc;
  (void)hipSetDevice(c->device);
  return submit_plain(c, g, false, problem, sched, S, steps, seed, out_id);
}

int qqa_set_engine(qqa_ctx* c, qqa_engine policy) {
  if (!c) return QQA_E_ARG;
  if (policy < QQA_ENGINE_AUTO || policy > QQA_ENGINE_COMPACT || policy == QQA_ENGINE_BATCH)
    return set_err(c, QQA_E_ARG, "unknown engine policy");
  c->engine_policy = policy;
  return QQA_OK;
}

int qqa_set_replica_layout(qqa_ctx* c, int32_t S, int32_t lanes_per_row) {
  if (!c) return QQA_E_ARG;
  if (S <= 0 || S > kMaxReplicas) return set_err(c, QQA_E_ARG, "S must be in [1, 4096]");
  if (lanes_per_row < 0 || lanes_per_row > 64 || !layout_supported(S, lanes_per_row))
    return set_err(c, QQA_E_ARG, "unsupported replica layout");
  if (lanes_per_row == 0) c->layout.erase(S);
  else c->layout[S] = replica_shape(S, lanes_per_row).lpr;
  return QQA_OK;
}

int qqa_autotune(qqa_ctx* c, qqa_graph_id gid, qqa_problem problem, int32_t S, int32_t* lanes_per_row) {
  if (!c) return QQA_E_ARG;
  auto git = c->graphs.find(gid);
  if (git == c->graphs.end()) return set_err(c, QQA_E_ARG, "unknown graph id");
  if (S <= 0 || S > kMaxReplicas) return set_err(c, QQA_E_ARG, "S must be in [1, 4096]");
  const DevGraph& g = git->second;
  if (g.dense) return set_err(c, QQA_E_ARG, "the dense path has no replica layout to tune");
  (void)hipSetDevice(c->device);
  Request r;
  r.problem = problem;
  qqa_schedule_default(&r.sched, problem, g.n);
  r.S = S;
  r.n = g.n;
  r.shape = replica_shape(S);
  // one replica per variable: time the compact engine, which the context then runs
  const bool compact = S == 1 && problem != QQA_MAXCLIQUE &&
                       (c->engine_policy < 0 || c->engine_policy == QQA_ENGINE_COMPACT);
  if (compact) r.engine = kEngineCompact;
  const size_t fp = request_footprint(g.n, S, r.sched.rule, problem) + (size_t)g.nchunks * r.shape.stride * sizeof(float) +
                    (compact ? 4 * (size_t)g.n * sizeof(float) : 0);
  if (!budget_fits(c, fp)) return set_err(c, QQA_E_NOMEM, "no budget left for tuning state");
  int rc = alloc_request_buffers(c, &r, &c->err, g.nchunks);
  if (rc) return rc;
  const int warm = 3, timed = 12;
  int best = 0;
  float best_ms = 1e30f;
  {
    // an instance that one workgroup runs with P in LDS keeps the default layout: that
    // engine is faster than any streaming layout and runs only whole-row layouts
    r.lanes_per_row = replica_shape(S).lpr;
    StepParams probe = request_step_params(&r, g);
    int rpg = 0, grid = 0;
    if (problem != QQA_MAXCLIQUE && persistent_plan(probe, g.nchunks > 0, 1, &rpg, &grid) == kEngineLdsBlock) {
      release_request_buffers(c, &r);
      c->layout[S] = 0;
      if (lanes_per_row) *lanes_per_row = replica_shape(S).lpr;
      return QQA_OK;
    }
  }
  hipError_t e = launch_init(1, g.n, S, r.P[0], r.m, r.v, c->stream);
  // max clique: valid per-replica sums for the timed updates (their values do not matter)
  if (e == hipSuccess && r.colsum) e = launch_colsum(r.P[0], g.n, r.shape.stride, r.colsum, c->stream);
  const size_t n = (size_t)g.n;
  float* Pc[2] = {r.compact, r.compact ? r.compact + n : nullptr};
  if (compact && e == hipSuccess) e = launch_compact_pack(r.P[0], r.shape.stride, g.n, Pc[0], c->stream);
  if (compact && r.m && e == hipSuccess) e = launch_compact_pack(r.m, r.shape.stride, g.n, r.compact + 2 * n, c->stream);
  if (compact && r.v && e == hipSuccess) e = launch_compact_pack(r.v, r.shape.stride, g.n, r.compact + 3 * n, c->stream);
  int last_lpr = -1;
  for (int want = 1; want <= 64 && e == hipSuccess; want <<= 1) {
    const ReplicaShape sh = replica_shape(S, want);
    if (sh.lpr == last_lpr || !layout_supported(S, want)) continue;
    last_lpr = sh.lpr;
    r.lanes_per_row = sh.lpr;
    StepParams p = request_step_params(&r, g);
    for (int t = 0; t < warm + timed && e == hipSuccess; ++t) {
      if (t == warm) e = hipEventRecord(r.ev[1], c->stream);
      p.P_in = r.P[t & 1];
      p.P_out = r.P[(t + 1) & 1];
      fill_step_scalars(p, r.sched, t, warm + timed);
      if (compact) {
        e = launch_compact_step(p, Pc[t & 1], Pc[(t + 1) & 1], r.compact + 2 * n, r.compact + 3 * n, c->stream);
        continue;
      }
      if (g.nchunks) e = launch_hub_partials(p, g.chunks, g.nchunks, c->stream);
      if (e == hipSuccess) e = launch_step(p, c->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(r.ev[2], c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(r.ev[2]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.ev[1], r.ev[2]);
    if (e == hipSuccess && ms < best_ms) {
      best_ms = ms;
      best = sh.lpr;
    }
  }
  (void)hipStreamSynchronize(c->stream);
  release_request_buffers(c, &r);
  if (e != hipSuccess) return set_err(c, QQA_E_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
  c->layout[S] = best;
  if (lanes_per_row) *lanes_per_row = best;
  return QQA_OK;
}

int qqa_poll(qqa_ctx* c, qqa_req id, qqa_result* out, int32_t timeout_us) {
  if (!c) return QQA_E_ARG;
  (void)hipSetDevice(c->device);
  if (c->server) {
    int rc = serve_poll(c, id, out, timeout_us);
    if (rc != QQA_E_UNKNOWN_REQ) return rc;
  }
  auto it = c->reqs.find(id);
  if (it == c->reqs.end()) return set_err(c, QQA_E_UNKNOWN_REQ, "unknown request id");
  Request* r = it->second.get();
  const auto t0 = Clock::now();
  for (;;) {
    hipError_t q = hipEventQuery(r->ev[3]);
    if (q == hipSuccess) break;
    if (q != hipErrorNotReady) return set_err(c, QQA_E_DEVICE, std::string("poll: ") + hipGetErrorString(q));
    if (timeout_us == 0) return QQA_PENDING;
    if (timeout_us < 0) {
      hipError_t s = hipEventSynchronize(r->ev[3]);
      if (s != hipSuccess) return set_err(c, QQA_E_DEVICE, std::string("poll: ") + hipGetErrorString(s));
      break;
    }
    if (std::chrono::duration<double, std::micro>(Clock::now() - t0).count() > timeout_us) return QQA_PENDING;
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  const auto t_done = Clock::now();
  int rc = QQA_OK;
  if (r->cancelled) {
    rc = set_err(c, QQA_E_CANCELLED, "request was cancelled");
  } else if ((r->engine == kEnginePersistent || r->engine == kEngineLdsBlock) && out_bar(r->out_host, r->S)[1] != 0u) {
    rc = set_err(c, QQA_E_DEVICE, "persistent engine: grid barrier timed out");
  } else if (r->engine == kEngineResident && out_bar(r->out_host, r->S)[1] != 0u) {
    rc = set_err(c, QQA_E_DEVICE, "resident batch engine: a team barrier timed out");
  } else if (out) {
    fill_result(r, out);
    out->engine = r->engine;
    float ms = 0.f;
    out->queue_ms = r->queue_ms;
    out->first_update_ms = r->queue_ms;
    out->device_ms = hipEventElapsedTime(&ms, r->ev[0], r->ev[3]) == hipSuccess ? ms : -1.0;
    out->step_loop_ms = hipEventElapsedTime(&ms, r->ev[1], r->ev[2]) == hipSuccess ? ms : -1.0;
    out->latency_ms = std::chrono::duration<double, std::milli>(t_done - r->t_submit).count();
    out->kernel_us = -1.0;
    if (!r->probe.empty()) {
      double sum = 0.0;
      bool ok = true;
      for (size_t i = 0; i + 1 < r->probe.size(); i += 2)
        ok = ok && hipEventElapsedTime(&ms, r->probe[i], r->probe[i + 1]) == hipSuccess && (sum += ms, true);
      if (ok) out->kernel_us = sum * 1e3 / (double)(r->probe.size() / 2);
    }
  }
  release_request_buffers(c, r);
  c->in_use -= r->footprint;
  graph_unref(c, r->graph);
  c->reqs.erase(it);
  return rc;
}

int qqa_cancel(qqa_ctx* c, qqa_req id) {
  if (!c) return QQA_E_ARG;
  if (c->server) {
    int rc = serve_cancel(c, id);
    if (rc != QQA_E_UNKNOWN_REQ) return rc;
  }
  auto it = c->reqs.find(id);
  if (it == c->reqs.end()) return set_err(c, QQA_E_UNKNOWN_REQ, "unknown request id");
  it->second->cancelled = true;  // device work already enqueued runs out; poll reports it
  return QQA_OK;
}

}  // extern "C"

namespace qqa {

void fill_result(const Request* r, qqa_result* out) {
  out->kernel_us = -1.0;
  int64_t *a, *b, *o;
  int32_t* best;
  uint8_t* x;
  out_views(r->out_host, r->n, r->S, &a, &b, &o, &best, &x);
  const int s = *best;
  out->best_replica = s;
  out->best_objective = o[s];
  out->best_size_or_cut = a[s];
  out->best_violations = b[s];
  out->feasible = b[s] == 0;
  if (out->replica_objective) std::memcpy(out->replica_objective, o, sizeof(int64_t) * r->S);
  if (out->replica_size_or_cut) std::memcpy(out->replica_size_or_cut, a, sizeof(int64_t) * r->S);
  if (out->replica_violations) std::memcpy(out->replica_violations, b, sizeof(int64_t) * r->S);
  if (out->best_x) std::memcpy(out->best_x, x, r->n);
}

}  // namespace qqa
