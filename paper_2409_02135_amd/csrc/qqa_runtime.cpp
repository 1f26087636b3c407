// Host runtime behind include/qqa.h: argument and graph validation, device uploads,
// a size-keyed buffer pool, and the request lifecycle (submit -> device work -> poll).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "qqa.h"
#include "qqa_internal.h"
#include "qqa_runtime.h"

using namespace qqa;

namespace qqa {

// ---------------------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------------------
static thread_local std::string g_dev_error;

int fail(std::string* where, int code, const std::string& msg) {
  if (where) *where = msg;
  return code;
}

// ---------------------------------------------------------------------------------------
// schedule helpers
// ---------------------------------------------------------------------------------------
bool schedule_valid(const qqa_schedule& s, std::string* why) {
  auto finite = [](float x) { return std::isfinite(x); };
  if (!finite(s.gamma_min) || !finite(s.gamma_max) || !finite(s.lr) || !finite(s.weight_decay) ||
      !finite(s.temperature) || !finite(s.comm_alpha) || !finite(s.beta1) || !finite(s.beta2) ||
      !finite(s.adam_eps)) {
    *why = "schedule has a non-finite value";
    return false;
  }
  if (s.gamma_min > s.gamma_max) { *why = "gamma_min > gamma_max"; return false; }
  if (s.entropy_alpha < 2 || s.entropy_alpha > 64 || (s.entropy_alpha & 1)) {
    *why = "entropy_alpha must be even and in [2, 64]";
    return false;
  }
  if (!(s.lr > 0.f) || s.weight_decay < 0.f || s.temperature < 0.f || s.comm_alpha < 0.f) {
    *why = "need lr > 0, weight_decay >= 0, temperature >= 0, comm_alpha >= 0";
    return false;
  }
  if (s.beta1 < 0.f || s.beta1 >= 1.f || s.beta2 < 0.f || s.beta2 >= 1.f || s.adam_eps < 0.f) {
    *why = "need 0 <= beta < 1 and adam_eps >= 0";
    return false;
  }
  if (s.penalty_lambda < 0 || s.penalty_lambda > (1 << 20)) { *why = "penalty_lambda out of range"; return false; }
  if (s.rule != QQA_STEP_ADAMW && s.rule != QQA_STEP_LANGEVIN) { *why = "unknown step rule"; return false; }
  return true;
}

// Fill the per-update scalars of update t (0-based) of a K-update schedule.  gamma_t
// rises linearly from gamma_min (t = 0) to gamma_max (t = K-1); bias corrections use
// k = t + 1.  Everything is computed in double and rounded once to float.
void fill_step_scalars(StepParams& p, const qqa_schedule& s, int t, int K) {
  const double gmin = s.gamma_min, gmax = s.gamma_max;
  const double gamma = K <= 1 ? gmin : gmin + (gmax - gmin) * (double)t / (double)(K - 1);
  const double k = (double)t + 1.0;
  p.ce = (float)(-2.0 * (double)s.entropy_alpha * gamma);
  p.inv_bc1 = (float)(1.0 / (1.0 - std::pow((double)s.beta1, k)));
  p.inv_bc2 = (float)(1.0 / (1.0 - std::pow((double)s.beta2, k)));
  p.k = (uint32_t)(t + 1);
}

void fill_static_scalars(StepParams& p, const qqa_schedule& s, int problem, int S, uint64_t seed) {
  p.S = S;
  p.inv_S = (float)(1.0 / (double)S);
  p.stride = replica_shape(S).stride;
  p.problem = problem;
  p.rule = s.rule;
  p.alpha_e = s.entropy_alpha;
  p.lambda = (float)s.penalty_lambda;
  p.lr = s.lr;
  p.wd_factor = (float)(1.0 - (double)s.lr * (double)s.weight_decay);
  p.comm_alpha = s.comm_alpha;
  p.beta1 = s.beta1;
  p.omb1 = (float)(1.0 - (double)s.beta1);
  p.beta2 = s.beta2;
  p.omb2 = (float)(1.0 - (double)s.beta2);
  p.eps = s.adam_eps;
  p.noise_scale = (float)std::sqrt(2.0 * (double)s.lr * (double)s.temperature);
  p.key0 = (uint32_t)seed;
  p.key1 = (uint32_t)(seed >> 32);
}

// ---------------------------------------------------------------------------------------
// graph validation (host)
// ---------------------------------------------------------------------------------------
static bool on_grid(float w) {
  const double q = (double)w * 65536.0;
  return std::fabs(w) < 128.f && q == std::rint(q);
}

int validate_graph(const qqa_graph& g, int problem, std::string* why) {
  if (g.n <= 0) return fail(why, QQA_E_GRAPH, "graph needs n > 0");
  if (g.dense && problem == QQA_COLORING) return fail(why, QQA_E_GRAPH, "graph coloring takes a CSR graph");
  if (g.dense) {
    const int n = g.n;
    if ((int64_t)n * n > (int64_t)1 << 31) return fail(why, QQA_E_GRAPH, "dense graph too large");
    for (int i = 0; i < n; ++i) {
      if (g.dense[(size_t)i * n + i] != 0.f) return fail(why, QQA_E_GRAPH, "dense graph has a nonzero diagonal");
      for (int j = i + 1; j < n; ++j) {
        const float a = g.dense[(size_t)i * n + j], b = g.dense[(size_t)j * n + i];
        if (a != b) return fail(why, QQA_E_GRAPH, "dense graph is not symmetric");
        if (!std::isfinite(a)) return fail(why, QQA_E_GRAPH, "dense graph has a non-finite weight");
        if ((problem == QQA_MIS || problem == QQA_MAXCLIQUE) && a != 0.f && a != 1.f)
          return fail(why, QQA_E_GRAPH, "MIS / max-clique dense adjacency must be 0/1");
        if (problem == QQA_MAXCUT && !on_grid(a))
          return fail(why, QQA_E_GRAPH, "max-cut weight not a multiple of 2^-16 with |w| < 128");
      }
    }
    return QQA_OK;
  }
  if (!g.row_ptr || (g.nnz > 0 && !g.col_idx)) return fail(why, QQA_E_GRAPH, "CSR arrays missing");
  if (g.nnz < 0 || g.nnz >= ((int64_t)1 << 31)) return fail(why, QQA_E_GRAPH, "nnz out of range");
  if (g.row_ptr[0] != 0 || g.row_ptr[g.n] != g.nnz) return fail(why, QQA_E_GRAPH, "row_ptr must run from 0 to nnz");
  for (int i = 0; i < g.n; ++i)
    if (g.row_ptr[i + 1] < g.row_ptr[i]) return fail(why, QQA_E_GRAPH, "row_ptr is not monotone");
  // sorted copy of each row for duplicate and symmetry checks
  std::vector<int32_t> cols(g.col_idx, g.col_idx + g.nnz);
  std::vector<float> ws;
  const bool weighted = g.weight != nullptr && problem == QQA_MAXCUT;
  if (weighted) ws.assign(g.weight, g.weight + g.nnz);
  for (int i = 0; i < g.n; ++i) {
    const int64_t a = g.row_ptr[i], b = g.row_ptr[i + 1];
    for (int64_t e = a; e < b; ++e) {
      if (cols[e] < 0 || cols[e] >= g.n) return fail(why, QQA_E_GRAPH, "column index out of range");
      if (cols[e] == i) return fail(why, QQA_E_GRAPH, "self-loop");
      if (weighted && !on_grid(ws[e]))
        return fail(why, QQA_E_GRAPH, "max-cut weight not a multiple of 2^-16 with |w| < 128");
    }
    if (weighted) {
      std::vector<std::pair<int32_t, float>> row;
      row.reserve(b - a);
      for (int64_t e = a; e < b; ++e) row.emplace_back(cols[e], ws[e]);
      std::sort(row.begin(), row.end());
      for (int64_t e = a; e < b; ++e) { cols[e] = row[e - a].first; ws[e] = row[e - a].second; }
    } else {
      std::sort(cols.begin() + a, cols.begin() + b);
    }
    for (int64_t e = a + 1; e < b; ++e)
      if (cols[e] == cols[e - 1]) return fail(why, QQA_E_GRAPH, "duplicate edge");
  }
  for (int i = 0; i < g.n; ++i) {
    for (int64_t e = g.row_ptr[i]; e < g.row_ptr[i + 1]; ++e) {
      const int j = cols[e];
      auto first = cols.begin() + g.row_ptr[j], last = cols.begin() + g.row_ptr[j + 1];
      auto it = std::lower_bound(first, last, i);
      if (it == last || *it != i) return fail(why, QQA_E_GRAPH, "graph is not symmetric");
      if (weighted && ws[it - cols.begin()] != ws[e]) return fail(why, QQA_E_GRAPH, "weights are not symmetric");
    }
  }
  return QQA_OK;
}

void build_hub_plan(const int32_t* row_ptr, int n, std::vector<HubChunk>* chunks, std::vector<int32_t>* hub_first) {
  chunks->clear();
  hub_first->assign(n, -1);
  bool any = false;
  for (int i = 0; i < n; ++i) {
    const int deg = row_ptr[i + 1] - row_ptr[i];
    if (deg <= kHubDegree) continue;
    any = true;
    (*hub_first)[i] = (int32_t)chunks->size();
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; e += kHubChunk) chunks->push_back(HubChunk{i, e});
  }
  if (!any) hub_first->clear();
}

// ---------------------------------------------------------------------------------------
// buffer pool: size-class reuse, so repeated solves of one shape, and of nearby shapes,
// do not call hipMalloc / hipFree (both of which synchronise) after the first
// ---------------------------------------------------------------------------------------
size_t Pool::class_size(size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes <= 4096) return bytes;
  // eight classes between consecutive powers of two: m * 2^e with m in [8, 16)
  int e = 63 - __builtin_clzll((unsigned long long)bytes) - 3;
  const size_t step = size_t(1) << e;
  return (bytes + step - 1) & ~(step - 1);
}

hipError_t Pool::get(size_t bytes, void** out) {
  bytes = class_size(bytes);
  {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = free_.find(bytes);
    if (it != free_.end()) {
      *out = it->second;
      cached_ -= bytes;
      free_.erase(it);
      return hipSuccess;
    }
  }
  hipError_t e = pinned_ ? hipHostMalloc(out, bytes, hipHostMallocDefault) : hipMalloc(out, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim();
    e = pinned_ ? hipHostMalloc(out, bytes, hipHostMallocDefault) : hipMalloc(out, bytes);
  }
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lk(mu_);
    held_ += bytes;
  }
  return e;
}

void Pool::release_locked(std::multimap<size_t, void*>::iterator it) {
  if (pinned_) (void)hipHostFree(it->second);
  else (void)hipFree(it->second);
  held_ -= it->first;
  cached_ -= it->first;
  free_.erase(it);
}

void Pool::put(void* p, size_t bytes) {
  if (!p) return;
  bytes = class_size(bytes);
  std::lock_guard<std::mutex> lk(mu_);
  free_.emplace(bytes, p);
  cached_ += bytes;
  // over the cap: free the largest idle buffers first
  while (cached_ > cap_ && !free_.empty()) release_locked(std::prev(free_.end()));
}

void Pool::trim() {
  std::lock_guard<std::mutex> lk(mu_);
  while (!free_.empty()) release_locked(free_.begin());
}

size_t Pool::held() const {
  std::lock_guard<std::mutex> lk(mu_);
  return held_;
}

size_t Pool::cached() const {
  std::lock_guard<std::mutex> lk(mu_);
  return cached_;
}

void Pool::set_cap(size_t bytes) {
  std::lock_guard<std::mutex> lk(mu_);
  cap_ = bytes;
  while (cached_ > cap_ && !free_.empty()) release_locked(std::prev(free_.end()));
}

}  // namespace qqa

// =========================================================================================
// C ABI
// =========================================================================================
extern "C" {

void qqa_schedule_default(qqa_schedule* s, qqa_problem problem, int32_t n) {
  if (!s) return;
  s->gamma_min = problem == QQA_MAXCUT ? (n >= 1000 ? -20.f : -5.f) : -2.f;
  s->gamma_max = 0.1f;
  s->lr = 0.1f;
  s->weight_decay = 0.01f;
  s->temperature = 1e-3f;
  s->comm_alpha = 0.1f;
  s->entropy_alpha = 4;
  s->beta1 = 0.9f;
  s->beta2 = 0.999f;
  s->adam_eps = 1e-8f;
  s->penalty_lambda = 2;
  s->rule = QQA_STEP_ADAMW;
}

int qqa_graph_validate(const qqa_graph* g, qqa_problem problem, char* why, size_t why_len) {
  std::string msg;
  int rc = g ? validate_graph(*g, problem, &msg) : fail(&msg, QQA_E_GRAPH, "graph is NULL");
  if (why && why_len) {
    std::snprintf(why, why_len, "%s", msg.c_str());
  }
  return rc;
}

int32_t qqa_replica_stride(int32_t S) { return S <= 0 ? 0 : replica_shape(S).stride; }

const char* qqa_dev_last_error(void) { return g_dev_error.c_str(); }

#define DEV_CHECK(expr)                                                                        \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(&g_dev_error, QQA_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

int qqa_dev_philox(uint64_t seed, int32_t n, int32_t nquads, uint32_t k, uint32_t stream_id, uint32_t* out,
                   void* stream) {
  if (n < 0 || nquads < 0 || (!out && (int64_t)n * nquads > 0)) return fail(&g_dev_error, QQA_E_ARG, "bad philox arguments");
  DEV_CHECK(launch_philox(seed, n, nquads, k, stream_id, out, (hipStream_t)stream));
  return QQA_OK;
}

int qqa_dev_noise(uint64_t seed, int32_t n, int32_t S, uint32_t k, float* xi, void* stream) {
  if (n < 0 || S <= 0 || S > kMaxReplicas || (!xi && n > 0)) return fail(&g_dev_error, QQA_E_ARG, "bad noise arguments");
  DEV_CHECK(launch_noise(seed, n, S, k, xi, (hipStream_t)stream));
  return QQA_OK;
}

int qqa_dev_init(uint64_t seed, int32_t n, int32_t S, float* P, float* m, float* v, void* stream) {
  if (n < 0 || S <= 0 || S > kMaxReplicas || (!P && n > 0)) return fail(&g_dev_error, QQA_E_ARG, "bad init arguments");
  DEV_CHECK(launch_init(seed, n, S, P, m, v, (hipStream_t)stream));
  return QQA_OK;
}

static int dev_graph_check(const qqa_dev_graph* g) {
  if (!g || g->n < 0) return fail(&g_dev_error, QQA_E_ARG, "graph is NULL or n < 0");
  if (g->dense) return QQA_OK;
  if (g->n > 0 && !g->row_ptr) return fail(&g_dev_error, QQA_E_ARG, "row_ptr missing");
  if (g->nnz > 0 && !g->col_idx) return fail(&g_dev_error, QQA_E_ARG, "col_idx missing");
  return QQA_OK;
}

// max clique: per-replica sums of P_in for the update that reads it (stream-ordered buffer)
static hipError_t colsum_for(StepParams& p, int problem, unsigned long long** T, hipStream_t st) {
  if (problem != QQA_MAXCLIQUE) return hipSuccess;
  if (!*T) {
    hipError_t e = hipMallocAsync((void**)T, (size_t)p.stride * sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
  }
  p.colsum = *T;
  return launch_colsum(p.P_in, p.n, p.stride, *T, st);
}

int qqa_dev_step(const qqa_dev_graph* g, qqa_problem problem, const qqa_schedule* sched, int32_t S, int32_t t,
                 int32_t K, uint64_t seed, const float* P_in, float* P_out, float* m, float* v,
                 int32_t lanes_per_row, void* stream) {
  int rc = dev_graph_check(g);
  if (rc) return rc;
  if (!known_problem(problem)) return fail(&g_dev_error, QQA_E_ARG, "unknown problem");
  if (S <= 0 || S > kMaxReplicas) return fail(&g_dev_error, QQA_E_ARG, "S must be in [1, 4096]");
  if (K <= 0 || t < 0 || t >= K) return fail(&g_dev_error, QQA_E_ARG, "need 0 <= t < K");
  qqa_schedule s;
  if (sched) s = *sched; else qqa_schedule_default(&s, problem, g->n);
  std::string why;
  if (!schedule_valid(s, &why)) return fail(&g_dev_error, QQA_E_ARG, why);
  if (g->n > 0 && (!P_in || !P_out)) return fail(&g_dev_error, QQA_E_ARG, "P_in/P_out missing");
  if (P_in == P_out && g->n > 0) return fail(&g_dev_error, QQA_E_ARG, "P_out must not alias P_in");
  if (s.rule == QQA_STEP_ADAMW && g->n > 0 && (!m || !v)) return fail(&g_dev_error, QQA_E_ARG, "AdamW needs m and v");
  if (lanes_per_row < 0 || lanes_per_row > 64 || !layout_supported(S, lanes_per_row))
    return fail(&g_dev_error, QQA_E_ARG, "unsupported replica layout");
  hipStream_t st = (hipStream_t)stream;
  StepParams p{};
  p.row_ptr = g->row_ptr;
  p.col = g->col_idx;
  p.w = problem == QQA_MAXCUT ? g->weight : nullptr;
  p.coupling = nullptr;
  p.P_in = P_in;
  p.P_out = P_out;
  p.m = m;
  p.v = v;
  p.n = g->n;
  fill_static_scalars(p, s, problem, S, seed);
  fill_step_scalars(p, s, t, K);
  p.lanes_per_row = lanes_per_row;
  if (g->n == 0) return QQA_OK;
  unsigned long long* T = nullptr;
  DEV_CHECK(colsum_for(p, problem, &T, st));
  if (g->dense) {
    float* C = nullptr;  // the product's split-K parts, added by the update kernel
    const int parts = dense_splits(g->n, p.stride);
    DEV_CHECK(hipMallocAsync((void**)&C, (size_t)parts * g->n * p.stride * sizeof(float), st));
    p.row_ptr = nullptr;
    p.col = nullptr;
    p.w = nullptr;
    p.coupling = C;
    p.coupling_parts = parts;
    hipError_t e = launch_dense_parts(g->dense, P_in, C, g->n, p.stride, problem, st);
    if (e == hipSuccess) e = launch_step(p, st);
    (void)hipFreeAsync(C, st);
    if (T) (void)hipFreeAsync(T, st);
    DEV_CHECK(e);
    return QQA_OK;
  }
  // the same row split the solver uses: read the row pointers back to plan it
  std::vector<int32_t> rp(g->n + 1);
  DEV_CHECK(hipMemcpyAsync(rp.data(), g->row_ptr, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  DEV_CHECK(hipStreamSynchronize(st));
  std::vector<HubChunk> chunks;
  std::vector<int32_t> hub_first;
  build_hub_plan(rp.data(), g->n, &chunks, &hub_first);
  HubChunk* d_chunks = nullptr;
  int32_t* d_first = nullptr;
  float* d_part = nullptr;
  if (!chunks.empty()) {
    DEV_CHECK(hipMallocAsync((void**)&d_chunks, chunks.size() * sizeof(HubChunk), st));
    DEV_CHECK(hipMallocAsync((void**)&d_first, hub_first.size() * sizeof(int32_t), st));
    DEV_CHECK(hipMallocAsync((void**)&d_part, chunks.size() * (size_t)p.stride * sizeof(float), st));
    DEV_CHECK(hipMemcpyAsync(d_chunks, chunks.data(), chunks.size() * sizeof(HubChunk), hipMemcpyHostToDevice, st));
    DEV_CHECK(hipMemcpyAsync(d_first, hub_first.data(), hub_first.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    p.hub_first = d_first;
    p.hub_partial = d_part;
    DEV_CHECK(launch_hub_partials(p, d_chunks, (int)chunks.size(), st));
  }
  hipError_t e = launch_step(p, st);
  if (T) (void)hipFreeAsync(T, st);
  if (!chunks.empty()) {
    (void)hipFreeAsync(d_chunks, st);
    (void)hipFreeAsync(d_first, st);
    (void)hipFreeAsync(d_part, st);
    // host vectors go out of scope: the copies above must have completed
    DEV_CHECK(hipStreamSynchronize(st));
  }
  DEV_CHECK(e);
  return QQA_OK;
}

int qqa_dev_run(const qqa_dev_graph* g, qqa_problem problem, const qqa_schedule* sched, int32_t S, int32_t t0,
                int32_t t1, int32_t K, uint64_t seed, float* P0, float* P1, float* m, float* v, int32_t engine,
                int32_t lanes_per_row, void* stream) {
  int rc = dev_graph_check(g);
  if (rc) return rc;
  if (!known_problem(problem)) return fail(&g_dev_error, QQA_E_ARG, "unknown problem");
  if (S <= 0 || S > kMaxReplicas) return fail(&g_dev_error, QQA_E_ARG, "S must be in [1, 4096]");
  if (K <= 0 || t0 < 0 || t1 < t0 || t1 > K) return fail(&g_dev_error, QQA_E_ARG, "need 0 <= t0 <= t1 <= K");
  qqa_schedule s;
  if (sched) s = *sched; else qqa_schedule_default(&s, problem, g->n);
  std::string why;
  if (!schedule_valid(s, &why)) return fail(&g_dev_error, QQA_E_ARG, why);
  if (g->n > 0 && (!P0 || !P1 || P0 == P1)) return fail(&g_dev_error, QQA_E_ARG, "need two distinct P buffers");
  if (s.rule == QQA_STEP_ADAMW && g->n > 0 && (!m || !v)) return fail(&g_dev_error, QQA_E_ARG, "AdamW needs m and v");
  if (lanes_per_row < 0 || lanes_per_row > 64 || !layout_supported(S, lanes_per_row))
    return fail(&g_dev_error, QQA_E_ARG, "unsupported replica layout");
  if (g->n == 0 || t0 == t1) return QQA_OK;
  hipStream_t st = (hipStream_t)stream;
  if (problem == QQA_MAXCLIQUE && engine > 0 && engine != kEngineSliced)
    return fail(&g_dev_error, QQA_E_ARG, "max clique runs on the streaming and sliced engines");
  unsigned long long* T = nullptr;
  if (g->dense) {
    if (engine > 0) return fail(&g_dev_error, QQA_E_ARG, "dense coupling runs on the streaming engine");
    StepParams p{};
    p.m = m;
    p.v = v;
    p.n = g->n;
    fill_static_scalars(p, s, problem, S, seed);
    p.lanes_per_row = lanes_per_row;
    float* C = nullptr;  // the product's split-K parts, added by the update kernel
    const int parts = dense_splits(g->n, p.stride);
    DEV_CHECK(hipMallocAsync((void**)&C, (size_t)parts * g->n * p.stride * sizeof(float), st));
    p.coupling = C;
    p.coupling_parts = parts;
    float* P[2] = {P0, P1};
    hipError_t e = hipSuccess;
    for (int t = t0; t < t1 && e == hipSuccess; ++t) {
      p.P_in = P[t & 1];
      p.P_out = P[(t + 1) & 1];
      fill_step_scalars(p, s, t, K);
      e = colsum_for(p, problem, &T, st);
      if (e == hipSuccess) e = launch_dense_parts(g->dense, p.P_in, C, g->n, p.stride, problem, st);
      if (e == hipSuccess) e = launch_step(p, st);
    }
    (void)hipFreeAsync(C, st);
    if (T) (void)hipFreeAsync(T, st);
    DEV_CHECK(e);
    return QQA_OK;
  }
  StepParams p{};
  p.row_ptr = g->row_ptr;
  p.col = g->col_idx;
  p.w = problem == QQA_MAXCUT ? g->weight : nullptr;
  p.m = m;
  p.v = v;
  p.n = g->n;
  fill_static_scalars(p, s, problem, S, seed);
  p.lanes_per_row = lanes_per_row;
  std::vector<int32_t> rp(g->n + 1);
  DEV_CHECK(hipMemcpyAsync(rp.data(), g->row_ptr, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  DEV_CHECK(hipStreamSynchronize(st));
  std::vector<HubChunk> chunks;
  std::vector<int32_t> hub_first;
  build_hub_plan(rp.data(), g->n, &chunks, &hub_first);
  int rpg = 0, grid = 0;
  int use = kEngineStream;
  const bool sliceable = slice_shape(S).sq > 0;
  const bool compactable = S == 1 && problem != QQA_MAXCLIQUE;
  if (engine == kEngineSliced) {
    if (!sliceable) return fail(&g_dev_error, QQA_E_ARG, "engine cannot run this instance");
    use = kEngineSliced;
  } else if (engine == kEngineCompact) {
    if (!compactable) return fail(&g_dev_error, QQA_E_ARG, "engine cannot run this instance");
    use = kEngineCompact;
  } else if (engine != kEngineStream && problem != QQA_MAXCLIQUE) {
    // allow mask: 1 = one workgroup with P in LDS, 2 = many workgroups with registers
    const int allow = engine < 0 ? 3 : (engine == kEngineLdsBlock ? 1 : (engine == kEnginePersistent ? 2 : 0));
    if (!allow) return fail(&g_dev_error, QQA_E_ARG, "unknown engine");
    use = persistent_plan(p, !chunks.empty(), allow, &rpg, &grid);
    if (engine >= 0 && use != engine) return fail(&g_dev_error, QQA_E_ARG, "engine cannot run this instance");
  }
  if (engine < 0 && use == kEngineStream && compactable) use = kEngineCompact;
  if (engine < 0 && use == kEngineStream && sliceable && slice_by_default(g->n, S, false)) use = kEngineSliced;
  float* P[2] = {P0, P1};
  if (use == kEngineCompact) {
    const size_t n = (size_t)g->n;
    const bool adam = s.rule == QQA_STEP_ADAMW;
    int32_t* d_first = nullptr;
    if (!chunks.empty()) {
      DEV_CHECK(hipMallocAsync((void**)&d_first, hub_first.size() * sizeof(int32_t), st));
      DEV_CHECK(hipMemcpyAsync(d_first, hub_first.data(), hub_first.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
      p.hub_first = d_first;
    }
    float* cbuf = nullptr;
    DEV_CHECK(hipMallocAsync((void**)&cbuf, 4 * n * sizeof(float), st));
    float* Pc[2] = {cbuf, cbuf + n};
    float* mc = cbuf + 2 * n;
    float* vc = cbuf + 3 * n;
    hipError_t e = launch_compact_pack(P[t0 & 1], p.stride, g->n, Pc[t0 & 1], st);
    if (adam && e == hipSuccess) e = launch_compact_pack(m, p.stride, g->n, mc, st);
    if (adam && e == hipSuccess) e = launch_compact_pack(v, p.stride, g->n, vc, st);
    for (int t = t0; t < t1 && e == hipSuccess; ++t) {
      fill_step_scalars(p, s, t, K);
      e = launch_compact_step(p, Pc[t & 1], Pc[(t + 1) & 1], mc, vc, st);
    }
    if (e == hipSuccess) e = launch_compact_unpack(Pc[t1 & 1], g->n, p.stride, P[t1 & 1], st);
    if (adam && e == hipSuccess) e = launch_compact_unpack(mc, g->n, p.stride, m, st);
    if (adam && e == hipSuccess) e = launch_compact_unpack(vc, g->n, p.stride, v, st);
    (void)hipFreeAsync(cbuf, st);
    if (d_first) (void)hipFreeAsync(d_first, st);
    DEV_CHECK(hipStreamSynchronize(st));
    DEV_CHECK(e);
    return QQA_OK;
  }
  if (use == kEngineStream || use == kEngineSliced) {
    HubChunk* d_chunks = nullptr;
    int32_t* d_first = nullptr;
    float* d_part = nullptr;
    if (!chunks.empty()) {
      DEV_CHECK(hipMallocAsync((void**)&d_chunks, chunks.size() * sizeof(HubChunk), st));
      DEV_CHECK(hipMallocAsync((void**)&d_first, hub_first.size() * sizeof(int32_t), st));
      DEV_CHECK(hipMallocAsync((void**)&d_part, chunks.size() * (size_t)p.stride * sizeof(float), st));
      DEV_CHECK(hipMemcpyAsync(d_chunks, chunks.data(), chunks.size() * sizeof(HubChunk), hipMemcpyHostToDevice, st));
      DEV_CHECK(hipMemcpyAsync(d_first, hub_first.data(), hub_first.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
      p.hub_first = d_first;
      p.hub_partial = d_part;
    }
    float2* stats = nullptr;  // sliced engine: partial statistics, ping-pong
    float2* part[2] = {nullptr, nullptr};
    hipError_t e = hipSuccess;
    if (use == kEngineSliced) {
      const size_t count = (size_t)g->n * kReplicaSlices;
      DEV_CHECK(hipMallocAsync((void**)&stats, 2 * count * sizeof(float2), st));
      part[0] = stats;
      part[1] = stats + count;
      p.P_in = P[t0 & 1];
      e = launch_slice_stats(p, part[t0 & 1], st);
    }
    for (int t = t0; t < t1 && e == hipSuccess; ++t) {
      p.P_in = P[t & 1];
      p.P_out = P[(t + 1) & 1];
      fill_step_scalars(p, s, t, K);
      e = colsum_for(p, problem, &T, st);
      if (e == hipSuccess && !chunks.empty()) e = launch_hub_partials(p, d_chunks, (int)chunks.size(), st);
      if (e == hipSuccess) e = stats ? launch_slice_step(p, part[t & 1], part[(t + 1) & 1], st) : launch_step(p, st);
    }
    if (T) (void)hipFreeAsync(T, st);
    if (stats) (void)hipFreeAsync(stats, st);
    if (!chunks.empty()) {
      (void)hipFreeAsync(d_chunks, st);
      (void)hipFreeAsync(d_first, st);
      (void)hipFreeAsync(d_part, st);
      DEV_CHECK(hipStreamSynchronize(st));
    }
    DEV_CHECK(e);
    return QQA_OK;
  }
  // persistent engines: per-update table and barrier words
  std::vector<float4> table((size_t)K);
  for (int t = 0; t < K; ++t) {
    StepParams q{};
    fill_step_scalars(q, s, t, K);
    table[t] = make_float4(q.ce, q.inv_bc1, q.inv_bc2, 0.f);
  }
  float4* d_table = nullptr;
  unsigned* d_bar = nullptr;
  DEV_CHECK(hipMallocAsync((void**)&d_table, table.size() * sizeof(float4), st));
  DEV_CHECK(hipMallocAsync((void**)&d_bar, 256, st));
  DEV_CHECK(hipMemcpyAsync(d_table, table.data(), table.size() * sizeof(float4), hipMemcpyHostToDevice, st));
  DEV_CHECK(launch_fill_u64(reinterpret_cast<unsigned long long*>(d_bar), 1, st));
  PersistParams pp{};
  pp.a = p;
  pp.P[0] = P0;
  pp.P[1] = P1;
  pp.table = d_table;
  pp.t0 = t0;
  pp.t1 = t1;
  pp.bar = d_bar;
  hipError_t e = hipSuccess;
  float4* d_noise = nullptr;
  if (use == kEngineLdsBlock && t1 > t0) {
    // the normals of a bounded chunk of updates at a time, then the chunk's updates
    const size_t per_update = (size_t)g->n * (p.stride / 4) * sizeof(float4);
    const int chunk = (int)std::min<size_t>((size_t)(t1 - t0), std::max<size_t>(1, kNoiseTableMaxBytes / per_update));
    pp.nnz = g->nnz;
    e = hipMallocAsync((void**)&d_noise, per_update * (size_t)chunk, st);
    pp.noise = d_noise;
    for (int c0 = t0; c0 < t1 && e == hipSuccess; c0 += chunk) {
      pp.t0 = c0;
      pp.t1 = std::min(t1, c0 + chunk);
      e = launch_noise_table(p, pp.t0, pp.t1, d_noise, st);
      if (e == hipSuccess) e = launch_persistent(pp, use, rpg, grid, st);
    }
  } else if (use != kEngineLdsBlock) {
    e = launch_persistent(pp, use, rpg, grid, st);
  }
  unsigned bar[2] = {0, 0};
  hipError_t e2 = hipMemcpyAsync(bar, d_bar, sizeof(bar), hipMemcpyDeviceToHost, st);
  hipError_t e3 = hipStreamSynchronize(st);
  (void)hipFreeAsync(d_table, st);
  (void)hipFreeAsync(d_bar, st);
  if (d_noise) (void)hipFreeAsync(d_noise, st);
  DEV_CHECK(e);
  DEV_CHECK(e2);
  DEV_CHECK(e3);
  if (bar[1] != 0u) return fail(&g_dev_error, QQA_E_DEVICE, "persistent engine: grid barrier timed out");
  return QQA_OK;
}

int qqa_dev_dense_coupling(const float* W, const float* P, float* C, int32_t n, int32_t S, qqa_problem problem,
                           void* stream) {
  if (n < 0 || S <= 0 || S > kMaxReplicas || (n > 0 && (!W || !P || !C)))
    return fail(&g_dev_error, QQA_E_ARG, "bad dense coupling arguments");
  if (!known_problem(problem)) return fail(&g_dev_error, QQA_E_ARG, "unknown problem");
  const int stride = replica_shape(S).stride;
  const size_t wb = dense_workspace_bytes(n, stride);
  hipStream_t st = (hipStream_t)stream;
  float* work = nullptr;
  if (wb) DEV_CHECK(hipMallocAsync((void**)&work, wb, st));
  const hipError_t e = launch_dense_coupling(W, P, C, n, stride, problem, work, st);
  if (work) (void)hipFreeAsync(work, st);
  DEV_CHECK(e);
  return QQA_OK;
}

int qqa_dev_color_step(const qqa_dev_graph* g, int32_t colors, const qqa_schedule* sched, int32_t S, int32_t t,
                       int32_t K, uint64_t seed, const float* V_in, float* V_out, float* m, float* v,
                       int32_t lanes_per_row, void* stream) {
  int rc = dev_graph_check(g);
  if (rc) return rc;
  if (g->dense) return fail(&g_dev_error, QQA_E_ARG, "graph coloring takes a CSR graph");
  if (colors < 2 || colors > 255) return fail(&g_dev_error, QQA_E_ARG, "colours must be in [2, 255]");
  if (S <= 0 || S > kMaxReplicas) return fail(&g_dev_error, QQA_E_ARG, "S must be in [1, 4096]");
  if (K <= 0 || t < 0 || t >= K) return fail(&g_dev_error, QQA_E_ARG, "need 0 <= t < K");
  qqa_schedule s;
  if (sched) s = *sched; else qqa_schedule_default(&s, QQA_COLORING, g->n);
  std::string why;
  if (!schedule_valid(s, &why)) return fail(&g_dev_error, QQA_E_ARG, why);
  if (g->n > 0 && (!V_in || !V_out || V_in == V_out)) return fail(&g_dev_error, QQA_E_ARG, "need distinct V_in, V_out");
  if (s.rule == QQA_STEP_ADAMW && g->n > 0 && (!m || !v)) return fail(&g_dev_error, QQA_E_ARG, "AdamW needs m and v");
  if (lanes_per_row < 0 || lanes_per_row > 64 || !layout_supported(S, lanes_per_row))
    return fail(&g_dev_error, QQA_E_ARG, "unsupported replica layout");
  if (g->n == 0) return QQA_OK;
  hipStream_t st = (hipStream_t)stream;
  StepParams base{};
  base.row_ptr = g->row_ptr;
  base.col = g->col_idx;
  base.m = m;
  base.v = v;
  base.n = g->n;
  fill_static_scalars(base, s, QQA_COLORING, S, seed);
  base.lanes_per_row = lanes_per_row;
  const size_t state = (size_t)g->n * colors * base.stride * sizeof(float);
  float *sig = nullptr, *G = nullptr;
  DEV_CHECK(hipMallocAsync((void**)&sig, state, st));
  DEV_CHECK(hipMallocAsync((void**)&G, state, st));
  const double gamma = K <= 1 ? s.gamma_min
                              : (double)s.gamma_min + ((double)s.gamma_max - (double)s.gamma_min) * t / (double)(K - 1);
  const double cK = 1.0 / ((double)(colors - 1) * (std::pow((double)(colors - 1), s.entropy_alpha - 1) + 1.0));
  StepParams pg = base;
  pg.n = g->n * colors;
  pg.P_in = sig;
  pg.ce = (float)(-gamma * cK * (double)s.entropy_alpha * (double)colors);
  StepParams pu = base;
  pu.P_in = V_in;
  pu.P_out = V_out;
  fill_step_scalars(pu, s, t, K);
  hipError_t e = launch_cat_sigma(V_in, sig, g->n, colors, base.stride, S, st);
  if (cat_fused_shape(S, lanes_per_row, colors)) {
    // one launch; G's buffer takes the new sigma
    if (e == hipSuccess) e = launch_cat_fused(pu, colors, pg.ce, sig, G, g->nnz, st);
  } else {
    if (e == hipSuccess) e = launch_cat_grad(pg, colors, G, st);
    if (e == hipSuccess) e = launch_cat_update(pu, colors, G, sig, st);
  }
  (void)hipFreeAsync(sig, st);
  (void)hipFreeAsync(G, st);
  DEV_CHECK(e);
  return QQA_OK;
}

int qqa_dev_color_eval(const qqa_dev_graph* g, int32_t colors, int32_t S, const float* V, uint8_t* X,
                       int64_t* conflicts, int32_t* best, void* stream) {
  if (!g || g->n < 0) return fail(&g_dev_error, QQA_E_ARG, "graph is NULL or n < 0");
  if (g->dense) return fail(&g_dev_error, QQA_E_ARG, "graph coloring takes a CSR graph");
  if (g->n > 0 && !g->row_ptr) return fail(&g_dev_error, QQA_E_ARG, "row_ptr missing");
  if (colors < 2 || colors > 255) return fail(&g_dev_error, QQA_E_ARG, "colours must be in [2, 255]");
  if (S <= 0 || S > kMaxReplicas) return fail(&g_dev_error, QQA_E_ARG, "S must be in [1, 4096]");
  if (!X || !conflicts || !best || (g->n > 0 && !V)) return fail(&g_dev_error, QQA_E_ARG, "output missing");
  hipStream_t st = (hipStream_t)stream;
  const ReplicaShape r = replica_shape(S);
  unsigned long long* acc = nullptr;
  int64_t* tmp = nullptr;
  DEV_CHECK(hipMallocAsync((void**)&acc, 2 * (size_t)r.stride * sizeof(unsigned long long), st));
  DEV_CHECK(hipMallocAsync((void**)&tmp, 2 * (size_t)S * sizeof(int64_t), st));
  hipError_t e = launch_cat_eval(g->row_ptr, g->col_idx, V, X, g->n, colors, r.stride, S, acc, st);
  EvalParams ep{};
  ep.n = g->n;
  ep.S = S;
  ep.stride = r.stride;
  ep.problem = QQA_COLORING;
  ep.acc = acc;
  ep.size_or_cut = conflicts;
  ep.viol = tmp;
  ep.obj = tmp + S;
  ep.best = best;
  if (e == hipSuccess) e = launch_finalize(ep, st);
  hipError_t e2 = hipFreeAsync(acc, st);
  hipError_t e3 = hipFreeAsync(tmp, st);
  DEV_CHECK(e);
  DEV_CHECK(e2);
  DEV_CHECK(e3);
  return QQA_OK;
}

int qqa_dev_replica_sums(const float* P, int32_t n, int32_t S, uint64_t* T, void* stream) {
  if (n < 0 || S <= 0 || S > kMaxReplicas || !T || (n > 0 && !P))
    return fail(&g_dev_error, QQA_E_ARG, "bad replica-sum arguments");
  DEV_CHECK(launch_colsum(P, n, replica_shape(S).stride, reinterpret_cast<unsigned long long*>(T), (hipStream_t)stream));
  return QQA_OK;
}

static int eval_args(const qqa_dev_graph* g, qqa_problem problem, int32_t S, const float* P, int64_t* size_or_cut,
                     int64_t* viol, int64_t* obj, int32_t* best) {
  if (!g || g->n < 0) return fail(&g_dev_error, QQA_E_ARG, "graph is NULL or n < 0");
  if (!g->dense && g->n > 0 && !g->row_ptr) return fail(&g_dev_error, QQA_E_ARG, "row_ptr missing");
  if (!known_problem(problem)) return fail(&g_dev_error, QQA_E_ARG, "unknown problem");
  if (S <= 0 || S > kMaxReplicas) return fail(&g_dev_error, QQA_E_ARG, "S must be in [1, 4096]");
  if (!size_or_cut || !viol || !obj || !best || (g->n > 0 && !P)) return fail(&g_dev_error, QQA_E_ARG, "output missing");
  return QQA_OK;
}

static EvalParams eval_params(const qqa_dev_graph* g, qqa_problem problem, int32_t penalty_lambda, int32_t S,
                              const float* P, int64_t* size_or_cut, int64_t* viol, int64_t* obj, int32_t* best,
                              unsigned long long* acc) {
  EvalParams p{};
  p.row_ptr = g->row_ptr;
  p.col = g->col_idx;
  p.w = problem == QQA_MAXCUT ? g->weight : nullptr;
  p.dense = g->dense;
  p.P = P;
  p.n = g->n;
  p.S = S;
  p.stride = replica_shape(S).stride;
  p.problem = problem;
  p.lambda = penalty_lambda;
  p.acc = acc;
  p.size_or_cut = size_or_cut;
  p.viol = viol;
  p.obj = obj;
  p.best = best;
  return p;
}

int qqa_dev_eval(const qqa_dev_graph* g, qqa_problem problem, int32_t penalty_lambda, int32_t S, const float* P,
                 int64_t* size_or_cut, int64_t* viol, int64_t* obj, int32_t* best, void* stream) {
  int rc = eval_args(g, problem, S, P, size_or_cut, viol, obj, best);
  if (rc) return rc;
  const ReplicaShape r = replica_shape(S);
  unsigned long long* acc = nullptr;
  DEV_CHECK(hipMallocAsync((void**)&acc, 2 * (size_t)r.stride * sizeof(unsigned long long), (hipStream_t)stream));
  const EvalParams p = eval_params(g, problem, penalty_lambda, S, P, size_or_cut, viol, obj, best, acc);
  hipError_t e = launch_eval(p, (hipStream_t)stream);
  hipError_t e2 = hipFreeAsync(acc, (hipStream_t)stream);
  DEV_CHECK(e);
  DEV_CHECK(e2);
  return QQA_OK;
}

int qqa_dev_eval_noalloc(const qqa_dev_graph* g, qqa_problem problem, int32_t penalty_lambda, int32_t S,
                         const float* P, int64_t* size_or_cut, int64_t* viol, int64_t* obj, int32_t* best,
                         void* stream) {
  int rc = eval_args(g, problem, S, P, size_or_cut, viol, obj, best);
  if (rc) return rc;
  unsigned long long* acc = nullptr;
  size_t words = 0;
  DEV_CHECK(eval_scratch(&acc, &words));
  const ReplicaShape r = replica_shape(S);
  if (2 * (size_t)r.stride > words)
    return fail(&g_dev_error, QQA_E_ARG, "replica stride exceeds the fixed evaluation scratch (2 x 4096 words)");
  // launch_eval clears the accumulators with a fill kernel before the counts
  DEV_CHECK(launch_eval(eval_params(g, problem, penalty_lambda, S, P, size_or_cut, viol, obj, best, acc),
                        (hipStream_t)stream));
  return QQA_OK;
}

}  // extern "C"
