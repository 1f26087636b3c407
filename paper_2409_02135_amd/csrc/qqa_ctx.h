// Context, resident-graph and request records shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <memory>
#include <vector>
#include <string>
#include <unordered_map>

#include "qqa.h"
#include "qqa_internal.h"
#include "qqa_runtime.h"

namespace qqa {

struct DevGraph {
  int n = 0;
  int64_t nnz = 0;
  int problem = 0;
  int32_t* row_ptr = nullptr;
  int32_t* col = nullptr;
  float* w = nullptr;
  float* dense = nullptr;
  HubChunk* chunks = nullptr;  // split plan of rows above kHubDegree neighbours
  int32_t* hub_first = nullptr;
  int nchunks = 0;
  size_t bytes = 0;
  int refs = 0;
  bool release_pending = false;
};

// updates whose dominant launch (the update kernel, or the dense product) is timed per
// streaming request
constexpr int kProbes = 32;

struct Request {
  enum State { kQueued = 0, kRunning = 1, kDone = 2 };
  int64_t id = 0;
  int state = kQueued;
  bool cancelled = false;
  int64_t graph = 0;
  bool temp_graph = false;
  int problem = 0;
  qqa_schedule sched{};
  int S = 0, K = 0, n = 0;
  uint64_t seed = 0;
  ReplicaShape shape{};
  int lanes_per_row = 0;
  int engine = 0;               // PersistEngine of the update loop (3: batch slots)
  int rows_per_group = 0, grid = 0;
  float4* table_dev = nullptr;  // per-update scalars (persistent engines)
  float4* table_host = nullptr;
  size_t table_bytes = 0;
  float4* noise_dev = nullptr;  // LDS-block engine: the normals of a chunk of updates
  size_t noise_bytes = 0;
  int noise_chunk = 0;          // updates per noise table
  size_t footprint = 0;
  float* P[2] = {nullptr, nullptr};
  float* m = nullptr;
  float* v = nullptr;
  unsigned long long* acc = nullptr;
  float* hub_partial = nullptr;  // nchunks x stride
  size_t hub_bytes = 0;
  float* coupling = nullptr;     // dense graphs: n x stride coupling product
  unsigned long long* colsum = nullptr;  // max clique: per-replica sums of P (2^-32 fixed point)
  float2* stats = nullptr;               // sliced engine: 2 x n x 8 partial statistics (ping-pong)
  float* compact = nullptr;              // compact engine: P[2], m, v as n floats each
  // graph coloring: colours K; state rows are n * K; sigma and G (n * K x stride), colours
  // of every replica (n x stride bytes)
  int colors = 0;
  float* cat_sigma = nullptr;
  float* cat_grad = nullptr;
  uint8_t* cat_colors = nullptr;
  size_t coupling_bytes = 0;
  char* out_dev = nullptr;
  char* out_host = nullptr;
  size_t out_size = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // start, loop start, loop end, done
  // streaming engine: event pairs around the dominant launch of sampled updates
  std::vector<hipEvent_t> probe;
  int probe_every = 0;
  std::chrono::steady_clock::time_point t_submit, t_admit;
  // set when the buffers and events belong to a shared owner (a batch or the server);
  // releasing the request then only drops its reference
  std::shared_ptr<void> owner;
  double queue_ms = 0.0;
};

struct Server;

}  // namespace qqa

struct qqa_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0;
  size_t in_use = 0;
  std::string err;
  // idle buffers kept for reuse: up to 8 GiB of device memory, 1 GiB pinned
  qqa::Pool dpool{false, size_t(8) << 30};
  qqa::Pool hpool{true, size_t(1) << 30};
  std::unordered_map<int64_t, qqa::DevGraph> graphs;
  int64_t next_graph = 1;
  std::unordered_map<int64_t, std::unique_ptr<qqa::Request>> reqs;
  int64_t next_req = 1;
  std::unique_ptr<qqa::Server> server;
  std::unordered_map<int, int> layout;  // S -> lanes per row (absent: default)
  int engine_policy = -1;                // qqa_engine: -1 auto, 0 stream only
  // S -> what the batch autotuner found faster for a batch of one layout class under the
  // automatic policy: 1 the resident engine, 0 the slot launches (absent: resident if it fits)
  std::unordered_map<int, int> batch_resident;
  int layout_for(int S) const {
    auto it = layout.find(S);
    return it == layout.end() ? 0 : it->second;
  }
  qqa_ctx();
  ~qqa_ctx();
};

namespace qqa {

size_t request_footprint(int n, int S, int rule, int problem);
size_t out_bytes(int n, int S);
void out_views(char* base, int n, int S, int64_t** a, int64_t** b, int64_t** o, int32_t** best, uint8_t** x);
// barrier words of a persistent launch inside a result record: [0] arrivals, [1] abort
unsigned* out_bar(char* base, int S);
int upload_graph(qqa_ctx* c, const qqa_graph& g, int problem, DevGraph* out, std::string* why);
int upload_graph_on(hipStream_t stream, const qqa_graph& g, int problem, DevGraph* out, std::string* why,
                    bool validate);
void free_graph(DevGraph& d);
void graph_unref(qqa_ctx* c, int64_t gid);
bool budget_fits(qqa_ctx* c, size_t bytes);  // frees idle pooled buffers when they crowd the budget
int alloc_request_buffers(qqa_ctx* c, Request* r, std::string* why, int nchunks);
void release_request_buffers(qqa_ctx* c, Request* r);
StepParams request_step_params(const Request* r, const DevGraph& g);
hipError_t enqueue_finish(qqa_ctx* c, Request* r, const DevGraph& g, const float* final_P);
void fill_result(const Request* r, qqa_result* out);
int set_err(qqa_ctx* c, int code, const std::string& msg);

// continuous-batching server hooks (qqa_serve.cpp)
int serve_poll(qqa_ctx* c, int64_t id, qqa_result* out, int32_t timeout_us);
int serve_cancel(qqa_ctx* c, int64_t id);
void server_shutdown(qqa_ctx* c);  // drain, then free everything the server holds

}  // namespace qqa
