// Host-side construction of multi-instance slot state, shared by ragged batches and the
// continuous-batching server.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "qqa_ctx.h"
#include "qqa_internal.h"

namespace qqa {

// Per-update scalars {ce, inv_bc1, inv_bc2, 0} of a K-update schedule, from the same host
// function the single-instance path uses (so both follow identical arithmetic).
std::vector<float4> schedule_table(const qqa_schedule& s, int K);

// Byte offsets of one instance's buffers inside a device arena.
struct SlotLayout {
  size_t P0, P1, m, v, hub, acc, out, bytes;  // out: out_bytes(n, S) bytes
  size_t out_size;
};
SlotLayout slot_layout(int n, int S, int rule, int nchunks);

// A slot descriptor for instance `g` solved with (problem, sched, S, K, seed), its buffers
// at `arena + L.*` and its update table at `table`.
SlotDesc make_slot(const DevGraph& g, int problem, const qqa_schedule& sched, int S, int K, uint64_t seed,
                   int lanes_per_row, char* arena, const SlotLayout& L, char* out, const float4* table, int start);

// Work lists (row blocks, split-row chunks) of one slot.
void append_items(int slot, const DevGraph& g, int lanes_per_row, std::vector<WorkItem>* items,
                  std::vector<HubItem>* hubs);

// A ragged batch in flight: owns its device arena, result arena, events and graph; every
// request of the batch holds a reference and the last one collected frees it.
struct BatchRun {
  qqa_ctx* c = nullptr;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  char* host_out = nullptr;
  size_t host_out_bytes = 0;
  size_t footprint = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  ~BatchRun();
};

}  // namespace qqa
