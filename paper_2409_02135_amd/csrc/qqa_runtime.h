// Internal host-runtime declarations shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "qqa.h"
#include "qqa_internal.h"

namespace qqa {

int fail(std::string* where, int code, const std::string& msg);
bool schedule_valid(const qqa_schedule& s, std::string* why);
void fill_step_scalars(StepParams& p, const qqa_schedule& s, int t, int K);
void fill_static_scalars(StepParams& p, const qqa_schedule& s, int problem, int S, uint64_t seed);
int validate_graph(const qqa_graph& g, int problem, std::string* why);
inline bool known_problem(int problem) {
  return problem == QQA_MIS || problem == QQA_MAXCUT || problem == QQA_MAXCLIQUE || problem == QQA_COLORING;
}
// Split plan for rows with more than kHubDegree neighbours (see qqa_internal.h).
void build_hub_plan(const int32_t* row_ptr, int n, std::vector<HubChunk>* chunks, std::vector<int32_t>* hub_first);

// Free list over hipMalloc (device) or hipHostMalloc (pinned host), safe to use from
// several threads.  Sizes are rounded up to a size class (eight classes per power of two,
// at most 12.5% above the request) so that buffers of nearby sizes are reused, and the
// bytes held in the free list are capped: a buffer put back beyond the cap is freed at
// once.  A failed allocation frees every cached buffer and tries once more.
class Pool {
 public:
  explicit Pool(bool pinned, size_t cap_bytes) : pinned_(pinned), cap_(cap_bytes) {}
  ~Pool() = default;
  Pool(const Pool&) = delete;
  Pool& operator=(const Pool&) = delete;
  // the bytes a request of `bytes` takes in the pool
  static size_t class_size(size_t bytes);
  hipError_t get(size_t bytes, void** out);
  void put(void* p, size_t bytes);
  void trim();
  size_t held() const;        // every byte the pool has allocated and not freed
  size_t cached() const;      // of which idle in the free list
  void set_cap(size_t bytes);

 private:
  void release_locked(std::multimap<size_t, void*>::iterator it);
  bool pinned_;
  size_t cap_;
  size_t held_ = 0, cached_ = 0;
  std::multimap<size_t, void*> free_;
  mutable std::mutex mu_;
};

}  // namespace qqa
