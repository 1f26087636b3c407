// Internal host-runtime declarations shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
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

// Size-keyed free list over hipMalloc (device) or hipHostMalloc (pinned host).
class Pool {
 public:
  explicit Pool(bool pinned) : pinned_(pinned) {}
  hipError_t get(size_t bytes, void** out);
  void put(void* p, size_t bytes);
  void trim();
  size_t held() const { return held_; }

 private:
  bool pinned_;
  size_t held_ = 0;
  std::multimap<size_t, void*> free_;
};

}  // namespace qqa
