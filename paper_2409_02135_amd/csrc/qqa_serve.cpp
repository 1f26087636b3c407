// Ragged multi-instance batches and the continuous-batching server.
#include <hip/hip_runtime.h>

#include "qqa.h"
#include "qqa_ctx.h"

using namespace qqa;

namespace qqa {
struct Server {};

int serve_poll(qqa_ctx*, int64_t, qqa_result*, int32_t) { return QQA_E_UNKNOWN_REQ; }
int serve_cancel(qqa_ctx*, int64_t) { return QQA_E_UNKNOWN_REQ; }
}  // namespace qqa

qqa_ctx::qqa_ctx() = default;
qqa_ctx::~qqa_ctx() = default;

extern "C" {

int qqa_solve_batch(qqa_ctx* c, int32_t, const qqa_graph_id*, const qqa_problem*, const qqa_schedule*, const int32_t*,
                    const int32_t*, const uint64_t*, qqa_req*) {
  return c ? set_err(c, QQA_E_ARG, "batched solves are not available in this build") : QQA_E_ARG;
}

int qqa_serve_start(qqa_ctx* c, int32_t) {
  return c ? set_err(c, QQA_E_ARG, "the server is not available in this build") : QQA_E_ARG;
}

int qqa_serve_submit(qqa_ctx* c, const qqa_graph*, qqa_problem, const qqa_schedule*, int32_t, int32_t, uint64_t,
                     qqa_req*) {
  return c ? set_err(c, QQA_E_ARG, "the server is not available in this build") : QQA_E_ARG;
}

int qqa_serve_stop(qqa_ctx* c) { return c ? QQA_OK : QQA_E_ARG; }

}  // extern "C"
