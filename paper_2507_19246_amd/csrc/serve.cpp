// Continuous-batching request server (placeholder until the scheduler lands).
#include "mq_internal.h"

extern "C" {
int mq_server_create(const mq_server_desc*, void*, mq_server** out) {
  if (out) *out = nullptr;
  return MQ_ERR_INVALID_ARG;
}
int mq_submit(mq_server*, const mq_request*, uint64_t*) { return MQ_ERR_INVALID_ARG; }
int mq_poll(mq_server*, mq_result*, int32_t, int32_t* n_out) {
  if (n_out) *n_out = 0;
  return MQ_ERR_INVALID_ARG;
}
int mq_server_pending(const mq_server*, int32_t* n) {
  if (n) *n = 0;
  return MQ_ERR_INVALID_ARG;
}
int mq_server_destroy(mq_server*) { return MQ_OK; }
}
