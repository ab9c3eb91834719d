// km_server.cpp -- continuous-batching server (placeholder until implemented).
#include "../../include/kmeans.h"

extern "C" {
int32_t kmeans_server_create(km_context*, size_t, int32_t, km_server** out) {
  if (out) *out = nullptr;
  return KM_ERR_UNSUPPORTED;
}
int32_t kmeans_submit(km_server*, const km_problem*, const km_precision*, uint64_t*) { return KM_ERR_UNSUPPORTED; }
int32_t kmeans_poll(km_server*, uint64_t, int32_t) { return KM_ERR_UNSUPPORTED; }
int32_t kmeans_cancel(km_server*, uint64_t) { return KM_ERR_UNSUPPORTED; }
int32_t kmeans_server_destroy(km_server*) { return KM_ERR_UNSUPPORTED; }
}
