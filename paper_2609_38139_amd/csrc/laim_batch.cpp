// laim_batch.cpp -- batched persistent launch and serving loop (placeholder
// entry points until the implementations land).
#include "laim_internal.h"

using namespace laim;

extern "C" {
laim_status laim_batch_plan_create(const laim_batch_item*, int32_t, laim_stream, laim_batch_plan** out) {
  if (out) *out = nullptr;
  set_error("batched plans are not available in this build");
  return LAIM_EUNSUP;
}
laim_status laim_batch_plan_launch(laim_batch_plan*, laim_stream) {
  set_error("batched plans are not available in this build");
  return LAIM_EUNSUP;
}
void laim_batch_plan_destroy(laim_batch_plan*) {}
laim_status laim_server_create(int32_t, size_t, int32_t, laim_server** out) {
  if (out) *out = nullptr;
  set_error("the server is not available in this build");
  return LAIM_EUNSUP;
}
laim_status laim_server_submit(laim_server*, const laim_code*, const laim_decode_params*, uint64_t,
                               const uint8_t*, uint64_t*) { return LAIM_EUNSUP; }
laim_status laim_server_step(laim_server*, laim_server_event*, int32_t, int32_t*) { return LAIM_EUNSUP; }
laim_status laim_server_result(laim_server*, uint64_t, uint8_t*, uint8_t*, int32_t*) { return LAIM_EUNSUP; }
laim_status laim_server_stats(const laim_server*, int32_t*, int32_t*, size_t*) { return LAIM_EUNSUP; }
void laim_server_destroy(laim_server*) {}
}
