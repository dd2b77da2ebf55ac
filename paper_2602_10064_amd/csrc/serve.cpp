// Serving loop (continuous batching of jobs).  Placeholder until the loop lands.
#include "runtime.h"

using namespace tacaw;

extern "C" {

void tacaw_serve_shutdown(tacaw_ctx*) {}

tacaw_status tacaw_submit(tacaw_ctx*, tacaw_job*) {
  set_error("serving loop not built yet");
  return TACAW_EUNSUPPORTED;
}
tacaw_status tacaw_poll(tacaw_job*, int* done) {
  if (done) *done = 0;
  set_error("serving loop not built yet");
  return TACAW_EUNSUPPORTED;
}
tacaw_status tacaw_wait(tacaw_job*) {
  set_error("serving loop not built yet");
  return TACAW_EUNSUPPORTED;
}
tacaw_status tacaw_cancel(tacaw_job*) {
  set_error("serving loop not built yet");
  return TACAW_EUNSUPPORTED;
}
}
