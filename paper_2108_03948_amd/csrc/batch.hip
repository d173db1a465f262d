// Uneven batch API (persistent launch over a job table).
#include <hip/hip_runtime.h>

#include "internal.h"
#include "thzspec.h"

struct tz_batch {
  int unused;
};

extern "C" {
tz_status tz_batch_create(const tz_job *, int64_t, const tz_opts *, tz_batch **batch) {
  if (batch) *batch = nullptr;
  return TZ_EUNSUPPORTED;
}
tz_status tz_batch_launch(tz_batch *, const void *, void *, void *) { return TZ_EUNSUPPORTED; }
void tz_batch_destroy(tz_batch *) {}
}
