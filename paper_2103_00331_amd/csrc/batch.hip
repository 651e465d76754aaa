// Batched solver: placeholder entry points until the persistent kernel lands.
#include "handle.h"

extern "C" {
int cpmdp_batch_create(cpmdp_batch_t** out, cpmdp_t* const*, int32_t) {
  if (out) *out = nullptr;
  return cpm::fail(nullptr, CPMDP_E_UNSUPPORTED, "batched solver not built");
}
int cpmdp_batch_workspace_bytes(const cpmdp_batch_t*, size_t*) { return CPMDP_E_UNSUPPORTED; }
int cpmdp_batch_bind(cpmdp_batch_t*, void*, size_t, void*) { return CPMDP_E_UNSUPPORTED; }
int cpmdp_batch_solve(cpmdp_batch_t*, double* const*, int32_t* const*, double, int64_t, int, int,
                      int64_t*, double*) {
  return CPMDP_E_UNSUPPORTED;
}
int cpmdp_batch_autotune(cpmdp_batch_t*, int, const char*) { return CPMDP_E_UNSUPPORTED; }
int cpmdp_batch_config(const cpmdp_batch_t*, int32_t*, int32_t*) { return CPMDP_E_UNSUPPORTED; }
void cpmdp_batch_destroy(cpmdp_batch_t*) {}
}
