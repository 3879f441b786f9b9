// Batched instances in one persistent launch (placeholder until the
// persistent kernel lands): every entry point validates and reports
// CG_EUNSUPPORTED.
#include <string.h>

#include "countgauss.h"
#include "cg_internal.hpp"

extern "C" {

int cg_batched_plan(cg_instance* inst, int32_t count, const cg_opts* opts,
                    size_t* workspace_bytes) {
  (void)inst; (void)count; (void)opts; (void)workspace_bytes;
  return CG_EUNSUPPORTED;
}

int cg_sketch_batched(const cg_instance* inst, int32_t count, const cg_opts* opts) {
  (void)inst; (void)count; (void)opts;
  return CG_EUNSUPPORTED;
}

int cg_set_tuning(const int32_t* rows_per_item, const int32_t* kc_per_item, int32_t classes) {
  (void)rows_per_item; (void)kc_per_item; (void)classes;
  return CG_EUNSUPPORTED;
}

}  // extern "C"
