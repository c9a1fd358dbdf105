// stubs.hip -- entry points not yet implemented (return FTK_ERR_ARG with a message).
#include <hip/hip_runtime.h>

#include "../../include/ftk.h"

extern "C" {
ftk_status ftk_cp_create(int32_t, const int64_t*, ftk_field_kind, const ftk_options*, ftk_stream_t, ftk_tracker** h) {
  if (h) *h = nullptr;
  return FTK_ERR_ARG;
}
ftk_status ftk_cp_push(ftk_tracker*, const float*) { return FTK_ERR_STATE; }
ftk_status ftk_cp_finish(ftk_tracker*, ftk_cp_result*) { return FTK_ERR_STATE; }
void ftk_cp_destroy(ftk_tracker*) {}
ftk_status ftk_track_cp2d_batched(int32_t, const float* const*, const int64_t*, const int64_t*, const int64_t*,
                                  ftk_field_kind, const ftk_options*, ftk_stream_t, ftk_cp_result*) {
  return FTK_ERR_ARG;
}
}
