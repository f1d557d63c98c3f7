// nn_batched.cpp — C ABI of the batched persistent inversion.
#include "nn_internal.h"

extern "C" {

size_t nn_batched_workspace_size(int32_t batch, nn_dtype dtype) {
  (void)batch;
  (void)dtype;
  return 0;
}

nn_status nn_invert_batched(nn_ctx*, const void*, void*, const int64_t*, const int32_t*, int32_t,
                            int32_t, nn_dtype, const nn_params*, void*, size_t, nn_info_dev*) {
  return NN_ERR_UNSUPPORTED;
}

}  // extern "C"
