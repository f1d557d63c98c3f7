// nn_mixed.cpp — mixed-precision NN schedule (BF16 -> FP32 -> FP64).
#include "nn_internal.h"

namespace nn {

size_t mixed_workspace_size(int64_t n, const nn_params* prm) {
  (void)n;
  (void)prm;
  return 0;
}

nn_status run_mixed(nn_ctx*, const void*, int64_t, void*, int64_t, int64_t, const nn_params*,
                    void*, size_t, nn_info*) {
  return NN_ERR_UNSUPPORTED;
}

}  // namespace nn
