// hf_mlp.hip -- learned cost model of the fused-kernel tuner (placeholder until
// the training and inference kernels land).
#include "hf_runtime.hpp"

namespace hf {
int mlp_rank(DeviceState*, const hf_pair*, const std::vector<hf_config>&, std::vector<int>*) {
  return HF_ENOMODEL;
}
}  // namespace hf
