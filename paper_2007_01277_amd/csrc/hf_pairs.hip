// hf_pairs.hip -- fused instantiations of one ordered pair of kernel kinds.
// Compiled once per pair with -DHF_KA=<kind> -DHF_KB=<kind> (HF_KA <= HF_KB), so
// the forty-five pairs build in parallel; each object exports hf_table_<KA>_<KB>.
#include "hf_kernels.hpp"

#if !defined(HF_KA) || !defined(HF_KB)
#error "compile with -DHF_KA=<kind> -DHF_KB=<kind>"
#endif

#define HF_CAT5(a, b, c, d, e) a##b##c##d##e
#define HF_TABLE_NAME(a, b) HF_CAT5(hf_table_, a, _, b, )

namespace hf {
HF_DEFINE_PAIR_TABLE(HF_KA, HF_KB, HF_TABLE_NAME(HF_KA, HF_KB))
}  // namespace hf
