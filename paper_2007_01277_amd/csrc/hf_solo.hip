// hf_solo.hip -- the original (unfused) kernels: every kind at every block size.
#include "hf_kernels.hpp"

namespace hf {

#define HF_SOLO_ENTRY(K, B) {K, -1, B, 0, reinterpret_cast<const void*>(&solo<BodyOf<K>::T, B>)},
#define HF_SOLO_KIND(K) HF_SOLO_ENTRY(K, 256) HF_SOLO_ENTRY(K, 512) HF_SOLO_ENTRY(K, 1024)

const KernelEntry* hf_table_solo(int* count) {
  static const KernelEntry tab[] = {HF_SOLO_KIND(0) HF_SOLO_KIND(1) HF_SOLO_KIND(2) HF_SOLO_KIND(3)
                                        HF_SOLO_KIND(4) HF_SOLO_KIND(5) HF_SOLO_KIND(6)
                                            HF_SOLO_KIND(7) HF_SOLO_KIND(8)};
  *count = (int)(sizeof(tab) / sizeof(tab[0]));
  return tab;
}

}  // namespace hf
