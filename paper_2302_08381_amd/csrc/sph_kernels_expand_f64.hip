// radial expansion kernels, double
#include <utility>

#include "sph_expand.inl"

namespace sph {
namespace {

using T = double;

template <bool NORM, int... Is>
void fill_expand(const void** out, std::integer_sequence<int, Is...>) {
  const void* tbl[] = {reinterpret_cast<const void*>(&k_expand<T, kBuckets[Is], NORM>)...};
  for (size_t i = 0; i < sizeof...(Is); ++i) out[i] = tbl[i];
}

struct Tables {
  const void* fn[2][kNumBuckets];
  Tables() {
    fill_expand<false>(fn[0], std::make_integer_sequence<int, kNumBuckets>{});
    fill_expand<true>(fn[1], std::make_integer_sequence<int, kNumBuckets>{});
  }
};

}  // namespace

KernelInfo expand_info_f64(int L, int normalize) {
  static const Tables t;
  if (L < 0 || L > kMaxLmax || (normalize != 0 && normalize != 1)) return KernelInfo{nullptr, 0, 0, 0, 0};
  return KernelInfo{t.fn[normalize][bucket_index(L)], 0, 0, 0, kExpandThreads};
}

}  // namespace sph
