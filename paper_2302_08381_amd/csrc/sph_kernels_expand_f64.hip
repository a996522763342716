// radial expansion kernels, double
#include <utility>

#include "sph_expand.inl"

namespace sph {
namespace {

using T = double;

// l_max <= 8: compile-time degrees; larger: the run-time-degree kernel of
// the m-extent bucket.
constexpr int kSpecMax = 8;

template <bool NORM, int... Is>
void fill_expand(const void** out, std::integer_sequence<int, Is...>) {
  const void* tbl[] = {reinterpret_cast<const void*>(&k_expand<T, kBuckets[Is], -1, NORM>)...};
  for (size_t i = 0; i < sizeof...(Is); ++i) out[i] = tbl[i];
}

template <bool NORM, int... Ls>
void fill_spec(const void** out, std::integer_sequence<int, Ls...>) {
  const void* tbl[] = {reinterpret_cast<const void*>(&k_expand<T, Ls, Ls, NORM>)...};
  for (size_t i = 0; i < sizeof...(Ls); ++i) out[i] = tbl[i];
}

struct Tables {
  const void* fn[2][kNumBuckets];
  const void* spec[2][kSpecMax + 1];
  Tables() {
    fill_expand<false>(fn[0], std::make_integer_sequence<int, kNumBuckets>{});
    fill_expand<true>(fn[1], std::make_integer_sequence<int, kNumBuckets>{});
    fill_spec<false>(spec[0], std::make_integer_sequence<int, kSpecMax + 1>{});
    fill_spec<true>(spec[1], std::make_integer_sequence<int, kSpecMax + 1>{});
  }
};

}  // namespace

KernelInfo expand_info_f64(int L, int normalize) {
  static const Tables t;
  if (L < 0 || L > kMaxLmax || (normalize != 0 && normalize != 1)) return KernelInfo{nullptr, 0, 0, 0, 0};
  const void* fn = L <= kSpecMax ? t.spec[normalize][L] : t.fn[normalize][bucket_index(L)];
  return KernelInfo{fn, 0, 0, 0, kExpandThreads};
}

}  // namespace sph
