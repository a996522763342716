// explicit Hessian kernels, float
#include <utility>

#include "sph_hess.inl"

namespace sph {
namespace {

using T = float;

// The degree-split block, for the buckets whose smallest l_max still fits a
// point's nine rows in one group of degrees.
template <bool NORM, int I>
const void* split_ptr() {
  constexpr int lo = I == 0 ? 0 : kBuckets[I - 1] + 1;
  if constexpr (group_end(0, lo, kHessBudget<T>) > lo)
    return reinterpret_cast<const void*>(&k_hess<T, kBuckets[I], NORM, 2>);
  else
    return nullptr;
}

template <bool NORM, int... Is>
void fill(const void** one, const void** split, std::integer_sequence<int, Is...>) {
  const void* a[] = {reinterpret_cast<const void*>(&k_hess<T, kBuckets[Is], NORM, 1>)...};
  const void* b[] = {split_ptr<NORM, Is>()...};
  for (size_t i = 0; i < sizeof...(Is); ++i) {
    one[i] = a[i];
    split[i] = b[i];
  }
}

struct Tables {
  const void* one[2][kNumBuckets];
  const void* split[2][kNumBuckets];
  Tables() {
    fill<false>(one[0], split[0], std::make_integer_sequence<int, kNumBuckets>{});
    fill<true>(one[1], split[1], std::make_integer_sequence<int, kNumBuckets>{});
  }
};

const Tables& tables() {
  static const Tables t;
  return t;
}

}  // namespace

KernelInfo hess_info_f32(int L, int normalize) {
  if (L < 0 || L > kMaxLmax || (normalize != 0 && normalize != 1)) return KernelInfo{nullptr, 0, 0, 0, 0};
  const Tables& t = tables();
  const int b = bucket_index(L);
  const size_t lds = sizeof(T) * static_cast<size_t>(kHessPoints * 9 * tile_stride<T>(L, kHessBudget<T>));
  const bool one_group = group_end(0, L, kHessBudget<T>) > L;
  if (one_group && t.split[normalize][b] != nullptr)
    return KernelInfo{t.split[normalize][b], lds, lds, kHessPoints, 2 * kWave};
  return KernelInfo{t.one[normalize][b], lds, lds, kHessPoints, kWave};
}

}  // namespace sph
