// Explicit kernel instantiations and lookup tables for one element type and
// one kernel family.  Included by sph_kernels_<family>_<type>.hip with
// SPH_T, SPH_SUFFIX and SPH_FAMILY (1 = forward, 2 = backward and double
// backward) defined.
#include <utility>

#include "sph_bwd.inl"
#include "sph_dbwd.inl"
#include "sph_fwd.inl"

#define SPH_CAT2(a, b) a##b
#define SPH_CAT(a, b) SPH_CAT2(a, b)

namespace sph {
namespace {

using T = SPH_T;
using Buckets = std::make_integer_sequence<int, kNumBuckets>;
bool in_range(int L) { return L >= 0 && L <= kMaxL; }

#if SPH_FAMILY == 1
template <bool NORM, int V, int... Is>
void fill_fwd(const void** out, std::integer_sequence<int, Is...>) {
  constexpr int B = kBudgets<T>[V];
  const void* tbl[] = {reinterpret_cast<const void*>(&k_fwd<T, kBuckets[Is], NORM, B>)...};
  for (size_t i = 0; i < sizeof...(Is); ++i) out[i] = tbl[i];
}

struct Tables {
  const void* fwd[2][kNumBudgetVariants][kNumBuckets];
  Tables() {
    fill_fwd<false, 0>(fwd[0][0], Buckets{});
    fill_fwd<false, 1>(fwd[0][1], Buckets{});
    fill_fwd<true, 0>(fwd[1][0], Buckets{});
    fill_fwd<true, 1>(fwd[1][1], Buckets{});
  }
};
#else
template <bool NORM, int... Is>
void fill_dbwd(const void** out, std::integer_sequence<int, Is...>) {
  const void* tbl[] = {reinterpret_cast<const void*>(&k_dbwd<T, kBuckets[Is], NORM>)...};
  for (size_t i = 0; i < sizeof...(Is); ++i) out[i] = tbl[i];
}

struct Tables {
  const void* dbwd[2][kNumBuckets];
  const void* bwd;
  Tables() {
    fill_dbwd<false>(dbwd[0], Buckets{});
    fill_dbwd<true>(dbwd[1], Buckets{});
    bwd = reinterpret_cast<const void*>(&k_bwd<T>);
  }
};
#endif

const Tables& tables() {
  static const Tables t;
  return t;
}

}  // namespace

#if SPH_FAMILY == 1
KernelInfo SPH_CAT(fwd_info_, SPH_SUFFIX)(int L, int normalize, int variant) {
  if (!in_range(L) || (normalize != 0 && normalize != 1) || variant < 0 ||
      variant >= kNumBudgetVariants)
    return KernelInfo{nullptr, 0, 0};
  const int b = kBudgets<T>[variant];
  return KernelInfo{tables().fwd[normalize][variant][bucket_index(L)],
                    sizeof(T) * kWave * static_cast<size_t>(plan_stride(L, b)), b};
}
#else
KernelInfo SPH_CAT(bwd_info_, SPH_SUFFIX)(int L) {
  if (!in_range(L)) return KernelInfo{nullptr, 0, 0};
  return KernelInfo{tables().bwd, 0, kBwdChunk<T>};
}

KernelInfo SPH_CAT(dbwd_info_, SPH_SUFFIX)(int L, int normalize) {
  if (!in_range(L) || (normalize != 0 && normalize != 1)) return KernelInfo{nullptr, 0, 0};
  const int b = kDbwdBudget<T>;
  return KernelInfo{tables().dbwd[normalize][bucket_index(L)],
                    sizeof(T) * kWave * static_cast<size_t>(plan_stride(L, b)), b};
}
#endif

}  // namespace sph
