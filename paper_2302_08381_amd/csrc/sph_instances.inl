// Explicit kernel instantiations and lookup tables for one element type and
// one kernel family.  Included by the sph_kernels_*.hip translation units with
// SPH_T, SPH_SUFFIX and SPH_FAMILY defined (1 = forward kernels for one
// normalisation SPH_NORM, 2 = backward and double backward).
#include <utility>

#include "sph_bwd.inl"
#include "sph_dbwd.inl"
#include "sph_fwd.inl"
#include "sph_fwd4.inl"

#define SPH_CAT2(a, b) a##b
#define SPH_CAT(a, b) SPH_CAT2(a, b)
#define SPH_CAT3(a, b, c) SPH_CAT(SPH_CAT(a, b), c)

namespace sph {
namespace {

using T = SPH_T;
using Buckets = std::make_integer_sequence<int, kNumBuckets>;
bool in_range(int L) { return L >= 0 && L <= kMaxL; }

#if SPH_FAMILY == 1
constexpr bool kNorm = SPH_NORM != 0;
// float32 specialises l_max <= 8 at compile time (degree loops unrolled,
// coefficients as literals); everything else uses the run-time-degree
// kernel of the smallest m-extent bucket that covers l_max.
constexpr int kSpecMax = std::is_same_v<T, float> ? 8 : -1;
constexpr int kSpecSlots = kSpecMax + 1 > 0 ? kSpecMax + 1 : 1;

template <int... Ls>
void fill_spec(const void** vals, const void** ders, std::integer_sequence<int, Ls...>) {
  if constexpr (kSpecMax >= 0) {
    const void* v[] = {reinterpret_cast<const void*>(&k_fwd<T, Ls, Ls, kNorm>)...};
    const void* d[] = {reinterpret_cast<const void*>(&k_fwd4<T, Ls, Ls, kNorm>)...};
    for (size_t i = 0; i < sizeof...(Ls); ++i) {
      vals[i] = v[i];
      ders[i] = d[i];
    }
  }
}

template <int... Is>
void fill_buckets(const void** vals, const void** ders, std::integer_sequence<int, Is...>) {
  const void* v[] = {reinterpret_cast<const void*>(&k_fwd<T, kBuckets[Is], -1, kNorm>)...};
  const void* d[] = {reinterpret_cast<const void*>(&k_fwd4<T, kBuckets[Is], -1, kNorm>)...};
  for (size_t i = 0; i < sizeof...(Is); ++i) {
    vals[i] = v[i];
    ders[i] = d[i];
  }
}

struct Tables {
  const void* spec_vals[kSpecSlots] = {};
  const void* spec_ders[kSpecSlots] = {};
  const void* vals[kNumBuckets] = {};
  const void* ders[kNumBuckets] = {};
  Tables() {
    if constexpr (kSpecMax >= 0) fill_spec(spec_vals, spec_ders, std::make_integer_sequence<int, kSpecSlots>{});
    fill_buckets(vals, ders, Buckets{});
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
KernelInfo SPH_CAT3(SPH_CAT(fwd_values_, SPH_SUFFIX), _n, SPH_NORM)(int L) {
  if (!in_range(L)) return KernelInfo{nullptr, 0, 0, 0};
  const void* fn = L <= kSpecMax ? tables().spec_vals[L] : tables().vals[bucket_index(L)];
  const size_t lds = sizeof(T) * kWave * static_cast<size_t>(plan_stride(L, kValueBudget<T>));
  return KernelInfo{fn, lds, lds, kWave};
}

KernelInfo SPH_CAT3(SPH_CAT(fwd_derivs_, SPH_SUFFIX), _n, SPH_NORM)(int L) {
  if (!in_range(L)) return KernelInfo{nullptr, 0, 0, 0};
  const void* fn = L <= kSpecMax ? tables().spec_ders[L] : tables().ders[bucket_index(L)];
  const size_t row = sizeof(T) * static_cast<size_t>(plan_stride(L, kQuadBudget<T>));
  return KernelInfo{fn, row * kWave, row * (kWave + kQuadPoints), kQuadPoints};
}
#else
KernelInfo SPH_CAT(bwd_info_, SPH_SUFFIX)(int L) {
  if (!in_range(L)) return KernelInfo{nullptr, 0, 0, 0};
  return KernelInfo{tables().bwd, 0, 0, kBwdPointsPerBlock};
}

KernelInfo SPH_CAT(dbwd_info_, SPH_SUFFIX)(int L, int normalize) {
  if (!in_range(L) || (normalize != 0 && normalize != 1)) return KernelInfo{nullptr, 0, 0, 0};
  const size_t lds = sizeof(T) * kWave * static_cast<size_t>(plan_stride(L, kDbwdBudget<T>));
  return KernelInfo{tables().dbwd[normalize][bucket_index(L)], lds, lds, kWave};
}
#endif

}  // namespace sph
