// Explicit kernel instantiations and lookup tables for one element type and
// one kernel family.  Included by the sph_kernels_*.hip translation units with
// SPH_T, SPH_SUFFIX and SPH_FAMILY defined: 1 = values-only forward and 3 =
// forward with derivatives (mode SPH_MODE), both for one normalisation
// SPH_NORM; 2 = backward and double backward.
#include <utility>

#include "sph_bwd.inl"
#include "sph_dbwd.inl"
#include "sph_fwd.inl"
#include "sph_fwd4.inl"

#define SPH_CAT2(a, b) a##b
#define SPH_CAT(a, b) SPH_CAT2(a, b)

namespace sph {
namespace {

using T = SPH_T;
using Buckets = std::make_integer_sequence<int, kNumBuckets>;
bool in_range(int L) { return L >= 0 && L <= kMaxL; }

#if SPH_FAMILY == 1 || SPH_FAMILY == 3
constexpr bool kNorm = SPH_NORM != 0;
// l_max <= 12 (float) and l_max <= 8 (double) are specialised at compile
// time (degree loops unrolled, coefficients as literals, order-m terms
// tabulated); larger l_max use the run-time-degree kernel of the smallest
// m-extent bucket that covers l_max.
constexpr int kSpecMax = std::is_same_v<T, float> ? 12 : 8;
constexpr int kSpecSlots = kSpecMax + 1 > 0 ? kSpecMax + 1 : 1;

#if SPH_FAMILY == 1
template <int MM, int LT>
const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&k_fwd<T, MM, LT, kNorm>);
}
template <int LT>
const void* alt_ptr() {
  return nullptr;
}
#else
constexpr bool kFused = SPH_MODE != kDerivStore;
constexpr bool kStore = SPH_MODE != kDerivFused;
template <int MM, int LT>
const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&k_fwd4<T, MM, LT, kNorm, kFused, kStore, quad_waves<T>(LT)>);
}
// The compile-time kernel on a one-wave tile where the default takes two.
template <int LT>
const void* alt_ptr() {
  if constexpr (quad_waves<T>(LT) == 2)
    return reinterpret_cast<const void*>(&k_fwd4<T, LT, LT, kNorm, kFused, kStore, 1>);
  else
    return nullptr;
}
#endif

template <int... Ls>
void fill_spec(const void** out, const void** alt, std::integer_sequence<int, Ls...>) {
  if constexpr (kSpecMax >= 0) {
    const void* v[] = {kernel_ptr<Ls, Ls>()...};
    const void* a[] = {alt_ptr<Ls>()...};
    for (size_t i = 0; i < sizeof...(Ls); ++i) {
      out[i] = v[i];
      alt[i] = a[i];
    }
  }
}

template <int... Is>
void fill_buckets(const void** out, std::integer_sequence<int, Is...>) {
  const void* v[] = {kernel_ptr<kBuckets[Is], -1>()...};
  for (size_t i = 0; i < sizeof...(Is); ++i) out[i] = v[i];
}

struct Tables {
  const void* spec[kSpecSlots] = {};
  const void* spec_alt[kSpecSlots] = {};
  const void* buckets[kNumBuckets] = {};
  Tables() {
    if constexpr (kSpecMax >= 0) fill_spec(spec, spec_alt, std::make_integer_sequence<int, kSpecSlots>{});
    fill_buckets(buckets, Buckets{});
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
  const void* bwd[2];  // one and two waves per block
  Tables() {
    fill_dbwd<false>(dbwd[0], Buckets{});
    fill_dbwd<true>(dbwd[1], Buckets{});
    bwd[0] = reinterpret_cast<const void*>(&k_bwd<T, 1>);
    bwd[1] = reinterpret_cast<const void*>(&k_bwd<T, 2>);
  }
};
#endif

const Tables& tables() {
  static const Tables t;
  return t;
}

#if SPH_FAMILY == 1 || SPH_FAMILY == 3
// Kernel of a variant (see FwdVariant) and its tile width in waves.
const void* pick(int L, int variant, int& nw, bool quad) {
  const bool ct = L <= kSpecMax;
  nw = 1;
  switch (variant) {
    case kVarDefault:
      if (ct && quad) nw = quad_waves<T>(L);
      return ct ? tables().spec[L] : tables().buckets[bucket_index(L)];
    case kVarTile16:
      return ct ? tables().spec_alt[L] : nullptr;
    case kVarRuntime:
      return ct ? tables().buckets[bucket_index(L)] : nullptr;
    default:
      return nullptr;
  }
}
#endif

}  // namespace

#if SPH_FAMILY == 1
KernelInfo SPH_CAT(SPH_CAT(SPH_CAT(fwd_values_, SPH_SUFFIX), _n), SPH_NORM)(int L, int variant) {
  if (!in_range(L)) return KernelInfo{nullptr, 0, 0, 0, 0};
  int nw = 1;
  const void* fn = pick(L, variant, nw, false);
  if (fn == nullptr) return KernelInfo{nullptr, 0, 0, 0, 0};
  const size_t lds = sizeof(T) * kWave * static_cast<size_t>(plan_stride(L, kValueBudget<T>));
  return KernelInfo{fn, lds, lds, kWave, kWave};
}
#elif SPH_FAMILY == 3
KernelInfo SPH_CAT(SPH_CAT(SPH_CAT(SPH_CAT(SPH_CAT(fwd_derivs_, SPH_SUFFIX), _n), SPH_NORM), _m), SPH_MODE)(
    int L, int variant) {
  if (!in_range(L)) return KernelInfo{nullptr, 0, 0, 0, 0};
  int nw = 1;
  const void* fn = pick(L, variant, nw, true);
  if (fn == nullptr) return KernelInfo{nullptr, 0, 0, 0, 0};
  const size_t row = sizeof(T) * static_cast<size_t>(plan_stride(L, kQuadBudget<T>));
  const int pts = kQuadWavePoints * nw, thr = kWave * nw;
  return KernelInfo{fn, row * static_cast<size_t>(4 * pts), row * static_cast<size_t>(5 * pts), pts, thr};
}
#else
KernelInfo SPH_CAT(bwd_info_, SPH_SUFFIX)(int L) {
  if (!in_range(L)) return KernelInfo{nullptr, 0, 0, 0, 0};
  const int nw = bwd_waves<T>((L + 1) * (L + 1));
  return KernelInfo{tables().bwd[nw - 1], 0, 0, 16 * nw, kWave * nw};
}

KernelInfo SPH_CAT(dbwd_info_, SPH_SUFFIX)(int L, int normalize) {
  if (!in_range(L) || (normalize != 0 && normalize != 1)) return KernelInfo{nullptr, 0, 0, 0, 0};
  const size_t lds = sizeof(T) * kWave * static_cast<size_t>(plan_stride(L, kDbwdBudget<T>));
  return KernelInfo{tables().dbwd[normalize][bucket_index(L)], lds, lds, kWave, kWave};
}
#endif

}  // namespace sph
