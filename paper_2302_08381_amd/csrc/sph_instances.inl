// Explicit kernel instantiations and lookup tables for one element type and
// one kernel family.  Included by the sph_kernels_*.hip translation units with
// SPH_T, SPH_SUFFIX and SPH_FAMILY defined: 1 = values-only forward and 3 =
// forward with derivatives (mode SPH_MODE), both for one normalisation
// SPH_NORM; 2 = backward and double backward.
#include <utility>

#include "sph_bwd.inl"
#include "sph_dbwd.inl"
#include "sph_fwd.inl"
#include "sph_fwd1.inl"
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
template <int LT>
const void* split_ptr() {
  return nullptr;
}
template <int MM>
const void* split_rt_ptr() {
  return nullptr;
}
template <int LT>
const void* lane_ptr() {
  return nullptr;
}
#else
constexpr bool kFused = SPH_MODE != kDerivStore;
constexpr bool kStore = SPH_MODE != kDerivFused;
template <int MM, int LT>
const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&k_fwd4<T, MM, LT, kNorm, kFused, kStore, quad_waves<T>(LT), 1>);
}
// The compile-time kernel on an unsplit one-wave tile.
template <int LT>
const void* alt_ptr() {
  return reinterpret_cast<const void*>(&k_fwd4<T, LT, LT, kNorm, kFused, kStore, 1, 1>);
}
// The compile-time one-wave tile with its degrees split between two waves
// (l_max >= 4, where the default tile is one wave).
template <int LT>
const void* split_ptr() {
  if constexpr (quad_waves<T>(LT) == 1 && LT >= 4)
    return reinterpret_cast<const void*>(&k_fwd4<T, LT, LT, kNorm, kFused, kStore, 1, 2>);
  else
    return nullptr;
}
// The run-time-degree kernel with each group's degrees split between two
// waves (no fused backward).
template <int MM>
const void* split_rt_ptr() {
  if constexpr (!kFused)
    return reinterpret_cast<const void*>(&k_fwd4<T, MM, -1, kNorm, kFused, kStore, 1, 2>);
  else
    return nullptr;
}
// The one-lane kernel (l_max <= 3).
template <int LT>
const void* lane_ptr() {
  if constexpr (LT <= kLaneMaxL)
    return reinterpret_cast<const void*>(&k_fwd1<T, LT, kNorm, kFused, kStore>);
  else
    return nullptr;
}
#endif

template <int... Ls>
void fill_spec(const void** out, const void** alt, const void** split, const void** lane,
               std::integer_sequence<int, Ls...>) {
  if constexpr (kSpecMax >= 0) {
    const void* v[] = {kernel_ptr<Ls, Ls>()...};
    const void* a[] = {alt_ptr<Ls>()...};
    const void* d[] = {split_ptr<Ls>()...};
    const void* o[] = {lane_ptr<Ls>()...};
    for (size_t i = 0; i < sizeof...(Ls); ++i) {
      out[i] = v[i];
      alt[i] = a[i];
      split[i] = d[i];
      lane[i] = o[i];
    }
  }
}

template <int... Is>
void fill_buckets(const void** out, const void** split, std::integer_sequence<int, Is...>) {
  const void* v[] = {kernel_ptr<kBuckets[Is], -1>()...};
  const void* d[] = {split_rt_ptr<kBuckets[Is]>()...};
  for (size_t i = 0; i < sizeof...(Is); ++i) {
    out[i] = v[i];
    split[i] = d[i];
  }
}

struct Tables {
  const void* spec[kSpecSlots] = {};
  const void* spec_alt[kSpecSlots] = {};
  const void* spec_split[kSpecSlots] = {};
  const void* spec_lane[kSpecSlots] = {};
  const void* buckets[kNumBuckets] = {};
  const void* buckets_split[kNumBuckets] = {};
  Tables() {
    if constexpr (kSpecMax >= 0)
      fill_spec(spec, spec_alt, spec_split, spec_lane, std::make_integer_sequence<int, kSpecSlots>{});
    fill_buckets(buckets, buckets_split, Buckets{});
  }
};

#else
// Double backward: one wave per 64-point tile, or (one group of degrees:
// l_max <= 12 float, <= 8 double) the degree-split block of two waves.
constexpr int kDbwdSplitMax = std::is_same_v<T, float> ? 12 : 8;

template <bool NORM, int MM, int DS>
const void* dbwd_ptr() {
  if constexpr (DS == 2 && MM > kDbwdSplitMax)
    return nullptr;
  else
    return reinterpret_cast<const void*>(&k_dbwd<T, MM, NORM, DS>);
}

template <bool NORM, int DS, int... Is>
void fill_dbwd(const void** out, std::integer_sequence<int, Is...>) {
  const void* tbl[] = {dbwd_ptr<NORM, kBuckets[Is], DS>()...};
  for (size_t i = 0; i < sizeof...(Is); ++i) out[i] = tbl[i];
}

struct Tables {
  const void* dbwd[2][kNumBuckets];
  const void* dbwd_split[2][kNumBuckets];
  const void* bwd[2];  // one and two waves per block
  Tables() {
    fill_dbwd<false, 1>(dbwd[0], Buckets{});
    fill_dbwd<true, 1>(dbwd[1], Buckets{});
    fill_dbwd<false, 2>(dbwd_split[0], Buckets{});
    fill_dbwd<true, 2>(dbwd_split[1], Buckets{});
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
// Whether the degree-split tile is the default for a compile-time l_max.
// Measured against the unsplit one-wave tile (Y+dY, N = 1e6): faster for
// float l_max 9, 11, 12 (18-28 %) and double 5, 7, 8 (7-17 %), even for
// double 6, 5 % slower for float 10.
bool split_by_default(int L) {
  return std::is_same_v<T, float> ? (L >= 9 && L != 10) : L >= 5;
}

// Kernel of a variant (see FwdVariant), its tile width in waves and its
// degree-split factor (waves per tile width).
const void* pick(int L, int variant, int& nw, int& ds, bool quad) {
  const bool ct = L <= kSpecMax;
  nw = 1;
  ds = 1;
  switch (variant) {
    case kVarDefault:
      // l_max <= 1: one lane per point.  GPU time on 1.36 M points (graph
      // replays, one tile per block), against the quad-lane tile: float
      // Y+dY 7.2 vs 17.2 us (l_max 0), 15.6 vs 19.7 us (1); with the fused
      // backward 13.8 vs 24.8 and 25.5 vs 32.8 us; double within 5 % or
      // faster.  At l_max 2 and 3 the two are even without the backward.
      if (ct && quad && L <= 1 && tables().spec_lane[L] != nullptr) {
        nw = 0;
        return tables().spec_lane[L];
      }
      if (ct && quad && tables().spec_split[L] != nullptr && split_by_default(L)) {
        ds = 2;
        return tables().spec_split[L];
      }
      // run-time degrees: the split groups measured 27-34 % faster (float
      // l_max 16 and 32, double 16); the fused backward has no split form
      if (!ct && quad && tables().buckets_split[bucket_index(L)] != nullptr) {
        ds = 2;
        return tables().buckets_split[bucket_index(L)];
      }
      if (ct && quad) nw = quad_waves<T>(L);
      return ct ? tables().spec[L] : tables().buckets[bucket_index(L)];
    case kVarTile16:
      return ct ? tables().spec_alt[L] : nullptr;
    case kVarRuntime:  // the unsplit run-time-degree kernel
      return (ct || quad) ? tables().buckets[bucket_index(L)] : nullptr;
    case kVarSplit:
      ds = 2;
      return ct ? tables().spec_split[L] : tables().buckets_split[bucket_index(L)];
    case kVarLane:  // nw = 0 marks the one-lane kernel
      nw = 0;
      return quad && ct ? tables().spec_lane[L] : nullptr;
    default:
      return nullptr;
  }
}
#endif

}  // namespace

#if SPH_FAMILY == 1
KernelInfo SPH_CAT(SPH_CAT(SPH_CAT(fwd_values_, SPH_SUFFIX), _n), SPH_NORM)(int L, int variant) {
  if (!in_range(L)) return KernelInfo{nullptr, 0, 0, 0, 0};
  int nw = 1, ds = 1;
  const void* fn = pick(L, variant, nw, ds, false);
  if (fn == nullptr) return KernelInfo{nullptr, 0, 0, 0, 0};
  const size_t lds = sizeof(T) * kWave * static_cast<size_t>(tile_stride<T>(L, kValueBudget<T>));
  return KernelInfo{fn, lds, lds, kWave, kWave};
}
#elif SPH_FAMILY == 3
KernelInfo SPH_CAT(SPH_CAT(SPH_CAT(SPH_CAT(SPH_CAT(fwd_derivs_, SPH_SUFFIX), _n), SPH_NORM), _m), SPH_MODE)(
    int L, int variant) {
  if (!in_range(L)) return KernelInfo{nullptr, 0, 0, 0, 0};
  int nw = 1, ds = 1;
  const void* fn = pick(L, variant, nw, ds, true);
  if (fn == nullptr) return KernelInfo{nullptr, 0, 0, 0, 0};
  const size_t row = sizeof(T) * static_cast<size_t>(tile_stride<T>(L, kQuadBudget<T>));
  if (nw == 0)  // one lane per point: 4 * 64 rows, plus 64 gY rows when fused
    return KernelInfo{fn, row * static_cast<size_t>(4 * kWave), row * static_cast<size_t>(5 * kWave), kWave, kWave};
  const int pts = kQuadWavePoints * nw, thr = kWave * nw * ds;
  // fused: the upstream-gradient tile, and the split kernel's partial sums
  const size_t fused = row * static_cast<size_t>(5 * pts) + (ds == 2 ? sizeof(T) * kWave : 0);
  return KernelInfo{fn, row * static_cast<size_t>(4 * pts), fused, pts, thr};
}
#else
KernelInfo SPH_CAT(bwd_info_, SPH_SUFFIX)(int L) {
  if (!in_range(L)) return KernelInfo{nullptr, 0, 0, 0, 0};
  const int K = (L + 1) * (L + 1);
  const int nw = bwd_waves<T>(K);
  const int stride = nw == 2 ? bwd_stride<T, 2>(K) : bwd_stride<T, 1>(K);
  const size_t lds = sizeof(T) * static_cast<size_t>(4 * 16 * nw * stride);  // sized by K: small l_max fit more blocks
  // The pipelined loop over tiles runs on a resident grid, except for float
  // tiles too wide for four blocks in a CU's 160 KiB of LDS (l_max = 8:
  // three blocks, 215 us resident against 202 us at one tile per block; at
  // l_max 4 and 6, where the waves bound residency, the resident grid is
  // 3-22 % faster, as it is for double at l_max = 8).
  const bool pipe = nw == 2 ? kBwdPipe<T, 2> : kBwdPipe<T, 1>;
  const bool lds_bound = std::is_same_v<T, float> && 4 * lds > 160 * 1024;
  const int bpc = pipe && !lds_bound ? 1 : 0;
  return KernelInfo{tables().bwd[nw - 1], lds, lds, 16 * nw, kWave * nw, bpc};
}

KernelInfo SPH_CAT(dbwd_info_, SPH_SUFFIX)(int L, int normalize) {
  if (!in_range(L) || (normalize != 0 && normalize != 1)) return KernelInfo{nullptr, 0, 0, 0, 0};
  const size_t lds = sizeof(T) * kWave * static_cast<size_t>(tile_stride<T>(L, kDbwdBudget<T>));
  const bool one_group = group_end(0, L, kDbwdBudget<T>) > L;
  const void* split = tables().dbwd_split[normalize][bucket_index(L)];
  if (one_group && split != nullptr)  // + wave 1's Hessian sums
    return KernelInfo{split, lds + 3 * kWave * sizeof(T), lds + 3 * kWave * sizeof(T), kWave, 2 * kWave};
  return KernelInfo{tables().dbwd[normalize][bucket_index(L)], lds, lds, kWave, kWave};
}
#endif

}  // namespace sph
