// radial expansion kernels, float
#include <utility>

#include "sph_expand.inl"

namespace sph {
namespace {

using T = float;

// l_max <= 12: compile-time degrees; larger: the run-time-degree kernel of
// the m-extent bucket.
constexpr int kSpecMax = 12;

template <bool NORM, int ACC, int... Is>
void fill_expand(const void** out, std::integer_sequence<int, Is...>) {
  const void* tbl[] = {reinterpret_cast<const void*>(&k_expand<T, kBuckets[Is], -1, NORM, ACC>)...};
  for (size_t i = 0; i < sizeof...(Is); ++i) out[i] = tbl[i];
}

template <bool NORM, int ACC, int... Ls>
void fill_spec(const void** out, std::integer_sequence<int, Ls...>) {
  const void* tbl[] = {reinterpret_cast<const void*>(&k_expand<T, Ls, Ls, NORM, ACC>)...};
  for (size_t i = 0; i < sizeof...(Ls); ++i) out[i] = tbl[i];
}

template <bool NORM, int NPC, int GS, bool STAGE, int... Is>
void fill_bwd(const void** out, std::integer_sequence<int, Is...>) {
  const void* tbl[] = {reinterpret_cast<const void*>(&k_expand_bwd<T, kBuckets[Is], NORM, NPC, GS, STAGE>)...};
  for (size_t i = 0; i < sizeof...(Is); ++i) out[i] = tbl[i];
}

struct Tables {
  const void* fn[2][2][kNumBuckets];  // [normalize][ACC == 8]
  const void* spec[2][2][kSpecMax + 1];
  const void* bwd[2][2][2][kNumBuckets];  // [normalize][NPC == 16][staged two groups, or one direct group]
  Tables() {
    fill_bwd<false, 8, 32, true>(bwd[0][0][0], std::make_integer_sequence<int, kNumBuckets>{});
    fill_bwd<true, 8, 32, true>(bwd[1][0][0], std::make_integer_sequence<int, kNumBuckets>{});
    fill_bwd<false, 16, 32, true>(bwd[0][1][0], std::make_integer_sequence<int, kNumBuckets>{});
    fill_bwd<true, 16, 32, true>(bwd[1][1][0], std::make_integer_sequence<int, kNumBuckets>{});
    fill_bwd<false, 8, 64, false>(bwd[0][0][1], std::make_integer_sequence<int, kNumBuckets>{});
    fill_bwd<true, 8, 64, false>(bwd[1][0][1], std::make_integer_sequence<int, kNumBuckets>{});
    fill_bwd<false, 16, 64, false>(bwd[0][1][1], std::make_integer_sequence<int, kNumBuckets>{});
    fill_bwd<true, 16, 64, false>(bwd[1][1][1], std::make_integer_sequence<int, kNumBuckets>{});
    fill_expand<false, 4>(fn[0][0], std::make_integer_sequence<int, kNumBuckets>{});
    fill_expand<true, 4>(fn[1][0], std::make_integer_sequence<int, kNumBuckets>{});
    fill_expand<false, 8>(fn[0][1], std::make_integer_sequence<int, kNumBuckets>{});
    fill_expand<true, 8>(fn[1][1], std::make_integer_sequence<int, kNumBuckets>{});
    fill_spec<false, 4>(spec[0][0], std::make_integer_sequence<int, kSpecMax + 1>{});
    fill_spec<true, 4>(spec[1][0], std::make_integer_sequence<int, kSpecMax + 1>{});
    fill_spec<false, 8>(spec[0][1], std::make_integer_sequence<int, kSpecMax + 1>{});
    fill_spec<true, 8>(spec[1][1], std::make_integer_sequence<int, kSpecMax + 1>{});
  }
};

const Tables& tables() {
  static const Tables t;
  return t;
}

}  // namespace

KernelInfo expand_info_f32(int L, int normalize, int n_max) {
  const Tables& t = tables();
  if (L < 0 || L > kMaxLmax || (normalize != 0 && normalize != 1) || n_max < 1) return KernelInfo{nullptr, 0, 0, 0, 0};
  const int a = expand_acc(L, n_max) == 8 ? 1 : 0;
  const void* fn = L <= kSpecMax ? t.spec[normalize][a][L] : t.fn[normalize][a][bucket_index(L)];
  return KernelInfo{fn, 0, 0, 0, kExpandThreads};
}

KernelInfo expand_bwd_info_f32(int L, int normalize, int n_max) {
  if (L < 0 || L > kMaxLmax || (normalize != 0 && normalize != 1) || n_max < 1 || n_max > 16)
    return KernelInfo{nullptr, 0, 0, 0, 0};
  const Tables& t = tables();
  const int w = n_max > 8 ? 1 : 0;
  const int npc = w ? 16 : 8;
  // Two staged groups of 32 lanes per wave where their G slices and radial
  // tiles take at most 32 KiB (five waves per CU), else one group of 64
  // lanes reading its rows directly, whose LDS holds only G.  Measured on
  // 20 000 environments: staged faster up to 29.8 KB (float32 l_max 8 with 8
  // channels 506 vs 517 us; float64 l_max 4, float32 16 channels l_max 4),
  // direct from 34 KB (float32 l_max 9 712 vs 546 us, l_max 12 1362 vs 773;
  // float64 l_max 8 1328 vs 678).  Padded channels (n_max < npc) copy
  // their tiles element by element, and float32 staging still paid at
  // 39-42 KB (12 channels l_max 6 1016 vs 1116 us, 5 channels l_max 10 873
  // vs 895) but not from 49 KB (l_max 12 1408 vs 1068); float64 lost at
  // 42 KB (5 channels l_max 6 692 vs 678).  The limit is the largest size
  // measured to gain, 42240 bytes.
  const size_t limit = n_max < npc && sizeof(T) == 4 ? 42240 : 32 * 1024;
  const int direct = expand_bwd_lds_bytes<T>(L, npc, 32, true) > limit ? 1 : 0;
  const int gs = direct ? 64 : 32;
  // one G slice per group where two would not fit (chunks then stop at
  // every environment's end)
  const int slices = expand_bwd_lds_bytes<T>(L, npc, gs, !direct, 2) <= 160 * 1024 ? 2 : 1;
  KernelInfo ki{t.bwd[normalize][w][direct][bucket_index(L)], expand_bwd_lds_bytes<T>(L, npc, gs, !direct, slices),
                0, 64 / gs, kWave};
  ki.slices = slices;
  return ki;
}

}  // namespace sph
