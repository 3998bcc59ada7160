// Kernel lookup shared by the instantiation units and the C-ABI layer.
#pragma once

#include "hjpd_kernels.hpp"

namespace hjpd {

// Persistent tiles (lanes per point L, nodes per lane K) that are compiled.
// Capacity L*K bounds the N a tile can hold.
struct Tile { int L, K; };
inline constexpr Tile kTiles[] = {{8, 1},  {16, 1}, {8, 2},  {8, 3},  {32, 1}, {16, 2}, {8, 4},  {16, 3},
                                  {64, 1}, {32, 2}, {16, 4}, {32, 3}, {64, 2}, {32, 4}, {64, 3}, {64, 4}};
inline constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);
inline constexpr int kMaxCapacity = 256;

// Persistent kernel variants: the general kernels (k_group_control for the
// quadrotor, the game kernels), the control kernel with the robustness
// recipes, the eikonal family's weighted discretisations (forward Euler,
// trapezoid), and the eikonal family's shifted-layout kernel for Algorithms 1
// and 2 (which kVarPlain also selects for that family).
enum Variant { kVarPlain = 0, kVarRecipe = 1, kVarMix = 2, kVarShift = 3, kVarShiftHopf = 4, kVarGameLax = 5 };

template <typename T, class F, int L, int K>
const void* group_ptr(int variant) {
  if constexpr (F::kGame) {
    if constexpr (F::kGameHopf) {
      // scalar-player game: Algorithm 4 (kVarPlain) or Algorithm 3 (kVarGameLax) in one kernel
      if (variant == kVarGameLax) return reinterpret_cast<const void*>(&k_group_game_hopf<T, F, L, K, true>);
      if (variant != kVarPlain) return nullptr;
      return reinterpret_cast<const void*>(&k_group_game_hopf<T, F, L, K>);
    } else {
      // Algorithm 3; with the sigma and value-change recipes (kVarRecipe)
      if (variant == kVarRecipe) return reinterpret_cast<const void*>(&k_group_game<T, F, L, K, true>);
      if (variant != kVarPlain) return nullptr;
      return reinterpret_cast<const void*>(&k_group_game<T, F, L, K>);
    }
  } else {
    if (variant == kVarRecipe) return reinterpret_cast<const void*>(&k_group_control_rec<T, F, L, K, true>);
    if constexpr (F::kMix) {
      // eikonal family: the shifted layout (Algorithms 1 and 2) or the weighted rules
      if (variant == kVarMix) return reinterpret_cast<const void*>(&k_group_control_shift<T, Weighted<F>, L, K, false>);
      if (variant == kVarShiftHopf) return reinterpret_cast<const void*>(&k_group_control_shift<T, F, L, K, true>);
      return reinterpret_cast<const void*>(&k_group_control_shift<T, F, L, K, false>);
    } else {
      // quadrotor: Algorithm 1 / 2, or the weighted rules (kVarMix; in FP64 built
      // for at most two nodes per lane, the wider tiles spill most of their state)
      if (variant == kVarMix) {
        if constexpr (sizeof(T) == 8 && K > 2) return nullptr;
        else return reinterpret_cast<const void*>(&k_group_control<T, F, L, K, true>);
      }
      if (variant != kVarPlain) return nullptr;
      return reinterpret_cast<const void*>(&k_group_control<T, F, L, K>);
    }
  }
}

// variant: kVarPlain (Algorithm 1 / 2 / 3), kVarRecipe (control kernel with
// the robustness recipes; the game kernel with the sigma and value-change
// recipes), kVarMix (weighted Euler discretisations),
// kVarShift / kVarShiftHopf (Algorithm 1 / 2 in the shifted layout, eikonal
// family), kVarGameLax (Algorithm 3 for the scalar-player game).
template <typename T, class F>
const void* pick_kernel(int plain, int L, int K, int variant) {
  if (plain) {
    if constexpr (F::kGame) {
      if constexpr (F::kGameHopf) return nullptr;  // no plain kernel for the game Hopf formulation
      else return reinterpret_cast<const void*>(&k_plain_game<T, F>);
    } else {
      return reinterpret_cast<const void*>(&k_plain_control<T, F>);
    }
  }
#define HJPD_TILE_CASE(LL, KK) \
  if (L == LL && K == KK) return group_ptr<T, F, LL, KK>(variant);
  HJPD_TILE_CASE(8, 1) HJPD_TILE_CASE(16, 1) HJPD_TILE_CASE(8, 2) HJPD_TILE_CASE(8, 3) HJPD_TILE_CASE(32, 1) HJPD_TILE_CASE(16, 2)
  HJPD_TILE_CASE(8, 4) HJPD_TILE_CASE(16, 3) HJPD_TILE_CASE(64, 1) HJPD_TILE_CASE(32, 2) HJPD_TILE_CASE(16, 4) HJPD_TILE_CASE(32, 3)
  HJPD_TILE_CASE(64, 2) HJPD_TILE_CASE(32, 4) HJPD_TILE_CASE(64, 3) HJPD_TILE_CASE(64, 4)
#undef HJPD_TILE_CASE
  return nullptr;
}

}  // namespace hjpd

// One lookup function per (family shape, dtype), defined in its own
// translation unit so the instantiations compile in parallel.
#define HJPD_DECLARE_LOOKUP(name) const void* hjpd_lookup_##name(int plain, int L, int K, int variant);
HJPD_DECLARE_LOOKUP(cnorm2_f32)
HJPD_DECLARE_LOOKUP(cnorm2_f64)
HJPD_DECLARE_LOOKUP(cnorm3_f32)
HJPD_DECLARE_LOOKUP(cnorm3_f64)
HJPD_DECLARE_LOOKUP(cnorm4_f32)
HJPD_DECLARE_LOOKUP(cnorm4_f64)
HJPD_DECLARE_LOOKUP(cnorm10_f32)
HJPD_DECLARE_LOOKUP(cnorm10_f64)
HJPD_DECLARE_LOOKUP(quad_f32)
HJPD_DECLARE_LOOKUP(quad_f64)
HJPD_DECLARE_LOOKUP(pursuit_f32)
HJPD_DECLARE_LOOKUP(pursuit_f64)
HJPD_DECLARE_LOOKUP(isaacs_f32)
HJPD_DECLARE_LOOKUP(isaacs_f64)
#undef HJPD_DECLARE_LOOKUP
