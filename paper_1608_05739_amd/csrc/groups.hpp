// Component groups of the fused z pass.
#pragma once

#include "internal.hpp"

namespace psatd {

// Input and output component groups.  In 2D (k_y = 0) the update splits into
// the s-polarized set (Ey, Bx, Bz; Jy) and the p-polarized set (Ex, Ez, By;
// Jx, Jz, rho), processed one after the other to halve the register state.
template <int G, int SRC>
struct Group;

// 2D s-polarization
template <int SRC>
struct Group<0, SRC> {
  static constexpr int nin = src_has_j(SRC) ? 4 : 3;
  static constexpr int in[4] = {kEy, kBx, kBz, kJy};
  static constexpr int nout = 3;
  static constexpr int out_slot[3] = {0, 1, 2};
};
// 2D p-polarization
template <int SRC>
struct Group<1, SRC> {
  static constexpr int nin = !src_has_j(SRC) ? 3 : (SRC == kRho ? 7 : 5);
  static constexpr int in[7] = {kEx, kEz, kBy, kJx, kJz, kRhoOld, kRhoNew};
  static constexpr int nout = 3;
  static constexpr int out_slot[3] = {0, 1, 2};
};
// 3D: everything couples
template <int SRC>
struct Group<2, SRC> {
  static constexpr int nin = !src_has_j(SRC) ? 6 : (SRC == kRho ? 11 : 9);
  static constexpr int in[11] = {kEx, kEy, kEz, kBx, kBy, kBz, kJx, kJy, kJz, kRhoOld, kRhoNew};
  static constexpr int nout = 6;
  static constexpr int out_slot[6] = {0, 1, 2, 3, 4, 5};
};

}  // namespace psatd
