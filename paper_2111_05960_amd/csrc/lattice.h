// Velocity sets.  g (for phi) runs on D2Q9, D3Q19, D2Q5 or D3Q7; h (for c)
// on the lattice of g or, under D2Q9 / D3Q19, on the light one of the same
// dimension, D2Q5 or D3Q7.
//
// D2Q9 is numbered as in Sec. 3.1 of the paper: rest, the four axis
// vectors (+x, +y, -x, -y), the four diagonals (+x+y, -x+y, -x-y, +x-y);
// weights 4/9, 1/9, 1/36.
//
// D3Q19 (not listed in the paper) is numbered by layers of e_z: the five
// e_z = +1 vectors, the rest vector, the eight in-plane vectors, the five
// e_z = -1 vectors; weights 1/3 (rest), 1/18 (axes), 1/36 (edges).  Moments
// are summed in this index order, so the numbering is part of the result at
// the last bit; a z-marching kernel receives the contributions to a node's
// moment in exactly this order (lower plane, same plane, upper plane).
//
// D2Q5 is the rest and the four axis vectors of D2Q9 (same order); weights
// 1/3, 1/6.  D3Q7 is numbered by layers of e_z like D3Q19: (0,0,1), rest,
// +x, -x, +y, -y, (0,0,-1); weights 1/4 (rest), 1/8.  cs2 is xi_s^2, the
// second moment of the weights (1/3, except 1/4 for D3Q7), inv_cs2 its
// inverse written exactly (3 or 4); the relaxation times are
// tau_g = M_phi inv_cs2 and tau_h = 1 / (gamma cs2), and the gradient is
// inv_cs2 sum_k w_k e_k d_k.
#pragma once

#include <cstdint>

namespace gplbm {

struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr double cs2 = 1.0 / 3.0;
  static constexpr double inv_cs2 = 3.0;
  static constexpr int D = 2;
  static constexpr int REST = 0;
  static constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  static constexpr double w[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                                  1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                                  1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr double cs2 = 1.0 / 3.0;
  static constexpr double inv_cs2 = 3.0;
  static constexpr int D = 3;
  static constexpr int REST = 5;
  static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 1, -1, 0, 0,
                                 1, -1, -1, 1, 0, -1, 1, 0, 0};
  static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 0, 1, -1,
                                 1, 1, -1, -1, 0, 0, 0, -1, 1};
  static constexpr int ez[19] = {1, 1, 1, 1, 1, 0, 0, 0, 0, 0,
                                 0, 0, 0, 0, -1, -1, -1, -1, -1};
  static constexpr int opp[19] = {14, 15, 16, 17, 18, 5, 7, 6, 9, 8,
                                  12, 13, 10, 11, 0, 1, 2, 3, 4};
  static constexpr double w[19] = {
      1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
      1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
      1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 18.0,
      1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

struct D2Q5 {
  static constexpr int Q = 5;
  static constexpr double cs2 = 1.0 / 3.0;
  static constexpr double inv_cs2 = 3.0;
  static constexpr int D = 2;
  static constexpr int REST = 0;
  static constexpr int ex[5] = {0, 1, 0, -1, 0};
  static constexpr int ey[5] = {0, 0, 1, 0, -1};
  static constexpr int ez[5] = {0, 0, 0, 0, 0};
  static constexpr int opp[5] = {0, 3, 4, 1, 2};
  static constexpr double w[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
};

struct D3Q7 {
  static constexpr int Q = 7;
  static constexpr double cs2 = 1.0 / 4.0;
  static constexpr double inv_cs2 = 4.0;
  static constexpr int D = 3;
  static constexpr int REST = 1;
  static constexpr int ex[7] = {0, 0, 1, -1, 0, 0, 0};
  static constexpr int ey[7] = {0, 0, 0, 0, 1, -1, 0};
  static constexpr int ez[7] = {1, 0, 0, 0, 0, 0, -1};
  static constexpr int opp[7] = {6, 1, 3, 2, 5, 4, 0};
  static constexpr double w[7] = {1.0 / 8.0, 1.0 / 4.0, 1.0 / 8.0, 1.0 / 8.0,
                                  1.0 / 8.0, 1.0 / 8.0, 1.0 / 8.0};
};

// Number of populations of a lattice numbered by layers of e_z with the
// given e_z (+1, 0, -1): the in-plane layer starts at index count(+1).
template <class L>
constexpr int count_ez(int v) {
  int n = 0;
  for (int k = 0; k < L::Q; ++k) n += L::ez[k] == v ? 1 : 0;
  return n;
}

// The populations of a lattice with the given e_z, as bits k.
template <class L>
constexpr uint32_t ez_mask(int v) {
  uint32_t m = 0;
  for (int k = 0; k < L::Q; ++k) m |= L::ez[k] == v ? (1u << k) : 0u;
  return m;
}

// The light lattice of the same dimension.
template <class L>
struct Light;
template <>
struct Light<D2Q9> {
  using type = D2Q5;
};
template <>
struct Light<D3Q19> {
  using type = D3Q7;
};

}  // namespace gplbm
