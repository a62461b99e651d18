// Velocity sets of the two lattices.  Both distributions (g for phi, h for
// c) use the same lattice.
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
#pragma once

#include <cstdint>

namespace gplbm {

struct D2Q9 {
  static constexpr int Q = 9;
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

}  // namespace gplbm
