// Velocity sets and Hermite coefficient layout for the HIP kernels.
//
// Textbook D2Q9, D3Q19 and D3Q27 sets with cs^2 = 1/3 (the paper names the
// lattices and cites the weights without printing them, Section 2).  Listed
// explicitly: rest, axis links, face diagonals, then (D3Q27) body diagonals.
#pragma once

#include <hip/hip_runtime.h>

namespace lbk {

struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr int D = 2;
  static constexpr int c[Q][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
  static constexpr double w[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                                  1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  static constexpr int wden = 36;
  static constexpr int wmul[Q] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
};

struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr int D = 3;
  static constexpr int c[Q][3] = {
      {0, 0, 0},   {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},  {0, 0, 1},  {0, 0, -1},
      {1, 1, 0},   {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},
      {-1, 0, 1},  {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  static constexpr double w[Q] = {
      1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
      1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
      1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  static constexpr int wden = 36;
  static constexpr int wmul[Q] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
};

struct D3Q27 {
  static constexpr int Q = 27;
  static constexpr int D = 3;
  static constexpr int c[Q][3] = {
      {0, 0, 0},    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},
      {0, 0, -1},   {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},  {1, 0, 1},
      {-1, 0, -1},  {1, 0, -1},  {-1, 0, 1},  {0, 1, 1},   {0, -1, -1}, {0, 1, -1},
      {0, -1, 1},   {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1},
      {-1, 1, -1},  {-1, 1, 1},  {1, -1, -1}};
  static constexpr double w[Q] = {
      8.0 / 27.0,  2.0 / 27.0,  2.0 / 27.0,  2.0 / 27.0,  2.0 / 27.0,  2.0 / 27.0,  2.0 / 27.0,
      1.0 / 54.0,  1.0 / 54.0,  1.0 / 54.0,  1.0 / 54.0,  1.0 / 54.0,  1.0 / 54.0,  1.0 / 54.0,
      1.0 / 54.0,  1.0 / 54.0,  1.0 / 54.0,  1.0 / 54.0,  1.0 / 54.0,  1.0 / 216.0, 1.0 / 216.0,
      1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0};
  static constexpr int wden = 216;
  static constexpr int wmul[Q] = {64, 16, 16, 16, 16, 16, 16, 4, 4, 4, 4, 4, 4, 4,
                                  4,  4,  4,  4,  4,  1,  1,  1, 1, 1, 1, 1, 1};
};

// t_a == wmul[a] / wden exactly, for every lattice.
template <class L>
constexpr bool weights_consistent() {
  for (int a = 0; a < L::Q; ++a)
    if (L::w[a] * L::wden != (double)L::wmul[a]) return false;
  return true;
}
static_assert(weights_consistent<D2Q9>(), "D2Q9 weights");
static_assert(weights_consistent<D3Q19>(), "D3Q19 weights");
static_assert(weights_consistent<D3Q27>(), "D3Q27 weights");

// Index of the link opposite to a (c_opp = -c_a).
template <class L>
__host__ __device__ constexpr int opposite(int a) {
  for (int b = 0; b < L::Q; ++b)
    if (L::c[b][0] == -L::c[a][0] && L::c[b][1] == -L::c[a][1] && L::c[b][2] == -L::c[a][2])
      return b;
  return -1;
}

// Moment storage (one array each, written by the moments sweep):
//   [0] drho = rho - rho0, [1..D] j, then Pi^neq: diagonal (D), off-diagonal
//   xy, (xz, yz).   M = 6 in 2D, 10 in 3D.
template <class L>
struct MomentLayout {
  static constexpr int D = L::D;
  static constexpr int M = 1 + D + D * (D + 1) / 2;
  static constexpr int RHO = 0;
  static constexpr int J = 1;
  static constexpr int PID = 1 + D;       // diagonal
  static constexpr int PIO = 1 + 2 * D;   // off-diagonal, (0,1), (0,2), (1,2)
};

// Post-collision Hermite coefficients of a node, prescaled by the smallest
// lattice weight 1/wden so that a link value is
//   f^pc_a - t_a rho0 = wmul[a] * (signed sum of coefficients)
// with wmul[a] a power of two (12 for the D3Q19 rest link).  The weights
// never enter as rounded constants: every coefficient is rounded once (by a
// correctly rounded division by a small odd integer, or exactly by a power of
// two), so the discrete moment sums of the rebuilt populations carry no
// fixed-sign bias from step to step.  Slots:
//   [0] r/wden,            r = drho - tr(A)/(2 cs^2)
//   [1..D] 3 J_b/wden      (order 3: minus 4.5 sum_{a != b} a3_aab / wden)
//   [1+D..] 4.5 A_aa/wden, then 9 A_ab/wden (a < b)
//   order 3 (D3Q27): 13.5 a3_aab/wden for (a,b) = xy, xz, yx, yz, zx, zy;
//   27 a3_xyz/wden
template <class L, int ORDER>
struct CoefLayout {
  static constexpr int D = L::D;
  static constexpr int R = 0;
  static constexpr int J = 1;
  static constexpr int AD = 1 + D;
  static constexpr int AO = 1 + 2 * D;
  static constexpr int T = 1 + D + D * (D + 1) / 2;
  static constexpr int K = T + (ORDER >= 3 ? 7 : 0);
};

// Off-diagonal slot of the pair (al, be), al != be, in the order xy, xz, yz.
__host__ __device__ constexpr int offdiag(int al, int be) {
  return (al > be) ? offdiag(be, al) : (al == 0 ? be - 1 : 2);
}

// Slot of a3_{al al be} (al != be) among the six third-order coefficients.
__host__ __device__ constexpr int t3slot(int al, int be) {
  return al * 2 + (be > al ? be - 1 : be);
}

}  // namespace lbk
