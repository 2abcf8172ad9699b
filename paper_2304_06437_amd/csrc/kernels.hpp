// HIP kernels of the thread-safe regularized lattice Boltzmann step (gfx950).
//
// One time step (Section 4: moments, then fused streaming + collision, then
// boundary conditions) is two sweeps over HBM:
//
//   moments        f -> m   pointwise: reads the Q population arrays of a node,
//                           writes its moments drho, j, Pi^neq (M arrays).
//   stream_collide m -> f   rebuilds every population of every node from the
//                           moments of the node it streams from (Section 3,
//                           eq. pushLB with the Hermite-regularized
//                           non-equilibrium), boundaries fused.  It never reads
//                           f, so it overwrites the single population set in
//                           place: no second population array, no even/odd
//                           step parity, no pointer swap.
//
// Work mapping of stream_collide: one 64-lane wavefront owns a segment of
// 64*V consecutive nodes of one x-row (V per lane).  It loads only that
// row's moments, turns each node's moments into its post-collision Hermite
// coefficients once, and then, for every link a,
//   - takes the source node x - c_a along x from its own registers or from the
//     neighbouring lane (cross-lane shuffle; the segment ends come from one
//     extra node on each side),
//   - stores the V link values into the row (y + c_ay, z + c_az) of array a.
// Transport along y and z is therefore a store into another row (push form
// of eq. pushLB), transport along x a register/lane shift (pull form).  Every
// population f_a(x) is written exactly once per step, by exactly one lane.
//
// Halfway bounce-back (Section 5.1): a link a of node x whose neighbour
// x + c_a lies beyond a wall is written back into the same node as the
// opposite link, f_abar(x) = f^pc_a(x).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"
#include "storage.hpp"

namespace lbk {

template <typename C>
struct StepParams {
  int64_t nx, ny, nz;
  int64_t px;          // row pitch: storage nodes per x-row (nx rounded up)
  int64_t npad;        // padded node count (a multiple of the block size)
  int64_t nseg;        // row segments per x-row in stream_collide
  int32_t bbx, bby, bbz;
  int32_t lb;          // log2 of the block size B (nodes)
  C rho0, inv_rho0;
  C F[3];
  C halfF[3];
  C omw;               // 1 - omega
  C omhw;              // 1 - omega/2
  // Moving walls: wall[2 axis + side] = -6 rho0 u_w / wden of the wall on
  // the low (side 0) or high (side 1) face of an axis; moving != 0 if any
  // is non-zero.
  int32_t moving;
  // Order in which a sweep's work units (wavefronts of stream-collide) are
  // mapped to row segments: 0 the natural one; otherwise unit u of U takes
  // segment (u * order_mul) mod U, a permutation (gcd(order_mul, U) = 1);
  // order_mul = U - 1 gives the reversed order.  For tests of the sweep's
  // independence of execution order.
  int32_t order_mul;
  C wall[6][3];
};

// Flat block number of a launch whose blocks are laid out x-fastest over a
// 2D grid (grid_of in handle.hpp): one grid dimension holds at most 2^32
// work-items, fewer than a large domain's wavefronts need.
__device__ __forceinline__ int64_t flat_block() {
  return (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
}

// -------------------------------------------------------------------------
// Blocked array layout.  The padded node range [0, npad) is cut into blocks of
// B = 2^lb consecutive nodes; a region of NA arrays stores, block after
// block, B elements of array 0, then B of array 1, and so on:
//   element (a, n) = (n >> lb) NA B + a B + (n & (B - 1)).
// The NA streams a sweep touches at one time then lie inside one contiguous
// NA B span instead of npad apart (plain structure of arrays), which the HBM
// system serves faster.  B is a power of two >= 1024, so a vector of up to
// 16 nodes that starts at a multiple of its length never crosses a block.
// -------------------------------------------------------------------------
template <int NA, typename C>
__device__ __forceinline__ int64_t slot(const StepParams<C>& p, int64_t n) {
  return (((n >> p.lb) * NA) << p.lb) + (n & ((int64_t(1) << p.lb) - 1));
}

template <typename C>
__device__ __forceinline__ int64_t astride(const StepParams<C>& p) {
  return int64_t(1) << p.lb;
}

// A value the same in every lane of the wavefront, so marked for the
// compiler (scalar registers and scalar arithmetic for what derives from it).
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// p + a 32-bit byte offset (a lane's offset from a wave-uniform base).
template <typename T>
__device__ __forceinline__ T* at_bytes(T* p, uint32_t bytes) {
  return (T*)((char*)p + bytes);
}
template <typename T>
__device__ __forceinline__ const T* at_bytes(const T* p, uint32_t bytes) {
  return (const T*)((const char*)p + bytes);
}

// Storage node of lattice node n = x + nx (y + ny z).  Rows are px >= nx
// storage nodes apart, so that every row starts on a vector boundary; nodes
// x in [nx, px) of a row are padding: zero populations (the stream-collide
// sweep writes only zeros there), never read into a lattice node.
template <typename C>
__device__ __forceinline__ int64_t node_at(const StepParams<C>& p, int64_t n) {
  if (p.px == p.nx) return n;
  return n + (n / p.nx) * (p.px - p.nx);
}

// -------------------------------------------------------------------------
// Node-level arithmetic.
// -------------------------------------------------------------------------

// Moments of one node from its shifted populations s_a = f_a - t_a rho0
// (Section 2 moment definitions; Section 4 moment snippet, where
// Pi^neq = sum_a f^neq_a c_a c_a, here in its closed form
// Pi^neq = sum_a s_a c_a c_a - drho cs2 I - rho0 u u, u = (j + F/2)/rho0).
template <class L, typename C>
__device__ __forceinline__ void node_moments(const C (&s)[L::Q], const StepParams<C>& p,
                                             C (&m)[MomentLayout<L>::M]) {
  // every operation rounded as written: no FMA contraction, whose choices
  // depend on the surrounding code, so that every kernel evaluating the
  // moments (and post_collision below) gets the same bits
#pragma clang fp contract(off)
  using ML = MomentLayout<L>;
  constexpr int D = L::D;
  C drho = s[0];
  C j[D];
  C P[D][D];
#pragma unroll
  for (int al = 0; al < D; ++al) {
    j[al] = C(0);
#pragma unroll
    for (int be = 0; be < D; ++be) P[al][be] = C(0);
  }
  if constexpr (D == 3) {
    // opposite links a, a' (c_a' = -c_a) enter every first moment with
    // opposite signs and every second moment with the same sign: sum their
    // difference and their sum once (54 additions per D3Q19 node instead
    // of 90)
#pragma unroll
    for (int a = 1; a < L::Q; ++a) {
      const int b = opposite<L>(a);
      if (b < a) continue;
      const C sp = s[a] + s[b];
      const C dp = s[a] - s[b];
      drho += sp;
#pragma unroll
      for (int al = 0; al < D; ++al) {
        if (L::c[a][al] > 0) j[al] += dp;
        if (L::c[a][al] < 0) j[al] -= dp;
        if (L::c[a][al] != 0) P[al][al] += sp;
#pragma unroll
        for (int be = al + 1; be < D; ++be) {
          const int cc = L::c[a][al] * L::c[a][be];
          if (cc > 0) P[al][be] += sp;
          if (cc < 0) P[al][be] -= sp;
        }
      }
    }
  } else {
#pragma unroll
    for (int a = 1; a < L::Q; ++a) {
      drho += s[a];
#pragma unroll
      for (int al = 0; al < D; ++al) {
        if (L::c[a][al] > 0) j[al] += s[a];
        if (L::c[a][al] < 0) j[al] -= s[a];
        if (L::c[a][al] != 0) P[al][al] += s[a];
#pragma unroll
        for (int be = al + 1; be < D; ++be) {
          const int cc = L::c[a][al] * L::c[a][be];
          if (cc > 0) P[al][be] += s[a];
          if (cc < 0) P[al][be] -= s[a];
        }
      }
    }
  }
  C u[D];
#pragma unroll
  for (int al = 0; al < D; ++al) u[al] = (j[al] + p.halfF[al]) * p.inv_rho0;
  const C cs2 = C(1.0 / 3.0);
  m[ML::RHO] = drho;
#pragma unroll
  for (int al = 0; al < D; ++al) {
    m[ML::J + al] = j[al];
    m[ML::PID + al] = P[al][al] - drho * cs2 - p.rho0 * u[al] * u[al];
#pragma unroll
    for (int be = al + 1; be < D; ++be)
      m[ML::PIO + offdiag(al, be)] = P[al][be] - p.rho0 * u[al] * u[be];
  }
}

// x * NUM / DEN with no bias: the odd part d of the reduced denominator is a
// division, the power-of-two part an exact scaling.  (A multiplication by
// the rounded reciprocal r = fl(1/d) alone carries r's rounding error, the
// same relative error with the same sign at every node and step, which
// accumulates as a drift of the conserved momentum.)  Two ways to divide:
//   FD = false: IEEE division, correctly rounded;
//   FD = true:  q = x r, then one correction with the exact FMA residual,
//               q' = q + (x - q d) r (Markstein's correction), with the sign
//               of x (it rounds -0 / d to +0 otherwise): four instructions
//               instead of about ten.  In FP32, for the odd divisors d = 3,
//               9, 27 that occur here, q' equals the IEEE quotient for every
//               finite input (checked exhaustively by lb_check_division), so
//               the choice changes speed, never a result bit.
// The sweeps bound by instruction issue (the fused step, D3Q27 third order
// with 16-bit storage) use FD = true; the bandwidth-bound ones measure
// faster with the IEEE sequence.
__host__ __device__ constexpr int gcd_int(int a, int b) { return b == 0 ? a : gcd_int(b, a % b); }

template <int NUM, int DEN, bool FD = false, typename C>
__device__ __forceinline__ C scaled(C x) {
  constexpr int g = gcd_int(NUM, DEN);
  constexpr int n = NUM / g, d = DEN / g;
  constexpr int d2 = d & -d;  // power-of-two part
  constexpr int dodd = d / d2;
  static_assert(n == 1 || dodd == 1, "scaled: single rounding needs n == 1 or odd part 1");
  C y = x;
  if constexpr (n != 1) y = y * C(n);
  if constexpr (dodd != 1) {
    if constexpr (FD) {
      constexpr C r = C(1) / C(dodd);
      const C q = y * r;
      const C e = fma(-q, C(dodd), y);  // exact: q is within an ulp of y / d
      y = copysign(fma(e, r, q), y);
    } else {
      y = y / C(dodd);
    }
  }
  if constexpr (d2 != 1) y = y * C(1.0 / d2);
  return y;
}

// Exhaustive check of the short division against the IEEE one: every
// finite FP32 input x (bit pattern i in [0, 2^32)), x / D both ways, counted
// where the bits differ.  Grid-stride; one counter per launch.
template <int D>
__global__ __launch_bounds__(256) void k_division_check(unsigned long long* mismatches) {
  const uint64_t nthr = (uint64_t)gridDim.x * blockDim.x;
  unsigned long long bad = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (uint64_t(1) << 32);
       i += nthr) {
    const float x = __uint_as_float((uint32_t)i);
    if (!isfinite(x)) continue;
    const float a = scaled<1, D, true, float>(x);
    const float b = scaled<1, D, false, float>(x);
    if (__float_as_uint(a) != __float_as_uint(b)) ++bad;
  }
  if (bad) atomicAdd(mismatches, bad);
}

// Post-collision Hermite coefficients of a node from its moments.  With
// J = j + F and u = (j + F/2)/rho0 the post-collision populations are
//   f^pc_a - t_a rho0 = t_a [ drho + c.J/cs2 + H2_a:A/(2 cs4) (+ H3_a:a3/(6 cs6)) ]
//   A  = rho0 u u + (1 - omega) Pi^neq + (1 - omega/2)(u F + F u)
//   a3 = rho0 u u u + (1 - omega)(u Pi^neq + perms)        (order 3, D3Q27)
// i.e. the equilibrium of eq. equil plus the regularized non-equilibrium of
// eq. hermite relaxed by (1 - omega) (eq. LBexp), with Guo's source in
// Hermite form.  The coefficients are prescaled (CoefLayout) so that a link
// value is a signed sum times a power of two, computed once per node instead
// of once per link.
template <class L, int ORDER, typename C, bool FD = false>
__device__ __forceinline__ void post_collision(const C (&m)[MomentLayout<L>::M],
                                               const StepParams<C>& p,
                                               C (&k)[CoefLayout<L, ORDER>::K]) {
#pragma clang fp contract(off)
  using ML = MomentLayout<L>;
  using CL = CoefLayout<L, ORDER>;
  constexpr int D = L::D;
  constexpr int W = L::wden;
  C u[D], Jt[D];
#pragma unroll
  for (int al = 0; al < D; ++al) {
    u[al] = (m[ML::J + al] + p.halfF[al]) * p.inv_rho0;
    Jt[al] = m[ML::J + al] + p.F[al];
  }
  C trA = C(0);
#pragma unroll
  for (int al = 0; al < D; ++al) {
    const C A = p.rho0 * u[al] * u[al] + p.omw * m[ML::PID + al] + p.omhw * C(2) * u[al] * p.F[al];
    trA += A;
    k[CL::AD + al] = scaled<9, 2 * W, FD>(A);   // 4.5 A / wden
#pragma unroll
    for (int be = al + 1; be < D; ++be) {
      const int o = offdiag(al, be);
      const C Ao = p.rho0 * u[al] * u[be] + p.omw * m[ML::PIO + o] +
                   p.omhw * (u[al] * p.F[be] + p.F[al] * u[be]);
      k[CL::AO + o] = scaled<9, W, FD>(Ao);
    }
  }
  k[CL::R] = scaled<1, W, FD>(m[ML::RHO] - C(1.5) * trA);
#pragma unroll
  for (int be = 0; be < D; ++be) k[CL::J + be] = scaled<3, W, FD>(Jt[be]);
  if constexpr (ORDER >= 3) {
    static_assert(L::Q == 27, "third-order terms need D3Q27");
    C B[3][3];
#pragma unroll
    for (int al = 0; al < 3; ++al) {
      B[al][al] = p.omw * m[ML::PID + al];
#pragma unroll
      for (int be = al + 1; be < 3; ++be) {
        B[al][be] = p.omw * m[ML::PIO + offdiag(al, be)];
        B[be][al] = B[al][be];
      }
    }
    C sum3[3] = {C(0), C(0), C(0)};
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
      for (int be = 0; be < 3; ++be) {
        if (be == al) continue;
        const C a3 = p.rho0 * u[al] * u[al] * u[be] + C(2) * u[al] * B[al][be] + u[be] * B[al][al];
        k[CL::T + t3slot(al, be)] = scaled<27, 2 * W, FD>(a3);  // 13.5 a3 / wden
        sum3[be] += a3;
      }
#pragma unroll
    for (int be = 0; be < 3; ++be) k[CL::J + be] -= scaled<9, 2 * W, FD>(sum3[be]);
    const C axyz = p.rho0 * u[0] * u[1] * u[2] + u[0] * B[1][2] + u[1] * B[0][2] + u[2] * B[0][1];
    k[CL::T + 6] = scaled<27, W, FD>(axyz);
  }
}

// Shifted post-collision value of link a from prescaled coefficients:
// wmul_a times a signed sum of coefficients (link_sum).
template <class L, int ORDER, int A, typename C>
__device__ __forceinline__ C link_sum(const C (&k)[CoefLayout<L, ORDER>::K]) {
  using CL = CoefLayout<L, ORDER>;
  constexpr int D = L::D;
  constexpr int c0 = L::c[A][0], c1 = L::c[A][1], c2 = L::c[A][2];
  constexpr int cv[3] = {c0, c1, c2};
  C v = k[CL::R];
#pragma unroll
  for (int al = 0; al < D; ++al) {
    if (cv[al] > 0) v += k[CL::J + al];
    if (cv[al] < 0) v -= k[CL::J + al];
  }
#pragma unroll
  for (int al = 0; al < D; ++al)
    if (cv[al] != 0) v += k[CL::AD + al];
#pragma unroll
  for (int al = 0; al < D; ++al)
#pragma unroll
    for (int be = al + 1; be < D; ++be) {
      if (cv[al] * cv[be] > 0) v += k[CL::AO + offdiag(al, be)];
      if (cv[al] * cv[be] < 0) v -= k[CL::AO + offdiag(al, be)];
    }
  if constexpr (ORDER >= 3) {
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
      for (int be = 0; be < 3; ++be) {
        if (be == al || cv[al] == 0) continue;
        if (cv[be] > 0) v += k[CL::T + t3slot(al, be)];
        if (cv[be] < 0) v -= k[CL::T + t3slot(al, be)];
      }
    if (c0 * c1 * c2 > 0) v += k[CL::T + 6];
    if (c0 * c1 * c2 < 0) v -= k[CL::T + 6];
  }
  return v;
}

template <class L, int ORDER, int A, typename C>
__device__ __forceinline__ C link_value(const C (&k)[CoefLayout<L, ORDER>::K]) {
  constexpr int mul = L::wmul[A];
  if constexpr (mul == 1) return link_sum<L, ORDER, A, C>(k);
  else return C(mul) * link_sum<L, ORDER, A, C>(k);
}

// Link value plus `extra` in the same prescaled units (wmul_a (sum + extra)).
template <class L, int ORDER, int A, typename C>
__device__ __forceinline__ C link_value_plus(const C (&k)[CoefLayout<L, ORDER>::K], C extra) {
  constexpr int mul = L::wmul[A];
  const C v = link_sum<L, ORDER, A, C>(k) + extra;
  if constexpr (mul == 1) return v;
  else return C(mul) * v;
}

// Moving-wall correction of link A leaving across face `face` (2 axis + side),
// in prescaled units: c_A . wall[face], so that wmul_A times it is
// -2 t_A rho0 (c_A . u_w)/cs2 (Ladd's momentum correction, which Bouzidi's
// interpolated bounce-back reduces to at the halfway wall).
template <class L, int A, typename C>
__device__ __forceinline__ C wall_dot(const StepParams<C>& p, int face) {
  C v = C(0);
#pragma unroll
  for (int al = 0; al < L::D; ++al) {
    if (L::c[A][al] > 0) v += p.wall[face][al];
    if (L::c[A][al] < 0) v -= p.wall[face][al];
  }
  return v;
}

// -------------------------------------------------------------------------
// Cross-lane shifts (64-lane wavefront).
// -------------------------------------------------------------------------
__device__ __forceinline__ float lane_from_below(float v) { return __shfl_up(v, 1, 64); }
__device__ __forceinline__ float lane_from_above(float v) { return __shfl_down(v, 1, 64); }
__device__ __forceinline__ double lane_from_below(double v) { return __shfl_up(v, 1, 64); }
__device__ __forceinline__ double lane_from_above(double v) { return __shfl_down(v, 1, 64); }
__device__ __forceinline__ float lane_bcast(float v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ double lane_bcast(double v, int src) { return __shfl(v, src, 64); }

// -------------------------------------------------------------------------
// Sweep 1: moments.  Each lane handles V consecutive nodes of the flattened
// (padded) arrays; all loads and stores are V-wide vectors.
// -------------------------------------------------------------------------
template <class L, typename S, typename C, int V>
__device__ __forceinline__ void moments_body(const S* __restrict__ f, C* __restrict__ m,
                                             const StepParams<C>& p, int64_t i0) {
  using ML = MomentLayout<L>;
  if (i0 >= p.npad) return;
  const int64_t B = astride(p), fs = slot<L::Q>(p, i0), ms = slot<ML::M>(p, i0);
  C s[L::Q][V];
#pragma unroll
  for (int a = 0; a < L::Q; ++a) load_pack<S, C, V>(f + fs + a * B, s[a]);
  C out[ML::M][V];
#pragma unroll
  for (int e = 0; e < V; ++e) {
    C se[L::Q], me[ML::M];
#pragma unroll
    for (int a = 0; a < L::Q; ++a) se[a] = s[a][e];
    node_moments<L, C>(se, p, me);
#pragma unroll
    for (int q = 0; q < ML::M; ++q) out[q][e] = me[q];
  }
#pragma unroll
  for (int q = 0; q < ML::M; ++q) store_plain<C, V>(m + ms + q * B, out[q]);
}

template <class L, typename S, typename C, int V>
__global__ __launch_bounds__(256) void k_moments(const S* __restrict__ f, C* __restrict__ m,
                                                 StepParams<C> p) {
  moments_body<L, S, C, V>(f, m, p, (flat_block() * blockDim.x + threadIdx.x) * V);
}

// -------------------------------------------------------------------------
// Sweep 2: fused streaming + collision with boundaries.
//
// Link indices ordered by target row offset (c_y, c_z): (0,0), (1,0),
// (-1,0), (0,1), (0,-1), then the four diagonal rows; lattice order within
// a row.  A permutation of 0..Q-1.
template <class L>
struct RowOrder {
  struct Table {
    int a[L::Q];
  };
  static constexpr Table make() {
    constexpr int rows[9][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1},
                                {1, 1}, {-1, -1}, {1, -1}, {-1, 1}};
    Table t{};
    int k = 0;
    for (int r = 0; r < 9; ++r)
      for (int a = 0; a < L::Q; ++a)
        if (L::c[a][1] == rows[r][0] && L::c[a][2] == rows[r][1]) t.a[k++] = a;
    return t;
  }
  static constexpr Table t = make();
  static constexpr const int (&a)[L::Q] = t.a;
};

template <class L>
constexpr bool row_order_is_permutation() {
  int seen[L::Q] = {};
  for (int i = 0; i < L::Q; ++i) {
    const int a = RowOrder<L>::make().a[i];
    if (a < 0 || a >= L::Q || seen[a]) return false;
    seen[a] = 1;
  }
  return true;
}
static_assert(row_order_is_permutation<D2Q9>(), "D2Q9 row order");
static_assert(row_order_is_permutation<D3Q19>(), "D3Q19 row order");
static_assert(row_order_is_permutation<D3Q27>(), "D3Q27 row order");

// Lane mapping: a wavefront's segment of 64 V nodes (V = E H) is split into H
// chunks of 64 E nodes; lane l owns nodes h*64E + l*E + e (e < E) of chunk h.
// Every vector load or store instruction therefore covers 64 E contiguous
// nodes (16 bytes per lane for E = 4 floats): whole cache lines per
// instruction.  Rows are px apart, nx rounded up to a multiple of E, so
// every vector is aligned; where px > nx the vector holding the row's last
// node (position tl < E - 1) reads padding moments and stores zeros into
// the padding populations.  PAD selects that handling at compile time: the
// PAD = false variant (fewer instructions per link) requires px == nx.
// RB = true requires every row to lie inside one block of the array layout
// (px divides the block size B): then element (a, row start + x) is
// slot(row start) + a B + x, a wave-uniform base (scalar arithmetic) plus a
// 32-bit lane offset, instead of a 64-bit slot computation per lane and link.
// -------------------------------------------------------------------------
template <class L, int ORDER, typename S, typename C, int E, int H, bool FD = false,
          bool PAD = true, bool RB = false>
struct StreamCollide {
  using ML = MomentLayout<L>;
  using CL = CoefLayout<L, ORDER>;
  static constexpr int M = ML::M;
  static constexpr int K = CL::K;
  static constexpr int W = 64 * E * H;  // nodes per segment

  struct Lane {
    int64_t xh[H];    // first node of this lane's chunk h
    bool act[H];      // chunk h starts inside the row
    int tl[H];        // position of the row's last node x = nx - 1 in chunk h, E if absent
    uint32_t bs[H];   // RB: byte offset of chunk h's first node from its row's slot (S)
    int64_t y, z, rowbase;
  };

  // Emit link A for this lane's nodes.
  template <int A>
  __device__ __forceinline__ static void link(S* __restrict__ f, const StepParams<C>& p,
                                              const C (&own)[H][E][K], const C (&left)[H][K],
                                              const C (&right)[H][K], const Lane& ln) {
    constexpr int cx = L::c[A][0], cy = L::c[A][1], cz = L::c[A][2];
    constexpr int AB = opposite<L>(A);
    int64_t ty = ln.y + cy, tz = ln.z + cz;
    bool row_in = true;
    if (cy != 0) {
      if (ty < 0 || ty >= p.ny) {
        if (p.bby) row_in = false;
        else ty = (ty < 0) ? p.ny - 1 : 0;
      }
    }
    if (cz != 0) {
      if (tz < 0 || tz >= p.nz) {
        if (p.bbz) row_in = false;
        else tz = (tz < 0) ? p.nz - 1 : 0;
      }
    }
    const int64_t trow = p.px * (ty + p.ny * tz);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      if (!ln.act[h]) continue;
      const int64_t xs = ln.xh[h];
      const int tl = ln.tl[h];
      if (row_in) {
        // value arriving at x (this lane's nodes) from source x - cx of this row
        C val[E];
        if constexpr (cx == 0) {
#pragma unroll
          for (int e = 0; e < E; ++e) val[e] = link_value<L, ORDER, A, C>(own[h][e]);
        } else if constexpr (cx > 0) {
#pragma unroll
          for (int e = 0; e < E; ++e)
            val[e] = (e > 0) ? link_value<L, ORDER, A, C>(own[h][e > 0 ? e - 1 : 0])
                             : link_value<L, ORDER, A, C>(left[h]);
        } else {
          const C rv = link_value<L, ORDER, A, C>(right[h]);
#pragma unroll
          for (int e = 0; e < E; ++e)
            val[e] = (e < E - 1) ? link_value<L, ORDER, A, C>(own[h][e < E - 1 ? e + 1 : 0]) : rv;
          if constexpr (PAD) {
            // source x + 1 of a padded row's last node (tl < E - 1) is the
            // node after the row end, which right holds
#pragma unroll
            for (int e = 0; e < E - 1; ++e)
              if (e == tl) val[e] = rv;
          }
        }
        S* dst;
        if constexpr (RB) dst = at_bytes(f + slot<L::Q>(p, trow) + A * astride(p), ln.bs[h]);
        else dst = f + slot<L::Q>(p, trow + xs) + A * astride(p);
        const bool cut_lo = (cx > 0) && p.bbx && (xs == 0);   // source x = -1
        const bool cut_hi = (cx < 0) && p.bbx && (tl < E);    // source x = nx
        if (!(cut_lo || cut_hi)) {
          if constexpr (PAD) {
            // the padding after a row's last node keeps zero populations
#pragma unroll
            for (int e = 1; e < E; ++e)
              if (e > tl) val[e] = C(0);
          }
          store_pack<S, C, E>(dst, val);
        } else {
          // x walls: skip the links the wall supplies, and the padding
#pragma unroll
          for (int e = 0; e < E; ++e) {
            if (e > tl || (cut_lo && e == 0) || (cut_hi && e == tl)) continue;
            dst[e] = Codec<S, C>::store(val[e]);
          }
        }
      } else {
        // every node of this row sends link A across a y/z wall: it comes
        // back into the same node as the opposite link
        C bv[E];
        if (!p.moving) {
#pragma unroll
          for (int e = 0; e < E; ++e) bv[e] = link_value<L, ORDER, A, C>(own[h][e]);
        } else {
          // corrections of every wall the link crosses (edges: the sum)
          C cw = C(0);
          if (cy != 0 && (ln.y + cy < 0 || ln.y + cy >= p.ny))
            cw += wall_dot<L, A, C>(p, 2 + (ln.y + cy < 0 ? 0 : 1));
          if (cz != 0 && (ln.z + cz < 0 || ln.z + cz >= p.nz))
            cw += wall_dot<L, A, C>(p, 4 + (ln.z + cz < 0 ? 0 : 1));
#pragma unroll
          for (int e = 0; e < E; ++e) {
            C extra = cw;
            if constexpr (cx != 0) {
              if (p.bbx && cx > 0 && xs + e == p.nx - 1) extra += wall_dot<L, A, C>(p, 1);
              if (p.bbx && cx < 0 && xs + e == 0) extra += wall_dot<L, A, C>(p, 0);
            }
            bv[e] = link_value_plus<L, ORDER, A, C>(own[h][e], extra);
          }
        }
        if constexpr (PAD) {
#pragma unroll
          for (int e = 1; e < E; ++e)
            if (e > tl) bv[e] = C(0);
        }
        if constexpr (RB)
          store_pack<S, C, E>(at_bytes(f + slot<L::Q>(p, ln.rowbase) + AB * astride(p), ln.bs[h]), bv);
        else
          store_pack<S, C, E>(f + slot<L::Q>(p, ln.rowbase + xs) + AB * astride(p), bv);
      }
      if constexpr (cx != 0) {
        if (row_in && p.bbx) {
          if (cx > 0 && tl < E) {
            // this vector holds x = nx - 1, node tl
#pragma unroll
            for (int e = 0; e < E; ++e)
              if (e == tl)
                f[slot<L::Q>(p, ln.rowbase + xs + e) + AB * astride(p)] = Codec<S, C>::store(
                    p.moving ? link_value_plus<L, ORDER, A, C>(own[h][e], wall_dot<L, A, C>(p, 1))
                             : link_value<L, ORDER, A, C>(own[h][e]));
          }
          if (cx < 0 && xs == 0)
            f[slot<L::Q>(p, ln.rowbase) + AB * astride(p)] = Codec<S, C>::store(
                p.moving ? link_value_plus<L, ORDER, A, C>(own[h][0], wall_dot<L, A, C>(p, 0))
                         : link_value<L, ORDER, A, C>(own[h][0]));
        }
      }
    }
  }

  // Links are emitted grouped by target row (c_y, c_z), so that a
  // wavefront finishes the stores into one row before the next (measured
  // 0.7 % faster than the lattice order for D3Q19 FP32 at 512^3).
  template <int I>
  __device__ __forceinline__ static void links(S* __restrict__ f, const StepParams<C>& p,
                                               const C (&own)[H][E][K], const C (&left)[H][K],
                                               const C (&right)[H][K], const Lane& ln) {
    if constexpr (I < L::Q) {
      link<RowOrder<L>::a[I]>(f, p, own, left, right, ln);
      links<I + 1>(f, p, own, left, right, ln);
    }
  }

  __device__ static void load_coef(const C* __restrict__ m, const StepParams<C>& p, int64_t idx,
                                   C (&k)[K]) {
    C mm[M];
    const int64_t ms = slot<M>(p, idx);
#pragma unroll
    for (int q = 0; q < M; ++q) mm[q] = m[ms + q * astride(p)];
    post_collision<L, ORDER, C, FD>(mm, p, k);
  }

  // One wavefront: row segment number `wave` of the domain (wave-uniform).
  __device__ static void run_wave(const C* __restrict__ m, S* __restrict__ f,
                                  const StepParams<C>& p, int64_t wave) {
    const int lane = threadIdx.x & 63;
    const int64_t rows = p.ny * p.nz;
    if (wave >= p.nseg * rows) return;  // whole wavefront leaves together
    const int64_t seg = wave % p.nseg;
    const int64_t row = wave / p.nseg;
    Lane ln;
    ln.y = row % p.ny;
    ln.z = row / p.ny;
    ln.rowbase = p.px * row;
    const int64_t x0 = seg * W;
    const int64_t xend = (x0 + W < p.nx) ? x0 + W : p.nx;
#pragma unroll
    for (int h = 0; h < H; ++h) {
      ln.xh[h] = x0 + (int64_t)h * 64 * E + (int64_t)lane * E;
      ln.act[h] = ln.xh[h] < p.nx;
      const int64_t rem = p.nx - 1 - ln.xh[h];
      ln.tl[h] = (rem >= 0 && rem < E) ? (int)rem : E;
      ln.bs[h] = (uint32_t)(x0 + h * 64 * E + lane * E) * (uint32_t)sizeof(S);
    }

    C own[H][E][K];
    {
      C mv[H][M][E];
#pragma unroll
      for (int h = 0; h < H; ++h)
#pragma unroll
        for (int q = 0; q < M; ++q) {
          if (ln.act[h]) {
            if constexpr (RB)
              load_plain<C, E, false>(
                  at_bytes(m + slot<M>(p, ln.rowbase) + q * astride(p),
                           (uint32_t)(ln.bs[h] / sizeof(S) * sizeof(C))),
                  mv[h][q]);
            else
              load_plain<C, E, false>(m + slot<M>(p, ln.rowbase + ln.xh[h]) + q * astride(p),
                                      mv[h][q]);
          } else {
#pragma unroll
            for (int e = 0; e < E; ++e) mv[h][q][e] = C(0);
          }
        }
#pragma unroll
      for (int h = 0; h < H; ++h)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          C mm[M];
#pragma unroll
          for (int q = 0; q < M; ++q) mm[q] = mv[h][q][e];
          post_collision<L, ORDER, C, FD>(mm, p, own[h][e]);
        }
    }
    // x-neighbours of each chunk's first and last node
    C left[H][K], right[H][K];
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int q = 0; q < K; ++q) {
        left[h][q] = lane_from_below(own[h][E - 1][q]);
        right[h][q] = lane_from_above(own[h][0][q]);
      }
    if constexpr (H > 1) {
      // chunk boundaries inside the segment: lane 0 of chunk h follows lane
      // 63 of chunk h-1
#pragma unroll
      for (int h = 0; h < H; ++h)
#pragma unroll
        for (int q = 0; q < K; ++q) {
          if (h > 0) {
            const C v = lane_bcast(own[h - 1][E - 1][q], 63);
            if (lane == 0) left[h][q] = v;
          }
          if (h < H - 1) {
            const C v = lane_bcast(own[h + 1][0][q], 0);
            if (lane == 63) right[h][q] = v;
          }
        }
    }
    if (lane == 0) {
      int64_t xl = x0 - 1;
      bool ok = true;
      if (xl < 0) {
        if (p.bbx) ok = false;
        else xl = p.nx - 1;
      }
      if (ok) load_coef(m, p, ln.rowbase + xl, left[0]);
    }
#pragma unroll
    for (int h = 0; h < H; ++h) {
      if (ln.act[h] && ln.xh[h] + E >= xend) {
        int64_t xr = xend;
        bool ok = true;
        if (xr >= p.nx) {
          if (p.bbx) ok = false;
          else xr = 0;
        }
        if (ok) load_coef(m, p, ln.rowbase + xr, right[h]);
      }
    }
    links<0>(f, p, own, left, right, ln);
  }
};

// Unit u of U under the order permutation of StepParams::order_mul (units
// past U stay past U).  The host sets order_mul only for U < 2^32, so the
// product fits 64 bits.
template <typename C>
__device__ __forceinline__ int64_t ordered_unit(const StepParams<C>& p, int64_t u, int64_t U) {
  if (p.order_mul == 0 || u >= U) return u;
  return (int64_t)(((uint64_t)u * (uint64_t)(uint32_t)p.order_mul) % (uint64_t)U);
}

template <class L, int ORDER, typename S, typename C, int E, int H, bool FD = false,
          bool PAD = true, bool RB = false>
__global__ __launch_bounds__(256) void k_stream_collide(const C* __restrict__ m,
                                                        S* __restrict__ f, StepParams<C> p) {
  int64_t w = flat_block() * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if constexpr (RB) w = uniform64(w);  // the row base in scalar registers
  StreamCollide<L, ORDER, S, C, E, H, FD, PAD, RB>::run_wave(
      m, f, p, ordered_unit(p, w, p.nseg * p.ny * p.nz));
}

// -------------------------------------------------------------------------
// Initialisation: populations at equilibrium of given fields (Pi^neq = 0).
// stage holds (1 + D) x cnt doubles: drho, then u.
// -------------------------------------------------------------------------
template <class L, int ORDER, typename S, typename C, int A>
__device__ __forceinline__ void init_links(S* __restrict__ f, int64_t B, int64_t fs,
                                           const C (&k)[CoefLayout<L, ORDER>::K]) {
  if constexpr (A < L::Q) {
    f[fs + A * B] = Codec<S, C>::store(link_value<L, ORDER, A, C>(k));
    init_links<L, ORDER, S, C, A + 1>(f, B, fs, k);
  }
}

template <class L, int ORDER, typename S, typename C>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ stage, int64_t n0,
                                              int64_t cnt, S* __restrict__ f, StepParams<C> p) {
  using ML = MomentLayout<L>;
  using CL = CoefLayout<L, ORDER>;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  C mm[ML::M];
#pragma unroll
  for (int q = 0; q < ML::M; ++q) mm[q] = C(0);
  mm[ML::RHO] = (C)stage[i];
#pragma unroll
  for (int al = 0; al < L::D; ++al) mm[ML::J + al] = p.rho0 * (C)stage[(int64_t)(1 + al) * cnt + i];
  StepParams<C> q = p;  // equilibrium: no force, no non-equilibrium part
#pragma unroll
  for (int al = 0; al < 3; ++al) {
    q.F[al] = C(0);
    q.halfF[al] = C(0);
  }
  C k[CL::K];
  post_collision<L, ORDER, C>(mm, q, k);
  init_links<L, ORDER, S, C, 0>(f, astride(p), slot<L::Q>(p, node_at(p, n0 + i)), k);
}

// -------------------------------------------------------------------------
// Moment read-out for the host: rho, u, Pi^neq of nodes [n0, n0 + cnt) as
// FP64, (1 + D + D(D+1)/2) x cnt.
// -------------------------------------------------------------------------
template <class L, typename S, typename C>
__global__ __launch_bounds__(256) void k_readout(const S* __restrict__ f, double* __restrict__ out,
                                                 int64_t n0, int64_t cnt, StepParams<C> p) {
  using ML = MomentLayout<L>;
  constexpr int D = L::D;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  C s[L::Q], me[ML::M];
  const int64_t fs = slot<L::Q>(p, node_at(p, n0 + i));
#pragma unroll
  for (int a = 0; a < L::Q; ++a) s[a] = Codec<S, C>::load(f[fs + a * astride(p)]);
  node_moments<L, C>(s, p, me);
  out[i] = (double)p.rho0 + (double)me[ML::RHO];  // keep the deviation's digits
#pragma unroll
  for (int al = 0; al < D; ++al)
    out[(int64_t)(1 + al) * cnt + i] = (double)((me[ML::J + al] + p.halfF[al]) * p.inv_rho0);
#pragma unroll
  for (int q = 0; q < D * (D + 1) / 2; ++q)
    out[(int64_t)(1 + D + q) * cnt + i] = (double)me[ML::PID + q];
}

// -------------------------------------------------------------------------
// FP64 conservation reductions: sum over nodes of drho and j.
// partial[block * 8 + {0: drho, 1..3: j}].
// -------------------------------------------------------------------------
template <class L, typename S, typename C>
__global__ __launch_bounds__(256) void k_conserved(const S* __restrict__ f,
                                                   double* __restrict__ partial, int64_t N,
                                                   StepParams<C> p) {
  __shared__ double red[4][256];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += stride) {
    const int64_t fs = slot<L::Q>(p, node_at(p, n));
#pragma unroll
    for (int a = 0; a < L::Q; ++a) {
      const double s = (double)Codec<S, C>::load(f[fs + a * astride(p)]);
      acc[0] += s;
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        if (L::c[a][al] > 0) acc[1 + al] += s;
        if (L::c[a][al] < 0) acc[1 + al] -= s;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 4; ++q) partial[(int64_t)blockIdx.x * 8 + q] = red[q][0];
}

}  // namespace lbk
