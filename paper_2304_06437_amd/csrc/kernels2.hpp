// Two-species colour-gradient kernels (Section 2.1), D2Q9 and D3Q19.
//
// The mixture g = f_R + f_B is relaxed with the regularized collision of
// kernels.hpp (one set of moments for the mixture), perturbed by
//   Omega1_a = (9/4) sigma omega |G| ( t_a (c_a.n)^2 - B_a ),  n = G/|G|,
// and recoloured (Latva-Kokko):
//   f_R,a = (rho_R/rho) g*_a + beta (rho_R rho_B / rho) t_a cos(theta_a),
//   f_B,a = g*_a - f_R,a,  cos(theta_a) = c_a.n / |c_a|,
// where G = grad phi, phi = (rho_R - rho_B)/rho, from the isotropic stencil
// G = (1/cs2) sum_b t_b c_b phi(x + c_b) (neighbours beyond a wall take the
// node's own phi).  No perturbation and cos(theta) = 0 where |G|^2 <= 1e-20.
//
// Storage: set 0 holds the mixture shifted, g_a - t_a rho0 (so its velocity
// keeps full precision).  Set 1 holds the red populations relative to a
// per-node reference colour ref(x) in {0, 1} (one byte per storage node):
//   r_a(x) = f_R,a(x) - ref(x) g_a(x),
// i.e. the red populations themselves at a blue-dominant node (ref 0) and
// minus the blue ones at a red-dominant node (ref 1): in both pure phases
// the stored values are small, so FP32 spends its digits on the colour
// field's deviations, not on t_a rho.  The stream-collide sweep sets ref(x)
// = [phi(x) > 0] from the phase it reads, for every node it owns, and
// encodes every link it writes into x with that same value; the next
// moments sweep decodes with it: rho_R = sum_a r_a + ref rho.  The moments
// sweep writes drho, j, Pi^neq and phi (M + 1 arrays).
//
// Near-contact interactions (Section 2.2, optional): after the moments
// sweep a flag pass marks the interface nodes on which a short-range
// repulsion acts; the stream-collide sweep adds the body force
// A rho_R n to the collision of every flagged node (see k_nci_flags).
#pragma once

#include "kernels.hpp"

namespace lbk {

// Lattice weights t_a and perturbation weights B_a as integers over one
// denominator (t_a = tmul/den, B_a = bmul/den), so that the perturbation
// and the colour split are formed with one rounding per node and their
// lattice sums carry no fixed-sign error from rounded constants.
template <class L>
struct ColourWeights;

// Reis & Phillips (2007) set for D2Q9: B = (-4/27, 2/27, 5/108).
template <>
struct ColourWeights<D2Q9> {
  static constexpr int den = 108;
  static constexpr int tmul[9] = {48, 12, 12, 12, 12, 3, 3, 3, 3};
  static constexpr int bmul[9] = {-16, 8, 8, 8, 8, 5, 5, 5, 5};
};

// Liu, Valocchi & Kang (2012) set for D3Q19: B = (-1/3, 1/18, 1/36).
template <>
struct ColourWeights<D3Q19> {
  static constexpr int den = 36;
  static constexpr int tmul[19] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
  static constexpr int bmul[19] = {-12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
};

template <class L>
constexpr bool colour_weights_consistent() {
  int tsum = 0, bsum = 0;
  for (int a = 0; a < L::Q; ++a) {
    if (ColourWeights<L>::tmul[a] * L::wden != L::wmul[a] * ColourWeights<L>::den) return false;
    tsum += ColourWeights<L>::tmul[a];
    bsum += ColourWeights<L>::bmul[a];
  }
  // sum t = 1 and sum B = cs2
  return tsum == ColourWeights<L>::den && 3 * bsum == ColourWeights<L>::den;
}
static_assert(colour_weights_consistent<D2Q9>(), "D2Q9 colour weights");
static_assert(colour_weights_consistent<D3Q19>(), "D3Q19 colour weights");

template <typename C>
struct ColourParams {
  C pert;                // (9/4) sigma omega / den
  C beta;                // beta / den
  unsigned char* ref;    // reference colour per storage node (see above)
};

// Per-node state carried along x in the two-species sweep:
// post-collision coefficients of the mixture, then S = (9/4) sigma omega |G|
// / den, the unit normal n (D), rho_R/rho, rho_R rho0 / den,
// beta rho_R rho_B / (rho den), rho_B/rho and rho_B rho0 / den.
template <class L>
struct ColourLayout {
  static constexpr int K = CoefLayout<L, 2>::K;
  static constexpr int S = K;
  static constexpr int N = K + 1;
  static constexpr int XR = K + 1 + L::D;
  static constexpr int R0 = K + 2 + L::D;
  static constexpr int RB = K + 3 + L::D;
  static constexpr int XB = K + 4 + L::D;
  static constexpr int B0 = K + 5 + L::D;
  static constexpr int KT = K + 6 + L::D;
};

// V reference-colour bytes of consecutive storage nodes (an aligned block).
template <int V>
__device__ __forceinline__ void load_ref(const unsigned char* __restrict__ ref, int64_t n,
                                         unsigned char (&out)[V]) {
  if constexpr (V == 1) out[0] = ref[n];
  else raw_load<V, false>(ref + n, out);
}

template <int V>
__device__ __forceinline__ void store_ref(unsigned char* __restrict__ ref, int64_t n,
                                          const unsigned char (&in)[V]) {
  if constexpr (V == 1) ref[n] = in[0];
  else raw_store<V, false>(ref + n, in);
}

// Moments sweep: mixture moments from set 0, red density from set 1 and
// the reference colour, rho_R = sum_a r_a + ref rho, and
// phi = (2 rho_R - rho)/rho = (2 ref - 1) + 2 (sum_a r_a)/rho.
template <class L, typename S, typename C, int V>
__device__ __forceinline__ void moments2_body(const S* __restrict__ f, C* __restrict__ m,
                                              const StepParams<C>& p, const ColourParams<C>& cp,
                                              int64_t i0) {
  using ML = MomentLayout<L>;
  if (i0 >= p.npad) return;
  // population region: 2Q arrays (set 0, then set 1); moment region: M + 1
  const int64_t B = astride(p), fs = slot<2 * L::Q>(p, i0), ms = slot<ML::M + 1>(p, i0);
  C s[L::Q][V];
  C rr[V];
#pragma unroll
  for (int a = 0; a < L::Q; ++a) load_pack<S, C, V>(f + fs + a * B, s[a]);
#pragma unroll
  for (int e = 0; e < V; ++e) rr[e] = C(0);
#pragma unroll
  for (int a = 0; a < L::Q; ++a) {
    C r[V];
    load_pack<S, C, V>(f + fs + (L::Q + a) * B, r);
#pragma unroll
    for (int e = 0; e < V; ++e) rr[e] += r[e];
  }
  unsigned char ref[V];
  load_ref<V>(cp.ref, i0, ref);
  C out[ML::M + 1][V];
#pragma unroll
  for (int e = 0; e < V; ++e) {
    C se[L::Q], me[ML::M];
#pragma unroll
    for (int a = 0; a < L::Q; ++a) se[a] = s[a][e];
    node_moments<L, C>(se, p, me);
#pragma unroll
    for (int q = 0; q < ML::M; ++q) out[q][e] = me[q];
    const C rho = p.rho0 + me[ML::RHO];
    out[ML::M][e] = (ref[e] ? C(1) : C(-1)) + C(2) * rr[e] / rho;
  }
#pragma unroll
  for (int q = 0; q <= ML::M; ++q) store_plain<C, V>(m + ms + q * B, out[q]);
}

template <class L, typename S, typename C, int V>
__global__ __launch_bounds__(256) void k_moments2(const S* __restrict__ f, C* __restrict__ m,
                                                  StepParams<C> p, ColourParams<C> cp) {
  moments2_body<L, S, C, V>(f, m, p, cp, (flat_block() * blockDim.x + threadIdx.x) * V);
}

// Index of the phase field of node n: the last of the M + 1 moment arrays.
template <class L, typename C>
__device__ __forceinline__ int64_t phi_index(const StepParams<C>& p, int64_t n) {
  return slot<MomentLayout<L>::M + 1>(p, n) + MomentLayout<L>::M * astride(p);
}

// Phase field of node (x + dx, ty, tz) given the wrapped/validated row
// (ty, tz): x wraps for periodic x; beyond an x wall the node's own phi.
template <class L, typename C>
__device__ __forceinline__ C phi_at(const C* __restrict__ m, const StepParams<C>& p,
                                    int64_t trow_base, int64_t x, int dx, C own) {
  int64_t xx = x + dx;
  if (xx < 0 || xx >= p.nx) {
    if (p.bbx) return own;
    xx = (xx < 0) ? p.nx - 1 : 0;
  }
  return m[phi_index<L>(p, trow_base + xx)];
}

// -------------------------------------------------------------------------
// Near-contact interactions (Section 2.2).
//
// Flag pass, gather form of the paper's rule.  The paper sits on a bulk node
// x of the continuous phase (phi(x) < -1 + eps), samples phi at x + d c_a
// and x - d c_a for each pair of opposite lattice directions, and flags both
// points when neither is bulk.  Seen from a node y, that is: y is flagged
// when it is not bulk and, for some direction c_a, the node y - d c_a is
// bulk while y - 2 d c_a is not.  Points beyond a bounce-back wall are not
// sampled; periodic axes wrap.  One thread per storage node, padding nodes
// get 0.
// Force: a flagged node with a defined phase gradient G carries
// F = A rho_R G/|G| (along the interface normal, into the dispersed red
// phase), added to the constant body force in its collision.
// -------------------------------------------------------------------------
template <typename C>
struct NciParams {
  C strength;      // A
  C thr;           // -1 + eps: phi below it is continuous-phase bulk
  int32_t reach;   // sampling distance d in lattice spacings
  int32_t pad_;
};

// Storage node of (x, y, z) + k c_A, or -1 when it lies beyond a wall.
template <class L, int A, typename C>
__device__ __forceinline__ int64_t shifted_node(const StepParams<C>& p, int64_t x, int64_t y,
                                                int64_t z, int64_t k) {
  int64_t t[3] = {x + k * L::c[A][0], y + k * L::c[A][1], z + k * L::c[A][2]};
  const int64_t n[3] = {p.nx, p.ny, p.nz};
  const int32_t bb[3] = {p.bbx, p.bby, p.bbz};
#pragma unroll
  for (int al = 0; al < 3; ++al) {
    if (t[al] < 0 || t[al] >= n[al]) {
      if (bb[al]) return -1;
      t[al] = ((t[al] % n[al]) + n[al]) % n[al];
    }
  }
  return t[0] + p.px * (t[1] + p.ny * t[2]);
}

// Is there a direction c_A (A >= A0, not the rest link) with y - d c_A bulk
// and y - 2 d c_A not bulk?
template <class L, typename C, int A = 1>
__device__ __forceinline__ bool nci_sees_pair(const C* __restrict__ m, const StepParams<C>& p,
                                              const NciParams<C>& q, int64_t x, int64_t y,
                                              int64_t z) {
  if constexpr (A < L::Q) {
    const int64_t s1 = shifted_node<L, A>(p, x, y, z, -(int64_t)q.reach);
    const int64_t s2 = shifted_node<L, A>(p, x, y, z, -2 * (int64_t)q.reach);
    if (s1 >= 0 && s2 >= 0 && m[phi_index<L>(p, s1)] < q.thr && m[phi_index<L>(p, s2)] > q.thr)
      return true;
    return nci_sees_pair<L, C, A + 1>(m, p, q, x, y, z);
  } else {
    return false;
  }
}

template <class L, typename C>
__global__ __launch_bounds__(256) void k_nci_flags(const C* __restrict__ m,
                                                   unsigned char* __restrict__ flag,
                                                   StepParams<C> p, NciParams<C> q) {
  const int64_t n = flat_block() * blockDim.x + threadIdx.x;
  if (n >= p.npad) return;
  const int64_t x = n % p.px, row = n / p.px;
  bool fl = false;
  if (x < p.nx && row < p.ny * p.nz) {
    const int64_t y = row % p.ny, z = row / p.ny;
    if (m[phi_index<L>(p, n)] > q.thr) fl = nci_sees_pair<L, C>(m, p, q, x, y, z);
  }
  flag[n] = fl ? 1 : 0;
}

// Post-collision coefficients of a flagged node: its collision sees the body
// force F + A rho_R G/|G| (G the phase gradient, |G| = Gn > 0, xr = rho_R/rho).
// The stored Pi^neq was formed with the velocity u = (j + F/2)/rho0 of the
// constant force; the extra half force shifts u, so Pi^neq = P - drho cs2 I
// - rho0 u u gains rho0 (u u - u' u').
template <class L, typename C>
__device__ __forceinline__ void nci_coefficients(const C (&m0)[MomentLayout<L>::M],
                                                 const C (&G)[3], C Gn, C xr,
                                                 const StepParams<C>& p, const NciParams<C>& q,
                                                 C (&k)[CoefLayout<L, 2>::K]) {
  using ML = MomentLayout<L>;
  constexpr int D = L::D;
  const C rho = p.rho0 + m0[ML::RHO];
  const C scale = q.strength * (xr * rho) / Gn;
  StepParams<C> pf = p;
  C mm[ML::M];
#pragma unroll
  for (int i = 0; i < ML::M; ++i) mm[i] = m0[i];
  C ug[D], un[D];
#pragma unroll
  for (int al = 0; al < D; ++al) {
    pf.F[al] = p.F[al] + scale * G[al];
    pf.halfF[al] = C(0.5) * pf.F[al];
    ug[al] = (mm[ML::J + al] + p.halfF[al]) * p.inv_rho0;
    un[al] = (mm[ML::J + al] + pf.halfF[al]) * p.inv_rho0;
  }
#pragma unroll
  for (int al = 0; al < D; ++al) {
    mm[ML::PID + al] += p.rho0 * (ug[al] * ug[al] - un[al] * un[al]);
#pragma unroll
    for (int be = al + 1; be < D; ++be)
      mm[ML::PIO + offdiag(al, be)] += p.rho0 * (ug[al] * ug[be] - un[al] * un[be]);
  }
  post_collision<L, 2, C>(mm, pf, k);
}

// Full per-node state of node (x, y, z) by scalar loads (segment halos).
template <class L, typename C, bool NCI = false>
__device__ void colour_state_scalar(const C* __restrict__ m, const StepParams<C>& p,
                                    const ColourParams<C>& cp, int64_t x, int64_t y, int64_t z,
                                    C (&st)[ColourLayout<L>::KT],
                                    const unsigned char* __restrict__ flag = nullptr,
                                    const NciParams<C>& q = NciParams<C>{}) {
  using ML = MomentLayout<L>;
  using XL = ColourLayout<L>;
  constexpr int D = L::D;
  const int64_t n = x + p.px * (y + p.ny * z);
  C mm[ML::M];
#pragma unroll
  for (int q = 0; q < ML::M; ++q) mm[q] = m[slot<ML::M + 1>(p, n) + q * astride(p)];
  C k[XL::K];
  post_collision<L, 2, C>(mm, p, k);
#pragma unroll
  for (int q = 0; q < XL::K; ++q) st[q] = k[q];
  const C own = m[phi_index<L>(p, n)];
  // same row-by-row summation order as the vector path in StreamCollide2
  C G[3] = {C(0), C(0), C(0)};
#pragma unroll
  for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      bool has[3] = {false, false, false};
      int wm[3] = {0, 0, 0};
#pragma unroll
      for (int b = 1; b < L::Q; ++b)
        if (L::c[b][1] == dy && L::c[b][2] == dz) {
          has[L::c[b][0] + 1] = true;
          wm[L::c[b][0] + 1] = L::wmul[b];
        }
      if (!(has[0] || has[1] || has[2])) continue;
      int64_t ty = y + dy, tz = z + dz;
      bool inside = true;
      if (ty < 0 || ty >= p.ny) {
        if (p.bby) inside = false;
        else ty = (ty < 0) ? p.ny - 1 : 0;
      }
      if (tz < 0 || tz >= p.nz) {
        if (p.bbz) inside = false;
        else tz = (tz < 0) ? p.nz - 1 : 0;
      }
      const int64_t tb = p.px * (ty + p.ny * tz);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if (!has[dx + 1]) continue;
        const C v = inside ? phi_at<L, C>(m, p, tb, x, dx, own) : own;
        const C wv = C(wm[dx + 1]) * v;
        if (dx > 0) G[0] += wv;
        if (dx < 0) G[0] -= wv;
        if (dy > 0) G[1] += wv;
        if (dy < 0) G[1] -= wv;
        if (D == 3) {
          if (dz > 0) G[2] += wv;
          if (dz < 0) G[2] -= wv;
        }
      }
    }
  const C rho = p.rho0 + mm[ML::RHO];
  const C xr = (C(1) + own) * C(0.5);
  const C xb = (C(1) - own) * C(0.5);
  // G = (1/cs2) sum t_b c_b phi = (3/wden) sum wmul_b c_b phi
  C G2 = C(0);
#pragma unroll
  for (int al = 0; al < D; ++al) {
    G[al] = scaled<3, L::wden>(G[al]);
    G2 += G[al] * G[al];
  }
  if (G2 > C(1e-20)) {
    const C Gn = sqrt(G2);
    st[XL::S] = cp.pert * Gn;
#pragma unroll
    for (int al = 0; al < D; ++al) st[XL::N + al] = G[al] / Gn;
    if constexpr (NCI) {
      if (flag[n]) {
        C kf[XL::K];
        nci_coefficients<L, C>(mm, G, Gn, xr, p, q, kf);
#pragma unroll
        for (int i = 0; i < XL::K; ++i) st[i] = kf[i];
      }
    }
  } else {
    st[XL::S] = C(0);
#pragma unroll
    for (int al = 0; al < D; ++al) st[XL::N + al] = C(0);
  }
  st[XL::XR] = xr;
  st[XL::R0] = scaled<1, ColourWeights<L>::den>(xr * p.rho0);
  st[XL::RB] = cp.beta * xr * xb * rho;
  st[XL::XB] = xb;
  st[XL::B0] = scaled<1, ColourWeights<L>::den>(xb * p.rho0);
}

// Value of link A from a source node's state: the shifted mixture gs and
// the stored red value fr for a destination of reference colour ref.
//   g*_a  = [regularized mixture]_a + S' (tmul_a (c_a.n)^2 - bmul_a)
//   rec   = beta' tmul_a (c_a.n)/|c_a|
//   ref 0: fr = f_R,a = (rho_R/rho)(g*_a + t_a rho0) + rec
//   ref 1: fr = f_R,a - (g*_a + t_a rho0) = -f_B,a = rec - (rho_B/rho)(g*_a + t_a rho0)
// with S' = S/den and beta' = beta rho_R rho_B/(rho den); both forms are
// evaluated from small terms (no cancellation of t_a rho0 sized values).
template <class L, int A, typename C>
__device__ __forceinline__ void colour_link(const C (&st)[ColourLayout<L>::KT], C& gs, C& fr,
                                            bool ref) {
  using XL = ColourLayout<L>;
  using CW = ColourWeights<L>;
  constexpr int D = L::D;
  const C (&k)[XL::K] = *reinterpret_cast<const C(*)[XL::K]>(&st[0]);
  C g = link_value<L, 2, A, C>(k);
  C cn = C(0);
#pragma unroll
  for (int al = 0; al < D; ++al) {
    if (L::c[A][al] > 0) cn += st[XL::N + al];
    if (L::c[A][al] < 0) cn -= st[XL::N + al];
  }
  constexpr int tm = CW::tmul[A];
  constexpr int bm = CW::bmul[A];
  constexpr int c2 = L::c[A][0] * L::c[A][0] + L::c[A][1] * L::c[A][1] + L::c[A][2] * L::c[A][2];
  g += st[XL::S] * (C(tm) * (cn * cn) - C(bm));
  C rec = C(0);
  if constexpr (c2 > 0) {
    constexpr double inv = c2 == 1 ? 1.0 : c2 == 2 ? 0.70710678118654752440 : 0.57735026918962576451;
    rec = st[XL::RB] * (C(tm) * (cn * C(inv)));
  }
  gs = g;
  fr = ref ? rec - (st[XL::XB] * g + C(tm) * st[XL::B0])
           : st[XL::XR] * g + C(tm) * st[XL::R0] + rec;
}

// Row index (0..8) of the target row offset (cy, cz) of a link.
__host__ __device__ constexpr int row_id(int cy, int cz) { return (cy + 1) + 3 * (cz + 1); }

// Stream-collide for two species.  One wavefront per x-row segment of 64 E
// nodes (E per lane), as in StreamCollide; the phase-field gradient reads
// phi from the 3 (2D) or 9 (3D) rows around the source row.  WHOLE: every
// row is one periodic, unpadded segment (nseg = 1, no x walls, px = nx), so
// the states beyond the row's two ends are those of its other end, taken
// from the lanes that hold them instead of recomputed.
template <class L, typename S, typename C, int E, bool WHOLE = false, bool NCI = false>
struct StreamCollide2 {
  using ML = MomentLayout<L>;
  using XL = ColourLayout<L>;
  static constexpr int M = ML::M;
  static constexpr int KT = XL::KT;
  static constexpr int W = 64 * E;

  // tl: position of the row's last node x = nx - 1 in this lane's vector,
  // E if the vector does not hold it (nodes after it are padding).
  // Reference colour (see the file header) of this lane's node e in the row
  // at offset (cy, cz): bit row_id(cy, cz) E + e of the lane's mask.  A row
  // beyond a wall holds the node's own value (its links come back into it).
  __device__ __forceinline__ static bool ref_bit(uint64_t mask, int row, int e) {
    return (mask >> (row * E + e)) & 1;
  }

  template <int A>
  __device__ __forceinline__ static void link(S* __restrict__ f, const StepParams<C>& p,
                                              const C (&own)[E][KT], const C (&left)[KT],
                                              const C (&right)[KT], int64_t xs, int tl,
                                              int64_t y, int64_t z, int64_t rowbase,
                                              uint64_t mask) {
    constexpr int cx = L::c[A][0], cy = L::c[A][1], cz = L::c[A][2];
    constexpr int AB = opposite<L>(A);
    constexpr int trow = row_id(cy, cz), orow = row_id(0, 0);
    int64_t ty = y + cy, tz = z + cz;
    bool row_in = true;
    if (cy != 0 && (ty < 0 || ty >= p.ny)) {
      if (p.bby) row_in = false;
      else ty = (ty < 0) ? p.ny - 1 : 0;
    }
    if (cz != 0 && (tz < 0 || tz >= p.nz)) {
      if (p.bbz) row_in = false;
      else tz = (tz < 0) ? p.nz - 1 : 0;
    }
    S* fr0 = f + A * astride(p);
    S* fr1 = f + (L::Q + A) * astride(p);
    if (row_in) {
      C gv[E], rv[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const bool rf = ref_bit(mask, trow, e);
        if constexpr (cx == 0) {
          colour_link<L, A, C>(own[e], gv[e], rv[e], rf);
        } else if constexpr (cx > 0) {
          if (e > 0) colour_link<L, A, C>(own[e > 0 ? e - 1 : 0], gv[e], rv[e], rf);
          else colour_link<L, A, C>(left, gv[e], rv[e], rf);
        } else {
          if (e < E - 1) colour_link<L, A, C>(own[e < E - 1 ? e + 1 : 0], gv[e], rv[e], rf);
          else colour_link<L, A, C>(right, gv[e], rv[e], rf);
        }
      }
      const bool padded = p.px != p.nx;  // wave-uniform
      if constexpr (cx < 0 && E > 1) {
        if (padded) {
          // the last node of a padded row takes source x + 1 from right
#pragma unroll
          for (int e = 0; e < E - 1; ++e)
            if (e == tl) colour_link<L, A, C>(right, gv[e], rv[e], ref_bit(mask, trow, e));
        }
      }
      // the E nodes from t on lie in one block
      const int64_t t = slot<2 * L::Q>(p, p.px * (ty + p.ny * tz) + xs);
      const bool cut_lo = (cx > 0) && p.bbx && (xs == 0);
      const bool cut_hi = (cx < 0) && p.bbx && (tl < E);
      if (!(cut_lo || cut_hi)) {
        if (padded) {
          // the padding after a row's last node keeps zero populations
#pragma unroll
          for (int e = 1; e < E; ++e)
            if (e > tl) gv[e] = rv[e] = C(0);
        }
        store_pack<S, C, E>(fr0 + t, gv);
        store_pack<S, C, E>(fr1 + t, rv);
      } else {
        // x walls: skip the links the wall supplies, and the padding
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (e > tl || (cut_lo && e == 0) || (cut_hi && e == tl)) continue;
          fr0[t + e] = Codec<S, C>::store(gv[e]);
          fr1[t + e] = Codec<S, C>::store(rv[e]);
        }
      }
    } else {
      C gv[E], rv[E];
#pragma unroll
      for (int e = 0; e < E; ++e)
        colour_link<L, A, C>(own[e], gv[e], rv[e], ref_bit(mask, orow, e));
      const int64_t t = slot<2 * L::Q>(p, rowbase + xs);
      if (p.px != p.nx) {
#pragma unroll
        for (int e = 1; e < E; ++e)
          if (e > tl) gv[e] = rv[e] = C(0);
      }
      store_pack<S, C, E>(f + t + AB * astride(p), gv);
      store_pack<S, C, E>(f + t + (L::Q + AB) * astride(p), rv);
    }
    if constexpr (cx != 0) {
      if (row_in && p.bbx) {
        // x walls: the node next to the wall gets the link back reversed
        if (cx > 0 && tl < E) {
#pragma unroll
          for (int e = 0; e < E; ++e)
            if (e == tl) {
              C g, r;
              colour_link<L, A, C>(own[e], g, r, ref_bit(mask, orow, e));
              const int64_t t = slot<2 * L::Q>(p, rowbase + xs + e);
              f[t + AB * astride(p)] = Codec<S, C>::store(g);
              f[t + (L::Q + AB) * astride(p)] = Codec<S, C>::store(r);
            }
        }
        if (cx < 0 && xs == 0) {
          C g, r;
          colour_link<L, A, C>(own[0], g, r, ref_bit(mask, orow, 0));
          const int64_t t = slot<2 * L::Q>(p, rowbase);
          f[t + AB * astride(p)] = Codec<S, C>::store(g);
          f[t + (L::Q + AB) * astride(p)] = Codec<S, C>::store(r);
        }
      }
    }
  }

  template <int A>
  __device__ __forceinline__ static void links(S* __restrict__ f, const StepParams<C>& p,
                                               const C (&own)[E][KT], const C (&left)[KT],
                                               const C (&right)[KT], int64_t xs, int tl,
                                               int64_t y, int64_t z, int64_t rowbase,
                                               uint64_t mask) {
    if constexpr (A < L::Q) {
      link<A>(f, p, own, left, right, xs, tl, y, z, rowbase, mask);
      links<A + 1>(f, p, own, left, right, xs, tl, y, z, rowbase, mask);
    }
  }

  // flag, q: near-contact flags (one byte per storage node) and parameters,
  // read only when NCI.
  __device__ static void run_wave(const C* __restrict__ m, S* __restrict__ f,
                                  const StepParams<C>& p, const ColourParams<C>& cp,
                                  int64_t wave, const unsigned char* __restrict__ flag = nullptr,
                                  const NciParams<C>& q = NciParams<C>{}) {
    constexpr int D = L::D;
    const int lane = threadIdx.x & 63;
    const int64_t rows = p.ny * p.nz;
    if (wave >= p.nseg * rows) return;
    const int64_t seg = wave % p.nseg;
    const int64_t row = wave / p.nseg;
    const int64_t y = row % p.ny, z = row / p.ny;
    const int64_t rowbase = p.px * row;
    const int64_t x0 = seg * W;
    const int64_t xend = (x0 + W < p.nx) ? x0 + W : p.nx;
    const int64_t xs = x0 + (int64_t)lane * E;
    const bool act = xs < p.nx;
    const int64_t rem = p.nx - 1 - xs;
    const int tl = (rem >= 0 && rem < E) ? (int)rem : E;

    C own[E][KT];
    C phio[E];
    C mv[M][E];  // the lane's moments (the near-contact force revisits them)
    {
#pragma unroll
      for (int q = 0; q < M; ++q) {
        if (act) load_plain<C, E, false>(m + slot<M + 1>(p, rowbase + xs) + q * astride(p), mv[q]);
        else
#pragma unroll
          for (int e = 0; e < E; ++e) mv[q][e] = C(0);
      }
      if (act) load_plain<C, E, false>(m + phi_index<L>(p, rowbase + xs), phio);
      else
#pragma unroll
        for (int e = 0; e < E; ++e) phio[e] = C(0);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        C mm[M];
#pragma unroll
        for (int q = 0; q < M; ++q) mm[q] = mv[q][e];
        C k[XL::K];
        post_collision<L, 2, C>(mm, p, k);
#pragma unroll
        for (int q = 0; q < XL::K; ++q) own[e][q] = k[q];
        const C rho = p.rho0 + mm[ML::RHO];
        const C xr = (C(1) + phio[e]) * C(0.5);
        const C xb = (C(1) - phio[e]) * C(0.5);
        own[e][XL::XR] = xr;
        own[e][XL::R0] = scaled<1, ColourWeights<L>::den>(xr * p.rho0);
        own[e][XL::RB] = cp.beta * xr * xb * rho;
        own[e][XL::XB] = xb;
        own[e][XL::B0] = scaled<1, ColourWeights<L>::den>(xb * p.rho0);
      }
    }
    // phase-field gradient of this lane's nodes from the rows around it
    C G[E][3];
    uint64_t mask = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) G[e][0] = G[e][1] = G[e][2] = C(0);
#pragma unroll
    for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        // links of the stencil reaching row (y + dy, z + dz): c_bx in {-1,0,1}
        bool has[3] = {false, false, false};
        int wm[3] = {0, 0, 0};
#pragma unroll
        for (int b = 1; b < L::Q; ++b)
          if (L::c[b][1] == dy && L::c[b][2] == dz) {
            has[L::c[b][0] + 1] = true;
            wm[L::c[b][0] + 1] = L::wmul[b];
          }
        if (!(has[0] || has[1] || has[2])) continue;
        int64_t ty = y + dy, tz = z + dz;
        bool inside = true;
        if (ty < 0 || ty >= p.ny) {
          if (p.bby) inside = false;
          else ty = (ty < 0) ? p.ny - 1 : 0;
        }
        if (tz < 0 || tz >= p.nz) {
          if (p.bbz) inside = false;
          else tz = (tz < 0) ? p.nz - 1 : 0;
        }
        const int64_t tb = p.px * (ty + p.ny * tz);
        C pv[E];
        if (inside) {
          if (act) load_plain<C, E, false>(m + phi_index<L>(p, tb + xs), pv);
          else
#pragma unroll
            for (int e = 0; e < E; ++e) pv[e] = C(0);
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) pv[e] = phio[e];
        }
        // reference colours of the nodes this lane writes into in this row
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (pv[e] > C(0)) mask |= uint64_t(1) << (row_id(dy, dz) * E + e);
        // x-neighbours of the lane's first and last node in this row
        C pl = lane_from_below(pv[E - 1]);
        C pr = lane_from_above(pv[0]);
        if (inside) {
          if (lane == 0) pl = phi_at<L, C>(m, p, tb, x0, -1, phio[0]);
          if (act && xs + E >= xend) pr = phi_at<L, C>(m, p, tb, xend - 1, 1, phio[E - 1]);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
          C vals[3];
          vals[1] = pv[e];
          vals[0] = (e > 0) ? pv[e > 0 ? e - 1 : 0] : pl;
          vals[2] = (e < E - 1 && e != tl) ? pv[e < E - 1 ? e + 1 : 0] : pr;
          if (!inside) {
            // the row lies beyond a y/z wall: every neighbour takes the own value
            vals[0] = vals[1] = vals[2] = phio[e];
          } else if (p.bbx) {
            // x walls: neighbours beyond x = 0 / nx - 1 take the own value
            if (xs + e == 0) vals[0] = phio[e];
            if (xs + e == p.nx - 1) vals[2] = phio[e];
          }
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            if (!has[dx + 1]) continue;
            const C wv = C(wm[dx + 1]) * vals[dx + 1];
            if (dx > 0) G[e][0] += wv;
            if (dx < 0) G[e][0] -= wv;
            if (dy > 0) G[e][1] += wv;
            if (dy < 0) G[e][1] -= wv;
            if (D == 3) {
              if (dz > 0) G[e][2] += wv;
              if (dz < 0) G[e][2] -= wv;
            }
          }
        }
      }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      C G2 = C(0);
#pragma unroll
      for (int al = 0; al < D; ++al) {
        G[e][al] = scaled<3, L::wden>(G[e][al]);
        G2 += G[e][al] * G[e][al];
      }
      if (G2 > C(1e-20)) {
        const C Gn = sqrt(G2);
        own[e][XL::S] = cp.pert * Gn;
#pragma unroll
        for (int al = 0; al < D; ++al) own[e][XL::N + al] = G[e][al] / Gn;
        if constexpr (NCI) {
          if (act && flag[rowbase + xs + e]) {
            C mm[M], kf[XL::K];
#pragma unroll
            for (int i = 0; i < M; ++i) mm[i] = mv[i][e];
            nci_coefficients<L, C>(mm, G[e], Gn, own[e][XL::XR], p, q, kf);
#pragma unroll
            for (int i = 0; i < XL::K; ++i) own[e][i] = kf[i];
          }
        }
      } else {
        own[e][XL::S] = C(0);
#pragma unroll
        for (int al = 0; al < D; ++al) own[e][XL::N + al] = C(0);
      }
    }
    C left[KT], right[KT];
#pragma unroll
    for (int q = 0; q < KT; ++q) {
      left[q] = lane_from_below(own[E - 1][q]);
      right[q] = lane_from_above(own[0][q]);
    }
    if constexpr (WHOLE) {
      // the whole periodic row is in this wavefront: the neighbours of its
      // ends are the states of its other end, already in registers (lane lt
      // holds x = nx - 1 as its last node)
      const int lt = (int)(p.nx / E) - 1;  // wave-uniform
#pragma unroll
      for (int q = 0; q < KT; ++q) {
        const C vl = lane_bcast(own[E - 1][q], lt);
        const C vr = lane_bcast(own[0][q], 0);
        if (lane == 0) left[q] = vl;
        if (lane == lt) right[q] = vr;
      }
    } else {
      if (lane == 0) {
        int64_t xl = x0 - 1;
        bool ok = true;
        if (xl < 0) {
          if (p.bbx) ok = false;
          else xl = p.nx - 1;
        }
        if (ok) colour_state_scalar<L, C, NCI>(m, p, cp, xl, y, z, left, flag, q);
      }
      if (act && xs + E >= xend) {
        int64_t xr = xend;
        bool ok = true;
        if (xr >= p.nx) {
          if (p.bbx) ok = false;
          else xr = 0;
        }
        if (ok) colour_state_scalar<L, C, NCI>(m, p, cp, xr, y, z, right, flag, q);
      }
    }
    if (!act) return;
    {
      // this lane's nodes keep the reference colour every link into them uses
      unsigned char rb[E];
#pragma unroll
      for (int e = 0; e < E; ++e) rb[e] = (e <= tl && phio[e] > C(0)) ? 1 : 0;
      store_ref<E>(cp.ref, rowbase + xs, rb);
    }
    links<0>(f, p, own, left, right, xs, tl, y, z, rowbase, mask);
  }
};

template <class L, typename S, typename C, int E, bool WHOLE = false, bool NCI = false>
__global__ __launch_bounds__(256) void k_stream_collide2(const C* __restrict__ m,
                                                         S* __restrict__ f, StepParams<C> p,
                                                         ColourParams<C> cp,
                                                         const unsigned char* __restrict__ flag,
                                                         NciParams<C> q) {
  const int64_t w = flat_block() * (blockDim.x >> 6) + (threadIdx.x >> 6);
  StreamCollide2<L, S, C, E, WHOLE, NCI>::run_wave(
      m, f, p, cp, ordered_unit(p, w, p.nseg * p.ny * p.nz), flag, q);
}

// Initialisation: set 0 = f^eq - t rho0; red f_R = (1 + phi)/2 f^eq stored
// relative to the reference colour [phi > 0]: (1 + phi)/2 f^eq, or
// -(1 - phi)/2 f^eq.  stage: (2 + D) x cnt doubles: drho, u, phi.
template <class L, typename S, typename C, int A>
__device__ __forceinline__ void init2_links(S* __restrict__ f, int64_t B, int64_t fs,
                                            const C (&k)[CoefLayout<L, 2>::K], C rho0, C xr,
                                            C xb, bool ref) {
  if constexpr (A < L::Q) {
    const C s = link_value<L, 2, A, C>(k);
    f[fs + A * B] = Codec<S, C>::store(s);
    const C feq = s + C(L::w[A]) * rho0;
    f[fs + (L::Q + A) * B] = Codec<S, C>::store(ref ? -(xb * feq) : xr * feq);
    init2_links<L, S, C, A + 1>(f, B, fs, k, rho0, xr, xb, ref);
  }
}

template <class L, typename S, typename C>
__global__ __launch_bounds__(256) void k_init2(const double* __restrict__ stage, int64_t n0,
                                               int64_t cnt, S* __restrict__ f, StepParams<C> p,
                                               ColourParams<C> cp) {
  using ML = MomentLayout<L>;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  C mm[ML::M];
#pragma unroll
  for (int q = 0; q < ML::M; ++q) mm[q] = C(0);
  mm[ML::RHO] = (C)stage[i];
#pragma unroll
  for (int al = 0; al < L::D; ++al) mm[ML::J + al] = p.rho0 * (C)stage[(int64_t)(1 + al) * cnt + i];
  const C phi = (C)stage[(int64_t)(1 + L::D) * cnt + i];
  const C xr = (C(1) + phi) * C(0.5);
  const C xb = (C(1) - phi) * C(0.5);
  const bool ref = phi > C(0);
  StepParams<C> q = p;
#pragma unroll
  for (int al = 0; al < 3; ++al) {
    q.F[al] = C(0);
    q.halfF[al] = C(0);
  }
  C k[CoefLayout<L, 2>::K];
  post_collision<L, 2, C>(mm, q, k);
  const int64_t n = node_at(p, n0 + i);
  init2_links<L, S, C, 0>(f, astride(p), slot<2 * L::Q>(p, n), k, p.rho0, xr, xb, ref);
  cp.ref[n] = ref ? 1 : 0;
}

// Read-out: rho, u, Pi^neq of the mixture and phi; (2 + D + D(D+1)/2) x cnt.
template <class L, typename S, typename C>
__global__ __launch_bounds__(256) void k_readout2(const S* __restrict__ f, double* __restrict__ out,
                                                  int64_t n0, int64_t cnt, StepParams<C> p,
                                                  ColourParams<C> cp) {
  using ML = MomentLayout<L>;
  constexpr int D = L::D;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  C s[L::Q], me[ML::M];
  C rr = C(0);
  const int64_t n = node_at(p, n0 + i);
  const int64_t fs = slot<2 * L::Q>(p, n);
#pragma unroll
  for (int a = 0; a < L::Q; ++a) {
    s[a] = Codec<S, C>::load(f[fs + a * astride(p)]);
    rr += Codec<S, C>::load(f[fs + (L::Q + a) * astride(p)]);
  }
  node_moments<L, C>(s, p, me);
  const C rho = p.rho0 + me[ML::RHO];
  out[i] = (double)p.rho0 + (double)me[ML::RHO];
#pragma unroll
  for (int al = 0; al < D; ++al)
    out[(int64_t)(1 + al) * cnt + i] = (double)((me[ML::J + al] + p.halfF[al]) * p.inv_rho0);
#pragma unroll
  for (int q = 0; q < D * (D + 1) / 2; ++q)
    out[(int64_t)(1 + D + q) * cnt + i] = (double)me[ML::PID + q];
  out[(int64_t)(1 + D + D * (D + 1) / 2) * cnt + i] =
      (double)((cp.ref[n] ? C(1) : C(-1)) + C(2) * rr / rho);
}

// FP64 reductions: drho, j (3), red mass.
template <class L, typename S, typename C>
__global__ __launch_bounds__(256) void k_conserved2(const S* __restrict__ f,
                                                    double* __restrict__ partial, int64_t N,
                                                    StepParams<C> p, ColourParams<C> cp) {
  __shared__ double red[5][256];
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += stride) {
    const int64_t sn = node_at(p, n);
    const int64_t fs = slot<2 * L::Q>(p, sn);
    double drho = 0.0, red = 0.0;
#pragma unroll
    for (int a = 0; a < L::Q; ++a) {
      const double s = (double)Codec<S, C>::load(f[fs + a * astride(p)]);
      drho += s;
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        if (L::c[a][al] > 0) acc[1 + al] += s;
        if (L::c[a][al] < 0) acc[1 + al] -= s;
      }
      red += (double)Codec<S, C>::load(f[fs + (L::Q + a) * astride(p)]);
    }
    acc[0] += drho;
    // red mass of the node: sum_a r_a + ref rho
    acc[4] += red + (cp.ref[sn] ? (double)p.rho0 + drho : 0.0);
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < 5; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 5; ++q) partial[(int64_t)blockIdx.x * 8 + q] = red[q][0];
}

}  // namespace lbk
