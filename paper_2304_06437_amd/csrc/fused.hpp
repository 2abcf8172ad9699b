// Fused step: the moments sweep and the stream-collide sweep in one pass
// (gfx950).
//
// The two-sweep step writes every node's moments to HBM and reads them
// back: 80 of the 232 bytes per lattice update (D3Q19 FP32).  This kernel
// computes the same quantities in the same arithmetic and keeps the
// moments in registers, so each update reads the node's Q populations once
// and writes Q populations once (152 B).  Its results equal the two-sweep
// step's bit for bit.
//
// Work mapping.  A tile is one x-row (y) and a run of consecutive planes
// [z0, z1); one 64-lane wavefront owns a tile and marches through it in z.
// The whole row is in the wavefront (nx = 64 E H: lane l holds nodes
// h 64E + l E + e), so the x-neighbours of every node are in registers of
// the same or the adjacent lane, with the periodic wrap between lanes 63
// and 0.  At plane z the wavefront
//   1. issues the loads of plane z+1 of its row,
//   2. writes the links of plane z that stay in its own row (c_y = 0,
//      c_z <= 0: planes z and z-1, both read already),
//   3. turns plane z+1 into moments and post-collision coefficients
//      (eq. for Pi^neq and the Hermite projection, as the two sweeps do),
//      and publishes that plane z+1 is read,
//   4. writes the links that leave its row (c_y != 0) and those into plane
//      z+1 of its own row (c_z = +1).
//
// Order between wavefronts.  The step is thread-safe in the paper's sense
// (Section 3): no update reads a value that another one writes in the same
// step.  Every population is written once, after the tile that owns its
// node has read it; the reads that a write must follow are the ones of the
// neighbouring rows y +- 1, which other wavefronts own.  Each tile
// publishes how many of its planes it has read (a progress word in device
// memory), and a wavefront writes into a neighbouring row's plane only
// after that row's tile has published it.  This is a write-after-read
// order: nothing the waiting wavefront reads depends on the other one, so
// the progress word needs no data to travel with it, only that the reads
// it announces have returned (s_waitcnt vmcnt(0) before the store of the
// word).  The links of a tile's first plane that go to plane z0 - 1 belong
// to the previous tile's last plane; they are held in registers and
// written when that tile has read its last plane.
//
// Progress.  Waits need every tile running at once: the host sizes the
// tiles so that all of them are resident and launches cooperatively (the
// launch fails instead of queueing tiles).  Every wait is bounded: past
// kFusedWaitLimit polls it raises the abort word and stops waiting (the
// step's result is then invalid and the host reports an error), so every
// wavefront ends.  The progress words count in epochs: a step reads the
// epoch at its start, counts from epoch x stride, and the last wavefront
// to finish advances the epoch, so every step is launched with the same
// arguments and the words are never cleared between steps.
#pragma once

#include "kernels.hpp"

namespace lbk {

struct FusedParams {
  int64_t tiles;       // ny * nzt
  int64_t nzt;         // tiles along z
  uint32_t* sync;      // progress[tiles], then done counter, epoch, abort
  int32_t stride;      // progress units per step (longest tile + 1)
  int32_t order_mul;   // tile order permutation (0 = natural), as StepParams::order_mul
  int32_t wait_limit;  // polls before a wait gives up (kFusedWaitLimit)
  int32_t pad_;
};

constexpr int32_t kFusedWaitLimit = 1 << 22;

__device__ __forceinline__ uint32_t sync_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void sync_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


template <class L, int ORDER, typename S, typename C, int E, int H, bool FD>
struct FusedSweep {
  using ML = MomentLayout<L>;
  using CL = CoefLayout<L, ORDER>;
  static constexpr int M = ML::M;
  static constexpr int K = CL::K;
  static constexpr int Q = L::Q;

  struct Tile {
    int64_t t, y, zt, z0, z1;
    uint32_t base;
    int lane;
  };

  __device__ __forceinline__ static int64_t z_start(const StepParams<C>& p, const FusedParams& fp, int64_t zt) {
    return zt * p.nz / fp.nzt;
  }
  __device__ __forceinline__ static int64_t tile_index(const StepParams<C>& p, const FusedParams& fp, int64_t y,
                                       int64_t zt) {
    y = (y % p.ny + p.ny) % p.ny;
    zt = (zt % fp.nzt + fp.nzt) % fp.nzt;
    return y + p.ny * zt;
  }

  // -- progress -------------------------------------------------------------
  // all vector memory operations of this wavefront (the plane loads) have
  // returned, then the word is stored
  __device__ __forceinline__ static void publish(const FusedParams& fp, const Tile& tl, uint32_t planes) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (tl.lane == 0) sync_store(fp.sync + tl.t, tl.base + planes);
    asm volatile("" ::: "memory");
  }
  // until tile u has read `planes` planes of this step, or the abort word is
  // up, or wait_limit polls have failed (then it raises the abort word)
  __device__ __forceinline__ static void wait_for(const FusedParams& fp, const Tile& tl, int64_t u,
                                  uint32_t planes) {
    const uint32_t need = tl.base + planes;
    uint32_t* abort_word = fp.sync + fp.tiles + 2;
    for (int32_t it = 0;; ++it) {
      if ((int32_t)(sync_load(fp.sync + u) - need) >= 0) break;
      if (sync_load(abort_word) != 0) break;
      if (it >= fp.wait_limit) {
        if (tl.lane == 0) sync_store(abort_word, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    asm volatile("" ::: "memory");
  }

  // -- one plane of the row --------------------------------------------------
  // Storage node of the row's first node.  A row never straddles a block of
  // the array layout (the row pitch, 64 E H = nx, divides the block size,
  // both powers of two; the host checks it), so element (a, row start + x)
  // is at slot(row start) + a B + x: a wave-uniform base plus the lane's
  // offset, with no per-lane 64-bit index arithmetic.
  __device__ __forceinline__ static int64_t row_of(const StepParams<C>& p, int64_t y, int64_t z) {
    return p.px * (y + p.ny * z);
  }

  __device__ __forceinline__ static void load_plane(const S* f, const StepParams<C>& p, int64_t rowbase, int lane,
                                    C (&raw)[Q][H][E]) {
#pragma unroll
    for (int a = 0; a < Q; ++a)
#pragma unroll
      for (int h = 0; h < H; ++h)
        load_pack<S, C, E>(f + slot<Q>(p, rowbase) + a * astride(p) + (h * 64 * E + lane * E),
                           raw[a][h]);
  }

  // Moments and post-collision coefficients of the lane's nodes, with the
  // two sweeps' arithmetic: node_moments and post_collision round every
  // operation as written (no FMA contraction), so computing the
  // coefficients straight from the moments in registers, with whatever
  // values the compiler shares between the two, gives the bits that the
  // two sweeps get through the moment arrays.
  __device__ __forceinline__ static void coef_of(const C (&raw)[Q][H][E], const StepParams<C>& p,
                                 C (&k)[H][E][K]) {
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        C s[Q], m[M];
#pragma unroll
        for (int a = 0; a < Q; ++a) s[a] = raw[a][h][e];
        node_moments<L, C>(s, p, m);
        post_collision<L, ORDER, C, FD>(m, p, k[h][e]);
      }
  }

  // Values of link A arriving at this lane's nodes from x - c_x (periodic
  // wrap; an x wall replaces the wrapped values, see store_arriving).
  template <int A>
  __device__ __forceinline__ static void arriving(const C (&k)[H][E][K], int lane, C (&val)[H][E]) {
    constexpr int cx = L::c[A][0];
    if constexpr (cx == 0) {
#pragma unroll
      for (int h = 0; h < H; ++h)
#pragma unroll
        for (int e = 0; e < E; ++e) val[h][e] = link_value<L, ORDER, A, C>(k[h][e]);
    } else if constexpr (cx > 0) {
      C last[H];
#pragma unroll
      for (int h = 0; h < H; ++h) last[h] = link_value<L, ORDER, A, C>(k[h][E - 1]);
#pragma unroll
      for (int h = 0; h < H; ++h) {
        // lane 0 of chunk h takes lane 63 of chunk h - 1 (chunk H-1 for h = 0)
        const C give = (lane == 63) ? last[(h + H - 1) % H] : last[h];
        val[h][0] = __shfl(give, (lane + 63) & 63, 64);
#pragma unroll
        for (int e = 1; e < E; ++e) val[h][e] = link_value<L, ORDER, A, C>(k[h][e - 1]);
      }
    } else {
      C first[H];
#pragma unroll
      for (int h = 0; h < H; ++h) first[h] = link_value<L, ORDER, A, C>(k[h][0]);
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const C give = (lane == 0) ? first[(h + 1) % H] : first[h];
        val[h][E - 1] = __shfl(give, (lane + 1) & 63, 64);
#pragma unroll
        for (int e = 0; e < E - 1; ++e) val[h][e] = link_value<L, ORDER, A, C>(k[h][e + 1]);
      }
    }
  }

  // Store link A's arriving values into row trow; where an x wall supplies
  // the value (x = 0 for c_x > 0, x = nx - 1 for c_x < 0) the element is
  // skipped: the wall's reflection writes it (own_row_walls).
  template <int A>
  __device__ __forceinline__ static void store_arriving(S* f, const StepParams<C>& p, int64_t trow, int lane,
                                        const C (&val)[H][E]) {
    constexpr int cx = L::c[A][0];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int64_t xs = (int64_t)h * 64 * E + lane * E;
      S* dst = f + slot<Q>(p, trow) + A * astride(p) + xs;
      const bool cut_lo = (cx > 0) && p.bbx && (xs == 0);
      const bool cut_hi = (cx < 0) && p.bbx && (xs + E == p.nx);
      if (!(cut_lo || cut_hi)) {
        store_pack<S, C, E>(dst, val[h]);
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if ((cut_lo && e == 0) || (cut_hi && e == E - 1)) continue;
          dst[e] = Codec<S, C>::store(val[h][e]);
        }
      }
    }
  }

  // Reflections at x walls of link A leaving this row's end nodes: into
  // the same node as the opposite link (halfway bounce-back, moving-wall
  // correction on the x faces).
  template <int A>
  __device__ __forceinline__ static void own_row_walls(S* f, const StepParams<C>& p, int64_t rowbase, int lane,
                                       const C (&k)[H][E][K]) {
    constexpr int cx = L::c[A][0];
    constexpr int AB = opposite<L>(A);
    if constexpr (cx > 0) {
      if (lane == 63) {
        const C v = p.moving ? link_value_plus<L, ORDER, A, C>(k[H - 1][E - 1], wall_dot<L, A, C>(p, 1))
                             : link_value<L, ORDER, A, C>(k[H - 1][E - 1]);
        f[slot<Q>(p, rowbase) + AB * astride(p) + (p.nx - 1)] = Codec<S, C>::store(v);
      }
    } else if constexpr (cx < 0) {
      if (lane == 0) {
        const C v = p.moving ? link_value_plus<L, ORDER, A, C>(k[0][0], wall_dot<L, A, C>(p, 0))
                             : link_value<L, ORDER, A, C>(k[0][0]);
        f[slot<Q>(p, rowbase) + AB * astride(p)] = Codec<S, C>::store(v);
      }
    }
  }

  // Link A leaving this row across a y or z wall: every node gets it back
  // as the opposite link (edges: the corrections of every wall crossed).
  template <int A>
  __device__ __forceinline__ static void bounce_row(S* f, const StepParams<C>& p, const Tile& tl, int64_t z,
                                    int64_t rowbase, const C (&k)[H][E][K]) {
    constexpr int cx = L::c[A][0], cy = L::c[A][1], cz = L::c[A][2];
    constexpr int AB = opposite<L>(A);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int64_t xs = (int64_t)h * 64 * E + tl.lane * E;
      C bv[E];
      if (!p.moving) {
#pragma unroll
        for (int e = 0; e < E; ++e) bv[e] = link_value<L, ORDER, A, C>(k[h][e]);
      } else {
        C cw = C(0);
        if (cy != 0 && (tl.y + cy < 0 || tl.y + cy >= p.ny))
          cw += wall_dot<L, A, C>(p, 2 + (tl.y + cy < 0 ? 0 : 1));
        if (cz != 0 && (z + cz < 0 || z + cz >= p.nz))
          cw += wall_dot<L, A, C>(p, 4 + (z + cz < 0 ? 0 : 1));
#pragma unroll
        for (int e = 0; e < E; ++e) {
          C extra = cw;
          if constexpr (cx != 0) {
            if (p.bbx && cx > 0 && xs + e == p.nx - 1) extra += wall_dot<L, A, C>(p, 1);
            if (p.bbx && cx < 0 && xs + e == 0) extra += wall_dot<L, A, C>(p, 0);
          }
          bv[e] = link_value_plus<L, ORDER, A, C>(k[h][e], extra);
        }
      }
      store_pack<S, C, E>(f + slot<Q>(p, rowbase) + AB * astride(p) + xs, bv);
    }
  }

  // does link A from row (y, z) leave through a y or z wall?
  template <int A>
  __device__ __forceinline__ static bool crosses_wall(const StepParams<C>& p, int64_t y, int64_t z) {
    constexpr int cy = L::c[A][1], cz = L::c[A][2];
    if (cy != 0 && p.bby && (y + cy < 0 || y + cy >= p.ny)) return true;
    if (cz != 0 && p.bbz && (z + cz < 0 || z + cz >= p.nz)) return true;
    return false;
  }

  __device__ __forceinline__ static int64_t wrap(int64_t v, int64_t n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

  // group 0: c_y = 0, c_z <= 0;  group 1: c_y != 0;  group 2: c_y = 0, c_z = +1
  template <int A>
  static constexpr int group() {
    return L::c[A][1] != 0 ? 1 : (L::c[A][2] > 0 ? 2 : 0);
  }
  // held back: links of the first plane into plane z0 - 1 (another tile's last plane)
  template <int A>
  __device__ __forceinline__ static bool deferred(const StepParams<C>& p, const Tile& tl, int64_t z) {
    return L::c[A][2] < 0 && z == tl.z0 && !crosses_wall<A>(p, tl.y, z);
  }

  template <int G, int I = 0>
  __device__ __forceinline__ static void emit(S* f, const StepParams<C>& p, const Tile& tl, int64_t z,
                              const C (&k)[H][E][K], C (&dv)[Q][H][E]) {
    if constexpr (I < Q) {
      constexpr int A = RowOrder<L>::a[I];
      if constexpr (group<A>() == G) {
        constexpr int cx = L::c[A][0], cy = L::c[A][1], cz = L::c[A][2];
        const int64_t rowbase = row_of(p, tl.y, z);
        if (crosses_wall<A>(p, tl.y, z)) {
          bounce_row<A>(f, p, tl, z, rowbase, k);
        } else {
          C val[H][E];
          arriving<A>(k, tl.lane, val);
          if (deferred<A>(p, tl, z)) {
#pragma unroll
            for (int h = 0; h < H; ++h)
#pragma unroll
              for (int e = 0; e < E; ++e) dv[A][h][e] = val[h][e];
          } else {
            const int64_t trow = row_of(p, wrap(tl.y + cy, p.ny), wrap(z + cz, p.nz));
            store_arriving<A>(f, p, trow, tl.lane, val);
          }
          if constexpr (cx != 0) {
            if (p.bbx) own_row_walls<A>(f, p, rowbase, tl.lane, k);
          }
        }
      }
      emit<G, I + 1>(f, p, tl, z, k, dv);
    }
  }

  template <int I = 0>
  __device__ __forceinline__ static void emit_deferred(S* f, const StepParams<C>& p, const Tile& tl,
                                       const C (&dv)[Q][H][E]) {
    if constexpr (I < Q) {
      constexpr int A = I;
      if constexpr (L::c[A][2] < 0) {
        if (deferred<A>(p, tl, tl.z0)) {
          const int64_t trow = row_of(p, wrap(tl.y + L::c[A][1], p.ny), wrap(tl.z0 - 1, p.nz));
          store_arriving<A>(f, p, trow, tl.lane, dv[A]);
        }
      }
      emit_deferred<I + 1>(f, p, tl, dv);
    }
  }

  __device__ __forceinline__ static void run(S* f, const StepParams<C>& p, const FusedParams& fp, int64_t t) {
    Tile tl;
    tl.lane = threadIdx.x & 63;
    tl.t = t;
    tl.y = t % p.ny;
    tl.zt = t / p.ny;
    tl.z0 = z_start(p, fp, tl.zt);
    tl.z1 = z_start(p, fp, tl.zt + 1);
    const uint32_t epoch = __builtin_amdgcn_readfirstlane(sync_load(fp.sync + fp.tiles + 1));
    tl.base = epoch * (uint32_t)fp.stride;
    const bool ylo = !(p.bby && tl.y == 0), yhi = !(p.bby && tl.y == p.ny - 1);
    const int64_t tdn = tile_index(p, fp, tl.y - 1, tl.zt), tup = tile_index(p, fp, tl.y + 1, tl.zt);

    C raw[Q][H][E];
    C k[H][E][K];
    C dv[Q][H][E];
    load_plane(f, p, row_of(p, tl.y, tl.z0), tl.lane, raw);
    coef_of(raw, p, k);
    publish(fp, tl, 1);
    for (int64_t z = tl.z0; z < tl.z1; ++z) {
      const bool has_next = z + 1 < tl.z1;
      if (has_next) load_plane(f, p, row_of(p, tl.y, z + 1), tl.lane, raw);
      emit<0>(f, p, tl, z, k, dv);
      C kn[H][E][K];
      if (has_next) {
        coef_of(raw, p, kn);
        publish(fp, tl, (uint32_t)(z + 2 - tl.z0));
      }
      // rows y +- 1 have read this tile's planes through z + 1 (through z
      // at the last plane, whose c_z = +1 links go to the next tile's first
      // plane)
      const uint32_t through = (uint32_t)((has_next ? z + 2 : z + 1) - tl.z0);
      if (ylo) wait_for(fp, tl, tdn, through);
      if (yhi) wait_for(fp, tl, tup, through);
      if (!has_next && !(p.bbz && tl.z1 == p.nz)) {
        if (ylo) wait_for(fp, tl, tile_index(p, fp, tl.y - 1, tl.zt + 1), 1);
        if (yhi) wait_for(fp, tl, tile_index(p, fp, tl.y + 1, tl.zt + 1), 1);
        wait_for(fp, tl, tile_index(p, fp, tl.y, tl.zt + 1), 1);
      }
      emit<1>(f, p, tl, z, k, dv);
      emit<2>(f, p, tl, z, k, dv);
      if (has_next) {
#pragma unroll
        for (int h = 0; h < H; ++h)
#pragma unroll
          for (int e = 0; e < E; ++e)
#pragma unroll
            for (int q = 0; q < K; ++q) k[h][e][q] = kn[h][e][q];
      }
    }
    // the first plane's c_z = -1 links: the previous tile's last plane
    if (!(p.bbz && tl.z0 == 0)) {
      const int64_t zp = tl.zt - 1;
      const uint32_t len = (uint32_t)(z_start(p, fp, (zp + fp.nzt) % fp.nzt + 1) -
                                      z_start(p, fp, (zp + fp.nzt) % fp.nzt));
      if (ylo) wait_for(fp, tl, tile_index(p, fp, tl.y - 1, zp), len);
      if (yhi) wait_for(fp, tl, tile_index(p, fp, tl.y + 1, zp), len);
      wait_for(fp, tl, tile_index(p, fp, tl.y, zp), len);
      emit_deferred(f, p, tl, dv);
    }
    // the last wavefront to finish starts the next epoch
    if (tl.lane == 0) {
      const uint32_t done = __hip_atomic_fetch_add(fp.sync + fp.tiles, 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
      if (done == (uint32_t)fp.tiles - 1) {
        sync_store(fp.sync + fp.tiles, 0u);
        sync_store(fp.sync + fp.tiles + 1, epoch + 1);
      }
    }
  }
};

template <class L, int ORDER, typename S, typename C, int E, int H, bool FD>
__global__ __launch_bounds__(256) void k_fused_step(S* f, StepParams<C> p, FusedParams fp) {
  const int64_t w = uniform64((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  if (w >= fp.tiles) return;
  int64_t t = w;
  if (fp.order_mul != 0)
    t = (int64_t)(((uint64_t)w * (uint64_t)(uint32_t)fp.order_mul) % (uint64_t)fp.tiles);
  FusedSweep<L, ORDER, S, C, E, H, FD>::run(f, p, fp, uniform64(t));
}

}  // namespace lbk
