// Host side of liblb.so: the C ABI declared in include/lb.h.
//
// Device memory of one simulation (lb_required_bytes):
//   f  species*Q population arrays, storage type: f_a - t_a rho0 (one
//      species), or the mixture g_a - t_a rho0 and the red set stored
//      relative to each node's reference colour (two; see kernels2.hpp)
//   m  M moment arrays (drho, j, Pi^neq, and phi for two species), compute type
//   n  near-contact flags, one byte per storage node (two species, NCI on)
//   c  reference colours, one byte per storage node (two species)
//   r  FP64 partial sums of the conservation reduction
// f and m are blocked structures of arrays: the node range, padded to
// npad (a multiple of the block size B, a power of two >= 1024), is cut into
// blocks of B nodes, and block k of a region of NA arrays holds B elements of
// each array in turn: element (a, n) at (n / B) NA B + a B + n % B.  B is 32
// KiB of population storage (8192 nodes in FP32, 16384 in 16-bit, 4096 in
// FP64), or the next power of two >= N for a smaller domain.  Every block
// starts 256-byte aligned and the moments sweep needs no tail.
// lb_init and lb_moments stage their host transfers through m, which the
// next step's moments sweep rewrites anyway; the library allocates nothing
// beyond lb_required_bytes on the device.  A handle without moment arrays
// (keep_moments 0, fused step only) keeps a bounded m for that staging alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "handle.hpp"
#include "lb.h"

namespace {

using namespace lbk;

// -------------------------------------------------------------------------
// Plain copy (bandwidth ceiling and byte-counter scale): one 16-byte
// non-temporal load and store per lane, one pass over the grid (the fastest
// plain copy measured on MI355X, ~6.5 TB/s for 4 GiB; a grid-stride loop
// over 65536 blocks reaches ~5.1 TB/s).
// -------------------------------------------------------------------------
typedef unsigned int lb_u4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy(const lb_u4* __restrict__ src,
                                              lb_u4* __restrict__ dst, int64_t n16) {
  const int64_t i = flat_block() * blockDim.x + threadIdx.x;
  if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}


constexpr size_t kAlign = 256;
// Host transfers of lb_init / lb_moments move at most this many nodes per
// chunk, so their host staging buffer stays bounded (<= 1.2 GB).
constexpr int64_t kMaxStageNodes = int64_t(1) << 24;
// A handle without moment arrays keeps at most this much staging memory.
constexpr size_t kStageBytes = size_t(256) << 20;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int status_of(hipError_t e) {
  if (e == hipSuccess) return LB_OK;
  if (e == hipErrorOutOfMemory) return LB_ENOMEM;
  return LB_EDEVICE;
}

#define LB_TRY_HIP(expr)                  \
  do {                                    \
    hipError_t e_ = (expr);               \
    if (e_ != hipSuccess) return status_of(e_); \
  } while (0)

int lattice_q(int lattice) {
  return lattice == LB_D2Q9 ? 9 : lattice == LB_D3Q19 ? 19 : lattice == LB_D3Q27 ? 27 : 0;
}

// The caller's parameters as a full current-version struct: the first
// struct_size bytes (one of the known version sizes) copied over the
// defaults of the later fields.  False for an unknown size.
bool normalize(const lb_params* in, lb_params* out) {
  if (!in) return false;
  const size_t sz = in->struct_size;
  if (sz != sizeof(lb_params) && sz != LB_PARAMS_SIZE_V3 && sz != LB_PARAMS_SIZE_V2 &&
      sz != LB_PARAMS_SIZE_V1)
    return false;
  lb_params_default(out);
  std::memcpy(out, in, sz);
  if (sz < sizeof(lb_params)) {
    lb_params d;
    lb_params_default(&d);
    std::memcpy((char*)out + sz, (const char*)&d + sz, sizeof(lb_params) - sz);
  }
  out->struct_size = sizeof(lb_params);
  return true;
}

int validate_full(const lb_params* p);
int fused_rows(const lb_params* p);

int validate(const lb_params* in) {
  lb_params p;
  if (!normalize(in, &p)) return LB_EINVAL;
  return validate_full(&p);
}

int validate_full(const lb_params* p) {
  const int Q = lattice_q(p->lattice);
  if (!Q) return LB_EINVAL;
  if (p->hermite_order != 2 && p->hermite_order != 3) return LB_EINVAL;
  if (p->hermite_order == 3 && p->lattice != LB_D3Q27) return LB_EINVAL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return LB_EINVAL;
  if (p->lattice == LB_D2Q9 && p->nz != 1) return LB_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (p->bc[a] != LB_PERIODIC && p->bc[a] != LB_BOUNCEBACK) return LB_EINVAL;
  if (p->lattice == LB_D2Q9 && p->bc[2] != LB_PERIODIC) return LB_EINVAL;
  if (!(std::isfinite(p->tau) && p->tau > 0.5)) return LB_EINVAL;
  if (!(std::isfinite(p->rho0) && p->rho0 > 0.0)) return LB_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->force[a])) return LB_EINVAL;
  if (p->lattice == LB_D2Q9 && p->force[2] != 0.0) return LB_EINVAL;
  if (p->species != 1 && p->species != 2) return LB_EINVAL;
  if (p->species == 2) {
    if (!(std::isfinite(p->sigma) && p->sigma >= 0.0)) return LB_EINVAL;
    if (!(std::isfinite(p->beta) && p->beta >= 0.0 && p->beta <= 1.0)) return LB_EINVAL;
    if (p->lattice == LB_D3Q27) return LB_EINVAL;  // no colour weights B_a for D3Q27 here
    if (p->hermite_order != 2) return LB_EINVAL;
    if (p->storage != LB_STORE_F32 && p->storage != LB_STORE_F64) return LB_EUNSUPPORTED;
  }
  const bool f64 = p->compute == LB_COMPUTE_F64;
  const bool f32 = p->compute == LB_COMPUTE_F32;
  if (!f64 && !f32) return LB_EINVAL;
  switch (p->storage) {
    case LB_STORE_F64:
      if (!f64) return LB_EINVAL;
      break;
    case LB_STORE_F32:
    case LB_STORE_F16S:
    case LB_STORE_BF16S:
      if (!f32) return LB_EINVAL;
      break;
    default:
      return LB_EINVAL;
  }
  // moving walls: tangential velocities on bounce-back faces, one species
  const int D = p->lattice == LB_D2Q9 ? 2 : 3;
  bool moving = false;
  for (int a = 0; a < 3; ++a)
    for (int side = 0; side < 2; ++side)
      for (int b = 0; b < 3; ++b) {
        const double v = p->wall_velocity[a][side][b];
        if (!std::isfinite(v)) return LB_EINVAL;
        if (v == 0.0) continue;
        if (p->bc[a] != LB_BOUNCEBACK || b == a || b >= D) return LB_EINVAL;
        moving = true;
      }
  if (moving && p->species == 2) return LB_EUNSUPPORTED;
  // near-contact interactions: two species, finite constants in range
  if (!(std::isfinite(p->nci_strength) && p->nci_strength >= 0.0)) return LB_EINVAL;
  if (p->nci_strength > 0.0) {
    if (p->species != 2) return LB_EINVAL;
    if (!(std::isfinite(p->nci_eps) && p->nci_eps > 0.0 && p->nci_eps < 2.0)) return LB_EINVAL;
    if (p->nci_reach < 1 || p->nci_reach > 8) return LB_EINVAL;
  }
  // keep every index comfortably inside int64
  const double N = (double)p->nx * (double)p->ny * (double)p->nz;
  if (N > 4.0e12) return LB_EINVAL;
  // population set only: every step is the fused step
  if (p->keep_moments != 0 && p->keep_moments != 1) return LB_EINVAL;
  if (p->keep_moments == 0 && fused_rows(p) == 0) return LB_EUNSUPPORTED;
  return LB_OK;
}

const Impl* select_impl(const lb_params* p) {
  switch (p->lattice) {
    case LB_D2Q9: return impl_d2q9(p->storage, p->species);
    case LB_D3Q19: return impl_d3q19(p->storage, p->species);
    case LB_D3Q27: return impl_d3q27(p->hermite_order, p->storage);
  }
  return nullptr;
}

// Nodes per lane of the stream-collide sweep: the narrowest V <= vmax that
// needs no more wavefronts per x-row (64 V nodes each) than vmax does.  A
// wider vector moves more bytes per instruction, but a row split over fewer
// wavefronts with most lanes busy beats one wide vector on a few lanes.
int choose_v2(int64_t nx, int vmax) {
  const int64_t fewest = (nx + 64 * vmax - 1) / (64 * vmax);
  for (int v = 1; v < vmax; v <<= 1)
    if ((nx + 64 * v - 1) / (64 * v) == fewest) return v;
  return vmax;
}

// Nodes per lane of the fused step for this shape, 0 where it has none:
// one species, 3D, FP32 or 16-bit storage, and rows of exactly 64 v nodes
// (v = 2, 4, 8 for D3Q19; 2, 4 for D3Q27, whose 512-node rows would not fit
// one wavefront's registers).
int fused_rows(const lb_params* p) {
  if (p->species != 1 || p->lattice == LB_D2Q9) return 0;
  if (p->storage == LB_STORE_F64 || p->compute != LB_COMPUTE_F32) return 0;
  const int vmax = p->lattice == LB_D3Q27 ? 4 : 8;
  for (int v = 2; v <= vmax; v <<= 1)
    if (p->nx == 64 * (int64_t)v) return v;
  return 0;
}

Layout layout_of(const lb_params* p) {
  Layout L;
  L.Q = lattice_q(p->lattice);
  L.D = p->lattice == LB_D2Q9 ? 2 : 3;
  L.M = 1 + L.D + L.D * (L.D + 1) / 2 + (p->species == 2 ? 1 : 0);  // + phi
  L.species = p->species;
  L.ssize = p->storage == LB_STORE_F64 ? 8 : p->storage == LB_STORE_F32 ? 4 : 2;
  L.csize = p->compute == LB_COMPUTE_F64 ? 8 : 4;
  L.N = p->nx * p->ny * p->nz;
  // rows padded to a whole number of the sweep's contiguous lane chunks, so
  // that every vector access is aligned
  const Impl* impl = select_impl(p);
  L.v2 = impl ? choose_v2(p->nx, impl->v2max) : 1;
  const int64_t e = impl ? std::min(L.v2, impl->emax) : 1;
  L.px = (p->nx + e - 1) / e * e;
  const int64_t ns = L.px * p->ny * p->nz;  // storage nodes
  int lb = 10;  // block of B = 2^lb nodes: 32 KiB of populations, >= 1024 nodes
  while ((int64_t(1) << lb) < ns && (int64_t(1) << lb) * (int64_t)L.ssize < 32768) ++lb;
  L.lb = lb;
  const int64_t B = int64_t(1) << lb;
  L.npad = (ns + B - 1) / B * B;
  L.f_off = 0;
  L.m_off = align_up((size_t)L.species * L.Q * L.npad * L.ssize, kAlign);
  // the moment arrays, or (population set only) just the staging buffer of
  // lb_init / lb_moments
  const size_t mbytes = (size_t)L.M * L.npad * L.csize;
  L.n_off = L.m_off + align_up(p->keep_moments ? mbytes : std::min(mbytes, kStageBytes), kAlign);
  const bool nci = p->species == 2 && p->nci_strength > 0.0;
  L.c_off = L.n_off + (nci ? align_up((size_t)L.npad, kAlign) : 0);
  L.r_off = L.c_off + (p->species == 2 ? align_up((size_t)L.npad, kAlign) : 0);
  L.s_off = L.r_off + align_up((size_t)kRedBlocks * 8 * sizeof(double), kAlign);
  // progress words of the fused step: one per tile (at most one per row and
  // plane) and three more
  const size_t sync_words = fused_rows(p) ? (size_t)(p->ny * p->nz + 3) : 0;
  L.total = L.s_off + align_up(sync_words * sizeof(uint32_t), kAlign);
  return L;
}

template <typename C>
void fill_params(StepParams<C>& q, const lb_params* p, const Layout& L, int v2) {
  q.nx = p->nx;
  q.ny = p->ny;
  q.nz = p->nz;
  q.px = L.px;
  q.npad = L.npad;
  q.nseg = (p->nx + 64 * v2 - 1) / (64 * v2);
  q.bbx = p->bc[0] == LB_BOUNCEBACK;
  q.bby = p->bc[1] == LB_BOUNCEBACK;
  q.bbz = p->bc[2] == LB_BOUNCEBACK;
  q.lb = L.lb;
  q.rho0 = (C)p->rho0;
  q.inv_rho0 = (C)(1.0 / p->rho0);
  for (int a = 0; a < 3; ++a) {
    q.F[a] = (C)p->force[a];
    q.halfF[a] = (C)(0.5 * p->force[a]);
  }
  const double omega = 1.0 / p->tau;
  q.omw = (C)(1.0 - omega);
  q.omhw = (C)(1.0 - 0.5 * omega);
  // moving walls, prescaled like the momentum coefficient: -6 rho0 u_w / wden
  const double wden = p->lattice == LB_D3Q27 ? 216.0 : 36.0;
  q.moving = 0;
  q.order_mul = 0;
  for (int a = 0; a < 3; ++a)
    for (int side = 0; side < 2; ++side)
      for (int b = 0; b < 3; ++b) {
        const double v = p->wall_velocity[a][side][b];
        q.wall[2 * a + side][b] = (C)(-6.0 * p->rho0 * v / wden);
        if (v != 0.0) q.moving = 1;
      }
}

int launch_status(hipError_t e) { return status_of(e); }

// Host side of the FP64 conservation reduction: sum the per-block partial
// sums into [mass, j (3), red mass, blue mass]; LB_ENONFINITE if the mass or
// momentum is not finite (the outputs are filled either way).
int finish_conserved(const lb_handle* h, const double* part, double* out) {
  const bool two = h->p.species == 2;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int b = 0; b < kRedBlocks; ++b)
    for (int q = 0; q < 5; ++q) acc[q] += part[(size_t)b * 8 + q];
  out[0] = (double)h->L.N * h->p.rho0 + acc[0];
  out[1] = acc[1];
  out[2] = acc[2];
  out[3] = acc[3];
  out[4] = two ? acc[4] : out[0];
  out[5] = two ? out[0] - acc[4] : 0.0;
  for (int q = 0; q < 4; ++q)
    if (!std::isfinite(out[q])) return LB_ENONFINITE;
  return LB_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
// Multiplier of the order permutation u -> (u * mul) mod U of U work units
// (lb_set_sweep_order): 0 natural, U - 1 reversed, or a multiplier near
// U/phi that shares no factor with U (mixes distant rows into
// neighbouring units).
int64_t order_multiplier(int order, int64_t U) {
  if (order == 0 || U <= 1) return 0;
  if (order == 1) return U - 1;
  int64_t mul = (int64_t)(0.6180339887 * (double)U) | 1;
  auto gcd = [](int64_t a, int64_t b) { while (b) { const int64_t t = a % b; a = b; b = t; } return a; };
  while (mul > 1 && gcd(mul, U) != 1) mul += 2;
  if (mul >= U) mul = U - 1;
  return mul;
}

// Choose the path lb_step takes.  The fused step needs its shape
// (fused_rows), cooperative launch, and all its tiles resident at once:
// ny * nzt wavefronts within what the device holds of its kernel.
// Automatic: D3Q19 only (the D3Q27 fused kernels, one wavefront per SIMD
// with their larger arithmetic, measure slower than the two sweeps), at
// least 8 planes per tile, and the fused step only when its tiles fill at
// least half of the resident wavefronts.  The progress words are cleared
// whenever the tiling is set.
int configure_fused(lb_handle* h, int path, int64_t z_tiles) {
  if (path == 1) {
    h->use_fused = false;
    h->path = 1;
    return LB_OK;
  }
  const void* fn = (h->fv && h->impl->fused_kernel) ? h->impl->fused_kernel(h->fv) : nullptr;
  if (path == 0 && h->p.lattice != LB_D3Q19) fn = nullptr;
  // the kernel addresses a row from its first node: rows must not straddle
  // a block of the array layout
  if (((int64_t(1) << h->L.lb) % h->L.px) != 0) fn = nullptr;
  const int64_t ny = h->p.ny, nz = h->p.nz;
  int64_t nzt = 0;
  bool ok = fn != nullptr;
  if (ok) {
    int coop = 0, cus = 0, nb = 0;
    LB_TRY_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, h->device));
    LB_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    LB_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, 0));
    const int64_t resident = (int64_t)nb * cus * 4;  // wavefronts
    if (!coop || resident < 1) {
      ok = false;
    } else if (z_tiles > 0) {
      if (z_tiles > nz) return LB_EINVAL;
      nzt = z_tiles;
      ok = ny * nzt <= resident;
    } else {
      nzt = std::min(std::max<int64_t>(nz / 8, 1), resident / ny);
      ok = nzt >= 1 && (path == 2 || 2 * ny * nzt >= resident);
    }
  }
  if (!ok) {
    if (path == 2) return LB_EUNSUPPORTED;
    h->use_fused = false;
    h->path = 0;
    return LB_OK;
  }
  h->fp.tiles = ny * nzt;
  h->fp.nzt = nzt;
  h->fp.sync = (uint32_t*)((char*)h->base + h->L.s_off);
  h->fp.stride = (int32_t)((nz + nzt - 1) / nzt + 1);
  h->fp.order_mul = (int32_t)order_multiplier(h->order, h->fp.tiles);
  h->fp.wait_limit = h->wait_limit;
  LB_TRY_HIP(hipMemsetAsync(h->fp.sync, 0, (size_t)(h->fp.tiles + 3) * sizeof(uint32_t), h->stream));
  h->use_fused = true;
  h->path = path;
  return LB_OK;
}

// LB_EDEVICE (once) if a fused step gave up waiting since the last check:
// its result is invalid.  Called after the stream has drained.
int fused_status(lb_handle* h) {
  if (!h->use_fused) return LB_OK;
  uint32_t* word = h->fp.sync + h->fp.tiles + 2;
  uint32_t v = 0;
  LB_TRY_HIP(hipMemcpyAsync(&v, word, sizeof(v), hipMemcpyDeviceToHost, h->stream));
  LB_TRY_HIP(hipStreamSynchronize(h->stream));
  if (v == 0) return LB_OK;
  LB_TRY_HIP(hipMemsetAsync(word, 0, sizeof(v), h->stream));
  LB_TRY_HIP(hipStreamSynchronize(h->stream));
  return LB_EDEVICE;
}

extern "C" {

void lb_params_default(lb_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(lb_params);
  p->lattice = LB_D3Q19;
  p->hermite_order = 2;
  p->nx = p->ny = p->nz = 32;
  p->bc[0] = p->bc[1] = p->bc[2] = LB_PERIODIC;
  p->species = 1;
  p->tau = 0.6;
  p->rho0 = 1.0;
  p->sigma = 0.0;
  p->beta = 0.0;
  p->storage = LB_STORE_F32;
  p->compute = LB_COMPUTE_F32;
  p->nci_strength = 0.0;
  p->nci_eps = 0.1;
  p->nci_reach = 1;
  p->keep_moments = 1;
}

int lb_validate(const lb_params* p) { return validate(p); }

size_t lb_required_bytes(const lb_params* in) {
  lb_params p;
  if (!normalize(in, &p) || validate_full(&p) != LB_OK) return 0;
  return layout_of(&p).total;
}

int lb_create(const lb_params* in, void* dev_mem, size_t dev_bytes, void* hip_stream,
              lb_handle** out) {
  if (!out) return LB_EINVAL;
  *out = nullptr;
  lb_params pn;
  if (!normalize(in, &pn)) return LB_EINVAL;
  const lb_params* p = &pn;
  const int st = validate_full(p);
  if (st != LB_OK) return st;
  try {
    lb_handle* h = new lb_handle();
    h->p = *p;
    h->L = layout_of(p);
    h->impl = select_impl(p);
    if (!h->impl) {
      delete h;
      return LB_EUNSUPPORTED;
    }
    h->stream = (hipStream_t)hip_stream;
    h->v2 = h->L.v2;
    {
      const hipError_t de = hipGetDevice(&h->device);
      if (de != hipSuccess) {
        delete h;
        return status_of(de);
      }
    }
    if (dev_mem) {
      if (((uintptr_t)dev_mem % kAlign) != 0) {
        delete h;
        return LB_EINVAL;
      }
      if (dev_bytes < h->L.total) {
        delete h;
        return LB_ENOMEM;
      }
      h->base = dev_mem;
      h->owned = false;
    } else {
      hipError_t e = hipMalloc(&h->base, h->L.total);
      if (e != hipSuccess) {
        delete h;
        return status_of(e);
      }
      h->owned = true;
    }
    h->f = (char*)h->base + h->L.f_off;
    h->m = (char*)h->base + h->L.m_off;
    h->partial = (double*)((char*)h->base + h->L.r_off);
    fill_params(h->p32, p, h->L, h->v2);
    fill_params(h->p64, p, h->L, h->v2);
    // (9/4) sigma omega and beta over the colour-weight denominator
    const double cden = p->lattice == LB_D2Q9 ? 108.0 : 36.0;
    const double pert = 2.25 * p->sigma / p->tau / cden;
    const double beta = p->beta / cden;
    unsigned char* ref = p->species == 2 ? (unsigned char*)((char*)h->base + h->L.c_off) : nullptr;
    h->cp32 = {(float)pert, (float)beta, ref};
    h->cp64 = {pert, beta, ref};
    h->nci = p->species == 2 && p->nci_strength > 0.0;
    h->flag = h->nci ? (unsigned char*)((char*)h->base + h->L.n_off) : nullptr;
    h->nq32 = {(float)p->nci_strength, (float)(-1.0 + p->nci_eps), p->nci_reach, 0};
    h->nq64 = {p->nci_strength, -1.0 + p->nci_eps, p->nci_reach, 0};
    hipError_t e = hipMemsetAsync(h->base, 0, h->L.total, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
      if (h->owned) (void)hipFree(h->base);
      delete h;
      return status_of(e);
    }
    h->fv = fused_rows(p);
    const int fs = configure_fused(h, p->keep_moments ? 0 : 2, 0);
    if (fs != LB_OK) {
      if (h->owned) (void)hipFree(h->base);
      delete h;
      return fs;
    }
    *out = h;
    return LB_OK;
  } catch (const std::bad_alloc&) {
    return LB_ENOMEM;
  } catch (...) {
    return LB_EDEVICE;
  }
}

int lb_init(lb_handle* h, const double* rho, const double* u, const double* phi) {
  if (!h || !rho || !u) return LB_EINVAL;
  if (h->p.species == 2 && !phi) return LB_EINVAL;
  const Layout& L = h->L;
  const int64_t N = L.N;
  for (int64_t n = 0; n < N; ++n)
    if (!std::isfinite(rho[n])) return LB_ENONFINITE;
  for (int64_t n = 0; n < (int64_t)L.D * N; ++n)
    if (!std::isfinite(u[n])) return LB_ENONFINITE;
  const bool two = h->p.species == 2;
  if (two) {
    for (int64_t n = 0; n < N; ++n) {
      if (!std::isfinite(phi[n])) return LB_ENONFINITE;
      if (phi[n] < -1.0 || phi[n] > 1.0) return LB_EINVAL;
    }
  }
  try {
    const int per = 1 + L.D + (two ? 1 : 0);  // doubles staged per node
    const int64_t cap = (int64_t)((L.n_off - L.m_off) / (per * sizeof(double)));
    const int64_t chunk = std::min(std::min(cap, kMaxStageNodes), N);
    // uninitialised: every element staged is written before it is copied
    std::unique_ptr<double[]> hb(new double[(size_t)per * chunk]);
    double* stage = (double*)h->m;
    for (int64_t n0 = 0; n0 < N; n0 += chunk) {
      const int64_t cnt = (N - n0 < chunk) ? N - n0 : chunk;
      for (int64_t i = 0; i < cnt; ++i) hb[i] = rho[n0 + i] - h->p.rho0;
      for (int al = 0; al < L.D; ++al)
        std::memcpy(&hb[(size_t)(1 + al) * cnt], u + (size_t)al * N + n0, cnt * sizeof(double));
      if (two) std::memcpy(&hb[(size_t)(1 + L.D) * cnt], phi + n0, cnt * sizeof(double));
      LB_TRY_HIP(hipMemcpyAsync(stage, hb.get(), (size_t)per * cnt * sizeof(double),
                                hipMemcpyHostToDevice, h->stream));
      LB_TRY_HIP(h->impl->init(h, stage, n0, cnt));
      LB_TRY_HIP(hipStreamSynchronize(h->stream));
    }
  } catch (const std::bad_alloc&) {
    return LB_ENOMEM;
  }
  h->steps = 0;
  return LB_OK;
}

int lb_step(lb_handle* h, int64_t nsteps) {
  if (!h || nsteps < 0) return LB_EINVAL;
  for (int64_t s = 0; s < nsteps; ++s) {
    const bool timed = h->tcount < h->tcap;
    hipEvent_t* ev = timed ? &h->ev[(size_t)4 * h->tcount] : nullptr;
    if (timed) LB_TRY_HIP(hipEventRecord(ev[0], h->stream));
    if (!h->use_fused) LB_TRY_HIP(h->impl->moments(h));
    if (timed) LB_TRY_HIP(hipEventRecord(ev[1], h->stream));
    if (timed) LB_TRY_HIP(hipEventRecord(ev[2], h->stream));
    if (h->use_fused) LB_TRY_HIP(h->impl->fused(h));
    else LB_TRY_HIP(h->impl->stream_collide(h));
    if (timed) {
      LB_TRY_HIP(hipEventRecord(ev[3], h->stream));
      ++h->tcount;
    }
    ++h->steps;
  }
  return LB_OK;
}

int lb_sweep(lb_handle* h, int which) {
  if (!h || (which != 0 && which != 1)) return LB_EINVAL;
  if (!h->p.keep_moments) return LB_EUNSUPPORTED;
  if (which == 0) LB_TRY_HIP(h->impl->moments(h));
  else {
    LB_TRY_HIP(h->impl->stream_collide(h));
    ++h->steps;
  }
  return LB_OK;
}

int lb_set_sweep_order(lb_handle* h, int order) {
  if (!h || order < 0 || order > 2) return LB_EINVAL;
  const int64_t U = h->p32.nseg * h->p32.ny * h->p32.nz;  // stream-collide wavefronts
  if (order != 0 && U >= (int64_t(1) << 31)) return LB_EUNSUPPORTED;
  const int64_t mul = order_multiplier(order, U);
  h->p32.order_mul = (int32_t)mul;
  h->p64.order_mul = (int32_t)mul;
  h->order = order;
  if (h->use_fused) h->fp.order_mul = (int32_t)order_multiplier(order, h->fp.tiles);
  return LB_OK;
}

int lb_set_step_path(lb_handle* h, int path, int64_t z_tiles) {
  if (!h || path < 0 || path > 2 || z_tiles < 0) return LB_EINVAL;
  if (!h->p.keep_moments) {
    if (path == 1) return LB_EUNSUPPORTED;
    path = 2;  // the only path of a handle without moment arrays
  }
  // drain: the progress words are reset below
  LB_TRY_HIP(hipStreamSynchronize(h->stream));
  const int st = fused_status(h);
  const int prev_path = h->path;
  const bool prev_use = h->use_fused;
  const lbk::FusedParams prev = h->fp;
  const int cs = configure_fused(h, path, path == 1 ? 0 : z_tiles);
  if (cs != LB_OK) {
    h->path = prev_path;
    h->use_fused = prev_use;
    h->fp = prev;
    return cs;
  }
  LB_TRY_HIP(hipStreamSynchronize(h->stream));
  return st;
}

int lb_set_fused_wait_limit(lb_handle* h, int64_t polls) {
  if (!h || polls < 0 || polls > INT32_MAX) return LB_EINVAL;
  h->wait_limit = (int32_t)polls;
  h->fp.wait_limit = h->wait_limit;
  return LB_OK;
}

int lb_get_step_path(const lb_handle* h, int* path, int64_t* z_tiles) {
  if (!h || !path || !z_tiles) return LB_EINVAL;
  *path = h->use_fused ? 2 : 1;
  *z_tiles = h->use_fused ? h->fp.nzt : 0;
  return LB_OK;
}

int lb_layout(const lb_handle* h, size_t* pop_offset, size_t* moment_offset,
              int64_t* block_nodes, int64_t* padded_nodes, int64_t* row_pitch) {
  if (!h || !pop_offset || !moment_offset || !block_nodes || !padded_nodes || !row_pitch)
    return LB_EINVAL;
  *pop_offset = h->L.f_off;
  *moment_offset = h->L.m_off;
  *block_nodes = int64_t(1) << h->L.lb;
  *padded_nodes = h->L.npad;
  *row_pitch = h->L.px;
  return LB_OK;
}

int lb_synchronize(lb_handle* h) {
  if (!h) return LB_EINVAL;
  LB_TRY_HIP(hipStreamSynchronize(h->stream));
  return fused_status(h);
}

int lb_set_stream(lb_handle* h, void* hip_stream) {
  if (!h) return LB_EINVAL;
  h->stream = (hipStream_t)hip_stream;
  return LB_OK;
}

int64_t lb_step_count(const lb_handle* h) { return h ? h->steps : -1; }

int lb_moments(lb_handle* h, double* rho, double* u, double* pineq, double* phi,
               double* conserved) {
  if (!h) return LB_EINVAL;
  LB_TRY_HIP(hipStreamSynchronize(h->stream));
  {
    const int fst = fused_status(h);
    if (fst != LB_OK) return fst;
  }
  const Layout& L = h->L;
  const int64_t N = L.N;
  const bool two = h->p.species == 2;
  const int K = L.D * (L.D + 1) / 2;
  const int per = 1 + L.D + K + (two ? 1 : 0);
  if (!two) phi = nullptr;
  try {
    if (rho || u || pineq || phi) {
      const int64_t cap = (int64_t)((L.n_off - L.m_off) / (per * sizeof(double)));
      const int64_t chunk = std::min(std::min(cap, kMaxStageNodes), N);
      double* stage = (double*)h->m;
      // staged rows: rho, u (D), Pi^neq (K), phi; only the requested ones
      // cross PCIe, straight into the caller's arrays
      auto fetch = [&](double* dst, int row, int64_t cnt) -> hipError_t {
        return hipMemcpyAsync(dst, stage + (size_t)row * cnt, cnt * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream);
      };
      for (int64_t n0 = 0; n0 < N; n0 += chunk) {
        const int64_t cnt = (N - n0 < chunk) ? N - n0 : chunk;
        // keep the first error, but always drain the stream before returning:
        // no copy into the caller's arrays may still be in flight afterwards
        hipError_t err = h->impl->readout(h, stage, n0, cnt);
        auto keep = [&](hipError_t e) { if (err == hipSuccess) err = e; };
        if (err == hipSuccess) {
          if (rho) keep(fetch(rho + n0, 0, cnt));
          if (u)
            for (int al = 0; al < L.D; ++al) keep(fetch(u + (size_t)al * N + n0, 1 + al, cnt));
          if (pineq)
            for (int q = 0; q < K; ++q) keep(fetch(pineq + (size_t)q * N + n0, 1 + L.D + q, cnt));
          if (phi) keep(fetch(phi + n0, 1 + L.D + K, cnt));
        }
        keep(hipStreamSynchronize(h->stream));
        if (err != hipSuccess) return status_of(err);
      }
    }
    int st = LB_OK;
    if (conserved) {
      std::vector<double> part((size_t)kRedBlocks * 8);
      LB_TRY_HIP(h->impl->conserved(h));
      LB_TRY_HIP(hipMemcpyAsync(part.data(), h->partial, part.size() * sizeof(double),
                                hipMemcpyDeviceToHost, h->stream));
      LB_TRY_HIP(hipStreamSynchronize(h->stream));
      st = finish_conserved(h, part.data(), conserved);
    } else {
      LB_TRY_HIP(hipStreamSynchronize(h->stream));
    }
    return st;
  } catch (const std::bad_alloc&) {
    return LB_ENOMEM;
  }
}

int lb_destroy(lb_handle* h) {
  if (!h) return LB_OK;
  int st = LB_OK;
  hipError_t se = hipStreamSynchronize(h->stream);
  if (se != hipSuccess) st = status_of(se);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  if (h->owned && h->base) {
    hipError_t e = hipFree(h->base);
    if (e != hipSuccess && st == LB_OK) st = status_of(e);
  }
  delete h;
  return st;
}

const char* lb_strerror(int status) {
  switch (status) {
    case LB_OK: return "ok";
    case LB_EINVAL: return "invalid argument or parameter combination";
    case LB_ENOMEM: return "out of memory or buffer too small";
    case LB_EUNSUPPORTED: return "not supported by this build";
    case LB_EDEVICE: return "HIP runtime error";
    case LB_ENONFINITE: return "non-finite value";
  }
  return "unknown status";
}

int lb_timing_begin(lb_handle* h, int64_t max_steps) {
  if (!h || max_steps < 0) return LB_EINVAL;
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
  h->tcap = 0;
  h->tcount = 0;
  try {
    h->ev.resize((size_t)4 * max_steps, nullptr);
  } catch (const std::bad_alloc&) {
    return LB_ENOMEM;
  }
  for (auto& e : h->ev) LB_TRY_HIP(hipEventCreate(&e));
  h->tcap = max_steps;
  return LB_OK;
}

int lb_timing_end(lb_handle* h, double* ms, int64_t* launches) {
  if (!h || !ms || !launches) return LB_EINVAL;
  LB_TRY_HIP(hipStreamSynchronize(h->stream));
  double t[2] = {0.0, 0.0};
  for (int64_t s = 0; s < h->tcount; ++s) {
    float a = 0.f, b = 0.f;
    LB_TRY_HIP(hipEventElapsedTime(&a, h->ev[(size_t)4 * s], h->ev[(size_t)4 * s + 1]));
    LB_TRY_HIP(hipEventElapsedTime(&b, h->ev[(size_t)4 * s + 2], h->ev[(size_t)4 * s + 3]));
    t[0] += a;
    t[1] += b;
  }
  ms[0] = t[0];
  ms[1] = t[1];
  launches[0] = launches[1] = h->tcount;
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
  h->tcap = h->tcount = 0;
  return LB_OK;
}

int lb_check_division(void* hip_stream, uint64_t* mismatches) {
  if (!mismatches) return LB_EINVAL;
  const hipStream_t st = (hipStream_t)hip_stream;
  unsigned long long* d = nullptr;
  LB_TRY_HIP(hipMalloc(&d, 3 * sizeof(unsigned long long)));
  unsigned long long h[3] = {0, 0, 0};
  hipError_t e = hipMemsetAsync(d, 0, sizeof(h), st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_division_check<3>, dim3(16384), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_division_check<9>, dim3(16384), dim3(256), 0, st, d + 1);
    hipLaunchKernelGGL(k_division_check<27>, dim3(16384), dim3(256), 0, st, d + 2);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d);
  if (e != hipSuccess) return status_of(e);
  for (int i = 0; i < 3; ++i) mismatches[i] = h[i];
  return LB_OK;
}

int lb_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src || (bytes % 16) || ((uintptr_t)dst % 16) || ((uintptr_t)src % 16))
    return LB_EINVAL;
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return LB_OK;
  const int64_t blocks = (n16 + 255) / 256;
  hipLaunchKernelGGL(k_copy, grid_of(blocks), dim3(256), 0, (hipStream_t)hip_stream,
                     (const lb_u4*)src, (lb_u4*)dst, n16);
  return launch_status(hipGetLastError());
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched execution
// ---------------------------------------------------------------------------
struct lb_batch {
  hipStream_t stream = nullptr;
  void* d_buf = nullptr;
  size_t d_cap = 0;
  void* h_buf = nullptr;  // pinned staging for the descriptor tables
  size_t h_cap = 0;
  hipEvent_t copied = nullptr;
  bool copy_pending = false;
  int graphs = 1;
  // Instantiated one-step graphs, keyed by the launch configuration they
  // captured (kernels, table addresses, job and work-unit counts).  The
  // tables are rewritten before every run, so a graph serves every call
  // whose segments launch the same configuration, whichever handles it
  // holds.  Oldest first; cleared when the table buffer moves.
  std::vector<std::pair<std::vector<int64_t>, hipGraphExec_t>> graph_cache;
  double* c_buf = nullptr;  // pinned staging of lb_batch_conserved
  size_t c_cap = 0;
};

namespace {

struct BatchGroup {
  const Impl* impl;
  int v2;
  std::vector<int> jobs;    // indices into the handle array, input order
  size_t off_k1 = 0, off_k2 = 0;  // byte offsets of the two tables
  int64_t units_k1 = 0, units_k2 = 0;
};

struct BatchSegment {
  int64_t steps = 0;
  std::vector<BatchGroup> groups;
};

constexpr size_t kGraphCacheSize = 16;

std::vector<int64_t> graph_key(const lb_batch* b, const BatchSegment& seg) {
  std::vector<int64_t> k;
  k.push_back((int64_t)(intptr_t)b->d_buf);
  for (const auto& g : seg.groups) {
    k.push_back((int64_t)(intptr_t)g.impl);
    k.push_back(g.v2);
    k.push_back((int64_t)g.jobs.size());
    k.push_back((int64_t)g.off_k1);
    k.push_back((int64_t)g.off_k2);
    k.push_back(g.units_k1);
    k.push_back(g.units_k2);
  }
  return k;
}

void clear_graph_cache(lb_batch* b) {
  for (auto& e : b->graph_cache) (void)hipGraphExecDestroy(e.second);
  b->graph_cache.clear();
}

hipError_t launch_segment_step(const lb_batch* b, const BatchSegment& seg) {
  for (const auto& g : seg.groups) {
    hipError_t e = g.impl->batch_moments((const char*)b->d_buf + g.off_k1, (int)g.jobs.size(),
                                         g.units_k1, b->stream);
    if (e != hipSuccess) return e;
  }
  for (const auto& g : seg.groups) {
    hipError_t e = g.impl->batch_sc((const char*)b->d_buf + g.off_k2, (int)g.jobs.size(),
                                    g.units_k2, g.v2, b->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

int lb_batch_create(void* hip_stream, lb_batch** out) {
  if (!out) return LB_EINVAL;
  *out = nullptr;
  try {
    lb_batch* b = new lb_batch();
    b->stream = (hipStream_t)hip_stream;
    hipError_t e = hipEventCreateWithFlags(&b->copied, hipEventDisableTiming);
    if (e != hipSuccess) {
      delete b;
      return status_of(e);
    }
    *out = b;
    return LB_OK;
  } catch (const std::bad_alloc&) {
    return LB_ENOMEM;
  }
}

int lb_batch_set_graphs(lb_batch* b, int enable) {
  if (!b) return LB_EINVAL;
  b->graphs = enable ? 1 : 0;
  return LB_OK;
}

int lb_batch_step(lb_batch* b, lb_handle* const* hs, const int64_t* nsteps, int count) {
  if (!b || count < 0 || (count > 0 && (!hs || !nsteps))) return LB_EINVAL;
  for (int i = 0; i < count; ++i) {
    if (!hs[i] || nsteps[i] < 0) return LB_EINVAL;
    if (hs[i]->stream != b->stream) return LB_EINVAL;
    for (int k = 0; k < i; ++k)
      if (hs[k] == hs[i]) return LB_EINVAL;
  }
  // the batched sweeps have no near-contact flag pass
  for (int i = 0; i < count; ++i)
    if (hs[i]->nci || !hs[i]->p.keep_moments) return LB_EUNSUPPORTED;
  if (count == 0) return LB_OK;
  try {
    // segments of constant active set: jobs sorted by their step counts
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return nsteps[a] < nsteps[c]; });
    std::vector<BatchSegment> segs;
    int64_t done = 0;
    for (int k = 0; k < count; ++k) {
      const int64_t target = nsteps[order[k]];
      if (target <= done) continue;
      BatchSegment seg;
      seg.steps = target - done;
      // active: every job with nsteps > done, grouped by kernel configuration
      std::map<std::pair<const Impl*, int>, size_t> gidx;
      for (int i = 0; i < count; ++i) {
        if (nsteps[i] <= done) continue;
        const auto key = std::make_pair(hs[i]->impl, hs[i]->v2);
        auto it = gidx.find(key);
        if (it == gidx.end()) {
          gidx[key] = seg.groups.size();
          BatchGroup g;
          g.impl = hs[i]->impl;
          g.v2 = hs[i]->v2;
          seg.groups.push_back(g);
          it = gidx.find(key);
        }
        seg.groups[it->second].jobs.push_back(i);
      }
      segs.push_back(std::move(seg));
      done = target;
    }
    // descriptor tables of every segment in one staging block
    size_t bytes = 0;
    for (auto& seg : segs)
      for (auto& g : seg.groups) {
        const size_t tb = align_up(g.impl->desc_size * g.jobs.size(), 256);
        g.off_k1 = bytes;
        bytes += tb;
        g.off_k2 = bytes;
        bytes += tb;
      }
    if (b->copy_pending) {
      LB_TRY_HIP(hipEventSynchronize(b->copied));
      b->copy_pending = false;
    }
    if (bytes > b->h_cap) {
      if (b->h_buf) (void)hipHostFree(b->h_buf);
      b->h_buf = nullptr;
      b->h_cap = 0;
      LB_TRY_HIP(hipHostMalloc(&b->h_buf, bytes, hipHostMallocDefault));
      b->h_cap = bytes;
    }
    if (bytes > b->d_cap) {
      LB_TRY_HIP(hipStreamSynchronize(b->stream));  // old tables may still be in use
      clear_graph_cache(b);  // the cached graphs point into the old tables
      if (b->d_buf) (void)hipFree(b->d_buf);
      b->d_buf = nullptr;
      b->d_cap = 0;
      LB_TRY_HIP(hipMalloc(&b->d_buf, bytes));
      b->d_cap = bytes;
    }
    for (auto& seg : segs)
      for (auto& g : seg.groups) {
        int64_t u1 = 0, u2 = 0;
        for (size_t q = 0; q < g.jobs.size(); ++q) {
          const lb_handle* h = hs[g.jobs[q]];
          g.impl->fill_desc(h, (char*)b->h_buf + g.off_k1 + q * g.impl->desc_size, u1);
          g.impl->fill_desc(h, (char*)b->h_buf + g.off_k2 + q * g.impl->desc_size, u2);
          u1 += g.impl->units_moments(h);
          u2 += g.impl->units_sc(h);
        }
        g.units_k1 = u1;
        g.units_k2 = u2;
      }
    LB_TRY_HIP(hipMemcpyAsync(b->d_buf, b->h_buf, bytes, hipMemcpyHostToDevice, b->stream));
    LB_TRY_HIP(hipEventRecord(b->copied, b->stream));
    b->copy_pending = true;
    for (const auto& seg : segs) {
      const bool graph = b->graphs && b->stream != nullptr && seg.steps >= 3;
      if (graph) {
        const std::vector<int64_t> key = graph_key(b, seg);
        hipGraphExec_t ex = nullptr;
        for (const auto& e : b->graph_cache)
          if (e.first == key) ex = e.second;
        if (!ex) {
          hipGraph_t gr = nullptr;
          LB_TRY_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
          hipError_t le = launch_segment_step(b, seg);
          hipError_t ce = hipStreamEndCapture(b->stream, &gr);
          if (le != hipSuccess || ce != hipSuccess) {
            if (gr) (void)hipGraphDestroy(gr);
            return status_of(le != hipSuccess ? le : ce);
          }
          hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
          (void)hipGraphDestroy(gr);
          if (ie != hipSuccess) return status_of(ie);
          if (b->graph_cache.size() >= kGraphCacheSize) {
            (void)hipGraphExecDestroy(b->graph_cache.front().second);
            b->graph_cache.erase(b->graph_cache.begin());
          }
          b->graph_cache.emplace_back(key, ex);
        }
        hipError_t ge = hipSuccess;
        for (int64_t s = 0; s < seg.steps && ge == hipSuccess; ++s) ge = hipGraphLaunch(ex, b->stream);
        hipError_t se = hipStreamSynchronize(b->stream);
        if (ge != hipSuccess) return status_of(ge);
        if (se != hipSuccess) return status_of(se);
      } else {
        for (int64_t s = 0; s < seg.steps; ++s) LB_TRY_HIP(launch_segment_step(b, seg));
      }
    }
    for (int i = 0; i < count; ++i) hs[i]->steps += nsteps[i];
    return LB_OK;
  } catch (const std::bad_alloc&) {
    return LB_ENOMEM;
  }
}

int lb_step_batch(lb_handle* const* hs, const int64_t* nsteps, int count) {
  if (count < 0 || (count > 0 && (!hs || !nsteps))) return LB_EINVAL;
  if (count == 0) return LB_OK;
  if (!hs[0]) return LB_EINVAL;
  lb_batch* b = nullptr;
  int st = lb_batch_create(hs[0]->stream, &b);
  if (st != LB_OK) return st;
  st = lb_batch_step(b, hs, nsteps, count);
  const int dst = lb_batch_destroy(b);
  return st != LB_OK ? st : dst;
}

int lb_batch_conserved(lb_batch* b, lb_handle* const* hs, int count, double* out) {
  if (!b || count < 0 || (count > 0 && (!hs || !out))) return LB_EINVAL;
  for (int i = 0; i < count; ++i)
    if (!hs[i] || hs[i]->stream != b->stream) return LB_EINVAL;
  if (count == 0) return LB_OK;
  const size_t per = (size_t)kRedBlocks * 8;  // doubles of one handle's partial sums
  const size_t need = per * (size_t)count * sizeof(double);
  if (need > b->c_cap) {
    LB_TRY_HIP(hipStreamSynchronize(b->stream));
    if (b->c_buf) (void)hipHostFree(b->c_buf);
    b->c_buf = nullptr;
    b->c_cap = 0;
    LB_TRY_HIP(hipHostMalloc((void**)&b->c_buf, need, hipHostMallocDefault));
    b->c_cap = need;
  }
  for (int i = 0; i < count; ++i) {
    LB_TRY_HIP(hs[i]->impl->conserved(hs[i]));
    LB_TRY_HIP(hipMemcpyAsync(b->c_buf + per * i, hs[i]->partial, per * sizeof(double),
                              hipMemcpyDeviceToHost, b->stream));
  }
  LB_TRY_HIP(hipStreamSynchronize(b->stream));
  int st = LB_OK;
  for (int i = 0; i < count; ++i)
    if (finish_conserved(hs[i], b->c_buf + per * i, out + 6 * (size_t)i) != LB_OK)
      st = LB_ENONFINITE;
  return st;
}

int lb_batch_destroy(lb_batch* b) {
  if (!b) return LB_OK;
  int st = LB_OK;
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) st = status_of(e);
  clear_graph_cache(b);
  if (b->c_buf) (void)hipHostFree(b->c_buf);
  if (b->d_buf) (void)hipFree(b->d_buf);
  if (b->h_buf) (void)hipHostFree(b->h_buf);
  if (b->copied) (void)hipEventDestroy(b->copied);
  delete b;
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched step without allocation (lb_step_batch_noalloc)
//
// The descriptor tables live in a fixed per-device array instead of buffers
// allocated per call.  They are written there by small kernels that carry
// the descriptor bytes as kernel arguments, so no host staging buffer has to
// outlive the call and nothing waits: every write is ordered on the
// handles' stream after the previous segment's sweeps.  Host-side
// bookkeeping uses fixed-size arrays on the stack.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[LB_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kPutWords = 384;  // 3 KiB of descriptor bytes per write kernel
constexpr int kMaxDevices = 64;

struct ScratchPut {
  uint64_t w[kPutWords];
  uint32_t dst_word;  // first destination word in the scratch array
  uint32_t nwords;
};

__global__ __launch_bounds__(kPutWords) void k_scratch_put(uint64_t* __restrict__ base,
                                                           ScratchPut put) {
  const uint32_t t = threadIdx.x;
  if (t < put.nwords) base[put.dst_word + t] = put.w[t];
}

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device
// (the host-side name of the array is not a device address).
hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Accumulates descriptor bytes bound for consecutive scratch words and
// flushes them as one write kernel when full or when the next bytes go
// elsewhere.
struct Putter {
  uint64_t* base;
  hipStream_t stream;
  ScratchPut put;
  hipError_t err = hipSuccess;
  Putter(void* b, hipStream_t s) : base((uint64_t*)b), stream(s) {
    put.dst_word = 0;
    put.nwords = 0;
  }
  void flush() {
    if (put.nwords == 0 || err != hipSuccess) {
      put.nwords = 0;
      return;
    }
    hipLaunchKernelGGL(k_scratch_put, dim3(1), dim3(kPutWords), 0, stream, base, put);
    err = hipGetLastError();
    put.nwords = 0;
  }
  // bytes: a multiple of 8; byte_off: a multiple of 8
  void append(const void* src, size_t bytes, size_t byte_off) {
    const uint32_t word = (uint32_t)(byte_off / 8);
    const uint32_t n = (uint32_t)(bytes / 8);
    if (put.nwords && (put.dst_word + put.nwords != word || put.nwords + n > kPutWords)) flush();
    if (put.nwords == 0) put.dst_word = word;
    std::memcpy(&put.w[put.nwords], src, bytes);
    put.nwords += n;
  }
};

struct NoAllocGroup {
  const Impl* impl;
  int v2;
  int njobs;
  size_t off_k1, off_k2;
  int64_t units_k1, units_k2;
};

}  // namespace

extern "C" {

int lb_step_batch_noalloc(lb_handle* const* hs, const int64_t* nsteps, int count) {
  if (count < 0 || (count > 0 && (!hs || !nsteps))) return LB_EINVAL;
  if (count == 0) return LB_OK;
  if (count > LB_NOALLOC_MAX_HANDLES) return LB_ENOMEM;
  for (int i = 0; i < count; ++i) {
    if (!hs[i] || nsteps[i] < 0) return LB_EINVAL;
    if (hs[i]->stream != hs[0]->stream || hs[i]->device != hs[0]->device) return LB_EINVAL;
    for (int k = 0; k < i; ++k)
      if (hs[k] == hs[i]) return LB_EINVAL;
  }
  for (int i = 0; i < count; ++i)
    if (hs[i]->nci || !hs[i]->p.keep_moments) return LB_EUNSUPPORTED;
  int cur = -1;
  LB_TRY_HIP(hipGetDevice(&cur));
  if (cur != hs[0]->device) return LB_EINVAL;
  void* sbase = nullptr;
  LB_TRY_HIP(scratch_address(cur, &sbase));
  const hipStream_t stream = hs[0]->stream;

  // jobs by step count (ties in input order): each distinct count ends a
  // segment over a fixed set of active jobs
  int order[LB_NOALLOC_MAX_HANDLES];
  for (int i = 0; i < count; ++i) order[i] = i;
  std::sort(order, order + count, [&](int a, int c) {
    return nsteps[a] < nsteps[c] || (nsteps[a] == nsteps[c] && a < c);
  });

  NoAllocGroup groups[LB_NOALLOC_MAX_HANDLES];
  unsigned char desc[512];
  int64_t done = 0;
  for (int k = 0; k < count; ++k) {
    const int64_t target = nsteps[order[k]];
    if (target <= done) continue;
    // active jobs grouped by kernel configuration, groups in order of first job
    int ng = 0;
    for (int i = 0; i < count; ++i) {
      if (nsteps[i] <= done) continue;
      int g = 0;
      while (g < ng && !(groups[g].impl == hs[i]->impl && groups[g].v2 == hs[i]->v2)) ++g;
      if (g == ng) {
        groups[ng] = NoAllocGroup{hs[i]->impl, hs[i]->v2, 0, 0, 0, 0, 0};
        ++ng;
      }
      ++groups[g].njobs;
    }
    size_t bytes = 0;
    for (int g = 0; g < ng; ++g) {
      const size_t tb = align_up(groups[g].impl->desc_size * groups[g].njobs, 256);
      groups[g].off_k1 = bytes;
      bytes += tb;
      groups[g].off_k2 = bytes;
      bytes += tb;
    }
    // the first segment holds every job, later ones subsets: only the first
    // can exceed the array, and then nothing has been enqueued yet
    if (bytes > LB_NOALLOC_SCRATCH_BYTES) return LB_ENOMEM;
    Putter put(sbase, stream);
    for (int g = 0; g < ng; ++g) {
      NoAllocGroup& G = groups[g];
      const size_t ds = G.impl->desc_size;
      if (ds > sizeof(desc) || ds % 8) return LB_EUNSUPPORTED;
      int64_t u1 = 0, u2 = 0;
      int q = 0;
      for (int i = 0; i < count; ++i) {
        if (nsteps[i] <= done || hs[i]->impl != G.impl || hs[i]->v2 != G.v2) continue;
        G.impl->fill_desc(hs[i], desc, u1);
        put.append(desc, ds, G.off_k1 + (size_t)q * ds);
        u1 += G.impl->units_moments(hs[i]);
        ++q;
      }
      q = 0;
      for (int i = 0; i < count; ++i) {
        if (nsteps[i] <= done || hs[i]->impl != G.impl || hs[i]->v2 != G.v2) continue;
        G.impl->fill_desc(hs[i], desc, u2);
        put.append(desc, ds, G.off_k2 + (size_t)q * ds);
        u2 += G.impl->units_sc(hs[i]);
        ++q;
      }
      G.units_k1 = u1;
      G.units_k2 = u2;
    }
    put.flush();
    LB_TRY_HIP(put.err);
    const char* tables = (const char*)sbase;
    for (int64_t s = 0; s < target - done; ++s) {
      for (int g = 0; g < ng; ++g)
        LB_TRY_HIP(groups[g].impl->batch_moments(tables + groups[g].off_k1, groups[g].njobs,
                                                 groups[g].units_k1, stream));
      for (int g = 0; g < ng; ++g)
        LB_TRY_HIP(groups[g].impl->batch_sc(tables + groups[g].off_k2, groups[g].njobs,
                                            groups[g].units_k2, groups[g].v2, stream));
    }
    done = target;
  }
  for (int i = 0; i < count; ++i) hs[i]->steps += nsteps[i];
  return LB_OK;
}

}  // extern "C"
