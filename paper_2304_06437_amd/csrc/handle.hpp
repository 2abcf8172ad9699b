// Internal: simulation handle and per-configuration kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "kernels.hpp"
#include "kernels2.hpp"
#include "kernels_batch.hpp"
#include "fused.hpp"

#include <cstring>
#include "lb.h"

namespace lbk {

constexpr int kRedBlocks = 1024;  // blocks of the conservation reduction

// Grid of `blocks` 256-thread blocks: one dimension holds at most 2^32
// work-items, so larger launches lay their blocks out x-fastest over
// (x, y); kernels number them with flat_block() and drop the blocks past
// the end.  Enough for any domain lb_validate accepts (y <= 65535).
constexpr int64_t kMaxGridX = (int64_t(1) << 24) - 1;
inline dim3 grid_of(int64_t blocks) {
  if (blocks <= kMaxGridX) return dim3((unsigned)blocks);
  return dim3((unsigned)kMaxGridX, (unsigned)((blocks + kMaxGridX - 1) / kMaxGridX));
}

struct Layout {
  int Q = 0, D = 0, M = 0, species = 1;
  size_t ssize = 0, csize = 0;  // bytes per stored population / per moment
  int64_t N = 0, npad = 0;      // lattice nodes; storage nodes padded to whole blocks
  int64_t px = 0;               // row pitch: storage nodes per x-row (>= nx)
  int v2 = 1;                   // nodes per lane of the stream-collide sweep
  int lb = 10;                  // log2 of the block size of the array layout
  // regions: populations, moments, near-contact flags, reference colours,
  // reduction scratch, progress words of the fused step
  size_t f_off = 0, m_off = 0, n_off = 0, c_off = 0, r_off = 0, s_off = 0, total = 0;
};

struct Impl;

}  // namespace lbk

struct lb_handle {
  lb_params p;
  lbk::Layout L;
  const lbk::Impl* impl = nullptr;
  void* base = nullptr;
  bool owned = false;
  void* f = nullptr;
  void* m = nullptr;
  double* partial = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;  // HIP device current at lb_create
  int64_t steps = 0;
  int v2 = 1;  // nodes per lane of the stream-collide sweep
  lbk::StepParams<float> p32;
  lbk::StepParams<double> p64;
  lbk::ColourParams<float> cp32;
  lbk::ColourParams<double> cp64;
  // near-contact interactions (two species): flags, one byte per storage node
  bool nci = false;
  unsigned char* flag = nullptr;
  lbk::NciParams<float> nq32;
  lbk::NciParams<double> nq64;
  // fused step: nodes per lane of its kernel (row = 64 fv nodes, 0: the
  // shape has none), tiling and progress words, the path lb_step takes
  int fv = 0;
  int path = 0;         // requested: 0 automatic, 1 two sweeps, 2 fused
  bool use_fused = false;
  int order = 0;        // wavefront order of lb_set_sweep_order
  int32_t wait_limit = lbk::kFusedWaitLimit;  // lb_set_fused_wait_limit
  lbk::FusedParams fp{};
  // per-kernel timing
  std::vector<hipEvent_t> ev;
  int64_t tcap = 0, tcount = 0;
};

namespace lbk {

struct Impl {
  int v1;
  int v2max;  // widest lane vector (nodes per lane) of the stream-collide sweep
  int emax;   // widest contiguous chunk of it; rows are padded to a multiple
  hipError_t (*moments)(const lb_handle*);
  hipError_t (*stream_collide)(const lb_handle*);
  hipError_t (*init)(const lb_handle*, const double*, int64_t, int64_t);
  hipError_t (*readout)(const lb_handle*, double*, int64_t, int64_t);
  hipError_t (*conserved)(const lb_handle*);
  // batched execution (lb_batch_step)
  size_t desc_size;
  void (*fill_desc)(const lb_handle*, void* dst, int64_t start);
  int64_t (*units_moments)(const lb_handle*);
  int64_t (*units_sc)(const lb_handle*);
  hipError_t (*batch_moments)(const void* d_desc, int n, int64_t total, hipStream_t s);
  hipError_t (*batch_sc)(const void* d_desc, int n, int64_t total, int v2, hipStream_t s);
  // fused step for rows of 64 v nodes (nullptr: not built for this
  // configuration or this v)
  const void* (*fused_kernel)(int v) = nullptr;
  hipError_t (*fused)(const lb_handle*) = nullptr;
};

template <typename C>
inline void fill_job_desc(const lb_handle* h, void* dst, int64_t start);

template <typename C>
inline const StepParams<C>& params_of(const lb_handle* h);
template <>
inline const StepParams<float>& params_of<float>(const lb_handle* h) { return h->p32; }
template <>
inline const StepParams<double>& params_of<double>(const lb_handle* h) { return h->p64; }
template <typename C>
inline const ColourParams<C>& colour_of(const lb_handle* h);
template <>
inline const ColourParams<float>& colour_of<float>(const lb_handle* h) { return h->cp32; }
template <>
inline const ColourParams<double>& colour_of<double>(const lb_handle* h) { return h->cp64; }
template <typename C>
inline const NciParams<C>& nci_of(const lb_handle* h);
template <>
inline const NciParams<float>& nci_of<float>(const lb_handle* h) { return h->nq32; }
template <>
inline const NciParams<double>& nci_of<double>(const lb_handle* h) { return h->nq64; }

template <typename C>
inline void fill_job_desc(const lb_handle* h, void* dst, int64_t start) {
  JobDesc<C> d;
  std::memset(&d, 0, sizeof(d));
  d.p = params_of<C>(h);
  d.cp = colour_of<C>(h);
  d.m = h->m;
  d.f = h->f;
  d.start = start;
  std::memcpy(dst, &d, sizeof(d));
}

// V1: nodes per lane of the moments sweep.  V2MAX: the widest row
// vector (nodes per lane) of the stream-collide sweep; a lane's V nodes are
// H = V/E chunks of E <= EMAX consecutive nodes.  V2MAX and EMAX per lattice
// and storage type are the fastest measured at 512^3 (D3Q19, D3Q27) and
// 4096^2 (D2Q9) with the blocked layout.  FD: the short division of the
// coefficient prescaling (see scaled), for the instruction-bound D3Q27
// 16-bit sweeps.
template <class L, int ORDER, typename S, typename C, int V1, int V2MAX, int EMAX>
struct ImplT {
  static constexpr bool FD = L::Q == 27 && sizeof(S) == 2;
  static hipError_t moments(const lb_handle* h) {
    const auto& p = params_of<C>(h);
    const int64_t threads = p.npad / V1;
    hipLaunchKernelGGL((k_moments<L, S, C, V1>), grid_of((threads + 255) / 256), dim3(256), 0,
                       h->stream, (const S*)h->f, (C*)h->m, p);
    return hipGetLastError();
  }
  template <int V>
  static hipError_t sc(const lb_handle* h) {
    constexpr int E = V < EMAX ? V : EMAX;
    constexpr int HH = V / E;
    const auto& p = params_of<C>(h);
    const int64_t waves = p.nseg * p.ny * p.nz;
    const dim3 grid = grid_of((waves + 3) / 4);
    // the instruction-bound FD sweeps get a variant without the padded-row
    // selects for aligned rows; elsewhere the selects cost no measurable time.
    // D3Q27 rows inside one layout block (px divides B) take the variant that
    // addresses a row from its first node (measured 1-4 % faster at 512^3;
    // 1-3.5 % slower for D3Q19 and D2Q9, which keep 64-bit lane addresses).
    const bool rb = L::Q == 27 && ((int64_t(1) << p.lb) % p.px) == 0;
    if (FD && p.px == p.nx) {
      if (rb)
        hipLaunchKernelGGL((k_stream_collide<L, ORDER, S, C, E, HH, FD, !FD, L::Q == 27>), grid,
                           dim3(256), 0, h->stream, (const C*)h->m, (S*)h->f, p);
      else
        hipLaunchKernelGGL((k_stream_collide<L, ORDER, S, C, E, HH, FD, !FD>), grid, dim3(256),
                           0, h->stream, (const C*)h->m, (S*)h->f, p);
    } else {
      if (rb)
        hipLaunchKernelGGL((k_stream_collide<L, ORDER, S, C, E, HH, FD, true, L::Q == 27>), grid,
                           dim3(256), 0, h->stream, (const C*)h->m, (S*)h->f, p);
      else
        hipLaunchKernelGGL((k_stream_collide<L, ORDER, S, C, E, HH, FD, true>), grid, dim3(256),
                           0, h->stream, (const C*)h->m, (S*)h->f, p);
    }
    return hipGetLastError();
  }
  static hipError_t stream_collide(const lb_handle* h) {
    switch (h->v2) {
      case 8:
        if constexpr (V2MAX >= 8) return sc<8>(h);
        break;
      case 4:
        if constexpr (V2MAX >= 4) return sc<4>(h);
        break;
      case 2:
        return sc<2>(h);
      case 1:
        return sc<1>(h);
    }
    return hipErrorInvalidValue;
  }
  static hipError_t init(const lb_handle* h, const double* stage, int64_t n0, int64_t cnt) {
    const auto& p = params_of<C>(h);
    hipLaunchKernelGGL((k_init<L, ORDER, S, C>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                       h->stream, stage, n0, cnt, (S*)h->f, p);
    return hipGetLastError();
  }
  static hipError_t readout(const lb_handle* h, double* out, int64_t n0, int64_t cnt) {
    const auto& p = params_of<C>(h);
    hipLaunchKernelGGL((k_readout<L, S, C>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                       h->stream, (const S*)h->f, out, n0, cnt, p);
    return hipGetLastError();
  }
  static hipError_t conserved(const lb_handle* h) {
    const auto& p = params_of<C>(h);
    hipLaunchKernelGGL((k_conserved<L, S, C>), dim3(kRedBlocks), dim3(256), 0, h->stream,
                       (const S*)h->f, h->partial, h->L.N, p);
    return hipGetLastError();
  }
  static int64_t units_moments(const lb_handle* h) { return params_of<C>(h).npad / V1 / 256; }
  static int64_t units_sc(const lb_handle* h) {
    const auto& p = params_of<C>(h);
    return p.nseg * p.ny * p.nz;
  }
  static hipError_t batch_moments(const void* d, int n, int64_t total, hipStream_t s) {
    hipLaunchKernelGGL((k_moments_batch<L, 1, S, C, V1>), grid_of(total), dim3(256), 0, s,
                       (const JobDesc<C>*)d, n, total);
    return hipGetLastError();
  }
  template <int V>
  static hipError_t bsc(const void* d, int n, int64_t total, hipStream_t s) {
    constexpr int E = V < EMAX ? V : EMAX;
    constexpr int HH = V / E;
    hipLaunchKernelGGL((k_stream_collide_batch<L, ORDER, 1, S, C, E, HH, FD>),
                       grid_of((total + 3) / 4), dim3(256), 0, s, (const JobDesc<C>*)d,
                       n, total);
    return hipGetLastError();
  }
  static hipError_t batch_sc(const void* d, int n, int64_t total, int v2, hipStream_t s) {
    switch (v2) {
      case 8:
        if constexpr (V2MAX >= 8) return bsc<8>(d, n, total, s);
        break;
      case 4:
        if constexpr (V2MAX >= 4) return bsc<4>(d, n, total, s);
        break;
      case 2:
        return bsc<2>(d, n, total, s);
      case 1:
        return bsc<1>(d, n, total, s);
    }
    return hipErrorInvalidValue;
  }
  // Fused step (one species, 3D, FP32 or 16-bit storage): whole rows of
  // 64 V nodes per wavefront, chunks of up to FE nodes (16-byte accesses).
  static constexpr bool FUSED = L::D == 3 && sizeof(S) <= 4 && sizeof(C) == 4;
  static constexpr int FE = sizeof(S) == 2 ? 8 : 4;
  template <int V>
  static const void* fused_fn() {
    constexpr int E = V < FE ? V : FE;
    // the short division (same bits as the IEEE one in FP32, see scaled):
    // the fused step is bound by its arithmetic, not by bandwidth
    return (const void*)&k_fused_step<L, ORDER, S, C, E, V / E, true>;
  }
  static const void* fused_kernel(int v) {
    if constexpr (FUSED) {
      switch (v) {
        case 8:
          // D3Q27 rows of 512 nodes do not fit one wavefront's registers
          if constexpr (L::Q != 27) return fused_fn<8>();
          break;
        case 4: return fused_fn<4>();
        case 2: return fused_fn<2>();
      }
    }
    return nullptr;
  }
  static hipError_t fused(const lb_handle* h) {
    const void* fn = fused_kernel(h->fv);
    if (!fn) return hipErrorInvalidValue;
    S* f = (S*)h->f;
    StepParams<C> p = params_of<C>(h);
    FusedParams fp = h->fp;
    void* args[] = {(void*)&f, (void*)&p, (void*)&fp};
    return hipLaunchCooperativeKernel(fn, dim3((unsigned)((fp.tiles + 3) / 4)), dim3(256), args, 0,
                                      h->stream);
  }
  static const Impl* get() {
    static const Impl impl = {V1,           V2MAX,          EMAX < V2MAX ? EMAX : V2MAX,
                              &moments,     &stream_collide,
                              &init,        &readout,       &conserved,     sizeof(JobDesc<C>),
                              &fill_job_desc<C>, &units_moments, &units_sc, &batch_moments,
                              &batch_sc,    FUSED ? &fused_kernel : nullptr,
                              FUSED ? &fused : nullptr};
    return &impl;
  }
};

// Lane vectors per lattice and storage type: FP32 2 x 2 nodes per lane (4 x
// 1 for D3Q27); 16-bit storage one 16-byte chunk of 8 nodes (4 x 1 for
// D3Q27).  The 32/64-bit and the 16-bit storage types are instantiated by
// separate functions, so that the heavy lattices build them in separate
// translation units (which the build compiles in parallel).
template <class L>
struct LaneShape {
  static constexpr bool Q27 = L::Q == 27;
  static constexpr int V2D = Q27 ? 2 : 4;
  static constexpr int V2F = 4, EF = Q27 ? 4 : 2;
  static constexpr int V2H = Q27 ? 4 : 8, EH = Q27 ? 4 : 8;
};

inline bool half_storage(int storage) {
  return storage == LB_STORE_F16S || storage == LB_STORE_BF16S;
}

template <class L, int ORDER>
inline const Impl* impl_wide(int storage) {
  using LS = LaneShape<L>;
  switch (storage) {
    case LB_STORE_F64: return ImplT<L, ORDER, double, double, 2, LS::V2D, 2>::get();
    case LB_STORE_F32: return ImplT<L, ORDER, float, float, 4, LS::V2F, LS::EF>::get();
  }
  return nullptr;
}

template <class L, int ORDER>
inline const Impl* impl_half(int storage) {
  using LS = LaneShape<L>;
  switch (storage) {
    case LB_STORE_F16S: return ImplT<L, ORDER, _Float16, float, 4, LS::V2H, LS::EH>::get();
    case LB_STORE_BF16S: return ImplT<L, ORDER, __bf16, float, 4, LS::V2H, LS::EH>::get();
  }
  return nullptr;
}

template <class L, int ORDER>
inline const Impl* impl_for_storage(int storage) {
  return half_storage(storage) ? impl_half<L, ORDER>(storage) : impl_wide<L, ORDER>(storage);
}

// Two-species (colour-gradient) launchers: second-order Hermite terms only.
template <class L, typename S, typename C, int V1, int V2MAX>
struct ImplT2 {
  static hipError_t moments(const lb_handle* h) {
    const auto& p = params_of<C>(h);
    const int64_t threads = p.npad / V1;
    hipLaunchKernelGGL((k_moments2<L, S, C, V1>), grid_of((threads + 255) / 256), dim3(256), 0,
                       h->stream, (const S*)h->f, (C*)h->m, p, colour_of<C>(h));
    if (h->nci) {
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_nci_flags<L, C>), grid_of((p.npad + 255) / 256), dim3(256), 0,
                         h->stream, (const C*)h->m, h->flag, p, nci_of<C>(h));
    }
    return hipGetLastError();
  }
  template <int E>
  static hipError_t sc(const lb_handle* h) {
    const auto& p = params_of<C>(h);
    const int64_t waves = p.nseg * p.ny * p.nz;
    const dim3 grid = grid_of((waves + 3) / 4);
    const NciParams<C>& q = nci_of<C>(h);
    if (h->nci)
      hipLaunchKernelGGL((k_stream_collide2<L, S, C, E, false, true>), grid, dim3(256), 0,
                         h->stream, (const C*)h->m, (S*)h->f, p, colour_of<C>(h),
                         (const unsigned char*)h->flag, q);
    else if (p.nseg == 1 && !p.bbx && p.px == p.nx)
      hipLaunchKernelGGL((k_stream_collide2<L, S, C, E, true>), grid, dim3(256), 0, h->stream,
                         (const C*)h->m, (S*)h->f, p, colour_of<C>(h),
                         (const unsigned char*)nullptr, q);
    else
      hipLaunchKernelGGL((k_stream_collide2<L, S, C, E, false>), grid, dim3(256), 0, h->stream,
                         (const C*)h->m, (S*)h->f, p, colour_of<C>(h),
                         (const unsigned char*)nullptr, q);
    return hipGetLastError();
  }
  static hipError_t stream_collide(const lb_handle* h) {
    switch (h->v2) {
      case 4:
        if constexpr (V2MAX >= 4) return sc<4>(h);
        break;
      case 2:
        return sc<2>(h);
      case 1:
        return sc<1>(h);
    }
    return hipErrorInvalidValue;
  }
  static hipError_t init(const lb_handle* h, const double* stage, int64_t n0, int64_t cnt) {
    const auto& p = params_of<C>(h);
    hipLaunchKernelGGL((k_init2<L, S, C>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                       h->stream, stage, n0, cnt, (S*)h->f, p, colour_of<C>(h));
    return hipGetLastError();
  }
  static hipError_t readout(const lb_handle* h, double* out, int64_t n0, int64_t cnt) {
    const auto& p = params_of<C>(h);
    hipLaunchKernelGGL((k_readout2<L, S, C>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                       h->stream, (const S*)h->f, out, n0, cnt, p, colour_of<C>(h));
    return hipGetLastError();
  }
  static hipError_t conserved(const lb_handle* h) {
    const auto& p = params_of<C>(h);
    hipLaunchKernelGGL((k_conserved2<L, S, C>), dim3(kRedBlocks), dim3(256), 0, h->stream,
                       (const S*)h->f, h->partial, h->L.N, p, colour_of<C>(h));
    return hipGetLastError();
  }
  static int64_t units_moments(const lb_handle* h) { return params_of<C>(h).npad / V1 / 256; }
  static int64_t units_sc(const lb_handle* h) {
    const auto& p = params_of<C>(h);
    return p.nseg * p.ny * p.nz;
  }
  static hipError_t batch_moments(const void* d, int n, int64_t total, hipStream_t s) {
    hipLaunchKernelGGL((k_moments_batch<L, 2, S, C, V1>), grid_of(total), dim3(256), 0, s,
                       (const JobDesc<C>*)d, n, total);
    return hipGetLastError();
  }
  template <int E>
  static hipError_t bsc(const void* d, int n, int64_t total, hipStream_t s) {
    hipLaunchKernelGGL((k_stream_collide_batch<L, 2, 2, S, C, E, 1>),
                       grid_of((total + 3) / 4), dim3(256), 0, s, (const JobDesc<C>*)d,
                       n, total);
    return hipGetLastError();
  }
  static hipError_t batch_sc(const void* d, int n, int64_t total, int v2, hipStream_t s) {
    switch (v2) {
      case 4:
        if constexpr (V2MAX >= 4) return bsc<4>(d, n, total, s);
        break;
      case 2:
        return bsc<2>(d, n, total, s);
      case 1:
        return bsc<1>(d, n, total, s);
    }
    return hipErrorInvalidValue;
  }
  static const Impl* get() {
    static const Impl impl = {V1,           V2MAX,          V2MAX,
                              &moments,     &stream_collide,
                              &init,        &readout,       &conserved,     sizeof(JobDesc<C>),
                              &fill_job_desc<C>, &units_moments, &units_sc, &batch_moments,
                              &batch_sc};
    return &impl;
  }
};

template <class L>
inline const Impl* impl2_for_storage(int storage) {
  switch (storage) {
    case LB_STORE_F64: return ImplT2<L, double, double, 2, 2>::get();
    case LB_STORE_F32: return ImplT2<L, float, float, 4, 4>::get();
  }
  return nullptr;
}

// Translation units per lattice (and, for D3Q19 and D3Q27, per storage
// width) instantiate the kernels.
const Impl* impl_d2q9(int storage, int species);
const Impl* impl_d3q19(int storage, int species);
const Impl* impl_d3q19_half(int storage);
const Impl* impl_d3q27(int order, int storage);
const Impl* impl_d3q27_half(int storage);
const Impl* impl_d3q27_order3(int storage);
const Impl* impl_d3q27_order3_half(int storage);

}  // namespace lbk
