// Kernel instantiations for D3Q19 with 32/64-bit storage and two species; the
// 16-bit storage types live in their own translation unit (compiled in
// parallel).
#include "handle.hpp"

namespace lbk {
const Impl* impl_d3q19(int storage, int species) {
  if (species == 2) return impl2_for_storage<D3Q19>(storage);
  return half_storage(storage) ? impl_d3q19_half(storage) : impl_wide<D3Q19, 2>(storage);
}
}  // namespace lbk
