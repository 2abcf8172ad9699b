// Kernel instantiations for D3Q27, second-order Hermite terms, 32/64-bit
// storage; the 16-bit storage types and the third-order terms live in their
// own translation units (compiled in parallel).
#include "handle.hpp"

namespace lbk {
const Impl* impl_d3q27(int order, int storage) {
  if (order == 3) return impl_d3q27_order3(storage);
  return half_storage(storage) ? impl_d3q27_half(storage) : impl_wide<D3Q27, 2>(storage);
}
}  // namespace lbk
