// Kernel instantiations for D3Q27 with the recursive third-order Hermite
// terms, 32/64-bit storage (16-bit storage: kern_d3q27_o3_half.hip).
#include "handle.hpp"

namespace lbk {
const Impl* impl_d3q27_order3(int storage) {
  return half_storage(storage) ? impl_d3q27_order3_half(storage) : impl_wide<D3Q27, 3>(storage);
}
}  // namespace lbk
