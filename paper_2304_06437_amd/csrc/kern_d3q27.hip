// Kernel instantiations for D3Q27, second-order Hermite terms; the
// third-order ones live in their own translation unit (compiled in parallel).
#include "handle.hpp"

namespace lbk {
const Impl* impl_d3q27(int order, int storage) {
  return order == 3 ? impl_d3q27_order3(storage) : impl_for_storage<D3Q27, 2>(storage);
}
}  // namespace lbk
