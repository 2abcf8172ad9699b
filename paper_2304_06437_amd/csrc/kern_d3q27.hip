// Kernel instantiations for D3Q27 (second- and third-order Hermite terms).
#include "handle.hpp"

namespace lbk {
const Impl* impl_d3q27(int order, int storage) {
  return order == 3 ? impl_for_storage<D3Q27, 3>(storage) : impl_for_storage<D3Q27, 2>(storage);
}
}  // namespace lbk
