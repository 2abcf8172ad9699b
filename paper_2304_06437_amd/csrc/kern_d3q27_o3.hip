// Kernel instantiations for D3Q27 with the recursive third-order Hermite terms.
#include "handle.hpp"

namespace lbk {
const Impl* impl_d3q27_order3(int storage) { return impl_for_storage<D3Q27, 3>(storage); }
}  // namespace lbk
