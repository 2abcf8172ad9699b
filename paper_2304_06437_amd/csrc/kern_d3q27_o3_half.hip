// Kernel instantiations for D3Q27 with the recursive third-order Hermite
// terms, 16-bit storage.
#include "handle.hpp"

namespace lbk {
const Impl* impl_d3q27_order3_half(int storage) { return impl_half<D3Q27, 3>(storage); }
}  // namespace lbk
