// Kernel instantiations for D3Q27, second-order Hermite terms, 16-bit storage.
#include "handle.hpp"

namespace lbk {
const Impl* impl_d3q27_half(int storage) { return impl_half<D3Q27, 2>(storage); }
}  // namespace lbk
