// Kernel instantiations for D3Q19 with 16-bit (shifted FP16 / BF16) storage.
#include "handle.hpp"

namespace lbk {
const Impl* impl_d3q19_half(int storage) { return impl_half<D3Q19, 2>(storage); }
}  // namespace lbk
