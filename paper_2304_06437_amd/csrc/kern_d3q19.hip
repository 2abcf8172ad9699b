// Kernel instantiations for D3Q19.
#include "handle.hpp"

namespace lbk {
const Impl* impl_d3q19(int storage, int species) {
  return species == 2 ? impl2_for_storage<D3Q19>(storage) : impl_for_storage<D3Q19, 2>(storage);
}
}  // namespace lbk
