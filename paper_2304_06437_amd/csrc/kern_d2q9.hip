// Kernel instantiations for D2Q9.
#include "handle.hpp"

namespace lbk {
const Impl* impl_d2q9(int storage, int species) {
  return species == 2 ? impl2_for_storage<D2Q9>(storage) : impl_for_storage<D2Q9, 2>(storage);
}
}  // namespace lbk
