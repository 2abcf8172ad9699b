// Kernel instantiations for D2Q9.
#include "handle.hpp"

namespace lbk {
const Impl* impl_d2q9(int storage) { return impl_for_storage<D2Q9, 2>(storage); }
}  // namespace lbk
