// Kernels and launches of D2Q9 with F16 storage (both equilibria).
#include "kernels_impl.hpp"

namespace lbm {
template struct Ops<D2Q9, StoreF16, 0>;
template struct Ops<D2Q9, StoreF16, 1>;
}  // namespace lbm
