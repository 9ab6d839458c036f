// Kernels and launches of D2Q9 with F64 storage (both equilibria).
#include "kernels_impl.hpp"

namespace lbm {
template struct Ops<D2Q9, StoreF64, 0>;
template struct Ops<D2Q9, StoreF64, 1>;
}  // namespace lbm
