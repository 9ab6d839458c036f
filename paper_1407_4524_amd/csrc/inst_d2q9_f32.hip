// Kernels and launches of D2Q9 with F32 storage (both equilibria).
#include "kernels_impl.hpp"

namespace lbm {
template struct Ops<D2Q9, StoreF32, 0>;
template struct Ops<D2Q9, StoreF32, 1>;
}  // namespace lbm
