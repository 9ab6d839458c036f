// Kernels and launches of D3Q19 with F16 storage (both equilibria).
#include "kernels_impl.hpp"

namespace lbm {
template struct Ops<D3Q19, StoreF16, 0>;
template struct Ops<D3Q19, StoreF16, 1>;
}  // namespace lbm
