// Kernels and launches of D3Q19 with F64 storage (both equilibria).
#include "kernels_impl.hpp"

namespace lbm {
template struct Ops<D3Q19, StoreF64, 0>;
template struct Ops<D3Q19, StoreF64, 1>;
}  // namespace lbm
