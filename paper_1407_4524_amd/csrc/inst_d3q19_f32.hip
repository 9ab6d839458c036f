// Kernels and launches of D3Q19 with F32 storage (both equilibria).
#include "kernels_impl.hpp"

namespace lbm {
template struct Ops<D3Q19, StoreF32, 0>;
template struct Ops<D3Q19, StoreF32, 1>;
}  // namespace lbm
