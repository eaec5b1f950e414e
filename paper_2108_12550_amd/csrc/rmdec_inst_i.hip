// Kernel instantiations completing the domain m <= 10, L <= 8: codes of length 8 to 64
// (first-order and single-parity-check roots, higher orders, lists of 2 and 8).
// Shapes marked with a budget of 2 waves per SIMD (up to 256 VGPRs) spill at 3.
#include "rmdec_kernels.hpp"

namespace rmdec {
static const KernelEntry kEntries[] = {
    entry<3, 1, 2>(), entry<3, 1, 8>(), entry<3, 2, 2>(), entry<3, 2, 8>(), entry<4, 1, 2>(), entry<4, 1, 8>(),
    entry<4, 3, 2>(), entry<4, 3, 8>(), entry<5, 1, 2>(), entry<5, 1, 8>(), entry<5, 4, 2>(), entry<5, 4, 8>(),
    entry<6, 1, 2>(), entry<6, 1, 8>(), entry<6, 4, 1>(), entry<6, 4, 2>(), entry<6, 4, 4>(), entry<6, 4, 8>(),
    entry<6, 5, 1>(), entry<6, 5, 2>(), entry<6, 5, 4>(), entry<6, 5, 8>(),
};
KernelTable kernels_codes_i() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
