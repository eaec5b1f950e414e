// Kernel instantiations completing the domain m <= 10, L <= 8: codes of length
// 1024, orders 1 to 4
// (first-order and single-parity-check roots, higher orders, lists of 2 and 8).
// Shapes marked with a budget of 2 waves per SIMD (up to 256 VGPRs) spill at 3.
#include "rmdec_kernels.hpp"

namespace rmdec {
static const KernelEntry kEntries[] = {
    entry<10, 1, 1>(), entry<10, 1, 2>(), entry<10, 1, 4, decoders_per_wave(10, 4), 2>(), entry<10, 2, 2>(),
    entry<10, 3, 1>(), entry<10, 3, 2>(), entry<10, 3, 4>(), entry<10, 3, 8>(),
    entry<10, 4, 1, decoders_per_wave(10, 1), 2>(), entry<10, 4, 2>(), entry<10, 4, 4>(), entry<10, 4, 8>(),
};
KernelTable kernels_codes_l() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
