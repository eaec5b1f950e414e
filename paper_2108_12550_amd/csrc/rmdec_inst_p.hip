// Kernel instantiations completing the domain m <= 10, L <= 8: codes of length
// 1024, orders 5 to 9
// (first-order and single-parity-check roots, higher orders, lists of 2 and 8).
// Shapes marked with a budget of 2 waves per SIMD (up to 256 VGPRs) spill at 3.
#include "rmdec_kernels.hpp"

namespace rmdec {
static const KernelEntry kEntries[] = {
    entry<10, 5, 1, decoders_per_wave(10, 1), 2>(), entry<10, 5, 2>(), entry<10, 5, 4>(), entry<10, 5, 8>(),
    entry<10, 6, 1, decoders_per_wave(10, 1), 2>(), entry<10, 6, 2>(), entry<10, 6, 4>(), entry<10, 6, 8>(),
    entry<10, 7, 1, decoders_per_wave(10, 1), 2>(), entry<10, 7, 2>(), entry<10, 7, 4>(), entry<10, 7, 8>(),
    entry<10, 8, 1>(), entry<10, 8, 2>(), entry<10, 8, 4>(), entry<10, 8, 8>(), entry<10, 9, 1>(),
    entry<10, 9, 2, decoders_per_wave(10, 2), 2>(), entry<10, 9, 4, decoders_per_wave(10, 4), 2>(),
};
KernelTable kernels_codes_p() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
