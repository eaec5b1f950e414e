// Kernel instantiations completing the domain m <= 10, L <= 8: codes of length 128 and 256
// (first-order and single-parity-check roots, higher orders, lists of 2 and 8).
// Shapes marked with a budget of 2 waves per SIMD (up to 256 VGPRs) spill at 3.
#include "rmdec_kernels.hpp"

namespace rmdec {
static const KernelEntry kEntries[] = {
    entry<7, 1, 1>(), entry<7, 1, 2>(), entry<7, 1, 4>(), entry<7, 1, 8>(), entry<7, 4, 1>(), entry<7, 4, 2>(),
    entry<7, 4, 4>(), entry<7, 4, 8>(), entry<7, 5, 1>(), entry<7, 5, 2>(), entry<7, 5, 4>(), entry<7, 5, 8>(),
    entry<7, 6, 1>(), entry<7, 6, 2>(), entry<7, 6, 4>(), entry<7, 6, 8>(), entry<8, 1, 1>(), entry<8, 1, 2>(),
    entry<8, 1, 4, decoders_per_wave(8, 4), 2>(), entry<8, 1, 8>(), entry<8, 5, 1>(), entry<8, 5, 2>(),
    entry<8, 5, 4>(), entry<8, 5, 8>(), entry<8, 6, 1>(), entry<8, 6, 2>(),
    entry<8, 6, 4, decoders_per_wave(8, 4), 2>(), entry<8, 6, 8>(), entry<8, 7, 1>(), entry<8, 7, 2>(),
    entry<8, 7, 4, decoders_per_wave(8, 4), 2>(), entry<8, 7, 8>(),
};
KernelTable kernels_codes_j() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
