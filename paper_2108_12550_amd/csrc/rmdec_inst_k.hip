// Kernel instantiations completing the domain m <= 10, L <= 8: codes of length 512
// (first-order and single-parity-check roots, higher orders, lists of 2 and 8).
// Shapes marked with a budget of 2 waves per SIMD (up to 256 VGPRs) spill at 3.
#include "rmdec_kernels.hpp"

namespace rmdec {
static const KernelEntry kEntries[] = {
    entry<9, 1, 1>(), entry<9, 1, 2>(), entry<9, 1, 4, decoders_per_wave(9, 4), 2>(),
    entry<9, 1, 8, decoders_per_wave(9, 8), 2>(), entry<9, 5, 1, decoders_per_wave(9, 1), 2>(), entry<9, 5, 2>(),
    entry<9, 5, 4>(), entry<9, 5, 8>(), entry<9, 6, 1, decoders_per_wave(9, 1), 2>(), entry<9, 6, 2>(),
    entry<9, 6, 4>(), entry<9, 6, 8>(), entry<9, 7, 1>(), entry<9, 7, 2>(), entry<9, 7, 4>(),
    entry<9, 7, 8, decoders_per_wave(9, 8), 2>(), entry<9, 8, 1>(), entry<9, 8, 2, decoders_per_wave(9, 2), 2>(),
    entry<9, 8, 4, decoders_per_wave(9, 4), 2>(), entry<9, 8, 8, decoders_per_wave(9, 8), 2>(),
};
KernelTable kernels_codes_k() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
