// Kernel instantiations: short codes RM(2,4..6), RM(3,5..7).
#include "rmdec_kernels.hpp"

namespace rmdec {
static const KernelEntry kEntries[] = {
    entry<4, 2, 1>(), entry<4, 2, 2>(), entry<4, 2, 4>(), entry<4, 2, 8>(),
    entry<5, 2, 1>(), entry<5, 2, 2>(), entry<5, 2, 4>(), entry<5, 2, 8>(),
    entry<6, 2, 1>(), entry<6, 2, 2>(), entry<6, 2, 4>(), entry<6, 2, 8>(),
    entry<5, 3, 1>(), entry<5, 3, 2>(), entry<5, 3, 4>(), entry<5, 3, 8>(),
    entry<6, 3, 1>(), entry<6, 3, 2>(), entry<6, 3, 4>(), entry<6, 3, 8>(),
    entry<7, 3, 1>(), entry<7, 3, 2>(), entry<7, 3, 4>(), entry<7, 3, 8>(),
};
KernelTable kernels_codes_c() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
