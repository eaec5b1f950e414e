// Kernel instantiations: RM(2,7), RM(2,8) and RM(3,8).
#include "rmdec_kernels.hpp"

namespace rmdec {
static const KernelEntry kEntries[] = {
    entry<7, 2, 1>(), entry<7, 2, 2>(), entry<7, 2, 4>(), entry<7, 2, 8>(),
    entry<8, 2, 1>(), entry<8, 2, 2>(), entry<8, 2, 4>(), entry<8, 2, 8>(),
    entry<8, 3, 1>(), entry<8, 3, 2>(), entry<8, 3, 4>(), entry<8, 3, 8>(),
};
KernelTable kernels_codes_b() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
