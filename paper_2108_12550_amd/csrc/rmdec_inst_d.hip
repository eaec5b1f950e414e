// Kernel instantiations: codes whose root is a leaf, RM(1,m) and RM(m-1,m).
#include "rmdec_kernels.hpp"

namespace rmdec {
static const KernelEntry kEntries[] = {
    entry<3, 1, 1>(), entry<3, 1, 4>(), entry<4, 1, 1>(), entry<4, 1, 4>(),
    entry<5, 1, 1>(), entry<5, 1, 4>(), entry<6, 1, 1>(), entry<6, 1, 4>(),
    entry<3, 2, 1>(), entry<3, 2, 4>(), entry<4, 3, 1>(), entry<4, 3, 4>(),
    entry<5, 4, 1>(), entry<5, 4, 4>(),
};
KernelTable kernels_codes_d() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
