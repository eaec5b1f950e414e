// Kernel instantiations: RM(4,9) and RM(4,8).
#include "rmdec_kernels.hpp"

namespace rmdec {
static const KernelEntry kEntries[] = {
    entry<9, 4, 1>(), entry<9, 4, 2>(), entry<9, 4, 4>(), entry<9, 4, 8>(),
    entry<8, 4, 1>(), entry<8, 4, 2>(), entry<8, 4, 4>(), entry<8, 4, 8>(),
};
KernelTable kernels_codes_f() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
