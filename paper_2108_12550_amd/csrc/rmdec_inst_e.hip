// Kernel instantiations: RM(3,9), the higher-order length-512 code.
#include "rmdec_kernels.hpp"

namespace rmdec {
static const KernelEntry kEntries[] = {
    entry<9, 3, 1>(), entry<9, 3, 2>(), entry<9, 3, 4>(), entry<9, 3, 8>(),
};
KernelTable kernels_codes_e() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
