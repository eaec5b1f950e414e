// Kernel instantiations: RM(2,9) and RM(2,10), the length-512/1024 codes.
#include "rmdec_kernels.hpp"

namespace rmdec {
static const KernelEntry kEntries[] = {
    entry<9, 2, 1>(), entry<9, 2, 2>(), entry<9, 2, 4>(), entry<9, 2, 8>(),
    entry<10, 2, 1>(), entry<10, 2, 4>(), entry<10, 2, 8>(),
};
KernelTable kernels_codes_a() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
