// Kernel instantiations: lists of 32 paths for RM(5,9), RM(6,9) and RM(7,9)
// (one workgroup of 512 threads per frame, LDS-resident list).
#include "rmdec_biglist.hpp"

namespace rmdec {
namespace {
const KernelEntry kEntries[] = {
    big::big_entry<9, 5, 32>(), big::big_entry<9, 6, 32>(), big::big_entry<9, 7, 32>(),
};
} // namespace

KernelTable kernels_codes_t() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
