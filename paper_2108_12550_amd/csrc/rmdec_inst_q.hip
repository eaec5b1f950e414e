// Kernel instantiations: lists of 16 and 32 paths for the other internal
// codes of length 1024, orders 6 to 8 (one workgroup of 512 threads per frame,
// LDS-resident list).
#include "rmdec_biglist.hpp"

namespace rmdec {
namespace {
const KernelEntry kEntries[] = {
    big::big_entry<10, 6, 16>(), big::big_entry<10, 6, 32>(), big::big_entry<10, 7, 16>(),
    big::big_entry<10, 7, 32>(), big::big_entry<10, 8, 16>(), big::big_entry<10, 8, 32>(),
};
} // namespace

KernelTable kernels_codes_q() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
