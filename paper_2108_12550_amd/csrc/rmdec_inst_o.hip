// Kernel instantiations: lists of 16 and 32 paths for the other internal
// codes of length 1024, orders 2 to 5 (one workgroup of 512 threads per frame,
// LDS-resident list).
#include "rmdec_biglist.hpp"

namespace rmdec {
namespace {
const KernelEntry kEntries[] = {
    big::big_entry<10, 2, 16>(), big::big_entry<10, 2, 32>(), big::big_entry<10, 3, 16>(),
    big::big_entry<10, 3, 32>(), big::big_entry<10, 4, 16>(), big::big_entry<10, 4, 32>(),
    big::big_entry<10, 5, 16>(), big::big_entry<10, 5, 32>(),
};
} // namespace

KernelTable kernels_codes_o() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
