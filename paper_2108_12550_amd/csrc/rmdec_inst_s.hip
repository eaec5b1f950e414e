// Kernel instantiations: lists of 16 and 32 paths for the internal codes of
// lengths 16 and 32 (one workgroup of 512 threads per frame, LDS-resident
// list).
#include "rmdec_biglist.hpp"

namespace rmdec {
namespace {
const KernelEntry kEntries[] = {
    big::big_entry<4, 2, 16>(), big::big_entry<4, 2, 32>(), big::big_entry<5, 2, 16>(), big::big_entry<5, 2, 32>(),
    big::big_entry<5, 3, 16>(), big::big_entry<5, 3, 32>(),
};
} // namespace

KernelTable kernels_codes_s() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
