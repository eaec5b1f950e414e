// Kernel instantiations: lists of 16 and 32 paths for the other internal
// codes of length 64 to 256 (one workgroup of 512 threads per frame,
// LDS-resident list).
#include "rmdec_biglist.hpp"

namespace rmdec {
namespace {
const KernelEntry kEntries[] = {
    big::big_entry<6, 2, 32>(), big::big_entry<6, 3, 16>(), big::big_entry<6, 3, 32>(), big::big_entry<6, 4, 16>(),
    big::big_entry<6, 4, 32>(), big::big_entry<7, 2, 32>(), big::big_entry<7, 3, 32>(), big::big_entry<7, 4, 16>(),
    big::big_entry<7, 4, 32>(), big::big_entry<7, 5, 16>(), big::big_entry<7, 5, 32>(), big::big_entry<8, 5, 16>(),
    big::big_entry<8, 5, 32>(), big::big_entry<8, 6, 16>(), big::big_entry<8, 6, 32>(),
};
} // namespace

KernelTable kernels_codes_m() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
