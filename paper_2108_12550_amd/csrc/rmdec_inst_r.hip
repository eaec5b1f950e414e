// Kernel instantiations: leaf roots RM(1, m) and RM(m-1, m) with lists of
// 16 and 32 paths for every length, and of 8 paths at length 1024 (one
// workgroup of 512 threads per frame, the paths' rows in LDS).
#include "rmdec_biglist.hpp"

namespace rmdec {
namespace {
const KernelEntry kEntries[] = {
    big::bigleaf_entry<3, 1, 16>(), big::bigleaf_entry<3, 1, 32>(), big::bigleaf_entry<3, 2, 16>(),
    big::bigleaf_entry<3, 2, 32>(), big::bigleaf_entry<4, 1, 16>(), big::bigleaf_entry<4, 1, 32>(),
    big::bigleaf_entry<4, 3, 16>(), big::bigleaf_entry<4, 3, 32>(), big::bigleaf_entry<5, 1, 16>(),
    big::bigleaf_entry<5, 1, 32>(), big::bigleaf_entry<5, 4, 16>(), big::bigleaf_entry<5, 4, 32>(),
    big::bigleaf_entry<6, 1, 16>(), big::bigleaf_entry<6, 1, 32>(), big::bigleaf_entry<6, 5, 16>(),
    big::bigleaf_entry<6, 5, 32>(), big::bigleaf_entry<7, 1, 16>(), big::bigleaf_entry<7, 1, 32>(),
    big::bigleaf_entry<7, 6, 16>(), big::bigleaf_entry<7, 6, 32>(), big::bigleaf_entry<8, 1, 16>(),
    big::bigleaf_entry<8, 1, 32>(), big::bigleaf_entry<8, 7, 16>(), big::bigleaf_entry<8, 7, 32>(),
    big::bigleaf_entry<9, 1, 16>(), big::bigleaf_entry<9, 1, 32>(), big::bigleaf_entry<9, 8, 16>(),
    big::bigleaf_entry<9, 8, 32>(), big::bigleaf_entry<10, 1, 16>(), big::bigleaf_entry<10, 1, 32>(),
    big::bigleaf_entry<10, 9, 16>(), big::bigleaf_entry<10, 9, 32>(), big::bigleaf_entry<10, 1, 8>(),
    big::bigleaf_entry<10, 9, 8>(),
};
} // namespace

KernelTable kernels_codes_r() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
