// Kernel instantiations: lists of 16, 32 and 64 paths (one workgroup of 512
// threads per frame, LDS-resident list).
#include "rmdec_biglist.hpp"

namespace rmdec {
namespace {
const KernelEntry kEntries[] = {
    big::big_entry<8, 2, 16>(), big::big_entry<8, 2, 32>(), big::big_entry<8, 2, 64>(),
    big::big_entry<8, 3, 16>(), big::big_entry<8, 3, 32>(), big::big_entry<8, 3, 64>(),
    big::big_entry<8, 4, 16>(), big::big_entry<8, 4, 32>(), big::big_entry<8, 4, 64>(),
    big::big_entry<9, 2, 16>(), big::big_entry<9, 2, 32>(),
    big::big_entry<9, 3, 16>(), big::big_entry<9, 3, 32>(),
    big::big_entry<9, 4, 16>(), big::big_entry<9, 4, 32>(),
    big::big_entry<7, 2, 16>(), big::big_entry<7, 3, 16>(), big::big_entry<6, 2, 16>(),
};
} // namespace

KernelTable kernels_codes_g() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
