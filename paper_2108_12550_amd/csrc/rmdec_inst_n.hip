// Kernel instantiations: lists of 16 and 32 paths for the other internal
// codes of length 512 (one workgroup of 512 threads per frame,
// LDS-resident list).
#include "rmdec_biglist.hpp"

namespace rmdec {
namespace {
const KernelEntry kEntries[] = {
    big::big_entry<9, 5, 16>(), big::big_entry<9, 6, 16>(), big::big_entry<9, 7, 16>(),
};
} // namespace

KernelTable kernels_codes_n() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
