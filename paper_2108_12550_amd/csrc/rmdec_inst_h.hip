// Kernel instantiations: lists of 64 paths for RM(r, 9) (one workgroup of
// 512 threads per frame; the list takes 157 KB of LDS, within the 160 KB a
// workgroup may hold).
#include "rmdec_biglist.hpp"

namespace rmdec {
namespace {
const KernelEntry kEntries[] = {
    big::big_entry<9, 2, 64>(), big::big_entry<9, 3, 64>(), big::big_entry<9, 4, 64>(),
};
} // namespace

KernelTable kernels_codes_h() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
