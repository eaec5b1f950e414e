// Kernel instantiations: lists of 16, 32 and 64 paths (one workgroup of 512
// threads per frame, LDS-resident list).  The list's LLR stack takes
// 4*L*N bytes of LDS, so L*N is at most 16384 here.
#include "rmdec_biglist.hpp"
#include "rmdec_kernels.hpp"

namespace rmdec {
namespace {

template <int M, int R, int L>
hipError_t launch_big(const KernelArgs &args, int blocks, hipStream_t stream)
{
    constexpr size_t lds = big::Lay<M, L>::BYTES;
    static const hipError_t attr = hipFuncSetAttribute((const void *)&big::rm_biglist_kernel<M, R, L>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL((big::rm_biglist_kernel<M, R, L>), dim3(blocks), dim3(big::kThreads), lds, stream, args);
    return hipGetLastError();
}

template <int M, int R, int L>
constexpr KernelEntry big_entry()
{
    return KernelEntry{M, R, L, 1, 0, 2 * L + 4 * L * perm_spine(M, R), &launch_big<M, R, L>,
                       big::Lay<M, L>::BYTES};
}

const KernelEntry kEntries[] = {
    big_entry<8, 2, 16>(), big_entry<8, 2, 32>(), big_entry<8, 2, 64>(),
    big_entry<8, 3, 16>(), big_entry<8, 3, 32>(), big_entry<8, 3, 64>(),
    big_entry<8, 4, 16>(), big_entry<8, 4, 32>(), big_entry<8, 4, 64>(),
    big_entry<9, 2, 16>(), big_entry<9, 2, 32>(),
    big_entry<9, 3, 16>(), big_entry<9, 3, 32>(),
    big_entry<9, 4, 16>(), big_entry<9, 4, 32>(),
    big_entry<7, 2, 16>(), big_entry<7, 3, 16>(), big_entry<6, 2, 16>(),
};
} // namespace

KernelTable kernels_codes_g() { return {kEntries, (int)(sizeof kEntries / sizeof kEntries[0])}; }
} // namespace rmdec
