// rmdec_kernels.hpp -- registry of the compiled (m, r, L) decoder kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "rmdec_device.hpp"

namespace rmdec {

using LaunchFn = hipError_t (*)(const KernelArgs &args, int blocks, hipStream_t stream);

struct KernelEntry {
    int m, r, L;
    int D; // decoders per wavefront
    int lds_bytes_per_wave;
    int maps_per_dec; // maps stored per decoder in p-FHT mode
    LaunchFn launch;
    // kernels that run one workgroup per frame (lists of 16 or more paths):
    // the workgroup's LDS bytes; 0 for the one-wave-per-frame kernels
    int block_lds_bytes = 0;
    // frame-packed kernel for P = 1 (D frames per wave, one per decoder
    // slot) and its LDS bytes per wave with maps per slot (fresh tables per
    // frame) and with one shared copy; null where D = 1
    LaunchFn launch_packed = nullptr;
    int lds_bytes_packed = 0;
    int lds_bytes_packed_shared = 0;
};

template <int M, int R, int L, int D, int WPE>
hipError_t launch_decode(const KernelArgs &args, int blocks, hipStream_t stream)
{
    const size_t lds = (size_t)args.waves * Shape<M, R, L, D>::BYTES;
    hipLaunchKernelGGL((rm_decode_kernel<M, R, L, D, WPE>), dim3(blocks), dim3(kWave * args.waves), lds, stream, args);
    return hipGetLastError();
}

template <int M, int R, int L, int D, int WPE>
hipError_t launch_packed(const KernelArgs &args, int blocks, hipStream_t stream)
{
    using Pk = Packed<M, R, L, D>;
    const size_t lds = (size_t)args.waves * (args.frame_stride == 0 ? Pk::BYTES_SHARED : Pk::BYTES);
    hipLaunchKernelGGL((rm_decode_packed_kernel<M, R, L, D, WPE>), dim3(blocks), dim3(kWave * args.waves), lds, stream,
                       args);
    return hipGetLastError();
}

// Decoders per wavefront: D*L = 8 paths share the 64 lanes (8 lanes per
// path); for N <= 256 at L = 4, 16 paths (4 lanes per path: per-node fixed
// costs are shared by twice the decoders); for N = 1024 only 4 paths (16
// lanes per path), which keeps a half-length node vector at 32 registers.
// WPE: wavefronts per SIMD the register allocation must allow (4: at most
// 128 VGPRs; 3: 168; 2: 256).  These choices keep every kernel free of (or
// nearly free of) register spills; RM(2,9) and RM(2,10) at L = 4 and RM(3,8)
// at L = 8 fit the cap of four waves per SIMD without spilling.
constexpr int decoders_per_wave(int M, int L)
{
    return L >= 8 ? 1 : (M >= 10 ? 4 : (M <= 8 && L == 4) ? 16 : 8) / L;
}
constexpr int waves_per_eu(int M, int R, int L)
{
    return M >= 10 && L >= 8 ? 2
           : ((M == 9 && R == 2 && L == 4) || (M == 10 && R == 2 && L == 4) || (M == 8 && R == 3 && L == 8)) ? 4
                                                                                                            : 3;
}

template <int M, int R, int L, int D = decoders_per_wave(M, L), int WPE = waves_per_eu(M, R, L)>
constexpr KernelEntry entry()
{
    if constexpr (D > 1)
        return KernelEntry{M, R, L, D, Shape<M, R, L, D>::BYTES, Shape<M, R, L, D>::MAPS_PER_DEC,
                           &launch_decode<M, R, L, D, WPE>, 0, &launch_packed<M, R, L, D, WPE>,
                           Packed<M, R, L, D>::BYTES, Packed<M, R, L, D>::BYTES_SHARED};
    else
        return KernelEntry{M, R, L, D, Shape<M, R, L, D>::BYTES, Shape<M, R, L, D>::MAPS_PER_DEC,
                           &launch_decode<M, R, L, D, WPE>};
}

// Each translation unit rmdec_inst_*.hip defines one table (kernels_codes_a
// .. kernels_codes_t, which rmdec_host.hip searches).
struct KernelTable {
    const KernelEntry *entries;
    int count;
};


} // namespace rmdec
