// rmdec_kernels.hpp -- registry of the compiled (m, r, L) decoder kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "rmdec_device.hpp"

namespace rmdec {

using LaunchFn = hipError_t (*)(const KernelArgs &args, int blocks, hipStream_t stream);

struct KernelEntry {
    int m, r, L;
    int lds_bytes_per_wave;
    int maps_per_dec; // maps stored per decoder in p-FHT mode
    LaunchFn launch;
};

template <int M, int R, int L>
hipError_t launch_decode(const KernelArgs &args, int blocks, hipStream_t stream)
{
    const size_t lds = (size_t)args.waves * Shape<M, R, L>::BYTES;
    hipLaunchKernelGGL((rm_decode_kernel<M, R, L>), dim3(blocks), dim3(kWave * args.waves), lds, stream, args);
    return hipGetLastError();
}

template <int M, int R, int L>
constexpr KernelEntry entry()
{
    return KernelEntry{M, R, L, Shape<M, R, L>::BYTES, Shape<M, R, L>::MAPS_PER_DEC, &launch_decode<M, R, L>};
}

// Each translation unit rmdec_inst_*.hip defines one table.
struct KernelTable {
    const KernelEntry *entries;
    int count;
};

KernelTable kernels_codes_a();
KernelTable kernels_codes_b();
KernelTable kernels_codes_c();
KernelTable kernels_codes_d();

} // namespace rmdec
