// rmdec_serve.hpp -- the serving kernels, one per list size, and their
// registry (used by the request server in rmdec_serve.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "rmdec_kernels.hpp"

namespace rmdec {

// Codes every serving kernel decodes: RM(2,7), RM(2,8), RM(2,9), RM(2,10)
// and RM(3,8), as (m, r).
constexpr int kServeCodes[][2] = {{7, 2}, {8, 2}, {9, 2}, {10, 2}, {8, 3}};
constexpr int kNumServeCodes = 5;

struct ServeGroup {
    int L;                  // list size of every code in the kernel
    int lds_bytes_per_wave; // LDS slice of one wave
    const void *kernel;     // for occupancy queries (one wave per queue entry)
    const void *split_kernel; // the same with a request's decoders split over a workgroup
    hipError_t (*launch)(const ServeArgs &a, int blocks, int waves, hipStream_t stream);
    hipError_t (*launch_split)(const ServeArgs &a, int blocks, int waves, hipStream_t stream);
};

template <int WPE, int L>
struct ServeKernel {
    template <int M, int R>
    using C = Code<M, R, L, decoders_per_wave(M, L)>;
    using Slice = MaxBytes<C<7, 2>, C<8, 2>, C<9, 2>, C<10, 2>, C<8, 3>>;
    static const void *kernel() { return (const void *)&rm_serve_kernel<WPE, C<7, 2>, C<8, 2>, C<9, 2>, C<10, 2>, C<8, 3>>; }
    static const void *split_kernel()
    {
        return (const void *)&rm_serve_split_kernel<WPE, C<7, 2>, C<8, 2>, C<9, 2>, C<10, 2>, C<8, 3>>;
    }
    static hipError_t launch(const ServeArgs &a, int blocks, int waves, hipStream_t stream)
    {
        hipLaunchKernelGGL((rm_serve_kernel<WPE, C<7, 2>, C<8, 2>, C<9, 2>, C<10, 2>, C<8, 3>>), dim3(blocks),
                           dim3(kWave * waves), (size_t)waves * Slice::value, stream, a);
        return hipGetLastError();
    }
    static hipError_t launch_split(const ServeArgs &a, int blocks, int waves, hipStream_t stream)
    {
        hipLaunchKernelGGL((rm_serve_split_kernel<WPE, C<7, 2>, C<8, 2>, C<9, 2>, C<10, 2>, C<8, 3>>), dim3(blocks),
                           dim3(kWave * waves), (size_t)waves * Slice::value + kSplitXBytes, stream, a);
        return hipGetLastError();
    }
    static ServeGroup group() { return ServeGroup{L, Slice::value, kernel(), split_kernel(), &launch, &launch_split}; }
};

// index of (m, r) in kServeCodes, or -1
inline int serve_code_index(int m, int r)
{
    for (int i = 0; i < kNumServeCodes; i++)
        if (kServeCodes[i][0] == m && kServeCodes[i][1] == r)
            return i;
    return -1;
}

// one translation unit per list size: rmdec_serve_l{1,4,8}.hip
ServeGroup serve_group_l1();
ServeGroup serve_group_l4();
ServeGroup serve_group_l8();

} // namespace rmdec
