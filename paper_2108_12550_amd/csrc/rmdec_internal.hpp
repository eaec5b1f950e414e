// rmdec_internal.hpp -- library-internal declarations shared by the host units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "rmdec.h"
#include "rmdec_kernels.hpp"

struct rm_decoder {
    rm_config cfg;
    int N, K, nperm, maps_per_dec;
    const rmdec::KernelEntry *kern;
    bool packed;     // P = 1 with a frame-packed kernel: D frames per wave
    int slice_bytes; // LDS bytes per wave of the kernel that runs
    uint32_t *d_maps;   // the map tables (fresh mode: one chunk of frames' tables)
    size_t table_bytes;
    int64_t fresh_chunk; // fresh mode: frames whose tables the buffer holds
    // fresh mode: recorded after each chunk's decode on the stream it ran on;
    // the next map draw waits on it, so tables still being read by a decode
    // queued on another stream are never overwritten
    hipEvent_t fresh_done;
    bool fresh_pending;
    hipStream_t stream;
    int device;
};

namespace rmdec {
extern thread_local std::string g_err;
int fail(int code, const std::string &msg);
int check_device_ptr(const void *p, const char *name);
int check_alignment(int N, const float *llr, const uint8_t *out_bits, const float *out_metric);
KernelArgs batch_args(const rm_decoder *d, const float *llr, int64_t n_frames, uint8_t *out_bits, float *out_metric);
// launch the decoder's batched kernel over n_frames frames (args from batch_args)
hipError_t launch_decoder(const rm_decoder *d, const KernelArgs &a, int64_t n_frames);
// fresh mode: draw each chunk's tables on the device, then decode the chunk
int fresh_decode(rm_decoder *d, const float *llr, int64_t n_frames, uint8_t *out_bits, float *out_metric);
} // namespace rmdec
