// gb_lds_peak.hip -- the LDS read bandwidth of the device, measured: the peak
// against which the segment kernel's LDS traffic is reported.
//
// Every workgroup (1024 threads, 64 KiB of LDS) fills its LDS, then each wave
// reads it back in a loop, lane l of a wave reading the l-th consecutive
// element of a different 64-element run each time, so no two lanes of a read
// share a bank.  The words read are summed by three-input adds (few VALU
// instructions per byte read), and only a sum that cannot occur is written,
// so no read is optimised away.  Two widths: 16-byte
// reads (the LDS data path's width) and 4-byte reads (the width of the probe's
// word reads).
#include <hip/hip_runtime.h>

#include <string>

#include "goldbach.h"
#include "gb_internal.h"

// Written only by a workgroup whose sum takes a value that cannot occur: it
// keeps the reads live without any memory for the call to allocate (a symbol
// with external linkage, so the stores to it are not dropped).
__device__ uint32_t gb_lds_sink;

namespace {

constexpr uint32_t kLdsThreads = 1024;
constexpr uint32_t kLdsElems16 = 4096;   // 64 KiB of 16-byte elements
constexpr uint32_t kLdsElems4 = 16384;   // the same 64 KiB as 4-byte words

__global__ __launch_bounds__(kLdsThreads) void lds_read16_kernel(uint32_t iters)
{
    __shared__ uint4 buf[kLdsElems16];
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < kLdsElems16; i += kLdsThreads)
        buf[i] = make_uint4(i, 3 * i + 1, 5 * i + 2, 7 * i + 3);
    __syncthreads();
    const uint32_t lane = tid & 63;
    uint32_t run = tid >> 6;   // 64-element run of this wave's next read
    uint32_t acc = 0;
    for (uint32_t k = 0; k < iters; ++k) {
        // four reads 16 KiB apart from one address (immediate offsets)
        const uint4 *q = buf + (run & 15) * 64 + lane;
        const uint4 a = q[0];
        const uint4 b = q[1024];
        const uint4 c = q[2048];
        const uint4 d = q[3072];
        const uint32_t x = a.x + a.y + a.z + a.w + b.x + b.y + b.z + b.w;
        const uint32_t y = c.x + c.y + c.z + c.w + d.x + d.y + d.z + d.w;
        acc += x + y;
        run += 1;
    }
    if (acc == 0x9E3779B9u)
        gb_lds_sink = acc;
}

__global__ __launch_bounds__(kLdsThreads) void lds_read4_kernel(uint32_t iters)
{
    __shared__ uint32_t buf[kLdsElems4];
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < kLdsElems4; i += kLdsThreads)
        buf[i] = 2654435761u * i;
    __syncthreads();
    const uint32_t lane = tid & 63;
    uint32_t run = tid >> 6;
    uint32_t acc = 0;
    for (uint32_t k = 0; k < iters; ++k) {
        // eight reads 8 KiB apart from one address (immediate offsets)
        const uint32_t *q = buf + (run & 31) * 64 + lane;
        uint32_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            v[j] = q[2048 * j];
        acc += v[0] + v[1] + v[2] + v[3] + v[4] + v[5] + v[6] + v[7];
        run += 1;
    }
    if (acc == 0x9E3779B9u)
        gb_lds_sink = acc;
}

}  // namespace

// Bytes read from LDS per second by the whole device (all CUs, two 1024-thread
// workgroups each), for 16- or 4-byte reads.
gb_status gb_lds_peak(uint32_t width, double *bytes_per_s)
{
    if (!bytes_per_s || (width != 16 && width != 4)) {
        gb_internal_set_error("gb_lds_peak: width must be 16 or 4 and the output non-null");
        return GB_EINVAL;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        gb_internal_set_error("gb_lds_peak: no device");
        return GB_EHIP;
    }
    const uint32_t grid = 2u * (uint32_t)cus;
    const uint32_t iters = 20000;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    float ms = 0;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // the first run warms up
        e = hipEventRecord(e0, nullptr);
        if (e == hipSuccess) {
            if (width == 16)
                hipLaunchKernelGGL(lds_read16_kernel, dim3(grid), dim3(kLdsThreads), 0, nullptr, iters);
            else
                hipLaunchKernelGGL(lds_read4_kernel, dim3(grid), dim3(kLdsThreads), 0, nullptr, iters);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess)
            e = hipEventSynchronize(e1);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, e0, e1);
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        const std::string msg = std::string("gb_lds_peak: ") + hipGetErrorString(e);
        gb_internal_set_error(msg.c_str());
        return GB_EHIP;
    }
    // reads per thread: 4 x 16 bytes or 8 x 4 bytes per iteration
    const double per_thread = (double)iters * (width == 16 ? 64.0 : 32.0);
    *bytes_per_s = per_thread * kLdsThreads * grid / (ms * 1e-3);
    return GB_OK;
}
