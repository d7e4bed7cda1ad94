// sat_upload.hip -- host-to-device copy of an image by a kernel that reads pinned host memory.
//
// Serving uploads each new image from a pinned host buffer while other requests' builds and
// gathers run on other streams.  Enqueued as a DMA copy (hipMemcpyAsync), such an upload has
// held the calling thread for several milliseconds whenever other copies were outstanding; a
// kernel launch only appends a packet to the stream's queue and returns.  The kernel reads the
// mapped host pages over the bus (16-byte loads, several in flight per lane to cover the bus
// latency) and writes device memory with 16-byte stores.  It needs no LDS and few registers, so
// it shares the CUs it runs on with the other streams' kernels.
#include "sat_internal.h"

namespace satk {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kUpThreads = 256;
constexpr int kUpUnroll = 4;                 // 16-byte loads in flight per lane
constexpr int kUpMaxBlocks = 128;

__global__ __launch_bounds__(kUpThreads) void upload_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                            int64_t n16, const uint8_t *__restrict__ src_tail,
                                                            uint8_t *__restrict__ dst_tail, int tail) {
    const int64_t step = (int64_t)gridDim.x * kUpThreads * kUpUnroll;
    for (int64_t base = (int64_t)blockIdx.x * kUpThreads * kUpUnroll + threadIdx.x; base < n16; base += step) {
        u32x4 v[kUpUnroll];
#pragma unroll
        for (int k = 0; k < kUpUnroll; ++k) {
            const int64_t i = base + (int64_t)k * kUpThreads;
            if (i < n16) v[k] = src[i];
        }
#pragma unroll
        for (int k = 0; k < kUpUnroll; ++k) {
            const int64_t i = base + (int64_t)k * kUpThreads;
            if (i < n16) __builtin_nontemporal_store(v[k], dst + i);
        }
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < tail) dst_tail[threadIdx.x] = src_tail[threadIdx.x];
}

}  // namespace

hipError_t launch_upload(const void *src_dev, void *dst, size_t nbytes, hipStream_t stream) {
    const int64_t n16 = (int64_t)(nbytes / 16);
    const int tail = (int)(nbytes % 16);
    int64_t blocks = (n16 + kUpThreads * kUpUnroll - 1) / (kUpThreads * kUpUnroll);
    if (blocks < 1) blocks = 1;
    if (blocks > kUpMaxBlocks) blocks = kUpMaxBlocks;
    const uint8_t *s8 = static_cast<const uint8_t *>(src_dev);
    uint8_t *d8 = static_cast<uint8_t *>(dst);
    hipLaunchKernelGGL(upload_kernel, dim3((unsigned)blocks), dim3(kUpThreads), 0, stream,
                       reinterpret_cast<const u32x4 *>(s8), reinterpret_cast<u32x4 *>(d8), n16, s8 + n16 * 16,
                       d8 + n16 * 16, tail);
    return hipGetLastError();
}

}  // namespace satk
