// Library-resident workspace of dock_local_search_batch_static: a
// file-scope device array (each GPU holds its own copy until the process
// ends) and the kernel that writes an item table into it. The table travels
// in kernel arguments, so filling the workspace needs no host staging buffer,
// no device allocation and no memset/memcpy node: the whole call is kernel
// launches on the caller's stream.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "dock.h"
#include "dock_launch.h"

namespace {

constexpr int64_t kScratchBytes =
    docklaunch::kWorkspaceHeader + (int64_t)DOCK_STATIC_MAX_ITEMS * (int64_t)sizeof(docklaunch::DevItem);

// Host code must not pass this name to a kernel: in host code it is a
// stand-in, not a device address. The per-device address comes from
// hipGetSymbolAddress below.
__device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Bytes of the table carried by one fill launch (kernel arguments).
constexpr int kChunkWords = 640;

struct FillChunk {
    uint32_t words[kChunkWords];
    uint32_t* dst;
    int32_t n_words;
};

__global__ __launch_bounds__(256) void table_fill_kernel(FillChunk c) {
    for (int i = threadIdx.x; i < c.n_words; i += blockDim.x) c.dst[i] = c.words[i];
}

}  // namespace

namespace docklaunch {

int64_t static_workspace_capacity() { return kScratchBytes; }

hipError_t static_workspace(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_table_fill(void* dst_dev, const void* src_host, int64_t bytes, hipStream_t stream) {
    if (bytes % 4 != 0 || (reinterpret_cast<uintptr_t>(dst_dev) & 3) != 0) return hipErrorInvalidValue;
    const uint8_t* src = static_cast<const uint8_t*>(src_host);
    uint32_t* dst = static_cast<uint32_t*>(dst_dev);
    const int64_t words = bytes / 4;
    for (int64_t w0 = 0; w0 < words; w0 += kChunkWords) {
        FillChunk c;
        c.n_words = (int32_t)(words - w0 < kChunkWords ? words - w0 : kChunkWords);
        c.dst = dst + w0;
        __builtin_memcpy(c.words, src + 4 * w0, 4 * (size_t)c.n_words);
        hipLaunchKernelGGL(table_fill_kernel, dim3(1), dim3(256), 0, stream, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace docklaunch
