// Fixed device area for the allocation-free ragged batch (bc_batch_run_static).
//
// The plan of a batch (header, segment table, tile offsets) normally lives in
// device memory the caller owns.  The allocation-free entry point keeps it in
// `scratch` instead: a file-scope device array of BC_STATIC_PLAN_BYTES that
// every GPU the library runs on holds once, until the process ends.  Host
// code never passes the array's name to a kernel or a copy (on the host it is
// only a stand-in for the device symbol): the device address comes from
// hipGetSymbolAddress, once per device with that device current, and is kept
// per device.
//
// The plan reaches the area through small upload kernels that carry up to
// 3 KiB of plan each as kernel arguments.  They are ordered on the caller's
// stream like any launch, read no host memory when they run (the bytes are in
// the launch itself) and allocate nothing, so a HIP graph that captures them
// replays the plan it was captured with.
#include <string.h>

#include <mutex>

#include "internal.h"

namespace bc {
namespace {

__device__ __align__(256) uint8_t scratch[BC_STATIC_PLAN_BYTES];

constexpr uint32_t kUploadWords = 384;   // 3 KiB of plan per upload launch

struct UploadArgs {
    uint64_t offset;                     // first 8-byte word of the area to write
    uint32_t nwords;                     // words carried, <= kUploadWords
    uint32_t reserved;
    uint64_t w[kUploadWords];
};

__global__ __launch_bounds__(256) void k_plan_upload(uint64_t* area, UploadArgs a) {
    for (uint32_t i = threadIdx.x; i < a.nwords; i += blockDim.x) area[a.offset + i] = a.w[i];
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_area[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// use per device and kept.
hipError_t area_of_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_area[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_area[dev] = p;
    }
    *out = g_area[dev];
    return hipSuccess;
}

}  // namespace

hipError_t static_plan_upload(const void* host_plan, uint64_t bytes, hipStream_t st, void** dev_plan) {
    if (bytes > BC_STATIC_PLAN_BYTES || bytes % 8) return hipErrorInvalidValue;
    void* area = nullptr;
    hipError_t e = area_of_current_device(&area);
    if (e != hipSuccess) return e;
    const uint8_t* src = static_cast<const uint8_t*>(host_plan);
    const uint64_t words = bytes / 8;
    UploadArgs a{};
    for (uint64_t off = 0; off < words; off += kUploadWords) {
        const uint64_t nw = words - off < kUploadWords ? words - off : kUploadWords;
        a.offset = off;
        a.nwords = (uint32_t)nw;
        memcpy(a.w, src + 8 * off, 8 * nw);      // the host plan need not be 8-byte aligned
        hipLaunchKernelGGL(k_plan_upload, dim3(1), dim3(256), 0, st, static_cast<uint64_t*>(area), a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    *dev_plan = area;
    return hipSuccess;
}

}  // namespace bc
