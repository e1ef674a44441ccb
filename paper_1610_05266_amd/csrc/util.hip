// Small fill kernels (used instead of hipMemsetAsync so that every clear is an
// ordinary kernel node if a caller captures the stream in a graph).
#include <mutex>

#include "kernels.h"

namespace p2m {

namespace {

__global__ void __launch_bounds__(256) k_fill_i32(int32_t* __restrict__ p, int32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void __launch_bounds__(256) k_fill_u64(unsigned long long* __restrict__ p, unsigned long long v,
                                                  int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void __launch_bounds__(256) k_zero_bytes(uint8_t* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = 0;
}

__global__ void __launch_bounds__(256) k_zero_u32(uint32_t* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = 0u;
}

int grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return static_cast<int>(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

}  // namespace

int fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return P2M_OK;
    k_fill_i32<<<grid_for(n), 256, 0, st>>>(p, v, n);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

int fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t st) {
    if (n <= 0) return P2M_OK;
    k_fill_u64<<<grid_for(n), 256, 0, st>>>(p, v, n);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

int fill_bytes_zero(void* p, int64_t nbytes, hipStream_t st) {
    if (nbytes <= 0) return P2M_OK;
    if ((reinterpret_cast<uintptr_t>(p) & 3u) == 0 && (nbytes & 3) == 0) {
        k_zero_u32<<<grid_for(nbytes / 4), 256, 0, st>>>(static_cast<uint32_t*>(p), nbytes / 4);
    } else {
        k_zero_bytes<<<grid_for(nbytes), 256, 0, st>>>(static_cast<uint8_t*>(p), nbytes);
    }
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

// One non-blocking stream per device for work the library overlaps with the
// caller's stream (default priority); created on first use, kept for the
// life of the process.
int side_stream(int device, hipStream_t* out) {
    constexpr int MAXDEV = 64;
    static hipStream_t streams[MAXDEV] = {};
    static std::mutex mu;
    if (device < 0 || device >= MAXDEV) {
        set_error("device %d out of range", device);
        return P2M_EINVAL;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[device]) P2M_HIP(hipStreamCreateWithFlags(&streams[device], hipStreamNonBlocking));
    *out = streams[device];
    return P2M_OK;
}

}  // namespace p2m
