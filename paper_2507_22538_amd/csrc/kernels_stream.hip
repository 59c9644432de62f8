// A plain streaming read of a device buffer: the achievable HBM read rate
// that the Bellman pass's bandwidth is set beside.  Every 16 bytes are loaded
// once, non-temporally (as the P arrays are), and folded into an XOR so that
// no load can be dropped; each workgroup stores its XOR in a slot of its own
// and one small kernel folds the slots into the caller's word.
#include <algorithm>
#include <mutex>

#include "device.hpp"
#include "internal.hpp"

using namespace ipi;
using ipi::dev::i4_t;

namespace {

constexpr int kUnroll = 8;  // 16-byte loads in flight per lane

// Each workgroup streams one contiguous region (its lanes on consecutive
// 16-byte pieces, kUnroll loads in flight per lane): 7.0 TB/s on MI355X
// against 6.2 for the same loads dealt round-robin over the whole grid.
__global__ __launch_bounds__(kBlock) void k_stream_read(const i4_t* __restrict__ p, int64_t n16,
                                                        unsigned int* __restrict__ part) {
    const int64_t b0 = (int64_t)blockIdx.x * n16 / gridDim.x, b1 = ((int64_t)blockIdx.x + 1) * n16 / gridDim.x;
    int64_t i = b0 + threadIdx.x;
    int x = 0;
    for (; i + (kUnroll - 1) * kBlock < b1; i += kUnroll * kBlock) {
        i4_t v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = dev::ldnt(p + i + u * kBlock);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) x ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < b1; i += kBlock) {
        const i4_t v = dev::ldnt(p + i);
        x ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    // the workgroup's XOR to its slot: one same-address atomic per wavefront
    // or workgroup serialises at the end of the launch (44-80 us of a
    // 616 us read measured)
    for (int off = 32; off >= 1; off >>= 1) x ^= __shfl_xor(x, off, dev::kWave);
    __shared__ int wx[kBlock / dev::kWave];
    if ((threadIdx.x & (dev::kWave - 1)) == 0) wx[threadIdx.x / dev::kWave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kBlock / dev::kWave; ++w) t ^= wx[w];
        part[blockIdx.x] = (unsigned int)t;
    }
}

__global__ __launch_bounds__(kBlock) void k_stream_fin(const unsigned int* __restrict__ part, int nb,
                                                       unsigned int* __restrict__ out) {
    unsigned int x = 0;
    for (int i = threadIdx.x; i < nb; i += kBlock) x ^= part[i];
    for (int off = 32; off >= 1; off >>= 1) x ^= __shfl_xor(x, off, dev::kWave);
    if ((threadIdx.x & (dev::kWave - 1)) == 0) atomicXor(out, x);
}

constexpr int kMaxStreamDevices = 64;
constexpr int kMaxStreamBlocks = 64 * 1024;  // workgroups of one launch (8 per CU)
std::mutex g_part_mu;
unsigned int* g_part[kMaxStreamDevices] = {};

// the per-workgroup slots on the current device, allocated at the first call
unsigned int* stream_parts() {
    int dev = 0;
    IPI_HIP(hipGetDevice(&dev));
    IPI_REQUIRE(dev >= 0 && dev < kMaxStreamDevices, IPI_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_part_mu);
    if (!g_part[dev]) IPI_HIP(hipMalloc(&g_part[dev], kMaxStreamBlocks * sizeof(unsigned int)));
    return g_part[dev];
}

}  // namespace

extern "C" ipi_status ipi_stream_read(const void* buf, int64_t bytes, uint32_t* xor_out, void* stream) {
    try {
        IPI_REQUIRE(buf && xor_out, IPI_E_INVALID_ARG, "NULL argument");
        IPI_REQUIRE(bytes > 0 && bytes % 16 == 0, IPI_E_INVALID_ARG, "bytes must be a positive multiple of 16");
        IPI_REQUIRE(reinterpret_cast<uintptr_t>(buf) % 16 == 0, IPI_E_INVALID_ARG, "buf must be 16-byte aligned");
        const int64_t n16 = bytes / 16;
        // up to 8 workgroups of 256 threads per CU (32 waves, full
        // occupancy), each lane keeping 128 bytes in flight
        const int64_t want = (n16 + (int64_t)kBlock * kUnroll - 1) / ((int64_t)kBlock * kUnroll);
        const int64_t cap = std::min<int64_t>(8 * (int64_t)device_cus(), kMaxStreamBlocks);
        const unsigned nb = (unsigned)(want < 1 ? 1 : (want > cap ? cap : want));
        unsigned int* part = stream_parts();
        hipLaunchKernelGGL(k_stream_read, dim3(nb), dim3(kBlock), 0, (hipStream_t)stream,
                           static_cast<const i4_t*>(buf), n16, part);
        IPI_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_stream_fin, dim3(1), dim3(kBlock), 0, (hipStream_t)stream, part, (int)nb,
                           reinterpret_cast<unsigned int*>(xor_out));
        IPI_HIP(hipGetLastError());
        return IPI_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.status;
    }
}
