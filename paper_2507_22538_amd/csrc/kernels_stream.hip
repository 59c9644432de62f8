// A plain streaming read of a device buffer: the achievable HBM read rate
// that the Bellman pass's bandwidth is set beside.  Every 16 bytes are loaded
// once, non-temporally (as the P arrays are), and folded into an XOR so that
// no load can be dropped; each wavefront adds its XOR to one 32-bit word.
#include "device.hpp"
#include "internal.hpp"

using namespace ipi;
using ipi::dev::i4_t;

namespace {

constexpr int kUnroll = 8;  // 16-byte loads in flight per lane

__global__ __launch_bounds__(kBlock) void k_stream_read(const i4_t* __restrict__ p, int64_t n16,
                                                        unsigned int* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int x = 0;
    for (; i + (kUnroll - 1) * stride < n16; i += kUnroll * stride) {
        i4_t v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = dev::ldnt(p + i + u * stride);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) x ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < n16; i += stride) {
        const i4_t v = dev::ldnt(p + i);
        x ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    for (int off = 32; off >= 1; off >>= 1) x ^= __shfl_xor(x, off, dev::kWave);
    if ((threadIdx.x & (dev::kWave - 1)) == 0) atomicXor(out, (unsigned int)x);
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
        const int64_t cap = 8 * (int64_t)device_cus();
        const unsigned nb = (unsigned)(want < 1 ? 1 : (want > cap ? cap : want));
        hipLaunchKernelGGL(k_stream_read, dim3(nb), dim3(kBlock), 0, (hipStream_t)stream,
                           static_cast<const i4_t*>(buf), n16, reinterpret_cast<unsigned int*>(xor_out));
        IPI_HIP(hipGetLastError());
        return IPI_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.status;
    }
}
