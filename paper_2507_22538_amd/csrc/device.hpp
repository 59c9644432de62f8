// Device-side helpers for gfx950 (wave64): vector loads, lane-group and
// block reductions, XCD-aware block remapping, atomic maxima.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ipi {
namespace dev {

typedef double d2_t __attribute__((ext_vector_type(2)));
typedef float f2_t __attribute__((ext_vector_type(2)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef int i2_t __attribute__((ext_vector_type(2)));
typedef int i4_t __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
constexpr int kNumXcd = 8;

// Streaming (non-temporal) loads for the P arrays: each byte is used once per pass.
template <typename T>
__device__ __forceinline__ T ldnt(const T* p) {
    return __builtin_nontemporal_load(p);
}

// P_pi loads: streamed, or with KEEP through the caches, for a P_pi small
// enough that the last-level cache still holds it at the next sweep.
template <bool KEEP, typename T>
__device__ __forceinline__ T ldp(const T* p) {
    if constexpr (KEEP) return *p;
    else return __builtin_nontemporal_load(p);
}

// VEC consecutive values of P (value type VT) and their columns, loaded as one
// vector per array, streamed or (KEEP) cached.  Requires the element index to
// be a multiple of VEC.
template <typename VT, int VEC, bool KEEP = false>
struct VecLoad;

template <bool KEEP>
struct VecLoad<double, 1, KEEP> {
    __device__ __forceinline__ static void load(const double* v, const int* c, int64_t j, double* vv, int* cc) {
        vv[0] = ldp<KEEP>(v + j);
        cc[0] = ldp<KEEP>(c + j);
    }
};
template <bool KEEP>
struct VecLoad<double, 2, KEEP> {
    __device__ __forceinline__ static void load(const double* v, const int* c, int64_t j, double* vv, int* cc) {
        d2_t a = ldp<KEEP>(reinterpret_cast<const d2_t*>(v + j));
        i2_t b = ldp<KEEP>(reinterpret_cast<const i2_t*>(c + j));
        vv[0] = a.x; vv[1] = a.y;
        cc[0] = b.x; cc[1] = b.y;
    }
};
template <bool KEEP>
struct VecLoad<float, 1, KEEP> {
    __device__ __forceinline__ static void load(const float* v, const int* c, int64_t j, double* vv, int* cc) {
        vv[0] = (double)ldp<KEEP>(v + j);
        cc[0] = ldp<KEEP>(c + j);
    }
};
template <bool KEEP>
struct VecLoad<float, 2, KEEP> {
    __device__ __forceinline__ static void load(const float* v, const int* c, int64_t j, double* vv, int* cc) {
        f2_t a = ldp<KEEP>(reinterpret_cast<const f2_t*>(v + j));
        i2_t b = ldp<KEEP>(reinterpret_cast<const i2_t*>(c + j));
        vv[0] = (double)a.x; vv[1] = (double)a.y;
        cc[0] = b.x; cc[1] = b.y;
    }
};
template <bool KEEP>
struct VecLoad<float, 4, KEEP> {
    __device__ __forceinline__ static void load(const float* v, const int* c, int64_t j, double* vv, int* cc) {
        f4_t a = ldp<KEEP>(reinterpret_cast<const f4_t*>(v + j));
        i4_t b = ldp<KEEP>(reinterpret_cast<const i4_t*>(c + j));
        vv[0] = (double)a.x; vv[1] = (double)a.y; vv[2] = (double)a.z; vv[3] = (double)a.w;
        cc[0] = b.x; cc[1] = b.y; cc[2] = b.z; cc[3] = b.w;
    }
};

// E consecutive values and columns as E/W independent 16-byte loads
// (W = 2 doubles or 4 floats per load), streamed or (KEEP) cached.  Requires
// the index to be a multiple of W.
template <typename VT, int E, bool KEEP = false>
struct FlatLoad {
    static constexpr int W = sizeof(VT) == 8 ? 2 : 4;
    static_assert(E % W == 0, "chunk must be a multiple of the load width");
    __device__ __forceinline__ static void load(const VT* v, const int* c, int64_t j, double* vv, int* cc) {
#pragma unroll
        for (int q = 0; q < E / W; ++q) VecLoad<VT, W, KEEP>::load(v, c, j + q * W, vv + q * W, cc + q * W);
    }
};

// rows of one entry: one value and one column per chunk
template <bool KEEP>
struct FlatLoad<double, 1, KEEP> {
    __device__ __forceinline__ static void load(const double* v, const int* c, int64_t j, double* vv, int* cc) {
        vv[0] = ldp<KEEP>(v + j);
        cc[0] = ldp<KEEP>(c + j);
    }
};
template <bool KEEP>
struct FlatLoad<float, 1, KEEP> {
    __device__ __forceinline__ static void load(const float* v, const int* c, int64_t j, double* vv, int* cc) {
        vv[0] = (double)ldp<KEEP>(v + j);
        cc[0] = ldp<KEEP>(c + j);
    }
};

// doubles: E/2 loads of 2 values and E/4 loads of 4 columns (16 bytes each)
template <int E, bool KEEP>
struct FlatLoad<double, E, KEEP> {
    static_assert(E % 2 == 0, "chunk must hold whole 16-byte loads");
    __device__ __forceinline__ static void load(const double* v, const int* c, int64_t j, double* vv, int* cc) {
#pragma unroll
        for (int q = 0; q < E / 2; ++q) {
            d2_t a = ldp<KEEP>(reinterpret_cast<const d2_t*>(v + j + 2 * q));
            vv[2 * q] = a.x;
            vv[2 * q + 1] = a.y;
        }
        if constexpr (E % 4 == 0) {
#pragma unroll
            for (int q = 0; q < E / 4; ++q) {
                i4_t b = ldp<KEEP>(reinterpret_cast<const i4_t*>(c + j + 4 * q));
                cc[4 * q] = b.x;
                cc[4 * q + 1] = b.y;
                cc[4 * q + 2] = b.z;
                cc[4 * q + 3] = b.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < E / 2; ++q) {
                i2_t b = ldp<KEEP>(reinterpret_cast<const i2_t*>(c + j + 2 * q));
                cc[2 * q] = b.x;
                cc[2 * q + 1] = b.y;
            }
        }
    }
};

// E consecutive values only (band form: the columns are computed), as E/W
// 16-byte loads, streamed or (KEEP) cached.
template <typename VT, int E, bool KEEP = false>
struct FlatVals {
    __device__ __forceinline__ static void load(const VT* v, int64_t j, double* vv) {
        if constexpr (sizeof(VT) == 8) {
#pragma unroll
            for (int q = 0; q < E / 2; ++q) {
                d2_t a = ldp<KEEP>(reinterpret_cast<const d2_t*>(v + j + 2 * q));
                vv[2 * q] = a.x;
                vv[2 * q + 1] = a.y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < E / 4; ++q) {
                f4_t a = ldp<KEEP>(reinterpret_cast<const f4_t*>(v + j + 4 * q));
                vv[4 * q] = (double)a.x;
                vv[4 * q + 1] = (double)a.y;
                vv[4 * q + 2] = (double)a.z;
                vv[4 * q + 3] = (double)a.w;
            }
        }
    }
};

// Sum over an aligned group of L lanes (L a power of two <= 64); every lane
// of the group ends with the group total.  Fixed butterfly order.
template <int L>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
    for (int off = L / 2; off >= 1; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

__device__ __forceinline__ double wave_sum(double x) { return group_sum<kWave>(x); }

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fmax(x, __shfl_xor(x, off, kWave));
    return x;
}

// Block-wide sum of one value per thread (blockDim.x == 256): fixed order.
__device__ __forceinline__ double block_sum(double x, double* lds4) {
    x = wave_sum(x);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) lds4[w] = x;
    __syncthreads();
    double t = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
    __syncthreads();
    return t;
}

// Block index remapping so that each XCD (blocks are dispatched round-robin
// over the 8 XCDs) works on one contiguous range of logical blocks.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb) {
    const int64_t q = nb / kNumXcd, r = nb % kNumXcd;
    const int64_t x = bid % kNumXcd, i = bid / kNumXcd;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// max of non-negative doubles through their bit patterns (order-preserving;
// NaN with cleared sign compares above +inf, so it propagates).
__device__ __forceinline__ void atomic_max_nonneg(uint64_t* p, double v) {
    uint64_t bits = (uint64_t)__double_as_longlong(fabs(v));
    __hip_atomic_fetch_max(p, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace dev
}  // namespace ipi
