// Fused Bellman pass (Sec. II Bellman optimality operator; greedy extraction
// "approach 2" of Sec. III-B.3 without materialising the S*A vector P V).
//
// A tile is a run of consecutive states [s0, s1).  Because P is row-stacked
// (row = s*A + a), the tile's rows [s0*A, s1*A) and their nonzeros are
// contiguous in memory, so a tile streams one contiguous range of col/val.
// The grid is capped at a few workgroups per CU; the tiles are dealt
// round-robin over the workgroups (or waves), so the tiles in flight are
// neighbours in memory and consecutive ones run on one XCD, and each
// workgroup folds its maxima into the device-wide ones once at the end, so
// the number of same-address atomics does not grow with S.
//
//   phase 0  row_ptr[r0..r1] and g[r0..r1) of the tile -> LDS (coalesced)
//   phase 1  lane groups of L lanes take rows round-robin; each lane loads
//            VEC consecutive (val, col) pairs per step (non-temporal vector
//            loads), gathers V[col], accumulates in FP64; the group sums its
//            lanes with a fixed butterfly; Q(s,a) = g + gamma * sum -> LDS
//   phase 2  one thread per state: min / lowest-index argmin over its A
//            values of Q; writes TV, pi, resid = TV - V; block max of |resid|
//            folded into a device-wide max through the bit pattern.
#include <algorithm>
#include <type_traits>

#include "device.hpp"
#include "internal.hpp"

namespace ipi {

namespace {

template <typename VT, typename PT>
struct BellmanParams {
    const PT* row_ptr;
    const int* col;
    const VT* val;
    const double* g;
    const double* V;
    double gamma;
    int A;
    int spt;  // states per tile
    int64_t S;
    int64_t ntiles;
    double* TV;
    int32_t* pi;
    double* resid;
    uint64_t* rho_bits;
    uint64_t* vmax_bits;
    const int32_t* band;  // band form: first column of each row (flat kernel only)
    // stencil form (flat workgroup tiles only): per row its first column and
    // pattern, and the patterns' column offsets (sten_np x k)
    const uint32_t* sten = nullptr;
    const int32_t* sten_off = nullptr;
    int sten_np = 0;
    bool sten_pairs = false;  // columns in adjacent pairs: one 16-byte load of V per pair
    const float* lo = nullptr;  // split values (VT = F32Split): lo, beside hi in val
};

// Values held as float32 hi and lo (IPI_VAL_SPLIT): VT = F32Split, val points
// at hi and the params' lo at lo; a value is hi + lo rounded once to FP64.
// Chunk widths and loads are those of float values.
struct F32Split {
    float hi;
};
template <typename VT>
constexpr bool kSplit = std::is_same<VT, F32Split>::value;
template <typename VT>
using HiT = typename std::conditional<kSplit<VT>, float, VT>::type;
template <typename VT>
__device__ __forceinline__ const HiT<VT>* hi_vals(const VT* v) {
    return reinterpret_cast<const HiT<VT>*>(v);
}

// vv[e] += lo[j + e] for the E values of a chunk at j (j a multiple of the
// load width, as for the hi values)
template <int E>
__device__ __forceinline__ void add_lo(const float* lo, int64_t j, double* vv) {
    if constexpr (E % 4 == 0) {
#pragma unroll
        for (int q = 0; q < E / 4; ++q) {
            const dev::f4_t a = dev::ldp<false>(reinterpret_cast<const dev::f4_t*>(lo + j + 4 * q));
            vv[4 * q] += (double)a.x;
            vv[4 * q + 1] += (double)a.y;
            vv[4 * q + 2] += (double)a.z;
            vv[4 * q + 3] += (double)a.w;
        }
    } else if constexpr (E % 2 == 0) {
#pragma unroll
        for (int q = 0; q < E / 2; ++q) {
            const dev::f2_t a = dev::ldp<false>(reinterpret_cast<const dev::f2_t*>(lo + j + 2 * q));
            vv[2 * q] += (double)a.x;
            vv[2 * q + 1] += (double)a.y;
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) vv[e] += (double)dev::ldp<false>(lo + j + e);
    }
}

// index forms of the flat kernels: columns loaded, band form, stencil form
enum : int { kFormCols = 0, kFormBand = 1, kFormSten = 2 };

__device__ __forceinline__ double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

// LDS written by one lane of a wavefront, visible to the wave's other lanes
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// phase 2: one thread per state, min / lowest-index argmin over the A values
// of Q held in LDS; TV, pi, resid = TV - V; running max |resid|, max |V|
template <typename VT, typename PT>
__device__ __forceinline__ void bellman_finish(const BellmanParams<VT, PT>& p, const double* q, int64_t s0, int ns,
                                               double& mx, double& vx) {
    const int A = p.A;
    const double* __restrict__ V = p.V;
    for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
        const double* qs = q + ls * A;
        double best = qs[0];
        int arg = 0;
        for (int a = 1; a < A; ++a) {
            const double x = qs[a];
            if (x < best) {
                best = x;
                arg = a;
            }
        }
        const int64_t s = s0 + ls;
        if (p.TV) p.TV[s] = best;
        p.pi[s] = arg;
        const double vs = V[s];
        const double res = best - vs;
        if (p.resid) p.resid[s] = res;
        mx = nanmax(mx, fabs(res));
        vx = nanmax(vx, fabs(vs));
    }
}

// the workgroup's maxima folded into the device-wide ones (one atomic each)
template <typename VT, typename PT>
__device__ __forceinline__ void bellman_block_max(const BellmanParams<VT, PT>& p, double mx, double vx) {
    if (!p.rho_bits) return;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        mx = nanmax(mx, __shfl_xor(mx, off, dev::kWave));
        vx = nanmax(vx, __shfl_xor(vx, off, dev::kWave));
    }
    __shared__ double wm[8];
    if ((threadIdx.x & 63) == 0) {
        wm[threadIdx.x >> 6] = mx;
        wm[4 + (threadIdx.x >> 6)] = vx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        dev::atomic_max_nonneg(p.rho_bits, nanmax(nanmax(wm[0], wm[1]), nanmax(wm[2], wm[3])));
        if (p.vmax_bits) dev::atomic_max_nonneg(p.vmax_bits, nanmax(nanmax(wm[4], wm[5]), nanmax(wm[6], wm[7])));
    }
}

template <typename VT, typename PT, int L, int VEC>
__global__ __launch_bounds__(256) void k_bellman(BellmanParams<VT, PT> p) {
    extern __shared__ double lds[];
    const int64_t lb = dev::xcd_remap(blockIdx.x, gridDim.x);
    const int A = p.A;
    double* q = lds;                                             // spt * A doubles
    PT* rp = reinterpret_cast<PT*>(lds + (size_t)p.spt * A);     // spt * A + 1 entries
    constexpr int G = 256 / L;
    const int grp = threadIdx.x / L;
    const int lane = threadIdx.x % L;
    const double* __restrict__ V = p.V;
    double mx = 0.0, vx = 0.0;
    // tiles dealt round-robin over the workgroups (see k_bellman_wave)
    for (int64_t tile = lb; tile < p.ntiles; tile += gridDim.x) {
        const int64_t s0 = tile * (int64_t)p.spt;
        const int64_t s1 = min(p.S, s0 + (int64_t)p.spt);
        const int ns = (int)(s1 - s0);
        const int R = ns * A;
        const int64_t r0 = s0 * (int64_t)A;
        for (int i = threadIdx.x; i <= R; i += blockDim.x) rp[i] = p.row_ptr[r0 + i];
        for (int i = threadIdx.x; i < R; i += blockDim.x) q[i] = p.g[r0 + i];
        __syncthreads();
        for (int rr = grp; rr < R; rr += G) {
            const int64_t b = rp[rr], e = rp[rr + 1];
            double acc = 0.0;
#pragma unroll 4
            for (int64_t j = b + (int64_t)lane * VEC; j < e; j += (int64_t)L * VEC) {
                double vv[VEC];
                int cc[VEC];
                dev::VecLoad<HiT<VT>, VEC>::load(hi_vals(p.val), p.col, j, vv, cc);
                if constexpr (kSplit<VT>) add_lo<VEC>(p.lo, j, vv);
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc = fma(vv[v], V[cc[v]], acc);
            }
            acc = dev::group_sum<L>(acc);
            if (lane == 0) q[rr] = q[rr] + p.gamma * acc;
        }
        __syncthreads();
        bellman_finish(p, q, s0, ns, mx, vx);
        __syncthreads();  // q and rp are rewritten by the next tile
    }
    bellman_block_max(p, mx, vx);
}

// Uniform row length k (known at create): the tile's nonzeros start at
// s0*A*k; each thread streams chunks of E values with independent 16-byte
// loads and no row-pointer dependency; chunk sums go to LDS; each row adds
// its k/E chunks in order.  The columns come from the column array, from
// the row's first column (band form: k consecutive columns) or from the
// row's first column plus its pattern's offsets (stencil form, the offsets
// staged in LDS); the same products are summed in the same order.  ONE
// (k == E, a row is one chunk): the row's g is loaded with its values and
// its Q written from the chunk, with no row-sum phase (the same arithmetic).
template <typename VT, int E, int FORM, int U, bool ONE>
__global__ __launch_bounds__(256) void k_bellman_flat(BellmanParams<VT, int32_t> p, int k) {
    constexpr bool BAND = FORM == kFormBand, STEN = FORM == kFormSten;
    extern __shared__ double lds[];
    __shared__ int soff[STEN ? kStenMaxPatterns * kStenMaxK : 1];
    if constexpr (STEN) {
        for (int i = threadIdx.x; i < p.sten_np * k; i += blockDim.x) soff[i] = p.sten_off[i];
        __syncthreads();
    }
    const int64_t lb = dev::xcd_remap(blockIdx.x, gridDim.x);
    const int A = p.A;
    double* q = lds;                           // spt * A doubles
    double* cp = lds + (size_t)p.spt * A;      // spt * A * k / E chunk sums and a spare slot
    const int cpr = k / E;
    const int spare = p.spt * A * cpr;
    const double* __restrict__ V = p.V;
    double mx = 0.0, vx = 0.0;
    // tiles dealt round-robin over the workgroups (see k_bellman_wave)
    for (int64_t tile = lb; tile < p.ntiles; tile += gridDim.x) {
        const int64_t s0 = tile * (int64_t)p.spt;
        const int64_t s1 = min(p.S, s0 + (int64_t)p.spt);
        const int ns = (int)(s1 - s0);
        const int R = ns * A;
        const int64_t r0 = s0 * (int64_t)A;
        const int nch = R * cpr;
        const int64_t base = r0 * (int64_t)k;
        // the thread's first row's g and first state's V, loaded with the
        // first batch
        const double g0 = ONE ? 0.0 : p.g[r0 + min((int)threadIdx.x, R - 1)];
        const double v0 = V[s0 + min((int)threadIdx.x, ns - 1)];
        // batches of U chunks per thread, every load issued before the first
        // use (chunks past the tile's end re-read its last chunk and store to
        // the spare slot)
        const int nbatch = (nch + (int)blockDim.x * U - 1) / ((int)blockDim.x * U);
        for (int bt = 0; bt < nbatch; ++bt) {
            double vv[U][E];
            int cc[U][E];
            double gg[ONE ? U : 1];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int cl = min((int)threadIdx.x + (int)blockDim.x * (bt * U + u), nch - 1);
                if constexpr (ONE) gg[u] = p.g[r0 + cl];
                if constexpr (BAND || STEN) {
                    dev::FlatVals<HiT<VT>, E>::load(hi_vals(p.val), base + (int64_t)cl * E, vv[u]);
                } else {
                    dev::FlatLoad<HiT<VT>, E>::load(hi_vals(p.val), p.col, base + (int64_t)cl * E, vv[u], cc[u]);
                }
                if constexpr (kSplit<VT>) add_lo<E>(p.lo, base + (int64_t)cl * E, vv[u]);
            }
            if constexpr (BAND) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int cl = min((int)threadIdx.x + (int)blockDim.x * (bt * U + u), nch - 1);
                    const int rr = cl / cpr;
                    const int c0 = p.band[r0 + rr] + (cl - rr * cpr) * E;
#pragma unroll
                    for (int e = 0; e < E; ++e) cc[u][e] = c0 + e;
                }
            } else if constexpr (STEN) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int cl = min((int)threadIdx.x + (int)blockDim.x * (bt * U + u), nch - 1);
                    const int rr = cl / cpr;
                    const uint32_t wd = p.sten[r0 + rr];
                    const int c0 = (int)(wd & ((1u << kStenColBits) - 1));
                    const int* o = soff + (int)(wd >> kStenColBits) * k + (cl - rr * cpr) * E;
#pragma unroll
                    for (int e = 0; e < E; ++e) cc[u][e] = c0 + o[e];
                }
            }
            double xg[U][E];
            if (STEN && E % 2 == 0 && p.sten_pairs) {
                // columns c and c + 1: one 16-byte load (8-byte aligned)
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int e = 0; e < E; e += 2) {
                        dev::d2_t t;
                        __builtin_memcpy(&t, V + cc[u][e], 16);
                        xg[u][e] = t.x;
                        xg[u][e + 1] = t.y;
                    }
                }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int e = 0; e < E; ++e) xg[u][e] = V[cc[u][e]];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                double acc = 0.0;
#pragma unroll
                for (int e = 0; e < E; ++e) acc = fma(vv[u][e], xg[u][e], acc);
                const int c = (int)threadIdx.x + (int)blockDim.x * (bt * U + u);
                if constexpr (ONE) {
                    // the row sum of one chunk, as the row-sum phase forms it
                    if (c < nch) q[c] = gg[u] + p.gamma * (0.0 + acc);
                } else {
                    cp[c < nch ? c : spare] = acc;
                }
            }
        }
        if constexpr (!ONE) {
            __syncthreads();
            for (int rr = threadIdx.x; rr < R; rr += blockDim.x) {
                double t = 0.0;
                for (int i = 0; i < cpr; ++i) t += cp[rr * cpr + i];
                q[rr] = (rr == (int)threadIdx.x ? g0 : p.g[r0 + rr]) + p.gamma * t;
            }
        }
        __syncthreads();
        // one thread per state: min / lowest-index argmin over its A values
        for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
            const double* qs = q + ls * A;
            double best = qs[0];
            int arg = 0;
            for (int a = 1; a < A; ++a) {
                const double x = qs[a];
                if (x < best) {
                    best = x;
                    arg = a;
                }
            }
            const int64_t s = s0 + ls;
            if (p.TV) p.TV[s] = best;
            p.pi[s] = arg;
            const double vs = ls == (int)threadIdx.x ? v0 : V[s];
            const double res = best - vs;
            if (p.resid) p.resid[s] = res;
            mx = nanmax(mx, fabs(res));
            vx = nanmax(vx, fabs(vs));
        }
        __syncthreads();  // q and cp are rewritten by the next tile
    }
    bellman_block_max(p, mx, vx);
}

// Wave tiles with batched loads (uniform rows, 16-byte chunks, A <= 64).
// Each wavefront takes every (4 x grid)-th tile of whole states (at most
// 64 RPL rows) and has its own LDS slice, so one wave's streaming never
// waits at a workgroup barrier.  Per tile: the lane's row's g (and band start) and
// its state's V are loaded first; then batches of U chunks per lane, whose
// value loads and V gathers are all issued before the first is used; chunk
// sums go to LDS, each row adds its k/E chunk sums in order (the same sums
// in the same order as the workgroup-tile kernel), and one lane per state
// takes the min / lowest-index argmin over its A values of Q.
template <typename VT, int E, bool BAND, int U, int RPL>
__global__ __launch_bounds__(256) void k_bellman_wave(BellmanParams<VT, int32_t> p, int k) {
    extern __shared__ double lds[];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int A = p.A;
    const int cpr = k / E;
    constexpr int RM = 64 * RPL;  // rows per tile at most
    double* __restrict__ cp = lds + (size_t)wid * ((size_t)RM * cpr + 1 + RM + kBandWindow);
    double* __restrict__ q = cp + (size_t)RM * cpr + 1;
    double* __restrict__ vw = q + RM;  // band form: the tile's window of V
    const int64_t nb = gridDim.x;
    const int64_t lb = dev::xcd_remap(blockIdx.x, nb);
    const HiT<VT>* __restrict__ val = hi_vals(p.val);
    const double* __restrict__ V = p.V;
    double mx = 0.0, vx = 0.0;
    // tiles dealt round-robin over the waves: the tiles in flight at any
    // time are neighbours in memory, and consecutive tiles run on the same
    // XCD (consecutive remapped workgroups share one), so the V windows of
    // neighbouring tiles meet in its L2.  One contiguous range of tiles per
    // wave measured 4% slower on c2 (thousands of streams far apart).
    for (int64_t t = lb * 4 + wid; t < p.ntiles; t += nb * 4) {
        const int64_t s0 = t * (int64_t)p.spt;
        const int ns = (int)min((int64_t)p.spt, p.S - s0);
        const int R = ns * A;
        const int64_t r0 = s0 * (int64_t)A;
        const int nch = R * cpr;
        const int64_t base = r0 * (int64_t)k;
        double gr[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) gr[i] = p.g[r0 + min(lane + 64 * i, R - 1)];
        int bw[RPL];  // band form: first columns of the lane's rows
#pragma unroll
        for (int i = 0; i < RPL; ++i) bw[i] = BAND ? p.band[r0 + min(lane + 64 * i, R - 1)] : 0;
        const double vo = V[s0 + min(lane, ns - 1)];
        const int nbatch = (nch + 64 * U - 1) / (64 * U);
        // band form: the tile's rows read V in one window [wlo, wlo + span)
        // of at most kBandWindow entries (the launch checks the MDP's bound),
        // staged in the wave's LDS once per tile
        int wlo = 0;
        for (int bt = 0; bt < nbatch; ++bt) {
            double vv[U][E];
            int cc[U][E];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int cl = min(lane + 64 * (bt * U + u), nch - 1);
                if constexpr (BAND) dev::FlatVals<HiT<VT>, E>::load(val, base + (int64_t)cl * E, vv[u]);
                else dev::FlatLoad<HiT<VT>, E>::load(val, p.col, base + (int64_t)cl * E, vv[u], cc[u]);
                if constexpr (kSplit<VT>) add_lo<E>(p.lo, base + (int64_t)cl * E, vv[u]);
            }
            if constexpr (BAND) {
                if (bt == 0) {
                    int whi = bw[0];
                    wlo = bw[0];
#pragma unroll
                    for (int i = 1; i < RPL; ++i) {
                        wlo = min(wlo, bw[i]);
                        whi = max(whi, bw[i]);
                    }
#pragma unroll
                    for (int off = 32; off >= 1; off >>= 1) {
                        wlo = min(wlo, __shfl_xor(wlo, off, dev::kWave));
                        whi = max(whi, __shfl_xor(whi, off, dev::kWave));
                    }
                    const int span = whi + k - wlo;
                    const int i0 = min(2 * lane, span - 1), i1 = min(2 * lane + 1, span - 1);
                    const double a0 = V[wlo + i0], a1 = V[wlo + i1];
                    vw[i0] = a0;
                    vw[i1] = a1;
                    wave_sync();
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int cl = min(lane + 64 * (bt * U + u), nch - 1);
                    const int rr = cl / cpr;
                    int b0 = __shfl(bw[0], rr & 63, dev::kWave);
#pragma unroll
                    for (int i = 1; i < RPL; ++i) {
                        const int bi = __shfl(bw[i], rr & 63, dev::kWave);
                        if ((rr >> 6) == i) b0 = bi;
                    }
                    const int c0 = b0 + (cl - rr * cpr) * E;
#pragma unroll
                    for (int e = 0; e < E; ++e) cc[u][e] = c0 + e;
                }
            }
            double xg[U][E];
            if constexpr (BAND) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int e = 0; e < E; ++e) xg[u][e] = vw[cc[u][e] - wlo];
                }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int e = 0; e < E; ++e) xg[u][e] = V[cc[u][e]];
                }
                // keep every gather of the batch ahead of the first use
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                double x = 0.0;
#pragma unroll
                for (int e = 0; e < E; ++e) x = fma(vv[u][e], xg[u][e], x);
                // chunks past the tile's end go to the wave's spare slot
                const int c = lane + 64 * (bt * U + u);
                cp[c < nch ? c : RM * cpr] = x;
            }
        }
        wave_sync();
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int rr = lane + 64 * i;
            if (rr < R) {
                double sum = 0.0;
                for (int j = 0; j < cpr; ++j) sum += cp[rr * cpr + j];
                q[rr] = gr[i] + p.gamma * sum;
            }
        }
        wave_sync();
        if (lane < ns) {
            const double* qs = q + lane * A;
            double best = qs[0];
            int arg = 0;
            for (int a = 1; a < A; ++a) {
                const double x = qs[a];
                if (x < best) {
                    best = x;
                    arg = a;
                }
            }
            const int64_t s = s0 + lane;
            if (p.TV) p.TV[s] = best;
            p.pi[s] = arg;
            const double res = best - vo;
            if (p.resid) p.resid[s] = res;
            mx = nanmax(mx, fabs(res));
            vx = nanmax(vx, fabs(vo));
        }
        wave_sync();  // cp and q are rewritten by the next tile
    }
    bellman_block_max(p, mx, vx);
}

template <typename VT, typename PT, int L, int VEC>
void launch_one(const BellmanParams<VT, PT>& p, int64_t nb, hipStream_t st) {
    const size_t lds = (size_t)p.spt * p.A * sizeof(double) + ((size_t)p.spt * p.A + 1) * sizeof(PT);
    hipLaunchKernelGGL((k_bellman<VT, PT, L, VEC>), dim3((unsigned)nb), dim3(kBlock), lds, st, p);
}

template <typename VT, typename PT, int VEC>
void dispatch_lanes(const BellmanParams<VT, PT>& p, int64_t nb, int lanes, hipStream_t st) {
    switch (lanes) {
        case 1: launch_one<VT, PT, 1, VEC>(p, nb, st); break;
        case 2: launch_one<VT, PT, 2, VEC>(p, nb, st); break;
        case 4: launch_one<VT, PT, 4, VEC>(p, nb, st); break;
        case 8: launch_one<VT, PT, 8, VEC>(p, nb, st); break;
        case 16: launch_one<VT, PT, 16, VEC>(p, nb, st); break;
        case 32: launch_one<VT, PT, 32, VEC>(p, nb, st); break;
        case 64: launch_one<VT, PT, 64, VEC>(p, nb, st); break;
        default: throw Error(IPI_E_INVALID_ARG, "lanes per row must be a power of two in [1, 64]");
    }
}

template <typename VT, typename PT>
void dispatch_vec(const BellmanParams<VT, PT>& p, int64_t nb, int lanes, int vec, hipStream_t st) {
    if constexpr (sizeof(VT) == 4) {
        if (vec >= 4) return dispatch_lanes<VT, PT, 4>(p, nb, lanes, st);
    }
    if (vec >= 2) return dispatch_lanes<VT, PT, 2>(p, nb, lanes, st);
    dispatch_lanes<VT, PT, 1>(p, nb, lanes, st);
}

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_rho_to_double(const uint64_t* bits, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = __longlong_as_double((long long)bits[0]);
}

__global__ void k_negate(const double* x, double* y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = -x[i];
}

}  // namespace

int bellman_vec(const ipi_mdp_s* m, bool fp32) {
    int v = m->vec_align;
    if (!fp32 && v > 2) v = 2;  // 16-byte loads: 2 doubles / 4 floats
    return v;
}

// chunk width of the flat kernel for this MDP, or 0 when rows are not uniform
// (or no admissible width divides the row length)
bool flat_chunk_ok(const ipi_mdp_s* m, bool fp32, int e) {
    if (!m->uniform_k || e <= 0) return false;
    const int w = fp32 ? 4 : 2;  // values per 16-byte load
    const bool supported = e == 2 || e == 4 || e == 8 || e == 12 || e == 16 || e == 24 || e == 32;
    return supported && e % w == 0 && m->k_max % e == 0 && m->vec_align >= w && m->vec_align % w == 0;
}

int bellman_flat_e(const ipi_mdp_s* m, bool fp32, int pref) {
    if (pref > 0 && flat_chunk_ok(m, fp32, pref)) return pref;  // else the automatic choice
    // one 16-byte load per chunk first (2 doubles or 4 floats: consecutive
    // lanes then read consecutive bytes), then wider chunks
    const int cand[] = {2, 4, 8, 12, 16};
    for (int e : cand)
        if (flat_chunk_ok(m, fp32, e)) return e;
    // rows of one entry (a deterministic step per action): one value per chunk
    if (m->uniform_k && m->k_max == 1) return 1;
    return 0;
}

int flat_spt(const ipi_mdp_s* m, int e) {
    // about six to eight chunks per thread, at most kMaxTileRows rows and 4096 chunk slots
    const int64_t row_chunks = m->k_max / e;
    int spt = 1;
    while (spt < 1024 && (int64_t)(2 * spt) * m->A * row_chunks <= 8 * kBlock &&
           (int64_t)(2 * spt) * m->A <= kMaxTileRows)
        spt *= 2;
    while (spt > 1 && (int64_t)spt * m->A * row_chunks > 4096) spt /= 2;
    return spt;
}

int default_bellman_lanes(const ipi_mdp_s* m, bool fp32) {
    const double kavg = m->nnz / (double)((int64_t)m->S * m->A);
    const int vec = bellman_vec(m, fp32);
    int L = 1;
    while (L < 64 && (double)(2 * L) * vec * 3.0 <= kavg) L *= 2;
    return L;
}

int default_bellman_spt(const ipi_mdp_s* m, int lanes) {
    const int groups = kBlock / lanes;
    int spt = 1;
    // at least ~4 rows per lane group, at most kMaxTileRows rows and 256 states
    while (spt < 256 && (int64_t)spt * m->A < 4 * groups && (int64_t)(2 * spt) * m->A <= kMaxTileRows) spt *= 2;
    return spt;
}


// chunk width of the flat Bellman pass: the tuned one, else one 16-byte
// load per chunk
int bellman_pass_e(const ipi_mdp_s* m, bool fp32) { return bellman_flat_e(m, fp32, m->tune.bellman_chunk); }

// states per wave tile of the Bellman pass at most: 64 RPL rows
int bellman_wave_smax(const ipi_mdp_s* m, int rpl) { return std::min(64, 64 * rpl / m->A); }

// rows per lane of a band-form wave tile: two for float values, so that a
// tile streams as many bytes as with doubles (one and four rows per lane for
// floats measured slower)
constexpr int kBandRowsPerLane64 = 1;
constexpr int kBandRowsPerLane32 = 2;
int bellman_band_rpl(bool fp32) { return fp32 ? kBandRowsPerLane32 : kBandRowsPerLane64; }

// the band form on wave tiles: detected, not disabled, and the V window of a
// tile of the largest size fits the wave's LDS slice
bool bellman_wave_band(const ipi_mdp_s* m, bool fp32) {
    return band_on(m) && band_window_fits(m, bellman_wave_smax(m, bellman_band_rpl(fp32)));
}

// wave tiles: 16-byte chunks and a state's A rows within one wave's tile;
// by default (lanes -1) only in the band form, where they measured faster
// (lanes -3 asks for them, -2 for workgroup tiles)
bool bellman_wave_ok(const ipi_mdp_s* m, bool fp32, int lanes, int e) {
    if (lanes == -2 || e * (fp32 ? 4 : 8) != 16 || m->A > 64) return false;
    return lanes == -3 || bellman_wave_band(m, fp32);
}

// Flat chunk streaming by default when admissible and either wave tiles
// apply or a state's chunks fit a modest workgroup tile (A k / E <= 2048
// chunk slots, so a few workgroups share a CU); lanes < 0 asks for it
// whenever it is admissible.
bool bellman_uses_flat(const ipi_mdp_s* m, bool fp32, int lanes) {
    if (lanes > 0) return false;
    const int e = bellman_pass_e(m, fp32);
    if (e <= 0) return false;
    return lanes < 0 || bellman_wave_ok(m, fp32, lanes, e) || (int64_t)m->A * (m->k_max / e) <= 2048;
}

template <typename VT>
void launch_flat(const BellmanParams<VT, int32_t>& p, int64_t nb, int e, int k, hipStream_t st) {
    const size_t lds = ((size_t)p.spt * p.A * (1 + (size_t)(k / e)) + 1) * sizeof(double);
    // chunks per thread in flight: eight single values, six of 16 bytes
    // (three for floats, whose gathered V values take twice the registers),
    // three of 32, else one or two (wider chunks already hold several loads)
#define FLAT(E)                                                                                      \
    do {                                                                                             \
        constexpr int U = E == 1 ? 8                                                                    \
                          : E * (int)sizeof(VT) == 16 ? (sizeof(VT) == 8 ? 6 : 3)                             \
                          : (E * (int)sizeof(VT) == 32 ? 3 : (E * (int)sizeof(VT) <= 64 ? 2 : 1));               \
        if (k == E && E <= 4) {                                                                      \
            if (p.band) hipLaunchKernelGGL((k_bellman_flat<VT, E, kFormBand, U, E <= 4>), dim3((unsigned)nb), dim3(kBlock), lds, st, p, k); \
            else if (p.sten) hipLaunchKernelGGL((k_bellman_flat<VT, E, kFormSten, U, E <= 4>), dim3((unsigned)nb), dim3(kBlock), lds, st, p, k); \
            else hipLaunchKernelGGL((k_bellman_flat<VT, E, kFormCols, U, E <= 4>), dim3((unsigned)nb), dim3(kBlock), lds, st, p, k); \
        } else if (p.band) hipLaunchKernelGGL((k_bellman_flat<VT, E, kFormBand, U, false>), dim3((unsigned)nb), dim3(kBlock), lds, st, p, k); \
        else if (p.sten) hipLaunchKernelGGL((k_bellman_flat<VT, E, kFormSten, U, false>), dim3((unsigned)nb), dim3(kBlock), lds, st, p, k); \
        else hipLaunchKernelGGL((k_bellman_flat<VT, E, kFormCols, U, false>), dim3((unsigned)nb), dim3(kBlock), lds, st, p, k); \
    } while (0)
    if (e == 1) {  // rows of one entry: never in the band or stencil form (which need two)
        IPI_REQUIRE(!p.band && !p.sten, IPI_E_INVALID_ARG, "the band and stencil forms need rows of at least two entries");
        hipLaunchKernelGGL((k_bellman_flat<VT, 1, kFormCols, 8, false>), dim3((unsigned)nb), dim3(kBlock), lds, st, p, k);
        return;
    }
    if constexpr (sizeof(VT) == 8) {
        if (e == 2) {
            FLAT(2);
            return;
        }
    }
    switch (e) {
        case 4: FLAT(4); break;
        case 8: FLAT(8); break;
        case 12: FLAT(12); break;
        case 16: FLAT(16); break;
        case 24: FLAT(24); break;
        case 32: FLAT(32); break;
        default: throw Error(IPI_E_INVALID_ARG, "unsupported chunk width");
    }
#undef FLAT
}

// workgroups of a Bellman launch: 16 per CU (about three rounds of resident
// workgroups at the usual LDS footprint), never more than there are tiles
int64_t bellman_grid(const ipi_mdp_s* m, int64_t ntiles) {
    const int64_t cap = (int64_t)std::max(1, m->arch_cus) * 16;
    return std::max<int64_t>(1, std::min(ntiles, cap));
}

// wave-tile launch: rows per tile 64 RPL (RPL = 4 when a row has at most 4
// chunks and no band form, else 1), states per tile min(64, 64 RPL / A) or
// the tuned count when it fits
// Algorithmic bytes of one pass with this tuning's kernel (lanes as in
// launch_bellman).
double bellman_alg_bytes(const ipi_mdp_s* m, bool fp32, int lanes) {
    const double bv = fp32 ? 4.0 : 8.0;  // split values: hi + lo, 8 bytes
    fp32 = fp32 || m->val == nullptr;    // the kernels of float values
    const bool flat = bellman_uses_flat(m, fp32, lanes);
    const double R = (double)m->S * m->A;
    const double bp = m->rp32 ? 4.0 : 8.0;
    // the band form is read unless wave tiles run without it
    const bool wave = flat && bellman_wave_ok(m, fp32, lanes, bellman_pass_e(m, fp32));
    bool band = flat && band_on(m);
    if (band && wave) band = bellman_wave_band(m, fp32);
    // the stencil form on workgroup tiles only
    const bool sten = flat && !wave && !band && sten_on(m);
    // P values + columns (band and stencil forms: one word per row instead),
    // row pointers (not read by the flat kernels: uniform rows), g, V (read
    // once), TV + pi + resid writes
    const double cols = band || sten ? 4.0 * R : 4.0 * (double)m->nnz;
    return m->nnz * bv + cols + (flat ? 0.0 : (R + 1.0) * bp) + 8.0 * R + 8.0 * m->S + 20.0 * m->S;
}

template <typename VT, int E>
void launch_wave_t(const BellmanParams<VT, int32_t>& p, int64_t nb, int rpl, int k, hipStream_t st) {
    const int cpr = k / E;
    const size_t lds = (size_t)4 * ((size_t)64 * rpl * cpr + 1 + (size_t)64 * rpl + kBandWindow) * sizeof(double);
    const int per_lane = (p.spt * p.A * cpr + 63) / 64;
    // six chunks in flight per lane for doubles; four for floats (whose
    // gathered V values take twice the registers of their loads: 123 VGPRs,
    // still four waves per SIMD; six would leave three); three for split
    // values (hi and lo: 96 bytes of values a lane, as for doubles; four
    // chunks on tiles of two rows a lane measured 9% slower on c2)
    constexpr int UB = kSplit<VT> ? 3 : (sizeof(VT) == 8 ? 6 : 4);
#define WAVE(B, U, R) hipLaunchKernelGGL((k_bellman_wave<VT, E, B, U, R>), dim3((unsigned)nb), dim3(kBlock), lds, st, p, k)
    if (p.band && rpl == 4) {
        if (per_lane >= UB) WAVE(true, UB, 4);
        else if (per_lane >= 2) WAVE(true, 2, 4);
        else WAVE(true, 1, 4);
    } else if (p.band && rpl == 2) {
        if (per_lane >= UB) WAVE(true, UB, 2);
        else if (per_lane >= 2) WAVE(true, 2, 2);
        else WAVE(true, 1, 2);
    } else if (p.band) {
        if (per_lane >= UB) WAVE(true, UB, 1);
        else if (per_lane >= 2) WAVE(true, 2, 1);
        else WAVE(true, 1, 1);
    } else if (rpl == 4) {
        if (per_lane >= UB) WAVE(false, UB, 4);
        else if (per_lane >= 2) WAVE(false, 2, 4);
        else WAVE(false, 1, 4);
    } else {
        if (per_lane >= UB) WAVE(false, UB, 1);
        else if (per_lane >= 2) WAVE(false, 2, 1);
        else WAVE(false, 1, 1);
    }
#undef WAVE
}

// fp32: the float32 values (or hi alone); split: hi + lo (fp32 false)
void launch_bellman_wave(const ipi_mdp_s* m, const double* g, const double* V, const BellmanOut& o, bool fp32,
                         bool split, int e, int spt, hipStream_t st) {
    const int cpr = m->k_max / e;
    fp32 = fp32 || split;  // the chunk widths of float values
    const bool band = bellman_wave_band(m, fp32);
    // band tiles: split values take the doubles' one row a lane (their bytes
    // a value are the doubles'; the window check above used the larger tile)
    const int rpl = band ? (split ? kBandRowsPerLane64 : bellman_band_rpl(fp32)) : ((256 * cpr <= 1024) ? 4 : 1);
    const int smax = bellman_wave_smax(m, rpl);
    if (spt <= 0 || spt > smax) spt = smax;
    const int64_t ntiles = (m->S + spt - 1) / spt;
    const int64_t nb = bellman_grid(m, (ntiles + 3) / 4);
    if (split) {
        BellmanParams<F32Split, int32_t> p{nullptr, m->col, reinterpret_cast<const F32Split*>(m->val32), g, V,
                                           m->gamma, m->A, spt, m->S, ntiles, o.TV, o.pi, o.resid, o.rho_bits,
                                           o.vmax_bits, band ? m->band : nullptr};
        p.lo = m->val_lo;
        launch_wave_t<F32Split, 4>(p, nb, rpl, m->k_max, st);
    } else if (fp32) {
        BellmanParams<float, int32_t> p{nullptr, m->col, m->val32, g, V, m->gamma, m->A, spt, m->S,
                                        ntiles, o.TV, o.pi, o.resid, o.rho_bits, o.vmax_bits,
                                        band ? m->band : nullptr};
        launch_wave_t<float, 4>(p, nb, rpl, m->k_max, st);
    } else {
        BellmanParams<double, int32_t> p{nullptr, m->col, m->val, g, V, m->gamma, m->A, spt, m->S,
                                         ntiles, o.TV, o.pi, o.resid, o.rho_bits, o.vmax_bits,
                                         band ? m->band : nullptr};
        launch_wave_t<double, 2>(p, nb, rpl, m->k_max, st);
    }
    IPI_HIP(hipGetLastError());
}

void launch_bellman(const ipi_mdp_s* m, const double* g, const double* V, const BellmanOut& o, bool fp32,
                    int lanes, int spt, hipStream_t st) {
    IPI_REQUIRE(!fp32 || m->val32 != nullptr, IPI_E_INVALID_ARG, "FP32 precision needs an MDP created with IPI_VAL_FP32");
    IPI_REQUIRE(fp32 || m->val != nullptr || m->val_lo != nullptr, IPI_E_INVALID_ARG,
                "an FP64 Bellman pass needs the FP64 values of P (the MDP keeps float32 values only)");
    // FP64 arithmetic on split values: hi + lo, laid out as float values
    const bool split = !fp32 && m->val == nullptr;
    const bool f4 = fp32 || split;
    if (bellman_uses_flat(m, f4, lanes)) {
        const int e = bellman_pass_e(m, f4);
        if (bellman_wave_ok(m, f4, lanes, e)) {
            launch_bellman_wave(m, g, V, o, fp32, split, e, spt, st);
            return;
        }
        if (spt <= 0 || (int64_t)spt * m->A * (m->k_max / e) > 4096 || (int64_t)spt * m->A > kMaxTileRows)
            spt = flat_spt(m, e);
        const int64_t ntiles = (m->S + spt - 1) / spt;
        IPI_REQUIRE(ntiles < (int64_t)1 << 31, IPI_E_INVALID_ARG, "too many tiles");
        const int64_t nb = bellman_grid(m, ntiles);
        if (split) {
            BellmanParams<F32Split, int32_t> p{nullptr, m->col, reinterpret_cast<const F32Split*>(m->val32), g,
                                               V, m->gamma, m->A, spt, m->S, ntiles, o.TV, o.pi, o.resid,
                                               o.rho_bits, o.vmax_bits, band_on(m) ? m->band : nullptr};
            p.lo = m->val_lo;
            if (!p.band && sten_on(m)) {
                p.sten = m->sten;
                p.sten_off = m->sten_off;
                p.sten_np = m->sten_np;
                p.sten_pairs = m->sten_pairs;
            }
            launch_flat(p, nb, e, m->k_max, st);
        } else if (fp32) {
            BellmanParams<float, int32_t> p{nullptr, m->col, m->val32, g, V, m->gamma, m->A, spt, m->S,
                                            ntiles, o.TV, o.pi, o.resid, o.rho_bits, o.vmax_bits,
                                            band_on(m) ? m->band : nullptr};
            if (!p.band && sten_on(m)) {
                p.sten = m->sten;
                p.sten_off = m->sten_off;
                p.sten_np = m->sten_np;
                p.sten_pairs = m->sten_pairs;
            }
            launch_flat(p, nb, e, m->k_max, st);
        } else {
            BellmanParams<double, int32_t> p{nullptr, m->col, m->val, g, V, m->gamma, m->A, spt, m->S,
                                             ntiles, o.TV, o.pi, o.resid, o.rho_bits, o.vmax_bits,
                                             band_on(m) ? m->band : nullptr};
            if (!p.band && sten_on(m)) {
                p.sten = m->sten;
                p.sten_off = m->sten_off;
                p.sten_np = m->sten_np;
                p.sten_pairs = m->sten_pairs;
            }
            launch_flat(p, nb, e, m->k_max, st);
        }
        IPI_HIP(hipGetLastError());
        return;
    }
    if (lanes <= 0) lanes = default_bellman_lanes(m, f4);
    if (spt <= 0) spt = default_bellman_spt(m, lanes);
    IPI_REQUIRE((int64_t)spt * m->A <= kMaxTileRows, IPI_E_INVALID_ARG, "states per tile * A exceeds the tile capacity");
    const int64_t ntiles = (m->S + spt - 1) / spt;
    IPI_REQUIRE(ntiles < (int64_t)1 << 31, IPI_E_INVALID_ARG, "too many tiles");
    const int64_t nb = bellman_grid(m, ntiles);
    const int vec = bellman_vec(m, f4);
    if (split) {
        const auto* hv = reinterpret_cast<const F32Split*>(m->val32);
        if (m->rp32) {
            BellmanParams<F32Split, int32_t> p{(const int32_t*)m->row_ptr, m->col, hv, g, V, m->gamma, m->A,
                                               spt, m->S, ntiles, o.TV, o.pi, o.resid, o.rho_bits, o.vmax_bits,
                                               nullptr};
            p.lo = m->val_lo;
            dispatch_vec(p, nb, lanes, vec, st);
        } else {
            BellmanParams<F32Split, int64_t> p{(const int64_t*)m->row_ptr, m->col, hv, g, V, m->gamma, m->A,
                                               spt, m->S, ntiles, o.TV, o.pi, o.resid, o.rho_bits, o.vmax_bits,
                                               nullptr};
            p.lo = m->val_lo;
            dispatch_vec(p, nb, lanes, vec, st);
        }
    } else if (fp32) {
        IPI_REQUIRE(m->val32 != nullptr, IPI_E_INVALID_ARG, "FP32 precision needs an MDP created with IPI_VAL_FP32");
        if (m->rp32) {
            BellmanParams<float, int32_t> p{(const int32_t*)m->row_ptr, m->col, m->val32, g, V, m->gamma, m->A,
                                            spt, m->S, ntiles, o.TV, o.pi, o.resid, o.rho_bits, o.vmax_bits, nullptr};
            dispatch_vec(p, nb, lanes, vec, st);
        } else {
            BellmanParams<float, int64_t> p{(const int64_t*)m->row_ptr, m->col, m->val32, g, V, m->gamma, m->A,
                                            spt, m->S, ntiles, o.TV, o.pi, o.resid, o.rho_bits, o.vmax_bits, nullptr};
            dispatch_vec(p, nb, lanes, vec, st);
        }
    } else {
        if (m->rp32) {
            BellmanParams<double, int32_t> p{(const int32_t*)m->row_ptr, m->col, m->val, g, V, m->gamma, m->A,
                                             spt, m->S, ntiles, o.TV, o.pi, o.resid, o.rho_bits, o.vmax_bits, nullptr};
            dispatch_vec(p, nb, lanes, vec, st);
        } else {
            BellmanParams<double, int64_t> p{(const int64_t*)m->row_ptr, m->col, m->val, g, V, m->gamma, m->A,
                                             spt, m->S, ntiles, o.TV, o.pi, o.resid, o.rho_bits, o.vmax_bits, nullptr};
            dispatch_vec(p, nb, lanes, vec, st);
        }
    }
    IPI_HIP(hipGetLastError());
}

void launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t st) {
    int64_t nb = (n + kBlock - 1) / kBlock;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)nb), dim3(kBlock), 0, st, p, n, v);
    IPI_HIP(hipGetLastError());
}

void launch_rho_to_double(const uint64_t* bits, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_rho_to_double, dim3(1), dim3(64), 0, st, bits, out);
    IPI_HIP(hipGetLastError());
}

void launch_negate(const double* x, double* y, int64_t n, hipStream_t st) {
    int64_t nb = (n + kBlock - 1) / kBlock;
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_negate, dim3((unsigned)nb), dim3(kBlock), 0, st, x, y, n);
    IPI_HIP(hipGetLastError());
}

}  // namespace ipi
