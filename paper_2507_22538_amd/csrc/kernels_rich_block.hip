// Temporally blocked Richardson sweeps for band-form P_pi.
//
// The Richardson inner solve of Algorithm 1 (Sec. III-A; Table 2's OPI is
// this iteration with a fixed sweep count) applies, in correction form,
//   delta_{i+1} = delta_i + a D (b - (delta_i - gamma P_pi delta_i))
// once per sweep, and every sweep streams P_pi from HBM.  When every row of
// P_pi holds k consecutive columns starting within [s + dlo, s + dhi] of its
// state s, sweep i+1 of state s reads delta_i only on [s - hl, s + hr] with
// hl = max(0, -dlo) and hr = max(0, dhi + k - 1).  A workgroup then owns
// kRB consecutive states, loads their P_pi rows into registers (one state per
// thread) and delta_i into LDS once, and runs T sweeps in LDS; after sweep t
// the states in [e0 + t hl, e0 + kRB - t hr) are exact, so each workgroup
// writes the kRB - T (hl + hr) states in the middle of its range.  Each
// state's arithmetic is that of the one-sweep kernel (chunks of FE values
// summed with fused multiply-adds, chunk sums added in order), so the
// iterates are bit for bit those of T separate sweeps; P_pi is read from HBM
// kRB / (kRB - T (hl + hr)) times per T sweeps instead of T times.
//
// Outputs: delta after sweep T - 1 (the last sweep's input, which the
// stopping test returns when it passes) and after sweep T, on the
// workgroup's own states; per-workgroup partial sums of |r|^2 of the last
// sweep's residual r = b - J delta_{T-1} (the quantity the test reads).
#include <algorithm>
#include <type_traits>

#include "device.hpp"
#include "krylov.hpp"

namespace ipi {

namespace {

constexpr int kRB = 1024;  // states per workgroup: its output plus both halos

struct RichBlockParams {
    const void* val;       // P_pi values, row s at s * K
    const int32_t* band;   // first column of each row
    const double* b;
    const double* x;       // delta before the block
    const double* dinv;    // Jacobi scaling or nullptr
    double* out_prev;      // delta after sweep T - 1
    double* out_last;      // delta after sweep T
    double* partials;      // one per workgroup
    Ctrl* ctrl;
    double gamma;
    int64_t S;
    int hl, hr;            // halo widths (states) per sweep
    int out;               // output states per block
    int64_t nblk;          // blocks of kRB states
    bool lds_prefetch;     // long rows: the persistent kernel prefetching through LDS
};

// Staged rows in LDS.  A ds_read_b128 serves 16 lanes per cycle from 64
// four-byte banks (16 groups of 16 bytes).  A lane reading piece j of its own
// row at a row stride of NP pieces (NP = 2..16, always even) meets only
// 16 / gcd(NP, 16) groups among 16 lanes: 4-way conflicts for NP = 12, 8- and
// 16-way for 8 and 16.  Rows are therefore staged NP + 1 pieces apart (an odd
// stride: 16 lanes, 16 groups); the pad piece of each row is never read.
template <int NP>
constexpr int staged_stride() {
    return NP + 1;
}

// The 16-byte pieces of a thread's wavefront's contiguous P_pi rows for one
// block (exchanged through LDS so that each lane then holds its own row).
template <typename VT, int K, bool KEEP>
__device__ __forceinline__ void load_rows(const RichBlockParams& p, int64_t blk, int T,
                                          dev::d2_t (&pc)[K * (int)sizeof(VT) / 16]) {
    constexpr int SZ = (int)sizeof(VT);
    constexpr int NP = K * SZ / 16;
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    const int64_t e0 = blk * p.out - (int64_t)T * p.hl;
    const char* vb = static_cast<const char*>(p.val);
    const int64_t lim = p.S * (int64_t)K * SZ - 16;
    const int64_t wbase = (e0 + 64 * wid) * (int64_t)K * SZ;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        int64_t off = wbase + 16 * (int64_t)(lane + 64 * i);
        off = off < 0 ? 0 : (off > lim ? lim : off);  // pieces of states outside [0, S) are never used
        pc[i] = dev::ldp<KEEP>(reinterpret_cast<const dev::d2_t*>(vb + off));
    }
}

// the thread's state's first column, rhs, Jacobi scale and delta_i
struct BlockScalars {
    int w;
    double bo, dv, x;
};

__device__ __forceinline__ BlockScalars load_scalars(const RichBlockParams& p, int64_t blk, int T) {
    const int64_t s = blk * p.out - (int64_t)T * p.hl + threadIdx.x;
    const int64_t sc = s < 0 ? 0 : (s >= p.S ? p.S - 1 : s);  // clamped: every load in bounds
    return BlockScalars{p.band[sc], p.b[sc], p.dinv ? p.dinv[sc] : 1.0, p.x[sc]};
}

template <typename VT, int K, int FE, int T, bool KEEP>
__global__ __launch_bounds__(kRB) void k_rich_block(RichBlockParams p) {
    if (p.ctrl->active == 0) return;
    constexpr int SZ = (int)sizeof(VT);
    constexpr int NP = K * SZ / 16;   // 16-byte pieces of a row
    constexpr int WB = 64 * 16 * staged_stride<NP>();  // staged bytes of a wavefront's 64 rows
    constexpr int WR = 8;             // wavefronts staged per round
    __shared__ double X[2][kRB];
    __shared__ double red[kRB / 64];
    __shared__ __align__(16) char stage[WR * WB];
    const int tid = threadIdx.x;
    const int wid = tid >> 6, lane = tid & 63;
    const int64_t S = p.S;
    // one block per workgroup; neighbouring blocks (which read each other's
    // halo rows) run on one XCD, so the second read of a halo row can come
    // from its L2
    const int64_t blk = dev::xcd_remap(blockIdx.x, gridDim.x);
    const int64_t o0 = blk * p.out;
    const int64_t o1 = min(S, o0 + p.out);
    const int64_t e0 = o0 - (int64_t)T * p.hl;  // state of thread 0
    const int64_t s = e0 + tid;
    const bool in = s >= 0 && s < S;
    const int64_t sc = s < 0 ? 0 : (s >= S ? S - 1 : s);  // clamped: every load in bounds
    // The rows of a wavefront's 64 states are contiguous: its lanes load them
    // in consecutive 16-byte pieces (offsets clamped into the array; pieces
    // of states outside [0, S) are never used), then pass them through LDS so
    // that each lane holds its own state's row.
    dev::d2_t pc[NP];
    {
        const char* vb = static_cast<const char*>(p.val);
        const int64_t lim = S * (int64_t)K * SZ - 16;
        const int64_t wbase = (e0 + 64 * wid) * (int64_t)K * SZ;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            int64_t off = wbase + 16 * (int64_t)(lane + 64 * i);
            off = off < 0 ? 0 : (off > lim ? lim : off);
            pc[i] = dev::ldp<KEEP>(reinterpret_cast<const dev::d2_t*>(vb + off));
        }
    }
    VT v[K];
#pragma unroll 1
    for (int r = 0; r < kRB / 64 / WR; ++r) {
        if (wid / WR == r) {
            char* my = stage + (wid % WR) * WB;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const int pp = lane + 64 * i;  // row pp / NP, piece pp % NP
                *reinterpret_cast<dev::d2_t*>(my + 16 * (pp + pp / NP)) = pc[i];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                const dev::d2_t t = *reinterpret_cast<const dev::d2_t*>(my + 16 * (staged_stride<NP>() * lane + j));
                __builtin_memcpy(&v[j * (16 / SZ)], &t, 16);
            }
        }
        __syncthreads();  // the next round reuses the staging area
    }
    const int w = p.band[sc];
    const double bo = p.b[sc];
    const double dv = p.dinv ? p.dinv[sc] : 1.0;
    X[0][tid] = in ? p.x[sc] : 0.0;
    const double a = p.ctrl->omega;
    // exact range after sweep t: [lo0 + t hl, hi0 - t hr), but a range end at
    // the first or last state never moves (no state lies beyond it)
    const bool cut_lo = e0 > 0, cut_hi = e0 + kRB < S;
    const int64_t win = w - e0;  // the row's first column, relative to thread 0
    double racc = 0.0;
    int cur = 0;
#pragma unroll 1
    for (int t = 1; t <= T; ++t) {
        __syncthreads();
        const int64_t lo = cut_lo ? e0 + (int64_t)t * p.hl : 0;
        const int64_t hi = cut_hi ? e0 + kRB - (int64_t)t * p.hr : S;
        if (in && s >= lo && s < hi) {
            const double* xs = &X[cur][win];
            double yv = 0.0;
#pragma unroll
            for (int c = 0; c < K / FE; ++c) {
                double x = 0.0;
#pragma unroll
                for (int e = 0; e < FE; ++e) x = fma((double)v[c * FE + e], xs[c * FE + e], x);
                yv += x;
            }
            const double xv = X[cur][tid];
            const double jx = xv - p.gamma * yv;
            const double r = bo - jx;
            const double pr = p.dinv ? r * dv : r;
            const double xn = xv + a * pr;
            X[cur ^ 1][tid] = xn;
            if (t == T && s >= o0 && s < o1) {
                p.out_prev[s] = xv;
                p.out_last[s] = xn;
                racc = fma(r, r, racc);
            }
        }
        cur ^= 1;
    }
    // workgroup sum in a fixed order: wave butterflies, then the waves in order
    racc = dev::wave_sum(racc);
    if ((tid & 63) == 0) red[tid >> 6] = racc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int i = 0; i < kRB / 64; ++i) t += red[i];
        p.partials[blk] = t;
    }
}

// Persistent workgroups, one per CU, each taking a contiguous run of blocks
// (neighbouring blocks share halo rows: the second read of a halo row comes
// from the L2 the first one filled).  With PF the loads of the next block are
// issued before the current block's sweeps, so the row stream of one block
// overlaps the LDS sweeps of the previous one; without PF (rows too long for
// two copies in registers) each block loads when it starts.
template <typename VT, int K, int FE, int T, bool KEEP, bool PF>
__global__ __launch_bounds__(kRB) void k_rich_block_pf(RichBlockParams p) {
    if (p.ctrl->active == 0) return;
    constexpr int SZ = (int)sizeof(VT);
    constexpr int NP = K * SZ / 16;   // 16-byte pieces of a row
    constexpr int WB = 64 * 16 * staged_stride<NP>();  // staged bytes of a wavefront's 64 rows
    constexpr int WR = 8;             // wavefronts staged per round
    __shared__ double X[2][kRB];
    __shared__ double red[kRB / 64];
    __shared__ __align__(16) char stage[WR * WB];
    const int tid = threadIdx.x;
    const int wid = tid >> 6, lane = tid & 63;
    const int64_t S = p.S;
    const int64_t G = gridDim.x;
    const int64_t g = dev::xcd_remap(blockIdx.x, G);
    const int64_t b0 = g * p.nblk / G, b1 = (g + 1) * p.nblk / G;
    const double a = p.ctrl->omega;
    dev::d2_t pc[NP];
    BlockScalars sn{};
    if (PF && b0 < b1) {
        load_rows<VT, K, KEEP>(p, b0, T, pc);
        sn = load_scalars(p, b0, T);
    }
#pragma unroll 1
    for (int64_t blk = b0; blk < b1; ++blk) {
        if (!PF) load_rows<VT, K, KEEP>(p, blk, T, pc);
        const int64_t o0 = blk * p.out;
        const int64_t o1 = min(S, o0 + p.out);
        const int64_t e0 = o0 - (int64_t)T * p.hl;  // state of thread 0
        const int64_t s = e0 + tid;
        const bool in = s >= 0 && s < S;
        // each lane takes its own state's row out of its wavefront's pieces
        VT v[K];
#pragma unroll 1
        for (int r = 0; r < kRB / 64 / WR; ++r) {
            if (wid / WR == r) {
                char* my = stage + (wid % WR) * WB;
#pragma unroll
                for (int i = 0; i < NP; ++i) {
                    const int pp = lane + 64 * i;  // row pp / NP, piece pp % NP
                    *reinterpret_cast<dev::d2_t*>(my + 16 * (pp + pp / NP)) = pc[i];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    const dev::d2_t t = *reinterpret_cast<const dev::d2_t*>(my + 16 * (staged_stride<NP>() * lane + j));
                    __builtin_memcpy(&v[j * (16 / SZ)], &t, 16);
                }
            }
            __syncthreads();  // the next round reuses the staging area
        }
        const BlockScalars sc = PF ? sn : load_scalars(p, blk, T);
        const int w = sc.w;
        const double bo = sc.bo;
        const double dv = sc.dv;
        X[0][tid] = in ? sc.x : 0.0;
        // the next block's loads fly while this block sweeps
        if (PF && blk + 1 < b1) {
            load_rows<VT, K, KEEP>(p, blk + 1, T, pc);
            sn = load_scalars(p, blk + 1, T);
        }
        // exact range after sweep t: [lo0 + t hl, hi0 - t hr), but a range end at
        // the first or last state never moves (no state lies beyond it)
        const bool cut_lo = e0 > 0, cut_hi = e0 + kRB < S;
        const int64_t win = w - e0;  // the row's first column, relative to thread 0
        double racc = 0.0;
        int cur = 0;
#pragma unroll 1
        for (int t = 1; t <= T; ++t) {
            __syncthreads();
            const int64_t lo = cut_lo ? e0 + (int64_t)t * p.hl : 0;
            const int64_t hi = cut_hi ? e0 + kRB - (int64_t)t * p.hr : S;
            if (in && s >= lo && s < hi) {
                const double* xs = &X[cur][win];
                double yv = 0.0;
#pragma unroll
                for (int c = 0; c < K / FE; ++c) {
                    double x = 0.0;
#pragma unroll
                    for (int e = 0; e < FE; ++e) x = fma((double)v[c * FE + e], xs[c * FE + e], x);
                    yv += x;
                }
                const double xv = X[cur][tid];
                const double jx = xv - p.gamma * yv;
                const double r = bo - jx;
                const double pr = p.dinv ? r * dv : r;
                const double xn = xv + a * pr;
                X[cur ^ 1][tid] = xn;
                if (t == T && s >= o0 && s < o1) {
                    p.out_prev[s] = xv;
                    p.out_last[s] = xn;
                    racc = fma(r, r, racc);
                }
            }
            cur ^= 1;
        }
        // the block's sum in a fixed order: wave butterflies, then the waves in order
        racc = dev::wave_sum(racc);
        if ((tid & 63) == 0) red[tid >> 6] = racc;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int i = 0; i < kRB / 64; ++i) t += red[i];
            p.partials[blk] = t;
        }
        // X and red are rewritten by the next block (after its staging barriers)
    }
}

// A workgroup barrier for LDS traffic only: the wavefront's LDS operations
// complete (lgkmcnt), then it meets the others.  A __syncthreads would also
// wait for the direct global-to-LDS loads still in flight (they count as
// pending LDS writes), which are meant to run under the sweeps.  Every
// wavefront of the workgroup executes it the same number of times.
__device__ __forceinline__ void lds_only_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0); vmcnt and expcnt at their maxima (no wait)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// One state's product with its row's window x[win .. win + K), read as
// aligned 16-byte pieces from x[win - Q ..] (Q = win mod 2; for Q = 1 the
// piece past the window's end is read and unused).  Chunks of FE values
// summed with fused multiply-adds, chunk sums added in order: the one-sweep
// kernel's sum.
template <int K, int FE, int Q>
__device__ __forceinline__ double band_dot(const double (&v)[K], const dev::d2_t* xp) {
    dev::d2_t r[K / 2 + Q];
#pragma unroll
    for (int j = 0; j < K / 2 + Q; ++j) r[j] = xp[j];
    double yv = 0.0;
#pragma unroll
    for (int c = 0; c < K / FE; ++c) {
        double x = 0.0;
#pragma unroll
        for (int e = 0; e < FE; ++e) {
            const int i = c * FE + e + Q;
            x = fma(v[c * FE + e], (i & 1) ? r[i >> 1].y : r[i >> 1].x, x);
        }
        yv += x;
    }
    return yv;
}

// One 16-byte piece per lane from global memory straight into LDS, lane l's
// at lds + 16 l (global_load_lds_dwordx4; M0 holds the LDS base and is
// restored after the issue).  Issued from inline asm so that the compiler
// does not see a direct-to-LDS load in flight during the sweeps: when it
// does, it waits for all of a wavefront's window reads before the first
// multiply instead of for each piece as it is used.  The loads count in
// vmcnt like any global load; the kernel waits for them explicitly before a
// slot is read.
__device__ __forceinline__ void lds_dma16(const void* g, unsigned lds) {
    unsigned saved;
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %2\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %1, off\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(saved)
        : "v"(g), "s"(lds)
        : "memory");
}

__device__ __forceinline__ unsigned lds_addr(const void* p) {
    return (unsigned)(size_t)(const __attribute__((address_space(3))) char*)p;
}

template <int K, int SZ>
constexpr int lds_prefetch_waves() {
    constexpr int budget = 160 * 1024 - 2 * kRB * 8 - (kRB / 64) * 8 - 256;
    constexpr int wp = budget / (64 * 16 * staged_stride<K * SZ / 16>());
    return wp > kRB / 64 ? kRB / 64 : wp;
}

// Long rows (FP64 rows of 24 or 32 entries: a second copy in registers would
// spill) prefetched through LDS instead: persistent workgroups as in
// k_rich_block_pf, and during a block's sweeps the first WP wavefronts issue
// direct global-to-LDS loads (global_load_lds_dwordx4: lane l's 16 bytes land
// at base + 16 l) of their rows of the next block into their staging slots,
// which the sweeps do not touch.  At the next block each of them waits for
// its own loads, and after a barrier the threads whose rows are in these
// slots take them; then the other 16 - WP wavefronts load their rows the
// same way into the freed slots, and after another barrier the remaining
// threads take theirs.  No row passes through registers on its way to LDS,
// so a row is held once.  WP is the number of 64-row slots (rows padded as
// in staged_stride) that fit beside the sweep arrays in 160 KB of LDS.  The
// sweeps synchronise on LDS traffic only, so the loads in flight do not hold
// them up.  Same sums in the same order.
template <typename VT, int K, int FE, int T, bool KEEP>
__global__ __launch_bounds__(kRB) void k_rich_block_lds(RichBlockParams p) {
    if (p.ctrl->active == 0) return;
    constexpr int SZ = (int)sizeof(VT);
    constexpr int NP = K * SZ / 16;   // 16-byte pieces of a row
    constexpr int NPP = staged_stride<NP>();
    constexpr int WB = 64 * 16 * NPP;  // staged bytes of a wavefront's 64 rows
    constexpr int WP = lds_prefetch_waves<K, SZ>();
    constexpr int NW = kRB / 64;
    static_assert(WP >= NW - WP, "the other wavefronts must fit the freed slots");
    __shared__ double X[2][kRB];
    __shared__ double red[kRB / 64];
    __shared__ __align__(16) char stage[WP * WB];
    const int tid = threadIdx.x;
    const int wid = tid >> 6, lane = tid & 63;
    const int64_t S = p.S;
    const int64_t G = gridDim.x;
    const int64_t g = dev::xcd_remap(blockIdx.x, G);
    const int64_t b0 = g * p.nblk / G, b1 = (g + 1) * p.nblk / G;
    const double a = p.ctrl->omega;
    const char* vb = static_cast<const char*>(p.val);
    const int64_t lim = S * (int64_t)K * SZ - 16;
    // the wavefront's rows of block blk straight into slot `slot`, each row
    // NPP pieces apart: instruction i fills slots 64 i .. 64 i + 63 (lane
    // order) from global pieces q - q / NPP (a pad slot takes the next row's
    // first piece; it is never read).  A wavefront whose 64 states and the
    // next one lie in [0, S) (the last pad reads that state's first piece)
    // addresses its loads from one uniform base with 32-bit offsets; the
    // others clamp every offset into the array.
    auto load_slot = [&](int64_t blk, int slot) {
        const int64_t e0 = blk * p.out - (int64_t)T * p.hl;
        const int64_t ws = e0 + 64 * (int64_t)__builtin_amdgcn_readfirstlane(wid);
        char* my = stage + __builtin_amdgcn_readfirstlane(slot) * WB;  // uniform: scalar registers
        // the per-lane offsets are recomputed at each call (a few integer
        // operations) rather than kept live across the block loop, where
        // they would be spilled and their reloads would queue ahead of the
        // loads they address
        int ln = lane;
        asm volatile("" : "+v"(ln));
        if (ws >= 0 && ws + 64 < S) {
            const char* wb = vb + ws * (int64_t)K * SZ;
#pragma unroll
            for (int i = 0; i < NPP; ++i) {
                const unsigned q = (unsigned)ln + 64u * i;
                lds_dma16(wb + 16u * (q - q / NPP), lds_addr(my + 1024 * i));
            }
        } else {
            const int64_t wbase = ws * (int64_t)K * SZ;
#pragma unroll
            for (int i = 0; i < NPP; ++i) {
                const int q = ln + 64 * i;
                int64_t off = wbase + 16 * (int64_t)(q - q / NPP);
                off = off < 0 ? 0 : (off > lim ? lim : off);  // pieces of states outside [0, S) are never used
                lds_dma16(vb + off, lds_addr(my + 1024 * i));
            }
        }
    };
    // The thread's state, relative to the block: wavefront w computes the even
    // (w < 8) or odd states of [128 (w mod 8), 128 (w mod 8) + 128), so that
    // with a fixed offset between a row's first column and its state all
    // lanes of a wavefront share the parity of their windows and read them as
    // aligned 16-byte pieces, 16 bytes apart from lane to lane (no bank
    // conflicts).  Its row was loaded by wavefront jl, row jr of that slot.
    const int sig = 2 * (tid & (kRB / 2 - 1)) + tid / (kRB / 2);
    const int jl = sig >> 6, jr = sig & 63;
    // the thread's row out of a slot whose loads have landed and are visible
    // (float32 rows are widened to FP64 here, once per block, instead of at
    // every use in the sweeps: the same values)
    auto take_row = [&](int slot, double (&v)[K]) {
        const char* my = stage + slot * WB;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const char* src = my + 16 * (NPP * jr + j);
            if constexpr (SZ == 8) {
                const dev::d2_t t = *reinterpret_cast<const dev::d2_t*>(src);
                v[2 * j] = t.x;
                v[2 * j + 1] = t.y;
            } else {
                const dev::f4_t t = *reinterpret_cast<const dev::f4_t*>(src);
                v[4 * j] = (double)t.x;
                v[4 * j + 1] = (double)t.y;
                v[4 * j + 2] = (double)t.z;
                v[4 * j + 3] = (double)t.w;
            }
        }
    };
    // the thread's state's first column, rhs, Jacobi scale and delta entry,
    // loaded one block ahead with clamped indices (used as loaded only when
    // the loads have landed: nothing waits for them here)
    int w_n = 0;
    double bo_n = 0.0, dv_n = 1.0, x_n = 0.0;
    auto load_scalars_of = [&](int64_t blk) {
        const int64_t s = blk * p.out - (int64_t)T * p.hl + sig;
        const int64_t sc = s < 0 ? 0 : (s >= S ? S - 1 : s);  // clamped: every load in bounds
        w_n = p.band[sc];
        bo_n = p.b[sc];
        dv_n = p.dinv ? p.dinv[sc] : 1.0;
        x_n = p.x[sc];
    };
    double v[K];  // the state's row (FP64, or float32 widened)
    // Each block starts with its prefetched rows already taken and its other
    // rows and scalars in flight: for the first block here, for the others at
    // the end of the previous block, where these loads overlap its output
    // stores and residual sum.
    if (b0 < b1) {
        if (wid < WP) load_slot(b0, wid);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();  // each wavefront's loads into LDS have landed
        if (jl < WP) take_row(jl, v);
        __syncthreads();  // every prefetched slot has been read
        if (wid >= WP) load_slot(b0, wid - WP);
        load_scalars_of(b0);
    }
#pragma unroll 1
    for (int64_t blk = b0; blk < b1; ++blk) {
        const int64_t o0 = blk * p.out;
        const int64_t o1 = min(S, o0 + p.out);
        const int64_t e0 = o0 - (int64_t)T * p.hl;  // state of relative index 0
        const int64_t s = e0 + sig;
        const bool in = s >= 0 && s < S;
        // the rows of the other 16 - WP wavefronts and the scalars have landed
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (jl >= WP) take_row(jl - WP, v);
        __syncthreads();  // the slots are free for the next block's loads
        const int w = w_n;
        const double bo = bo_n, dv = dv_n;
        double xv = in ? x_n : 0.0;  // the state's own entry of the current iterate (0 outside [0, S))
        X[0][sig] = xv;
        if (wid < WP && blk + 1 < b1) load_slot(blk + 1, wid);
        // Offsets relative to the block, in 32 bits.  Exact range after sweep
        // t: [t hl, kRB - t hr), but a range end at the first or last state
        // never moves (no state lies beyond it).  The thread's state is in the
        // range at sweep t iff t <= tmax: a moving low end passes it after
        // sweep sig / hl, a moving high end after (kRB - 1 - sig) / hr, and a
        // fixed end keeps out the states beyond it at every sweep.
        const bool cut_lo = e0 > 0, cut_hi = e0 + kRB < S;
        const int first = (int)-e0, last = (int)(S - e0);
        // (recomputed per block: kept live across the block loop it would be
        // spilled, and its reload would sit in front of the first sweep)
        int sg = sig, hl = p.hl, hr = p.hr;
        asm volatile("" : "+v"(sg), "+s"(hl), "+s"(hr));
        int tmax = T;
        if (!in || (!cut_lo && sg < first) || (!cut_hi && sg >= last)) {
            tmax = 0;
        } else {
            if (cut_lo && hl > 0) tmax = min(tmax, sg / hl);
            if (cut_hi && hr > 0) tmax = min(tmax, (kRB - 1 - sg) / hr);
        }
        const bool own = sig >= (int)(o0 - e0) && sig < (int)(o1 - e0);  // the block's own states
        const int win = (int)(w - e0);  // the row's first column
        const int q = win & 1;
        const int half = (win - q) >> 1;  // first aligned piece of the window
        double racc = 0.0, xprev = xv;
        // one sweep reading buffer RD and writing the other; the last one also
        // keeps its input and the residual's square
        auto sweep = [&](auto RD, auto LAST, int t) {
            constexpr int rd = decltype(RD)::value;
            lds_only_barrier();
            if (t <= tmax) {
                const dev::d2_t* xp = reinterpret_cast<const dev::d2_t*>(&X[rd][0]) + half;
                const double yv = q ? band_dot<K, FE, 1>(v, xp) : band_dot<K, FE, 0>(v, xp);
                const double jx = xv - p.gamma * yv;
                const double r = bo - jx;
                const double pr = p.dinv ? r * dv : r;
                const double xn = xv + a * pr;
                X[rd ^ 1][sig] = xn;
                if constexpr (decltype(LAST)::value) {
                    xprev = xv;
                    if (own) racc = fma(r, r, 0.0);
                }
                xv = xn;
            }
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using NL = std::false_type;
        // sweep t reads buffer (t - 1) mod 2; T is even
#pragma unroll 1
        for (int t = 1; t + 1 < T; t += 2) {
            sweep(I0{}, NL{}, t);
            sweep(I1{}, NL{}, t + 1);
        }
        sweep(I0{}, NL{}, T - 1);
        sweep(I1{}, std::true_type{}, T);
        // the next block: its prefetched rows (landed during the sweeps) are
        // taken, then its other rows and its scalars are loaded while this
        // block's outputs are stored and its residual summed
        if (blk + 1 < b1) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (jl < WP) take_row(jl, v);
            __syncthreads();  // every prefetched slot has been read
            if (wid >= WP) load_slot(blk + 1, wid - WP);
            load_scalars_of(blk + 1);
        }
        // the last sweep's input and output on the block's own states
        if (own) {
            p.out_prev[s] = xprev;
            p.out_last[s] = xv;
        }
        racc = dev::wave_sum(racc);
        if ((tid & 63) == 0) red[tid >> 6] = racc;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int i = 0; i < kRB / 64; ++i) t += red[i];
            p.partials[blk] = t;
        }
    }
}

// Two states per thread.  A 512-thread workgroup owns the same kRB states,
// thread tid the adjacent states 2 tid and 2 tid + 1.  Their windows (with
// the fixed offset of band rows inside the chain) overlap in all but one
// entry, so 13 aligned 16-byte pieces (for rows of 24) serve both states and
// a sweep reads half the LDS bytes of one state per thread; the per-sweep
// work that is not arithmetic (range test, addresses, the write of the new
// entries, barrier) is shared by two states, and the registers of a
// 512-thread workgroup (256 per lane) hold both rows.  A wavefront's 128
// rows are staged as 64 pairs of rows, 2 NP + 1 pieces apart (an odd
// stride: no bank conflicts when each lane reads its pair), so each
// wavefront takes its own rows from its own slot.  Prefetching as in
// k_rich_block_lds: the first WP wavefronts load their next rows into LDS
// during the sweeps, the others into the freed slots at the block's start.
// Each state's sum is that of the one-sweep kernel.
constexpr int kRT = kRB / 2;  // threads of the two-state kernel

template <int K, int SZ>
constexpr int pair_stride() {
    return 2 * (K * SZ / 16) + 1;
}

template <int K, int SZ>
constexpr int pair_prefetch_waves() {
    constexpr int budget = 160 * 1024 - 2 * (kRB + 8) * 8 - (kRT / 64) * 8 - 256;
    constexpr int wp = budget / (64 * 16 * pair_stride<K, SZ>());
    return wp > kRT / 64 ? kRT / 64 : wp;
}

// the products of two adjacent states whose windows start at x[w] and
// x[w + 1], read as the K / 2 + 1 aligned pieces from x[w - Q] (Q = w mod 2)
template <int K, int FE, int Q>
__device__ __forceinline__ void pair_dot(const double (&va)[K], const double (&vb)[K], const dev::d2_t* xp,
                                         double& ya, double& yb) {
    dev::d2_t r[K / 2 + 1];
#pragma unroll
    for (int j = 0; j < K / 2 + 1; ++j) r[j] = xp[j];
    ya = 0.0;
    yb = 0.0;
#pragma unroll
    for (int c = 0; c < K / FE; ++c) {
        double xa = 0.0, xb = 0.0;
#pragma unroll
        for (int e = 0; e < FE; ++e) {
            const int i = c * FE + e, ia = i + Q, ib = i + 1 + Q;
            xa = fma(va[i], (ia & 1) ? r[ia >> 1].y : r[ia >> 1].x, xa);
            xb = fma(vb[i], (ib & 1) ? r[ib >> 1].y : r[ib >> 1].x, xb);
        }
        ya += xa;
        yb += xb;
    }
}

template <typename VT, int K, int FE, int T, bool KEEP>
__global__ __launch_bounds__(kRT) void k_rich_block_pair(RichBlockParams p) {
    if (p.ctrl->active == 0) return;
    constexpr int SZ = (int)sizeof(VT);
    constexpr int NP = K * SZ / 16;  // 16-byte pieces of a row
    constexpr int PS = pair_stride<K, SZ>();
    constexpr int WB = 64 * 16 * PS;  // staged bytes of a wavefront's 64 pairs of rows
    constexpr int WP = pair_prefetch_waves<K, SZ>();
    constexpr int NW = kRT / 64;
    constexpr int XO = 4;  // entries before each iterate buffer (window reads of states out of range)
    static_assert(WP >= NW - WP, "the other wavefronts must fit the freed slots");
    __shared__ __align__(16) double Xs[2][kRB + 2 * XO];
    __shared__ double red[NW];
    __shared__ __align__(16) char stage[WP * WB];
    const int tid = threadIdx.x;
    const int wid = tid >> 6, lane = tid & 63;
    const int64_t S = p.S;
    const int64_t G = gridDim.x;
    const int64_t g = dev::xcd_remap(blockIdx.x, G);
    const int64_t b0 = g * p.nblk / G, b1 = (g + 1) * p.nblk / G;
    const double a = p.ctrl->omega;
    const char* vbase = static_cast<const char*>(p.val);
    const int64_t lim = S * (int64_t)K * SZ - 16;
    // the wavefront's 128 rows of block blk into slot `slot`: instruction i
    // fills slot pieces 64 i .. 64 i + 63 (lane order), slot piece P from
    // global piece P - P / PS (a pair's pad piece takes the next pair's first
    // piece; it is never read).  Fast path as in k_rich_block_lds.
    auto load_slot = [&](int64_t blk, int slot) {
        const int64_t e0 = blk * p.out - (int64_t)T * p.hl;
        const int64_t ws = e0 + 128 * (int64_t)__builtin_amdgcn_readfirstlane(wid);
        char* my = stage + __builtin_amdgcn_readfirstlane(slot) * WB;
        int ln = lane;
        asm volatile("" : "+v"(ln));
        if (ws >= 0 && ws + 128 < S) {
            const char* wb = vbase + ws * (int64_t)K * SZ;
#pragma unroll
            for (int i = 0; i < PS; ++i) {
                const unsigned q = (unsigned)ln + 64u * i;
                lds_dma16(wb + 16u * (q - q / PS), lds_addr(my + 1024 * i));
            }
        } else {
            const int64_t wbase = ws * (int64_t)K * SZ;
#pragma unroll
            for (int i = 0; i < PS; ++i) {
                const int q = ln + 64 * i;
                int64_t off = wbase + 16 * (int64_t)(q - q / PS);
                off = off < 0 ? 0 : (off > lim ? lim : off);  // pieces of states outside [0, S) are never used
                lds_dma16(vbase + off, lds_addr(my + 1024 * i));
            }
        }
    };
    // the lane's two rows from its wavefront's slot (after the wavefront's
    // own loads have landed); float32 widened once per block
    auto take_pair = [&](int slot, double (&ra)[K], double (&rb)[K]) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const char* my = stage + slot * WB + 16 * PS * lane;
#pragma unroll
        for (int j = 0; j < 2 * NP; ++j) {
            double* dst = j < NP ? ra : rb;
            const int jj = j < NP ? j : j - NP;
            if constexpr (SZ == 8) {
                const dev::d2_t t = *reinterpret_cast<const dev::d2_t*>(my + 16 * j);
                dst[2 * jj] = t.x;
                dst[2 * jj + 1] = t.y;
            } else {
                const dev::f4_t t = *reinterpret_cast<const dev::f4_t*>(my + 16 * j);
                dst[4 * jj] = (double)t.x;
                dst[4 * jj + 1] = (double)t.y;
                dst[4 * jj + 2] = (double)t.z;
                dst[4 * jj + 3] = (double)t.w;
            }
        }
    };
    // both states' first columns, rhs, Jacobi scales and delta entries, one
    // block ahead with clamped indices (used as loaded after the next wait)
    int wa_n = 0, wb_n = 0;
    double ba_n = 0.0, bb_n = 0.0, da_n = 1.0, db_n = 1.0, xa_n = 0.0, xb_n = 0.0;
    auto load_scalars_of = [&](int64_t blk) {
        const int64_t sa = blk * p.out - (int64_t)T * p.hl + 2 * tid;
        const int64_t ca = sa < 0 ? 0 : (sa >= S ? S - 1 : sa);
        const int64_t cb = sa + 1 < 0 ? 0 : (sa + 1 >= S ? S - 1 : sa + 1);
        wa_n = p.band[ca];
        wb_n = p.band[cb];
        ba_n = p.b[ca];
        bb_n = p.b[cb];
        if (p.dinv) {
            da_n = p.dinv[ca];
            db_n = p.dinv[cb];
        }
        xa_n = p.x[ca];
        xb_n = p.x[cb];
    };
    double ra[K], rb[K];  // the two states' rows (FP64, or float32 widened)
    if (b0 < b1) {
        if (wid < WP) {
            load_slot(b0, wid);
            __builtin_amdgcn_s_waitcnt(0);
            take_pair(wid, ra, rb);
        }
        __syncthreads();  // every prefetched slot has been read
        if (wid >= WP) load_slot(b0, wid - WP);
        load_scalars_of(b0);
    }
#pragma unroll 1
    for (int64_t blk = b0; blk < b1; ++blk) {
        const int64_t o0 = blk * p.out;
        const int64_t o1 = min(S, o0 + p.out);
        const int64_t e0 = o0 - (int64_t)T * p.hl;  // state of relative index 0
        const int64_t sa = e0 + 2 * tid;            // the thread's first state
        const bool ina = sa >= 0 && sa < S, inb = sa + 1 >= 0 && sa + 1 < S;
        // the other wavefronts' rows and everyone's scalars have landed
        __builtin_amdgcn_s_waitcnt(0);
        if (wid >= WP) take_pair(wid - WP, ra, rb);
        __syncthreads();  // the slots are free for the next block's loads
        const int wa = wa_n, wbn = wb_n;
        const double ba = ba_n, bb = bb_n, da = da_n, db = db_n;
        double xa = ina ? xa_n : 0.0, xb = inb ? xb_n : 0.0;
        *reinterpret_cast<dev::d2_t*>(&Xs[0][XO + 2 * tid]) = dev::d2_t{xa, xb};
        if (wid < WP && blk + 1 < b1) load_slot(blk + 1, wid);
        // exact range after sweep t as in k_rich_block_lds; each state is in
        // it at sweep t iff t <= its tmax (computed per block: kept live
        // across the block loop it would be spilled)
        const bool cut_lo = e0 > 0, cut_hi = e0 + kRB < S;
        const int first = (int)-e0, last = (int)(S - e0);
        int sg = 2 * tid, hl = p.hl, hr = p.hr;
        asm volatile("" : "+v"(sg), "+s"(hl), "+s"(hr));
        auto tmax_of = [&](int sig, bool in) {
            int tm = T;
            if (!in || (!cut_lo && sig < first) || (!cut_hi && sig >= last)) return 0;
            if (cut_lo && hl > 0) tm = min(tm, sig / hl);
            if (cut_hi && hr > 0) tm = min(tm, (kRB - 1 - sig) / hr);
            return tm;
        };
        const int tma = tmax_of(sg, ina), tmb = tmax_of(sg + 1, inb);
        const int tml = max(tma, tmb);
        const int rlo = (int)(o0 - e0), rhi = (int)(o1 - e0);
        const bool owna = sg >= rlo && sg < rhi, ownb = sg + 1 >= rlo && sg + 1 < rhi;
        // windows relative to the block; both from one read when adjacent
        const int wina = (int)(wa - e0), winb = (int)(wbn - e0);
        const bool adj = winb == wina + 1;
        const int qa = wina & 1;
        const int hfa = (wina - qa) >> 1;
        // apart (rows at the chain's ends): each window on its own, clamped
        // into the buffer (only a state out of range reads beyond it)
        const int wca = min(max(wina, 0), kRB - K), wcb = min(max(winb, 0), kRB - K);
        const int qca = wca & 1, qcb = wcb & 1;
        const int hca = (wca - qca) >> 1, hcb = (wcb - qcb) >> 1;
        double racc = 0.0, xpa = xa, xpb = xb;
        auto sweep = [&](auto RD, auto LAST, int t) {
            constexpr int rd = decltype(RD)::value;
            lds_only_barrier();
            if (t <= tml) {
                const dev::d2_t* xb0 = reinterpret_cast<const dev::d2_t*>(&Xs[rd][XO]);
                double ya, yb;
                if (adj) {
                    if (qa) pair_dot<K, FE, 1>(ra, rb, xb0 + hfa, ya, yb);
                    else pair_dot<K, FE, 0>(ra, rb, xb0 + hfa, ya, yb);
                } else {
                    ya = qca ? band_dot<K, FE, 1>(ra, xb0 + hca) : band_dot<K, FE, 0>(ra, xb0 + hca);
                    yb = qcb ? band_dot<K, FE, 1>(rb, xb0 + hcb) : band_dot<K, FE, 0>(rb, xb0 + hcb);
                }
                const double jxa = xa - p.gamma * ya, jxb = xb - p.gamma * yb;
                const double rra = ba - jxa, rrb = bb - jxb;
                const double pra = p.dinv ? rra * da : rra, prb = p.dinv ? rrb * db : rrb;
                const double xna = xa + a * pra, xnb = xb + a * prb;
                *reinterpret_cast<dev::d2_t*>(&Xs[rd ^ 1][XO + 2 * tid]) = dev::d2_t{xna, xnb};
                if constexpr (decltype(LAST)::value) {
                    xpa = xa;
                    xpb = xb;
                    if (owna) racc = fma(rra, rra, racc);
                    if (ownb) racc = fma(rrb, rrb, racc);
                }
                xa = xna;
                xb = xnb;
            }
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using NL = std::false_type;
#pragma unroll 1
        for (int t = 1; t + 1 < T; t += 2) {
            sweep(I0{}, NL{}, t);
            sweep(I1{}, NL{}, t + 1);
        }
        sweep(I0{}, NL{}, T - 1);
        sweep(I1{}, std::true_type{}, T);
        // the next block's prefetched rows (landed during the sweeps), then
        // its other rows and its scalars, loaded while this block's outputs
        // are stored and its residual summed
        if (blk + 1 < b1) {
            if (wid < WP) {
                __builtin_amdgcn_s_waitcnt(0);
                take_pair(wid, ra, rb);
            }
            __syncthreads();  // every prefetched slot has been read
            if (wid >= WP) load_slot(blk + 1, wid - WP);
            load_scalars_of(blk + 1);
        }
        if (owna) {
            p.out_prev[sa] = xpa;
            p.out_last[sa] = xa;
        }
        if (ownb) {
            p.out_prev[sa + 1] = xpb;
            p.out_last[sa + 1] = xb;
        }
        racc = dev::wave_sum(racc);
        if (lane == 0) red[wid] = racc;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int i = 0; i < NW; ++i) t += red[i];
            p.partials[blk] = t;
        }
    }
}

// the two-state kernel fits (both rows in registers, half the wavefronts'
// next rows in LDS)
template <typename VT, int K>
constexpr bool rich_pair_fits() {
    return pair_prefetch_waves<K, (int)sizeof(VT)>() >= kRT / 64 - pair_prefetch_waves<K, (int)sizeof(VT)>() &&
           2 * K * (int)sizeof(VT) <= 384;
}

// Rows whose two copies (pieces in flight, values in use) fit the 128
// registers per lane of a 1024-thread workgroup run on the persistent
// prefetching kernel; longer rows (FP64 rows of 24 or 32 entries) on the
// persistent kernels that prefetch most wavefronts' next rows through LDS,
// or, when asked, on one block per workgroup.  Where the LDS-prefetching
// kernel is used (long rows, or rows whose every next row fits its stage),
// the two-state kernel takes its place when it fits (FP64 rows up to 24
// entries, float32 rows up to 32; 5 of 8 wavefronts prefetched for FP64
// rows of 24, all for float32 rows of 24).  All form the same sums in the
// same order.
template <typename VT, int K>
constexpr bool rich_prefetch() {
    return K * (int)sizeof(VT) <= 128;
}

// every wavefront's next rows fit the LDS stage of the LDS-prefetching kernel
template <typename VT, int K>
constexpr bool rich_lds_all() {
    return lds_prefetch_waves<K, (int)sizeof(VT)>() == kRB / 64;
}

template <typename VT, int K>
constexpr bool rich_pair() {
    return rich_pair_fits<VT, K>() && (rich_lds_all<VT, K>() || !rich_prefetch<VT, K>());
}

template <typename VT, int K, int FE, bool KEEP>
void launch_t(const RichBlockParams& p, int T, hipStream_t st) {
    if constexpr (rich_pair<VT, K>()) {
        if (p.lds_prefetch) {
            const int nb = (int)std::min<int64_t>(p.nblk, device_cus());
            if (T == 16) hipLaunchKernelGGL((k_rich_block_pair<VT, K, FE, 16, KEEP>), dim3(nb), dim3(kRT), 0, st, p);
            else if (T == 8) hipLaunchKernelGGL((k_rich_block_pair<VT, K, FE, 8, KEEP>), dim3(nb), dim3(kRT), 0, st, p);
            else hipLaunchKernelGGL((k_rich_block_pair<VT, K, FE, 4, KEEP>), dim3(nb), dim3(kRT), 0, st, p);
            return;
        }
    }
    if (p.lds_prefetch && rich_lds_all<VT, K>()) {
        const int nb = (int)std::min<int64_t>(p.nblk, device_cus());
        if (T == 16) hipLaunchKernelGGL((k_rich_block_lds<VT, K, FE, 16, KEEP>), dim3(nb), dim3(kRB), 0, st, p);
        else if (T == 8) hipLaunchKernelGGL((k_rich_block_lds<VT, K, FE, 8, KEEP>), dim3(nb), dim3(kRB), 0, st, p);
        else hipLaunchKernelGGL((k_rich_block_lds<VT, K, FE, 4, KEEP>), dim3(nb), dim3(kRB), 0, st, p);
        return;
    }
    if constexpr (rich_prefetch<VT, K>()) {
        const int nb = (int)std::min<int64_t>(p.nblk, device_cus());
        if (T == 16) hipLaunchKernelGGL((k_rich_block_pf<VT, K, FE, 16, KEEP, true>), dim3(nb), dim3(kRB), 0, st, p);
        else if (T == 8) hipLaunchKernelGGL((k_rich_block_pf<VT, K, FE, 8, KEEP, true>), dim3(nb), dim3(kRB), 0, st, p);
        else hipLaunchKernelGGL((k_rich_block_pf<VT, K, FE, 4, KEEP, true>), dim3(nb), dim3(kRB), 0, st, p);
    } else if (p.lds_prefetch) {
        const int nb = (int)std::min<int64_t>(p.nblk, device_cus());
        if (T == 16) hipLaunchKernelGGL((k_rich_block_lds<VT, K, FE, 16, KEEP>), dim3(nb), dim3(kRB), 0, st, p);
        else if (T == 8) hipLaunchKernelGGL((k_rich_block_lds<VT, K, FE, 8, KEEP>), dim3(nb), dim3(kRB), 0, st, p);
        else hipLaunchKernelGGL((k_rich_block_lds<VT, K, FE, 4, KEEP>), dim3(nb), dim3(kRB), 0, st, p);
    } else {
        const int nb = (int)p.nblk;
        if (T == 16) hipLaunchKernelGGL((k_rich_block<VT, K, FE, 16, KEEP>), dim3(nb), dim3(kRB), 0, st, p);
        else if (T == 8) hipLaunchKernelGGL((k_rich_block<VT, K, FE, 8, KEEP>), dim3(nb), dim3(kRB), 0, st, p);
        else hipLaunchKernelGGL((k_rich_block<VT, K, FE, 4, KEEP>), dim3(nb), dim3(kRB), 0, st, p);
    }
}

template <typename VT, int K, int FE>
void launch_keep(const RichBlockParams& p, bool keep, int T, hipStream_t st) {
    if (keep) launch_t<VT, K, FE, true>(p, T, st);
    else launch_t<VT, K, FE, false>(p, T, st);
}

template <typename VT, int FE>
void launch_k(const RichBlockParams& p, bool keep, int k, int T, hipStream_t st) {
    switch (k) {
        case 8: launch_keep<VT, 8, FE>(p, keep, T, st); break;
        case 16: launch_keep<VT, 16, FE>(p, keep, T, st); break;
        case 24: launch_keep<VT, 24, FE>(p, keep, T, st); break;
        case 32: launch_keep<VT, 32, FE>(p, keep, T, st); break;
        default: throw Error(IPI_E_INVALID_ARG, "blocked sweeps need rows of 8, 16, 24 or 32 entries");
    }
}

// Halo widths of the blocked sweeps.  Block b covers [e0, e0 + kRB) with
// e0 = b out - T hl, out = kRB - T (hl + hr); after sweep t its exact range
// is [e0 + t hl, e0 + kRB - t hr) (an end at 0 or S stays put).  The bounds
// over all rows are always safe.  The interior bounds (rows of the states in
// [H, S - H), H the largest reach of any row) are smaller when the band
// windows are clamped at the edges and reach further there (the birth-death
// chain: 23 and 23 over all rows, 12 and 11 inside), and they are safe when
// no edge state comes within H of a moving end of any block's exact range:
//   moving low end  (e0 > 0):        e0 >= H and e0 + T hl + 2 H <= S
//   moving high end (e0 + kRB < S):  e0 + kRB <= S - H and e0 + kRB - T hr >= 2 H
// Then every state a range end passes reads only the interior halos, and an
// edge state inside a range reads within it.  Same arithmetic per state
// either way, so the same iterates; the interior halos only widen each
// block's output (fewer blocks, fewer halo rows read twice).
struct Halo {
    int hl, hr;
};

Halo rich_halos(const PpiView& P, int T) {
    const Halo all{P.band_hl, P.band_hr};
    const Halo in{P.band_hl_in, P.band_hr_in};
    if (in.hl >= all.hl && in.hr >= all.hr) return all;
    const int64_t H = std::max(all.hl, all.hr);
    const int64_t out = kRB - (int64_t)T * (in.hl + in.hr);
    if (out < kRB / 2) return all;
    const int64_t S = P.S;
    const int64_t nblk = (S + out - 1) / out;
    // e0 grows with b, so each condition holds for every block of its set
    // when it holds at the set's first and last block
    auto ok = [&](int64_t b) {
        const int64_t e0 = b * out - (int64_t)T * in.hl;
        if (e0 > 0 && (e0 < H || e0 + (int64_t)T * in.hl + 2 * H > S)) return false;
        if (e0 + kRB < S && (e0 + kRB > S - H || e0 + kRB - (int64_t)T * in.hr < 2 * H)) return false;
        return true;
    };
    int64_t b_lo = 0;  // first block with a moving low end
    while (b_lo < nblk && b_lo * out - (int64_t)T * in.hl <= 0) ++b_lo;
    int64_t b_hi = nblk - 1;  // last block with a moving high end
    while (b_hi >= 0 && b_hi * out - (int64_t)T * in.hl + kRB >= S) --b_hi;
    for (int64_t b : {(int64_t)0, b_lo, b_hi, nblk - 1})
        if (b >= 0 && b < nblk && !ok(b)) return all;
    return in;
}

int out_per_block(const PpiView& P, int T) {
    const Halo h = rich_halos(P, T);
    return kRB - T * (h.hl + h.hr);
}

}  // namespace

bool rich_block_ok(const PpiView& P, int T) {
    const bool k_ok = P.k == 8 || P.k == 16 || P.k == 24 || P.k == 32;
    const int fe = P.fp32 ? 4 : 2;
    // the chunk width must be the one-sweep kernel's, so the sums agree
    return P.band && k_ok && P.flat_e == fe && P.rp == nullptr && (T == 4 || T == 8 || T == 16) &&
           out_per_block(P, T) >= kRB / 2;
}

int rich_block_grid(const PpiView& P, int T) {
    const int64_t out = out_per_block(P, T);
    return (int)((P.S + out - 1) / out);
}

void k_launch_rich_block(const PpiView& P, int T, const double* b, const double* x, double* out_prev, double* out_last,
                         double* partials, Ctrl* c, hipStream_t st) {
    IPI_REQUIRE(rich_block_ok(P, T), IPI_E_INVALID_ARG, "blocked sweeps do not apply to this P_pi");
    const Halo h = rich_halos(P, T);
    const int out = kRB - T * (h.hl + h.hr);
    const int nblk = (int)((P.S + out - 1) / out);
    RichBlockParams p{P.val, P.band, b, x, P.dinv, out_prev, out_last, partials, c, P.gamma, P.S,
                      h.hl, h.hr, out, (int64_t)nblk, P.lds_prefetch};
    if (P.fp32) launch_k<float, 4>(p, P.keep_block, P.k, T, st);
    else launch_k<double, 2>(p, P.keep_block, P.k, T, st);
    IPI_HIP(hipGetLastError());
}

}  // namespace ipi
