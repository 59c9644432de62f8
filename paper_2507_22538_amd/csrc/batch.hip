// Batched iPI: many independent MDPs advanced together in rounds.
//
// Every member runs its own Algorithm 1 state machine (Bellman pass -> inner
// GMRES or Richardson -> update -> Bellman ...) as a sequence of phases.  A
// phase is split into tiles of states.  One round is three launches:
//   k_bwork  the current phase of every member, tile by tile; the grid walks
//            the concatenated tile list (member m owns items off[m] ..
//            off[m+1]-1), each workgroup a contiguous run of it, and writes
//            one set of partial sums per tile;
//   k_bfin   one workgroup per member: the fixed-order sum of its tile
//            partials, the scalar step (Givens rotation, forcing test, outer
//            stopping test), the next phase and its tile count;
//   k_bscan  the exclusive scan of the tile counts.
// Every member advances by one phase per round, small and large ones side by
// side.  The kernel boundaries order all memory traffic between phases, so
// no workgroup ever fences, spins or waits on another one: on gfx950 a
// device-scope fence writes back the XCD's L2, which made a persistent
// claim-and-signal design fence-bound.  Results do not depend on the other
// members (tile sums are reduced in tile order by the member's own
// finaliser).
//
// BatchEngine keeps the descriptors and states in slots of a fixed-capacity
// table in device memory, so the chunk of 32 rounds is captured once per
// kernel mix and replayed.  Between chunks the host reads the states back:
// a member whose state reached the end leaves (its slot is freed), and new
// members join free slots (their tiles enter at the next scan).  The
// serving loop uses this for continuous batching; ipi_solve_batch adds all
// members at once and runs until every one has left.
//
// Rows of one length get a compact P_pi (phase EXT) that the inner products
// stream; other rows are gathered in place (rows s*A + pi(s) of P).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "device.hpp"
#include "krylov_tiled.hpp"

namespace ipi {

namespace {

constexpr int kBMJ = 32;          // largest GMRES restart in a batch
constexpr int kBTileStates = 256; // states per tile of the vector phases
constexpr int kBMaxRows = 1024;   // rows per tile of the Bellman phase
constexpr int kBChunk = 1024;     // LDS slots for element products (uniform rows)

enum Phase : int32_t {
    PH_BELL = 0,
    PH_INIT = 1,
    PH_ARN = 2,
    PH_ORTH = 3,
    PH_UPD = 4,
    PH_RES = 5,
    PH_RICH = 6,
    PH_RAXPY = 7,
    PH_OUT = 8,
    PH_DONE = 9,
    PH_EXT = 10  // compact P_pi (uniform rows): row s*A + pi(s) copied to s*k
};

struct BDesc {
    const void* row_ptr;
    const int* col;
    const double* val;
    const float* val32;
    const double* g;
    int64_t S;
    int64_t nnz;
    int kuni;       // row length when every row has the same length, else 0
    int* ell_col;   // compact P_pi (kuni > 0): row s at s*kuni
    void* ell_val;  // double, or float in the mixed mode
    int A;
    int rp32;
    int fp32;       // float32 P values (mixed modes)
    int bell64;     // fp32_inner: the Bellman phase reads the FP64 values
    int lanes;      // lanes per row of the Bellman and product phases
    int spt_b;      // states per Bellman tile
    int nt_b;       // Bellman tiles
    int nt_v;       // vector-phase tiles
    int inner;      // IPI_INNER_GMRES or IPI_INNER_RICHARDSON
    int restart;
    int max_outer;
    int max_inner;
    double gamma;
    double atol, rtol_cert, alpha, omega;
    double* Va;
    double* Vb;
    double* b;
    double* d0;
    double* d1;
    double* basis;
    double* small;
    int32_t* pi;
    double* part;
    double* V_out;
    int32_t* pi_out;
};

struct BState {
    int32_t phase;
    int32_t j;
    int32_t cur;
    int32_t outer;
    int32_t first_cycle;
    int32_t status;
    int32_t pad_;
    int64_t inner_total;
    double rho;
    double vmax;
    double alg_bytes;
    int32_t ntiles;  // tiles of the current phase (0: done)
    int32_t pad2_;
    Ctrl c;
};

__device__ __forceinline__ double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

// next phase ph with nt tiles (finaliser, thread 0)
__device__ __forceinline__ void open_phase(BState* st, int32_t ph, int nt) {
    st->phase = ph;
    st->ntiles = nt;
}

// sum over one block, all threads get the total
__device__ __forceinline__ double bsum(double x, double* red) { return dev::block_sum(x, red); }

// ---------------------------------------------------------------------------
// tile bodies
// ---------------------------------------------------------------------------

// out[r] = sum_e val[(row0 + r) k + e] * x[col[(row0 + r) k + e]], r < nrows,
// for rows of one length k: coalesced element loads (consecutive threads,
// consecutive nonzeros) in chunks of whole rows that fill at most kBChunk
// LDS slots, then each row adds its k products in order.  Ends synced.
template <typename VT>
__device__ __forceinline__ void rows_uniform(const VT* __restrict__ val, const int* __restrict__ col, const double* __restrict__ x,
                             int64_t row0, int nrows, int k, double* out, double* cp) {
    const int rpc = max(1, kBChunk / k);
    for (int r0 = 0; r0 < nrows; r0 += rpc) {
        const int nr = min(rpc, nrows - r0);
        const int ne = nr * k;
        const int64_t base = (row0 + r0) * (int64_t)k;
#pragma unroll 4
        for (int c = threadIdx.x; c < ne; c += blockDim.x)
            cp[c] = (double)dev::ldnt(val + base + c) * x[dev::ldnt(col + base + c)];
        __syncthreads();
        for (int r = threadIdx.x; r < nr; r += blockDim.x) {
            double t = 0.0;
            for (int e = 0; e < k; ++e) t += cp[r * k + e];
            out[r0 + r] = t;
        }
        __syncthreads();
    }
}

// compact P_pi rows of one tile of states (uniform rows)
template <typename VT>
__device__ __forceinline__ void ext_tile(const BDesc& d, int t) {
    const int64_t s0 = (int64_t)t * kBTileStates;
    const int ns = (int)min((int64_t)kBTileStates, d.S - s0);
    const int k = d.kuni;
    const VT* __restrict__ val = sizeof(VT) == 4 ? (const VT*)d.val32 : (const VT*)d.val;
    VT* __restrict__ ev = (VT*)d.ell_val;
    const int ne = ns * k;
    for (int c = threadIdx.x; c < ne; c += blockDim.x) {
        const int ls = c / k, e = c - ls * k;
        const int64_t s = s0 + ls;
        const int64_t src = (s * d.A + d.pi[s]) * (int64_t)k + e;
        const int64_t dst = s * (int64_t)k + e;
        d.ell_col[dst] = d.col[src];
        ev[dst] = val[src];
    }
}

template <typename VT, typename PT, int L>
__device__ __forceinline__ void bell_tile(const BDesc& d, const BState* st, int t, double* q, int64_t* rp, double* red,
                          double* part_out, double* cp) {
    const int64_t s0 = (int64_t)t * d.spt_b;
    const int ns = (int)min((int64_t)d.spt_b, d.S - s0);
    const int A = d.A, R = ns * A;
    const int64_t r0 = s0 * A;
    const PT* __restrict__ rowp = (const PT*)d.row_ptr;
    const VT* __restrict__ val = sizeof(VT) == 4 ? (const VT*)d.val32 : (const VT*)d.val;
    const double* __restrict__ V = st->cur ? d.Vb : d.Va;
    if (d.kuni > 0) {
        rows_uniform<VT>(val, d.col, V, r0, R, d.kuni, q, cp);
        for (int i = threadIdx.x; i < R; i += blockDim.x) q[i] = d.g[r0 + i] + d.gamma * q[i];
        __syncthreads();
    } else {
        for (int i = threadIdx.x; i <= R; i += blockDim.x) rp[i] = (int64_t)rowp[r0 + i];
        for (int i = threadIdx.x; i < R; i += blockDim.x) q[i] = d.g[r0 + i];
        __syncthreads();
        constexpr int G = 256 / L;
        const int grp = threadIdx.x / L, lane = threadIdx.x % L;
        for (int rr = grp; rr < R; rr += G) {
            const int64_t b = rp[rr], e = rp[rr + 1];
            double acc = 0.0;
            for (int64_t j = b + lane; j < e; j += L) acc = fma((double)val[j], V[d.col[j]], acc);
            acc = dev::group_sum<L>(acc);
            if (lane == 0) q[rr] = q[rr] + d.gamma * acc;
        }
        __syncthreads();
    }
    double mx = 0.0, vx = 0.0;
    for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
        const double* qs = q + ls * A;
        double best = qs[0];
        int arg = 0;
        for (int a = 1; a < A; ++a)
            if (qs[a] < best) {
                best = qs[a];
                arg = a;
            }
        const int64_t s = s0 + ls;
        d.pi[s] = arg;
        const double res = best - V[s];
        d.b[s] = res;
        mx = nanmax(mx, fabs(res));
        vx = nanmax(vx, fabs(V[s]));
    }
    for (int off = 32; off >= 1; off >>= 1) {
        mx = nanmax(mx, __shfl_xor(mx, off, 64));
        vx = nanmax(vx, __shfl_xor(vx, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = mx;
        red[4 + (threadIdx.x >> 6)] = vx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part_out[0] = nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3]));
        part_out[1] = nanmax(nanmax(red[4], red[5]), nanmax(red[6], red[7]));
    }
    __syncthreads();
}

// y[ls] = (P_pi x)[s0 + ls], rows s*A + pi(s) gathered in place
template <typename VT, typename PT, int L>
__device__ __forceinline__ void ppi_tile(const BDesc& d, const double* __restrict__ x, int64_t s0, int ns, double* y, double* cp) {
    if (d.kuni > 0) {  // compact P_pi
        rows_uniform<VT>((const VT*)d.ell_val, d.ell_col, x, s0, ns, d.kuni, y, cp);
        return;
    }
    const PT* __restrict__ rowp = (const PT*)d.row_ptr;
    const VT* __restrict__ val = sizeof(VT) == 4 ? (const VT*)d.val32 : (const VT*)d.val;
    constexpr int G = 256 / L;
    const int grp = threadIdx.x / L, lane = threadIdx.x % L;
    for (int ls = grp; ls < ns; ls += G) {
        const int64_t s = s0 + ls;
        const int64_t r = s * d.A + d.pi[s];
        const int64_t b = rowp[r], e = rowp[r + 1];
        double acc = 0.0;
        for (int64_t j = b + lane; j < e; j += L) acc = fma((double)val[j], x[d.col[j]], acc);
        acc = dev::group_sum<L>(acc);
        if (lane == 0) y[ls] = acc;
    }
    __syncthreads();
}

template <typename VT, typename PT, int L>
__device__ __forceinline__ void vec_tile(const BDesc& d, const BState* st, int ph, int t, double* y, double* ylds, double* red,
                         double* part_out, double* cp) {
    const int64_t S = d.S;
    const int64_t s0 = (int64_t)t * kBTileStates;
    const int ns = (int)min((int64_t)kBTileStates, S - s0);
    const double gamma = d.gamma;
    const double* V = st->cur ? d.Vb : d.Va;
    double* Vn = st->cur ? d.Va : d.Vb;
    // one state per thread (kBTileStates == blockDim.x); acc0 is the phase's
    // single partial sum, the Arnoldi dots are reduced one by one below
    double acc0 = 0.0;
    int nred = 1;
    if (ph == PH_INIT) {
        for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
            const double r = d.b[s0 + ls];
            d.basis[s0 + ls] = r;
            acc0 = fma(r, r, acc0);
        }
    } else if (ph == PH_ARN) {
        const int j = st->j;
        const double* uj = d.basis + (size_t)j * S;
        double* un = d.basis + (size_t)(j + 1) * S;
        const double cj = d.small[kOffSC + j];
        ppi_tile<VT, PT, L>(d, uj, s0, ns, ylds, cp);
        const int ls = threadIdx.x;
        const int64_t s = s0 + ls;
        double w = 0.0;
        if (ls < ns) {
            w = cj * (uj[s] - gamma * ylds[ls]);
            un[s] = w;
        }
        // dots <u_i, w> for i <= j: per-wave butterflies, then the 4 wave
        // sums in the fixed order of block_sum; ylds is reused once every
        // thread has read its product value
        __syncthreads();
        const int wid = threadIdx.x >> 6;
        for (int i = 0; i <= j; ++i) {
            double v = ls < ns ? d.basis[(size_t)i * S + s] * w : 0.0;
            v = dev::wave_sum(v);
            if ((threadIdx.x & 63) == 0) ylds[4 * i + wid] = v;
        }
        __syncthreads();
        if ((int)threadIdx.x <= j) {
            const double* p4 = ylds + 4 * threadIdx.x;
            part_out[threadIdx.x] = (p4[0] + p4[1]) + (p4[2] + p4[3]);
        }
        __syncthreads();
        return;
    } else if (ph == PH_ORTH) {
        const int j = st->j;
        if ((int)threadIdx.x <= j) y[threadIdx.x] = d.small[kOffH + (size_t)j * kLdH + threadIdx.x] * d.small[kOffSC + threadIdx.x];
        __syncthreads();
        double* w = d.basis + (size_t)(j + 1) * S;
        for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
            const int64_t s = s0 + ls;
            double x = w[s];
#pragma unroll 8
            for (int i = 0; i <= j; ++i) x = fma(-y[i], d.basis[(size_t)i * S + s], x);
            w[s] = x;
            acc0 = fma(x, x, acc0);
        }
    } else if (ph == PH_UPD) {
        const int n = st->c.j;
        if (threadIdx.x == 0) {
            const double* H = d.small + kOffH;
            for (int i = n - 1; i >= 0; --i) {
                double tt = d.small[kOffGV + i];
                for (int l = i + 1; l < n; ++l) tt -= H[(size_t)l * kLdH + i] * y[l];
                y[i] = tt / H[(size_t)i * kLdH + i];
            }
            for (int i = 0; i < n; ++i) y[i] *= d.small[kOffSC + i];
        }
        __syncthreads();
        const bool first = st->first_cycle != 0;
        for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
            const int64_t s = s0 + ls;
            double dl = first ? 0.0 : d.d0[s];
#pragma unroll 8
            for (int i = 0; i < n; ++i) dl = fma(y[i], d.basis[(size_t)i * S + s], dl);
            d.d0[s] = dl;
            Vn[s] = V[s] + dl;
        }
        nred = 0;
    } else if (ph == PH_RES) {
        ppi_tile<VT, PT, L>(d, d.d0, s0, ns, ylds, cp);
        for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
            const int64_t s = s0 + ls;
            const double r = d.b[s] - (d.d0[s] - gamma * ylds[ls]);
            d.basis[s] = r;
            acc0 = fma(r, r, acc0);
        }
    } else if (ph == PH_RICH) {
        const int i = st->j;
        const double omega = d.omega;
        if (i == 0) {
            for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
                const int64_t s = s0 + ls;
                const double r = d.b[s];
                d.d1[s] = omega * r;
                acc0 = fma(r, r, acc0);
            }
        } else {
            const double* dp = (i & 1) ? d.d1 : d.d0;
            double* dq = (i & 1) ? d.d0 : d.d1;
            ppi_tile<VT, PT, L>(d, dp, s0, ns, ylds, cp);
            for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
                const int64_t s = s0 + ls;
                const double r = d.b[s] - (dp[s] - gamma * ylds[ls]);
                dq[s] = dp[s] + omega * r;
                acc0 = fma(r, r, acc0);
            }
        }
    } else if (ph == PH_RAXPY) {
        const int rb = st->c.result_buf;
        const double* dd = rb == 0 ? d.d0 : d.d1;
        for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
            const int64_t s = s0 + ls;
            Vn[s] = rb < 0 ? V[s] : V[s] + dd[s];
        }
        nred = 0;
    } else if (ph == PH_OUT) {
        for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
            const int64_t s = s0 + ls;
            d.V_out[s] = V[s];
            d.pi_out[s] = d.pi[s];
        }
        nred = 0;
    }
    // per-tile partial, tile-major: part[t * (kBMJ + 1)]
    if (nred > 0) {
        const double tsum = bsum(acc0, red);
        if (threadIdx.x == 0) part_out[0] = tsum;
    }
}

// reduce partial i over the tiles of the completed phase, fixed order
__device__ double tiles_sum(const double* part, int nt, int i, double* red) {
    double s = 0.0;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) s += part[(size_t)t * (kBMJ + 1) + i];
    return bsum(s, red);
}

__device__ double tiles_max(const double* part, int nt, int i, double* red) {
    double m = 0.0;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) m = nanmax(m, part[(size_t)t * (kBMJ + 1) + i]);
    for (int off = 32; off >= 1; off >>= 1) m = nanmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    const double r = nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3]));
    __syncthreads();
    return r;
}

// algorithmic bytes of one phase of member d (the counts of the single-MDP
// solver: P_pi rows gathered in place add their row pointers and pi)
__device__ double phase_bytes(const BDesc& d, int ph, int j, int n_upd, bool first) {
    const double S = (double)d.S, vb = 8.0 * S;
    const double bv = (d.fp32 && !(ph == PH_BELL && d.bell64)) ? 4.0 : 8.0, bp = d.rp32 ? 4.0 : 8.0;
    const double nnz = (double)d.nnz;
    const double prod = d.kuni > 0 ? S * d.kuni * (bv + 4.0) : nnz / d.A * (bv + 4.0) + S * (2.0 * bp + 4.0);
    switch (ph) {
        case PH_EXT: return 4.0 * S + 2.0 * S * d.kuni * (bv + 4.0);
        case PH_BELL:
            return nnz * (bv + 4.0) + (d.kuni > 0 ? 0.0 : (S * d.A + 1.0) * bp) + 8.0 * S * d.A + vb + 12.0 * S;
        case PH_INIT: return 2.0 * vb;
        case PH_ARN: return prod + (j + 2) * vb;
        case PH_ORTH: return (j + 3) * vb;
        case PH_UPD: return n_upd * vb + (first ? 0.0 : vb) + 3.0 * vb;
        case PH_RES: return prod + 3.0 * vb;
        case PH_RICH: return j == 0 ? 2.0 * vb : prod + 3.0 * vb;
        case PH_RAXPY: return 3.0 * vb;
        case PH_OUT: return 12.0 * S;
        default: return 0.0;
    }
}

// finaliser of member d's completed phase (whole block; thread 0 decides)
__device__ void finalize(const BDesc& d, BState* st, double* red) {
    const int ph = st->phase;
    const int nt = st->ntiles;
    Ctrl* c = &st->c;
    if (threadIdx.x == 0) st->alg_bytes += phase_bytes(d, ph, st->j, c->j, st->first_cycle != 0);
    if (ph == PH_BELL) {
        const double rho = tiles_max(d.part, nt, 0, red);
        const double vmax = tiles_max(d.part, nt, 1, red);
        if (threadIdx.x == 0) {
            st->rho = rho;
            st->vmax = vmax;
            if (!isfinite(rho) || !isfinite(vmax)) {
                st->status = IPI_E_NUMERICAL;
                open_phase(st, PH_OUT, d.nt_v);
            } else if (rho <= d.atol || (d.rtol_cert > 0.0 && rho <= d.rtol_cert * (1.0 - d.gamma) * vmax)) {
                st->status = IPI_OK;
                open_phase(st, PH_OUT, d.nt_v);
            } else if (st->outer >= d.max_outer) {
                st->status = IPI_E_NOT_CONVERGED;
                open_phase(st, PH_OUT, d.nt_v);
            } else {
                c->active = 1;
                c->j = 0;
                c->steps_total = 0;
                c->converged = 0;
                c->max_inner = d.max_inner;
                c->restart = d.restart;
                c->result_buf = 0;
                c->breakdown = 0;
                c->target = d.alpha * rho;
                c->omega = d.omega;
                st->first_cycle = 1;
                st->j = 0;
                if (d.kuni > 0) open_phase(st, PH_EXT, d.nt_v);
                else open_phase(st, d.inner == IPI_INNER_GMRES ? PH_INIT : PH_RICH, d.nt_v);
            }
        }
        return;
    }
    if (ph == PH_EXT) {
        if (threadIdx.x == 0) open_phase(st, d.inner == IPI_INNER_GMRES ? PH_INIT : PH_RICH, d.nt_v);
        return;
    }
    if (ph == PH_INIT || ph == PH_RES) {
        const double s = tiles_sum(d.part, nt, 0, red);
        if (threadIdx.x == 0) {
            tiled::cycle_start(d.small, c, sqrt(s));
            st->j = 0;
            open_phase(st, c->active ? PH_ARN : PH_UPD, d.nt_v);
        }
        return;
    }
    if (ph == PH_ARN) {
        const int j = st->j;
        for (int i = 0; i <= j; ++i) {
            const double s = tiles_sum(d.part, nt, i, red);
            if (threadIdx.x == 0) d.small[kOffH + (size_t)j * kLdH + i] = s * d.small[kOffSC + i];
        }
        if (threadIdx.x == 0) open_phase(st, PH_ORTH, d.nt_v);
        return;
    }
    if (ph == PH_ORTH) {
        const double s = tiles_sum(d.part, nt, 0, red);
        if (threadIdx.x == 0) {
            const int j = st->j;
            tiled::givens_step(d.small, c, j, sqrt(s));
            if (c->active) {
                st->j = j + 1;
                open_phase(st, PH_ARN, d.nt_v);
            } else {
                open_phase(st, PH_UPD, d.nt_v);
            }
        }
        return;
    }
    if (ph == PH_UPD) {
        if (threadIdx.x == 0) {
            st->first_cycle = 0;
            if (c->converged || c->steps_total >= c->max_inner) {
                st->inner_total += c->steps_total;
                st->cur ^= 1;
                st->outer += 1;
                open_phase(st, PH_BELL, d.nt_b);
            } else {
                open_phase(st, PH_RES, d.nt_v);
            }
        }
        return;
    }
    if (ph == PH_RICH) {
        const double s = tiles_sum(d.part, nt, 0, red);
        if (threadIdx.x == 0) {
            const double r = sqrt(s);
            const int i = st->j;
            c->resid = r;
            if (r < c->target) {
                c->converged = 1;
                c->result_buf = i == 0 ? -1 : (i & 1);
                c->active = 0;
            } else {
                c->steps_total = i + 1;
                c->result_buf = (i + 1) & 1;
                if (c->steps_total >= c->max_inner) c->active = 0;
            }
            if (c->active) {
                st->j = i + 1;
                open_phase(st, PH_RICH, d.nt_v);
            } else {
                open_phase(st, PH_RAXPY, d.nt_v);
            }
        }
        return;
    }
    if (ph == PH_RAXPY) {
        if (threadIdx.x == 0) {
            st->inner_total += c->steps_total;
            st->cur ^= 1;
            st->outer += 1;
            open_phase(st, PH_BELL, d.nt_b);
        }
        return;
    }
    if (ph == PH_OUT) {
        if (threadIdx.x == 0) open_phase(st, PH_DONE, 0);
        return;
    }
}

template <typename VT, typename PT, int L>
__device__ __forceinline__ void run_item(const BDesc& d, const BState* st, int ph, int t, double* q, int64_t* rp, double* y,
                         double* ylds, double* red, double* cp) {
    double* part = d.part + (size_t)t * (kBMJ + 1);
    if (ph == PH_BELL) bell_tile<VT, PT, L>(d, st, t, q, rp, red, part, cp);
    else if (ph == PH_EXT) ext_tile<VT>(d, t);
    else vec_tile<VT, PT, L>(d, st, ph, t, y, ylds, red, part, cp);
}

template <typename VT, typename PT>
__device__ __forceinline__ void run_lanes(const BDesc& d, const BState* st, int ph, int t, double* q, int64_t* rp, double* y,
                          double* ylds, double* red, double* cp) {
    switch (d.lanes) {
        case 1: run_item<VT, PT, 1>(d, st, ph, t, q, rp, y, ylds, red, cp); break;
        case 2: run_item<VT, PT, 2>(d, st, ph, t, q, rp, y, ylds, red, cp); break;
        case 4: run_item<VT, PT, 4>(d, st, ph, t, q, rp, y, ylds, red, cp); break;
        case 8: run_item<VT, PT, 8>(d, st, ph, t, q, rp, y, ylds, red, cp); break;
        default: run_item<VT, PT, 16>(d, st, ph, t, q, rp, y, ylds, red, cp); break;
    }
}

// one round of work: the tiles of every member's current phase.  Workgroup
// b takes the contiguous items [b*total/G, (b+1)*total/G) of the tile list.
// CSR = false takes the members whose rows all have one length (no lane
// groups: 8 waves per SIMD fit), CSR = true the others (lane groups of 1..16
// lanes per row); a round launches each kind that the batch holds.
template <bool CSR>
__global__ __launch_bounds__(256) void k_bwork(const BDesc* __restrict__ D, const BState* __restrict__ ST,
                                               const int64_t* __restrict__ off, int n) {
    // rp (CSR Bellman tiles) and cp (uniform-row element products) are never
    // live together, so they share one LDS region
    __shared__ double q[kBMaxRows];
    __shared__ int64_t rpcp[kBMaxRows + 1 > kBChunk ? kBMaxRows + 1 : kBChunk];
    __shared__ double ylds[kBTileStates];
    __shared__ double y[kBMJ + 1];
    __shared__ double red[8];
    int64_t* rp = rpcp;
    double* cp = reinterpret_cast<double*>(rpcp);
    const int64_t total = off[n];
    const int64_t G = gridDim.x;
    // The tile list is split into one contiguous range per XCD (workgroup b
    // runs on XCD b mod 8), and an XCD's workgroups take the tiles of its
    // range round-robin, so at any time they work on neighbouring tiles,
    // mostly of one member, whose value vector then stays in that XCD's L2
    // (one contiguous run per workgroup had every member of the range in
    // flight at once).  Which workgroup runs a tile does not change the
    // result: each tile writes its own partial sums.
    const int64_t x = blockIdx.x % dev::kNumXcd;
    const int64_t nx = (G - x + dev::kNumXcd - 1) / dev::kNumXcd;  // workgroups on XCD x
    const int64_t w0 = x * total / dev::kNumXcd + blockIdx.x / dev::kNumXcd;
    const int64_t w1 = (x + 1) * total / dev::kNumXcd;
    if (w0 >= w1) return;
    // member of item w0: the last m with off[m] <= w0
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (off[mid] <= w0) lo = mid;
        else hi = mid - 1;
    }
    int m = lo;
    int64_t mend = off[m + 1];
    for (int64_t w = w0; w < w1; w += nx) {
        while (w >= mend) {
            ++m;
            mend = off[m + 1];
        }
        const BDesc& d = D[m];
        if (CSR != (d.kuni == 0)) continue;  // the other kernel's member (uniform per block)
        const BState* st = ST + m;
        const int ph = st->phase;
        const int t = (int)(w - off[m]);
        const bool f32 = d.fp32 && !(ph == PH_BELL && d.bell64);
        if constexpr (CSR) {
            if (f32) {
                if (d.rp32) run_lanes<float, int32_t>(d, st, ph, t, q, rp, y, ylds, red, cp);
                else run_lanes<float, int64_t>(d, st, ph, t, q, rp, y, ylds, red, cp);
            } else {
                if (d.rp32) run_lanes<double, int32_t>(d, st, ph, t, q, rp, y, ylds, red, cp);
                else run_lanes<double, int64_t>(d, st, ph, t, q, rp, y, ylds, red, cp);
            }
        } else {
            // uniform rows never read row_ptr; the lane count is unused
            if (f32) run_item<float, int32_t, 1>(d, st, ph, t, q, rp, y, ylds, red, cp);
            else run_item<double, int32_t, 1>(d, st, ph, t, q, rp, y, ylds, red, cp);
        }
        __syncthreads();  // LDS reuse by the next item
    }
}

// one workgroup per member: finalise the phase that just ran
__global__ __launch_bounds__(256) void k_bfin(const BDesc* __restrict__ D, BState* __restrict__ ST, int n) {
    __shared__ double red[8];
    const int m = blockIdx.x;
    if (m >= n) return;
    BState* st = ST + m;
    if (st->ntiles == 0) return;  // finished
    finalize(D[m], st, red);
}

// exclusive scan of the members' tile counts into off[0..n] (one workgroup)
__global__ __launch_bounds__(1024) void k_bscan(const BState* __restrict__ ST, int64_t* __restrict__ off, int n) {
    __shared__ int64_t part[1024];
    int64_t carry = 0;
    for (int base = 0; base < n; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const int64_t v = i < n ? (int64_t)ST[i].ntiles : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        // Hillis-Steele inclusive scan in LDS
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t a = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
            __syncthreads();
            part[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < n) off[i] = carry + part[threadIdx.x] - v;
        carry += part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) off[n] = carry;
}

// one chunk of rounds (captured once per kernel mix, replayed)
struct RoundArgs {
    const BDesc* D;
    BState* S;
    int64_t* off;
    int n, grid, rounds;
    bool any_uniform, any_csr;
};

void enqueue_rounds(void* ctx, hipStream_t st) {
    const RoundArgs& a = *static_cast<const RoundArgs*>(ctx);
    for (int r = 0; r < a.rounds; ++r) {
        if (a.any_uniform)
            hipLaunchKernelGGL(k_bwork<false>, dim3((unsigned)a.grid), dim3(kBlock), 0, st, a.D, (const BState*)a.S,
                               (const int64_t*)a.off, a.n);
        if (a.any_csr)
            hipLaunchKernelGGL(k_bwork<true>, dim3((unsigned)a.grid), dim3(kBlock), 0, st, a.D, (const BState*)a.S,
                               (const int64_t*)a.off, a.n);
        hipLaunchKernelGGL(k_bfin, dim3((unsigned)a.n), dim3(kBlock), 0, st, a.D, a.S, a.n);
        hipLaunchKernelGGL(k_bscan, dim3(1), dim3(1024), 0, st, (const BState*)a.S, a.off, a.n);
    }
    IPI_HIP(hipGetLastError());
}

int batch_lanes(const ipi_mdp_s* m) {
    const double k = (double)m->nnz / ((double)m->S * m->A);
    int L = 1;
    while (L < 16 && 2.0 * L * 3.0 <= k) L *= 2;
    return L;
}

// a member joins slot `slot`: V_0 = 0 and a fresh state machine (its tiles
// enter the next scan); block 0 writes the state, all blocks clear V
__global__ __launch_bounds__(256) void k_batch_join(const BDesc* __restrict__ D, BState* __restrict__ ST, int slot) {
    const BDesc& d = D[slot];
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < d.S; s += (int64_t)gridDim.x * blockDim.x)
        d.Va[s] = 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        BState* st = ST + slot;
        *st = BState{};
        st->phase = PH_BELL;
        st->ntiles = d.nt_b;
        st->first_cycle = 1;
        st->status = IPI_E_DEVICE;
    }
}

// a member leaves before it finished (cancelled, or past its round bound):
// no more tiles, no outputs
__global__ void k_batch_stop(BState* __restrict__ ST, int slot, int32_t status) {
    BState* st = ST + slot;
    st->ntiles = 0;
    st->phase = PH_DONE;
    st->status = status;
}

// partial sums a member needs: one row of kBMJ + 1 per tile of its largest phase
size_t member_partials(const ipi_mdp_s* m, int* spt_b, int* nt_b, int* nt_v) {
    int spt = 1;
    while (spt < 256 && 2 * spt * m->A <= kBMaxRows) spt *= 2;
    *spt_b = spt;
    *nt_b = (int)((m->S + spt - 1) / spt);
    *nt_v = (int)((m->S + kBTileStates - 1) / kBTileStates);
    return (size_t)std::max(*nt_b, *nt_v) * (kBMJ + 1);
}

}  // namespace

BatchEngine::BatchEngine(int capacity, hipStream_t st) : cap_(capacity), st_(st) {
    IPI_REQUIRE(capacity >= 1, IPI_E_INVALID_ARG, "batch capacity must be >= 1");
    hd_.resize((size_t)cap_ * sizeof(BDesc));
    hs_.resize((size_t)cap_ * sizeof(BState));
    slots_.resize((size_t)cap_);
    const size_t bytes_desc = sizeof(BDesc) * (size_t)cap_;
    const size_t bytes_st = sizeof(BState) * (size_t)cap_;
    off_st_ = (bytes_desc + 255) & ~(size_t)255;
    off_off_ = (off_st_ + bytes_st + 255) & ~(size_t)255;
    const size_t total = off_off_ + sizeof(int64_t) * ((size_t)cap_ + 1);
    {
        std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
        IPI_HIP(hipMalloc(&buf_, total));
    }
    // empty slots: no tiles (the finaliser and the scan skip them)
    IPI_HIP(hipMemsetAsync(buf_, 0, total, st_));
    grid_ = 8 * device_cus();
}

BatchEngine::~BatchEngine() {
    hipStreamSynchronize(st_);
    std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
    for (auto& g : graph_)
        if (g) hipGraphExecDestroy(g);
    if (cap_stream_) hipStreamDestroy(cap_stream_);
    hipFree(buf_);
}

int BatchEngine::add(ipi_mdp_s* m, const ipi_solve_opts& o, double* V_out, int32_t* pi_out) {
    IPI_REQUIRE(m && V_out && pi_out, IPI_E_INVALID_ARG, "NULL member");
    IPI_REQUIRE(o.inner == IPI_INNER_GMRES || o.inner == IPI_INNER_RICHARDSON, IPI_E_INVALID_ARG,
                "batch members use gmres or richardson");
    IPI_REQUIRE(o.pc == IPI_PC_NONE, IPI_E_INVALID_ARG, "batch members use pc_type none");
    IPI_REQUIRE(o.mode == IPI_MINCOST, IPI_E_INVALID_ARG, "batch members minimise costs");
    IPI_REQUIRE(o.inner != IPI_INNER_GMRES || (o.gmres_restart >= 1 && o.gmres_restart <= kBMJ),
                IPI_E_INVALID_ARG, "batch GMRES restart must lie in [1, 32]");
    IPI_REQUIRE(o.alpha > 0.0 && o.alpha < 1.0 && o.max_outer >= 1 && o.max_inner >= 1, IPI_E_INVALID_ARG,
                "bad batch options");
    IPI_REQUIRE(o.precision == IPI_FP64 || o.precision == IPI_FP32_MIXED || o.precision == IPI_FP32_INNER,
                IPI_E_INVALID_ARG, "bad precision");
    IPI_REQUIRE(o.precision == IPI_FP64 || m->val32, IPI_E_INVALID_ARG,
                "batch members in fp32_mixed or fp32_inner need an MDP created with IPI_VAL_FP32");
    IPI_REQUIRE(o.precision == IPI_FP32_MIXED || m->val, IPI_E_INVALID_ARG,
                "fp64 and fp32_inner members need the FP64 values of P");
    IPI_REQUIRE(m->A <= kBMaxRows, IPI_E_INVALID_ARG, "batch members need A <= 1024");
    int slot = -1;
    for (int i = 0; i < cap_; ++i) {
        if (slots_[(size_t)i].m == m) throw Error(IPI_E_INVALID_ARG, "an MDP appears twice in the batch");
        if (slot < 0 && !slots_[(size_t)i].m) slot = i;
    }
    IPI_REQUIRE(slot >= 0, IPI_E_INVALID_ARG, "the batch is full");
    int spt = 0, nt_b = 0, nt_v = 0;
    const size_t npart = member_partials(m, &spt, &nt_b, &nt_v);
    workspace_ensure(m, kBMJ, 0, o.precision != IPI_FP64, st_, npart);
    Workspace& w = m->ws;
    BDesc& d = reinterpret_cast<BDesc*>(hd_.data())[slot];
    d = BDesc{};
    d.row_ptr = m->row_ptr;
    d.col = m->col;
    d.val = m->val;
    d.val32 = m->val32;
    d.g = m->g;
    d.S = m->S;
    d.nnz = m->nnz;
    d.kuni = m->uniform_k ? m->k_max : 0;
    d.A = m->A;
    d.rp32 = m->rp32 ? 1 : 0;
    d.fp32 = o.precision != IPI_FP64 ? 1 : 0;
    d.bell64 = o.precision == IPI_FP32_INNER ? 1 : 0;
    d.lanes = batch_lanes(m);
    d.spt_b = spt;
    d.nt_b = nt_b;
    d.nt_v = nt_v;
    d.inner = o.inner;
    d.restart = o.inner == IPI_INNER_GMRES ? o.gmres_restart : 1;
    d.max_outer = o.max_outer;
    d.max_inner = o.max_inner;
    d.gamma = m->gamma;
    d.atol = o.atol;
    d.rtol_cert = o.rtol_cert;
    d.alpha = o.alpha;
    d.omega = o.richardson_scale;
    d.Va = w.V;
    d.Vb = w.TV;
    d.b = w.b;
    d.d0 = w.delta;
    d.d1 = w.delta2;
    d.basis = w.basis;
    d.small = w.small;
    d.ell_col = w.ppi_col;
    d.ell_val = w.ppi_val;
    d.pi = w.pi;
    d.part = w.bpart;
    d.V_out = V_out;
    d.pi_out = pi_out;
    BDesc* dD = reinterpret_cast<BDesc*>(buf_);
    IPI_HIP(hipMemcpyAsync(dD + slot, &d, sizeof(BDesc), hipMemcpyHostToDevice, st_));
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (m->S + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_batch_join, dim3(nb), dim3(kBlock), 0, st_, (const BDesc*)dD,
                       reinterpret_cast<BState*>(buf_ + off_st_), slot);
    IPI_HIP(hipGetLastError());
    // rounds this member can need: per outer iteration a Bellman pass, the
    // inner phases (GMRES: two per Arnoldi step, two per restart cycle;
    // Richardson: one per sweep, one update) and the output
    const int64_t inner_ph = o.inner == IPI_INNER_GMRES
                                 ? 2 * (int64_t)o.max_inner + 2 * ((int64_t)o.max_inner / d.restart + 1)
                                 : (int64_t)o.max_inner + 2;
    Slot& sl = slots_[(size_t)slot];
    sl.m = m;
    sl.opts = o;
    sl.V_out = V_out;
    sl.uniform = d.kuni > 0;
    sl.join_round = rounds_;
    sl.max_rounds = (int64_t)o.max_outer * (inner_ph + 3) + 4 + 128;
    sl.t_join = std::chrono::steady_clock::now();
    sl.done = false;
    ++active_;
    dirty_ = true;
    return slot;
}

std::vector<int> BatchEngine::step() {
    std::vector<int> fin;
    if (active_ == 0) return fin;
    BDesc* dD = reinterpret_cast<BDesc*>(buf_);
    BState* dS = reinterpret_cast<BState*>(buf_ + off_st_);
    int64_t* dOff = reinterpret_cast<int64_t*>(buf_ + off_off_);
    if (dirty_) {
        // tile counts of the members that joined since the last chunk
        hipLaunchKernelGGL(k_bscan, dim3(1), dim3(1024), 0, st_, (const BState*)dS, dOff, cap_);
        IPI_HIP(hipGetLastError());
        dirty_ = false;
    }
    bool any_uniform = false, any_csr = false, profile = false;
    for (const Slot& sl : slots_)
        if (sl.m && !sl.done) {
            (sl.uniform ? any_uniform : any_csr) = true;
            profile = profile || sl.opts.profile != 0;
        }
    // one chunk of 32 rounds; unless a member asks for profiling, captured
    // once per kernel mix into a HIP graph (the launches are the same every
    // time: the state lives in device memory) and replayed; rounds after a
    // member finishes exit at once for it
    RoundArgs ra{(const BDesc*)dD, dS, dOff, cap_, grid_, kRoundsPerChunk, any_uniform, any_csr};
    const int mix = (any_uniform ? 1 : 0) | (any_csr ? 2 : 0);
    if (!profile && !graph_tried_[mix]) {
        std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
        graph_tried_[mix] = true;
        if (!cap_stream_) IPI_HIP(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking));
        graph_[mix] = capture_graph_on(cap_stream_, enqueue_rounds, &ra);
    }
    if (!profile && graph_[mix]) IPI_HIP(hipGraphLaunch(graph_[mix], st_));
    else enqueue_rounds(&ra, st_);
    rounds_ += kRoundsPerChunk;
    IPI_HIP(hipMemcpyAsync(hs_.data(), dS, sizeof(BState) * (size_t)cap_, hipMemcpyDeviceToHost, st_));
    IPI_HIP(hipStreamSynchronize(st_));
    const auto now = std::chrono::steady_clock::now();
    const BState* hs = reinterpret_cast<const BState*>(hs_.data());
    for (int i = 0; i < cap_; ++i) {
        Slot& sl = slots_[(size_t)i];
        if (!sl.m || sl.done) continue;
        if (hs[i].phase == PH_DONE) {
            sl.done = true;
            sl.t_done = now;
            fin.push_back(i);
        } else if (rounds_ - sl.join_round > sl.max_rounds) {
            // past its round bound: stopped, reported as a device error
            hipLaunchKernelGGL(k_batch_stop, dim3(1), dim3(1), 0, st_, dS, i, (int32_t)IPI_E_DEVICE);
            IPI_HIP(hipGetLastError());
            dirty_ = true;
            sl.done = true;
            sl.overrun = true;
            sl.t_done = now;
            fin.push_back(i);
        }
    }
    return fin;
}

void BatchEngine::take(int slot, ipi_status* status, ipi_solve_info* info) {
    Slot& sl = slots_[(size_t)slot];
    IPI_REQUIRE(slot >= 0 && slot < cap_ && sl.m && sl.done, IPI_E_INVALID_ARG, "no finished member in this slot");
    const BState& s = reinterpret_cast<const BState*>(hs_.data())[slot];
    ipi_mdp_s* m = sl.m;
    ipi_status r = sl.overrun ? IPI_E_DEVICE : (ipi_status)s.status;
    if (r != IPI_OK) {
        set_last_error("batch member in slot " + std::to_string(slot) + " ended with status " +
                       std::to_string((int)r) + " in phase " + std::to_string(s.phase) + " after " +
                       std::to_string(s.outer) + " outer iterations" +
                       (sl.overrun ? " (past its round bound)" : ""));
    }
    // the residual of the returned V on the FP64 values (fp32_mixed: one FP64
    // Bellman pass, policy to scratch; without FP64 values the bound from the
    // float32 copy's row perturbation)
    double rho64 = s.rho;
    double bound = s.rho / (1.0 - m->gamma);
    if (sl.opts.precision == IPI_FP32_MIXED && !sl.overrun && s.phase == PH_DONE) {
        if (!m->val) {
            rho64 = std::numeric_limits<double>::quiet_NaN();
            bound = (s.rho + m->gamma * m->val32_dp * s.vmax) / (1.0 - m->gamma);
        } else {
            Workspace& w = m->ws;
            launch_fill_u64(&w.ctrl->rho_bits, 1, 0, st_);
            BellmanOut bo{nullptr, reinterpret_cast<int32_t*>(w.delta), nullptr, &w.ctrl->rho_bits, nullptr};
            launch_bellman(m, m->g, sl.V_out, bo, false, m->tune.bellman_lanes, m->tune.bellman_spt, st_);
            uint64_t bits = 0;
            IPI_HIP(hipMemcpyAsync(&bits, &w.ctrl->rho_bits, 8, hipMemcpyDeviceToHost, st_));
            IPI_HIP(hipStreamSynchronize(st_));
            std::memcpy(&rho64, &bits, 8);
            bound = rho64 / (1.0 - m->gamma);
        }
    }
    *status = r;
    if (info) {
        ipi_solve_info& f = *info;
        std::memset(&f, 0, sizeof(f));
        f.outer_iters = s.outer;
        f.converged = r == IPI_OK ? 1 : 0;
        f.inner_iters = s.inner_total;
        f.final_rho = s.rho;
        f.device_ms = std::chrono::duration<double, std::milli>(sl.t_done - sl.t_join).count();
        f.precision = sl.opts.precision;
        f.inner = sl.opts.inner;
        f.bellman_calls = s.outer + 1;
        f.inner_resid = s.c.resid;
        f.alg_bytes = s.alg_bytes;
        f.fp64_rho = rho64;
        f.err_bound = bound;
    }
    sl = Slot{};
    --active_;
}

void BatchEngine::drop(int slot) {
    Slot& sl = slots_[(size_t)slot];
    IPI_REQUIRE(slot >= 0 && slot < cap_ && sl.m, IPI_E_INVALID_ARG, "empty batch slot");
    if (!sl.done) {
        BState* dS = reinterpret_cast<BState*>(buf_ + off_st_);
        hipLaunchKernelGGL(k_batch_stop, dim3(1), dim3(1), 0, st_, dS, slot, (int32_t)IPI_E_CANCELLED);
        IPI_HIP(hipGetLastError());
        dirty_ = true;
    }
    IPI_HIP(hipStreamSynchronize(st_));
    sl = Slot{};
    --active_;
}

ipi_status solve_batch(int n, ipi_mdp_s* const* mdps, const ipi_solve_opts* opts, double* const* V_out,
                       int32_t* const* pi_out, ipi_solve_info* infos, ipi_status* statuses, hipStream_t st) {
    IPI_REQUIRE(n >= 1, IPI_E_INVALID_ARG, "empty batch");
    BatchEngine eng(n, st);
    for (int i = 0; i < n; ++i) {
        const int slot = eng.add(mdps[i], opts[i], V_out[i], pi_out[i]);
        IPI_REQUIRE(slot == i, IPI_E_DEVICE, "batch slot order");
    }
    int64_t chunks = 0;
    std::string first_error;
    while (eng.active() > 0) {
        for (int slot : eng.step()) {
            eng.take(slot, &statuses[slot], infos ? &infos[slot] : nullptr);
            if (statuses[slot] != IPI_OK && first_error.empty()) first_error = ipi_last_error();
        }
        ++chunks;
    }
    if (std::getenv("IPI_TRACE"))
        std::fprintf(stderr, "[ipi] batch of %d: %lld rounds\n", n, (long long)chunks * BatchEngine::kRoundsPerChunk);
    set_last_error(first_error);
    return IPI_OK;
}

}  // namespace ipi
