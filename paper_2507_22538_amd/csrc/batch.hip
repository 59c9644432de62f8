// Batched persistent iPI: many independent MDPs solved by one resident grid.
//
// Every MDP runs its own Algorithm 1 state machine (Bellman pass -> inner
// GMRES or Richardson -> update -> Bellman ...) as a sequence of phases.  A
// phase is split into tiles of states; workgroups of the persistent grid
// claim (MDP, tile) work items from per-MDP counters, so small and large
// MDPs share the chip without a host round trip per phase.
//
// Per MDP:
//   open = (epoch << 32) | tiles of the open phase   (written by the finaliser)
//   ctr  = (epoch << 32) | next tile to hand out      (atomic add claims a tile)
//   done = tiles finished in the open epoch
// A claim (e, t) is valid iff open still says epoch e and t < tiles.  The
// block finishing the last tile of an epoch is that phase's finaliser: it
// reduces the tiles' partial sums in tile order (so results do not depend
// on which block ran which tile, nor on the other members of the batch),
// runs the scalar step (Givens rotation, forcing test, outer stopping
// test), writes the next phase and opens the next epoch.
//
// The inner products gather the rows s*A + pi(s) of P in place (no compact
// P_pi copy).  Blocks with nothing to claim sleep briefly; a wall-clock
// watchdog aborts the launch (status IPI_E_DEVICE) if no block finds work
// for longer than the limit, so the grid always drains.
#include <algorithm>
#include <cmath>
#include <vector>

#include "device.hpp"
#include "krylov_tiled.hpp"

namespace ipi {

namespace {

constexpr int kBMJ = 32;          // largest GMRES restart in a batch
constexpr int kBTileStates = 256; // states per tile of the vector phases
constexpr int kBMaxRows = 1024;   // rows per tile of the Bellman phase

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
    PH_DONE = 9
};

struct BDesc {
    const void* row_ptr;
    const int* col;
    const double* val;
    const float* val32;
    const double* g;
    int64_t S;
    int A;
    int rp32;
    int fp32;
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
    uint64_t open;
    uint64_t ctr;
    uint32_t done;
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
    uint64_t rho_bits;
    uint64_t vmax_bits;
    Ctrl c;
};

struct BGlobal {
    uint32_t finished;
    uint32_t abort;
};

__device__ __forceinline__ uint64_t ld_acq(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_acq32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

// open epoch e+1 for phase ph with nt tiles (called by the finaliser, thread 0)
__device__ void open_phase(BState* st, int32_t ph, int nt) {
    const uint64_t e = (st->open >> 32) + 1;
    st->phase = ph;
    st->done = 0;
    __threadfence();
    __hip_atomic_store(&st->open, (e << 32) | (uint64_t)(uint32_t)nt, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->ctr, e << 32, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// sum over one block, all threads get the total
__device__ __forceinline__ double bsum(double x, double* red) { return dev::block_sum(x, red); }

// ---------------------------------------------------------------------------
// tile bodies
// ---------------------------------------------------------------------------

template <typename VT, typename PT, int L>
__device__ void bell_tile(const BDesc& d, BState* st, int t, double* q, int64_t* rp, double* red) {
    const int64_t s0 = (int64_t)t * d.spt_b;
    const int ns = (int)min((int64_t)d.spt_b, d.S - s0);
    const int A = d.A, R = ns * A;
    const int64_t r0 = s0 * A;
    const PT* __restrict__ rowp = (const PT*)d.row_ptr;
    const VT* __restrict__ val = sizeof(VT) == 4 ? (const VT*)d.val32 : (const VT*)d.val;
    const double* __restrict__ V = st->cur ? d.Vb : d.Va;
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
        dev::atomic_max_nonneg(&st->rho_bits, nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3])));
        dev::atomic_max_nonneg(&st->vmax_bits, nanmax(nanmax(red[4], red[5]), nanmax(red[6], red[7])));
    }
    __syncthreads();
}

// y[ls] = (P_pi x)[s0 + ls], rows s*A + pi(s) gathered in place
template <typename VT, typename PT, int L>
__device__ void ppi_tile(const BDesc& d, const double* __restrict__ x, int64_t s0, int ns, double* y) {
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
__device__ void vec_tile(const BDesc& d, BState* st, int ph, int t, double* y, double* ylds, double* red,
                         double* part_out) {
    const int64_t S = d.S;
    const int64_t s0 = (int64_t)t * kBTileStates;
    const int ns = (int)min((int64_t)kBTileStates, S - s0);
    const double gamma = d.gamma;
    const double* V = st->cur ? d.Vb : d.Va;
    double* Vn = st->cur ? d.Va : d.Vb;
    double acc[kBMJ + 1];
#pragma unroll
    for (int i = 0; i <= kBMJ; ++i) acc[i] = 0.0;
    int nred = 1;
    if (ph == PH_INIT) {
        for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
            const double r = d.b[s0 + ls];
            d.basis[s0 + ls] = r;
            acc[0] = fma(r, r, acc[0]);
        }
    } else if (ph == PH_ARN) {
        const int j = st->j;
        const double* uj = d.basis + (size_t)j * S;
        double* un = d.basis + (size_t)(j + 1) * S;
        const double cj = d.small[kOffSC + j];
        ppi_tile<VT, PT, L>(d, uj, s0, ns, ylds);
        for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
            const int64_t s = s0 + ls;
            const double w = cj * (uj[s] - gamma * ylds[ls]);
            un[s] = w;
#pragma unroll
            for (int i = 0; i < kBMJ; ++i)
                if (i <= j) acc[i] = fma(d.basis[(size_t)i * S + s], w, acc[i]);
        }
        nred = j + 1;
    } else if (ph == PH_ORTH) {
        const int j = st->j;
        if ((int)threadIdx.x <= j) y[threadIdx.x] = d.small[kOffH + (size_t)j * kLdH + threadIdx.x] * d.small[kOffSC + threadIdx.x];
        __syncthreads();
        double* w = d.basis + (size_t)(j + 1) * S;
        for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
            const int64_t s = s0 + ls;
            double x = w[s];
#pragma unroll
            for (int i = 0; i < kBMJ; ++i)
                if (i <= j) x = fma(-y[i], d.basis[(size_t)i * S + s], x);
            w[s] = x;
            acc[0] = fma(x, x, acc[0]);
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
#pragma unroll
            for (int i = 0; i < kBMJ; ++i)
                if (i < n) dl = fma(y[i], d.basis[(size_t)i * S + s], dl);
            d.d0[s] = dl;
            Vn[s] = V[s] + dl;
        }
        nred = 0;
    } else if (ph == PH_RES) {
        ppi_tile<VT, PT, L>(d, d.d0, s0, ns, ylds);
        for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
            const int64_t s = s0 + ls;
            const double r = d.b[s] - (d.d0[s] - gamma * ylds[ls]);
            d.basis[s] = r;
            acc[0] = fma(r, r, acc[0]);
        }
    } else if (ph == PH_RICH) {
        const int i = st->j;
        const double omega = d.omega;
        if (i == 0) {
            for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
                const int64_t s = s0 + ls;
                const double r = d.b[s];
                d.d1[s] = omega * r;
                acc[0] = fma(r, r, acc[0]);
            }
        } else {
            const double* dp = (i & 1) ? d.d1 : d.d0;
            double* dq = (i & 1) ? d.d0 : d.d1;
            ppi_tile<VT, PT, L>(d, dp, s0, ns, ylds);
            for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
                const int64_t s = s0 + ls;
                const double r = d.b[s] - (dp[s] - gamma * ylds[ls]);
                dq[s] = dp[s] + omega * r;
                acc[0] = fma(r, r, acc[0]);
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
    // per-tile partials, tile-major: part[t * (kBMJ + 1) + i]
#pragma unroll
    for (int i = 0; i < kBMJ; ++i) {
        if (i < nred) {
            const double tsum = bsum(acc[i], red);
            if (threadIdx.x == 0) part_out[i] = tsum;
        }
    }
}

// reduce partial i over the tiles of the closed epoch, fixed order
__device__ double tiles_sum(const double* part, int nt, int i, double* red) {
    double s = 0.0;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) s += part[(size_t)t * (kBMJ + 1) + i];
    return bsum(s, red);
}

// finaliser of a closed epoch (whole block calls it; thread 0 decides)
__device__ void finalize(const BDesc& d, BState* st, BGlobal* G, double* red) {
    const int ph = st->phase;
    const int nt = (int)(st->open & 0xffffffffu);
    Ctrl* c = &st->c;
    if (ph == PH_BELL) {
        if (threadIdx.x == 0) {
            const double rho = __longlong_as_double((long long)st->rho_bits);
            const double vmax = __longlong_as_double((long long)st->vmax_bits);
            st->rho_bits = 0;
            st->vmax_bits = 0;
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
                open_phase(st, d.inner == IPI_INNER_GMRES ? PH_INIT : PH_RICH, d.nt_v);
            }
        }
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
        if (threadIdx.x == 0) {
            open_phase(st, PH_DONE, 0);
            __hip_atomic_fetch_add(&G->finished, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
}

template <typename VT, typename PT, int L>
__device__ void run_item(const BDesc& d, BState* st, BGlobal* G, int ph, int t, double* q, int64_t* rp, double* y,
                         double* ylds, double* red) {
    if (ph == PH_BELL) bell_tile<VT, PT, L>(d, st, t, q, rp, red);
    else vec_tile<VT, PT, L>(d, st, ph, t, y, ylds, red, d.part + (size_t)t * (kBMJ + 1));
}

template <typename VT, typename PT>
__device__ void run_lanes(const BDesc& d, BState* st, BGlobal* G, int ph, int t, double* q, int64_t* rp, double* y,
                          double* ylds, double* red) {
    switch (d.lanes) {
        case 1: run_item<VT, PT, 1>(d, st, G, ph, t, q, rp, y, ylds, red); break;
        case 2: run_item<VT, PT, 2>(d, st, G, ph, t, q, rp, y, ylds, red); break;
        case 4: run_item<VT, PT, 4>(d, st, G, ph, t, q, rp, y, ylds, red); break;
        case 8: run_item<VT, PT, 8>(d, st, G, ph, t, q, rp, y, ylds, red); break;
        default: run_item<VT, PT, 16>(d, st, G, ph, t, q, rp, y, ylds, red); break;
    }
}

__global__ __launch_bounds__(256) void k_batch(const BDesc* __restrict__ D, BState* __restrict__ ST,
                                               BGlobal* __restrict__ G, int n, uint64_t watchdog_ticks) {
    __shared__ double q[kBMaxRows];
    __shared__ int64_t rp[kBMaxRows + 1];
    __shared__ double ylds[kBTileStates];
    __shared__ double y[kBMJ + 1];
    __shared__ double red[8];
    __shared__ int s_m, s_t, s_ph, s_last;
    int m = (int)(((int64_t)blockIdx.x * n) / gridDim.x);
    uint64_t idle_since = wall_clock64();
    for (;;) {
        if (threadIdx.x == 0) {
            s_m = -1;
            if (ld_acq32(&G->abort) || ld_acq32(&G->finished) >= (uint32_t)n) {
                s_m = -2;
            } else {
                for (int k = 0; k < n; ++k) {
                    const int mm = (m + k) % n;
                    BState* st = ST + mm;
                    const uint64_t op = ld_acq(&st->open);
                    const uint64_t cr = ld_acq(&st->ctr);
                    const uint32_t nt = (uint32_t)op;
                    if ((cr >> 32) != (op >> 32) || (uint32_t)cr >= nt) continue;
                    const uint64_t got = __hip_atomic_fetch_add(&st->ctr, (uint64_t)1, __ATOMIC_ACQ_REL,
                                                                __HIP_MEMORY_SCOPE_AGENT);
                    const uint64_t op2 = ld_acq(&st->open);
                    if ((got >> 32) != (op2 >> 32) || (uint32_t)got >= (uint32_t)op2) continue;
                    s_m = mm;
                    s_t = (int)(uint32_t)got;
                    s_ph = st->phase;
                    break;
                }
                if (s_m == -1) {
                    __builtin_amdgcn_s_sleep(4);
                    if (wall_clock64() - idle_since > watchdog_ticks) {
                        __hip_atomic_store(&G->abort, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                        s_m = -2;
                    }
                } else {
                    idle_since = wall_clock64();
                }
            }
        }
        __syncthreads();
        const int mm = s_m;
        if (mm == -2) break;
        if (mm == -1) continue;
        __threadfence();  // acquire: see the phase fields written before the epoch opened
        m = mm;
        const BDesc& d = D[mm];
        BState* st = ST + mm;
        const int ph = s_ph, t = s_t;
        if (d.fp32) {
            if (d.rp32) run_lanes<float, int32_t>(d, st, G, ph, t, q, rp, y, ylds, red);
            else run_lanes<float, int64_t>(d, st, G, ph, t, q, rp, y, ylds, red);
        } else {
            if (d.rp32) run_lanes<double, int32_t>(d, st, G, ph, t, q, rp, y, ylds, red);
            else run_lanes<double, int64_t>(d, st, G, ph, t, q, rp, y, ylds, red);
        }
        // arrive; the block finishing the last tile finalises the epoch
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t nt = (uint32_t)ld_acq(&st->open);
            const uint32_t prev = __hip_atomic_fetch_add(&st->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            s_last = (prev == nt - 1) ? 1 : 0;
        }
        __syncthreads();
        if (s_last) {
            __threadfence();
            finalize(d, st, G, red);
            __syncthreads();
        }
    }
}

__global__ void k_batch_setup(const BDesc* __restrict__ D, BState* __restrict__ ST, BGlobal* G, int n) {
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const BDesc& d = D[i];
        for (int64_t s = threadIdx.x; s < d.S; s += blockDim.x) d.Va[s] = 0.0;
        if (threadIdx.x == 0) {
            BState* st = ST + i;
            st->open = ((uint64_t)1 << 32) | (uint64_t)(uint32_t)d.nt_b;
            st->ctr = (uint64_t)1 << 32;
            st->done = 0;
            st->phase = PH_BELL;
            st->j = 0;
            st->cur = 0;
            st->outer = 0;
            st->first_cycle = 1;
            st->status = IPI_E_DEVICE;
            st->inner_total = 0;
            st->rho = 0;
            st->vmax = 0;
            st->rho_bits = 0;
            st->vmax_bits = 0;
            st->c = Ctrl{};
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        G->finished = 0;
        G->abort = 0;
    }
}

int batch_lanes(const ipi_mdp_s* m) {
    const double k = (double)m->nnz / ((double)m->S * m->A);
    int L = 1;
    while (L < 16 && 2.0 * L * 3.0 <= k) L *= 2;
    return L;
}

}  // namespace

ipi_status solve_batch(int n, ipi_mdp_s* const* mdps, const ipi_solve_opts* opts, double* const* V_out,
                       int32_t* const* pi_out, ipi_solve_info* infos, ipi_status* statuses, hipStream_t st) {
    std::vector<BDesc> hd((size_t)n);
    size_t part_total = 0;
    std::vector<size_t> part_off((size_t)n);
    for (int i = 0; i < n; ++i) {
        ipi_mdp_s* m = mdps[i];
        const ipi_solve_opts& o = opts[i];
        IPI_REQUIRE(o.inner == IPI_INNER_GMRES || o.inner == IPI_INNER_RICHARDSON, IPI_E_INVALID_ARG,
                    "batch members use gmres or richardson");
        IPI_REQUIRE(o.pc == IPI_PC_NONE, IPI_E_INVALID_ARG, "batch members use pc_type none");
        IPI_REQUIRE(o.mode == IPI_MINCOST, IPI_E_INVALID_ARG, "batch members minimise costs");
        IPI_REQUIRE(o.inner != IPI_INNER_GMRES || (o.gmres_restart >= 1 && o.gmres_restart <= kBMJ),
                    IPI_E_INVALID_ARG, "batch GMRES restart must lie in [1, 32]");
        IPI_REQUIRE(o.alpha > 0.0 && o.alpha < 1.0 && o.max_outer >= 1 && o.max_inner >= 1, IPI_E_INVALID_ARG,
                    "bad batch options");
        IPI_REQUIRE(o.precision == IPI_FP64 || m->val32, IPI_E_INVALID_ARG,
                    "fp32_mixed needs an MDP created with IPI_VAL_FP32");
        IPI_REQUIRE(m->A <= kBMaxRows, IPI_E_INVALID_ARG, "batch members need A <= 1024");
        for (int k = 0; k < i; ++k) IPI_REQUIRE(mdps[k] != m, IPI_E_INVALID_ARG, "an MDP appears twice in the batch");
        workspace_ensure(m, kBMJ, 0, o.precision == IPI_FP32_MIXED, st);
        BDesc& d = hd[(size_t)i];
        d.row_ptr = m->row_ptr;
        d.col = m->col;
        d.val = m->val;
        d.val32 = m->val32;
        d.g = m->g;
        d.S = m->S;
        d.A = m->A;
        d.rp32 = m->rp32 ? 1 : 0;
        d.fp32 = o.precision == IPI_FP32_MIXED ? 1 : 0;
        d.lanes = batch_lanes(m);
        int spt = 1;
        while (spt < 256 && 2 * spt * m->A <= kBMaxRows) spt *= 2;
        d.spt_b = spt;
        d.nt_b = (int)((m->S + spt - 1) / spt);
        d.nt_v = (int)((m->S + kBTileStates - 1) / kBTileStates);
        d.inner = o.inner;
        d.restart = o.inner == IPI_INNER_GMRES ? o.gmres_restart : 1;
        d.max_outer = o.max_outer;
        d.max_inner = o.max_inner;
        d.gamma = m->gamma;
        d.atol = o.atol;
        d.rtol_cert = o.rtol_cert;
        d.alpha = o.alpha;
        d.omega = o.richardson_scale;
        Workspace& w = m->ws;
        d.Va = w.V;
        d.Vb = w.TV;
        d.b = w.b;
        d.d0 = w.delta;
        d.d1 = w.delta2;
        d.basis = w.basis;
        d.small = w.small;
        d.pi = w.pi;
        d.V_out = V_out[i];
        d.pi_out = pi_out[i];
        part_off[(size_t)i] = part_total;
        part_total += (size_t)d.nt_v * (kBMJ + 1);
    }
    // one scratch allocation per call: descriptors, states, partials
    const size_t bytes_desc = sizeof(BDesc) * (size_t)n;
    const size_t bytes_st = sizeof(BState) * (size_t)n;
    const size_t off_st = (bytes_desc + 255) & ~(size_t)255;
    const size_t off_g = (off_st + bytes_st + 255) & ~(size_t)255;
    const size_t off_part = (off_g + sizeof(BGlobal) + 255) & ~(size_t)255;
    const size_t total = off_part + part_total * sizeof(double);
    char* buf = nullptr;
    IPI_HIP(hipMalloc(&buf, total));
    struct Free {
        char* p;
        ~Free() { hipFree(p); }
    } guard{buf};
    for (int i = 0; i < n; ++i) hd[(size_t)i].part = (double*)(buf + off_part) + part_off[(size_t)i];
    BDesc* dD = (BDesc*)buf;
    BState* dS = (BState*)(buf + off_st);
    BGlobal* dG = (BGlobal*)(buf + off_g);
    IPI_HIP(hipMemcpyAsync(dD, hd.data(), bytes_desc, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_batch_setup, dim3((unsigned)std::min(n, 4096)), dim3(kBlock), 0, st, dD, dS, dG, n);
    IPI_HIP(hipGetLastError());

    int dev = 0, blocks_per_cu = 0, clock_khz = 0;
    IPI_HIP(hipGetDevice(&dev));
    IPI_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu, k_batch, kBlock, 0));
    IPI_HIP(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev));
    if (blocks_per_cu < 1) blocks_per_cu = 1;
    if (clock_khz <= 0) clock_khz = 100000;
    const int grid = device_cus() * blocks_per_cu;
    const uint64_t watchdog = (uint64_t)clock_khz * 1000ull * 20ull;  // 20 s without any work item
    hipEvent_t e0, e1;
    IPI_HIP(hipEventCreate(&e0));
    IPI_HIP(hipEventCreate(&e1));
    IPI_HIP(hipEventRecord(e0, st));
    hipLaunchKernelGGL(k_batch, dim3((unsigned)grid), dim3(kBlock), 0, st, dD, dS, dG, n, watchdog);
    IPI_HIP(hipGetLastError());
    IPI_HIP(hipEventRecord(e1, st));
    std::vector<BState> hs((size_t)n);
    BGlobal hg{};
    IPI_HIP(hipMemcpyAsync(hs.data(), dS, bytes_st, hipMemcpyDeviceToHost, st));
    IPI_HIP(hipMemcpyAsync(&hg, dG, sizeof(hg), hipMemcpyDeviceToHost, st));
    IPI_HIP(hipStreamSynchronize(st));
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    for (int i = 0; i < n; ++i) {
        const BState& s = hs[(size_t)i];
        ipi_status r = (ipi_status)s.status;
        if (s.phase != PH_DONE) r = IPI_E_DEVICE;
        statuses[i] = r;
        if (infos) {
            ipi_solve_info& f = infos[i];
            std::memset(&f, 0, sizeof(f));
            f.outer_iters = s.outer;
            f.converged = r == IPI_OK ? 1 : 0;
            f.inner_iters = s.inner_total;
            f.final_rho = s.rho;
            f.device_ms = ms;
            f.precision = opts[i].precision;
            f.inner = opts[i].inner;
            f.bellman_calls = s.outer + 1;
            f.inner_resid = s.c.resid;
        }
    }
    if (hg.abort) {
        set_last_error("batch watchdog: no work item could be claimed for 20 s; results of unfinished members are invalid");
        throw Error(IPI_E_DEVICE, "batch watchdog fired");
    }
    return IPI_OK;
}

}  // namespace ipi
