// Tiled P_pi product kernels shared by the inner solvers (included by the
// per-variant translation units so their instantiations compile in parallel).
// Each block writes its partial sums to partials[i * gridDim.x + block]; a
// separate finalise kernel reduces them in a fixed order (no cross-block
// fences inside a product kernel: on gfx950 an agent-scope release writes
// back the XCD's L2, which is far too costly to do once per block).
#pragma once

#include "device.hpp"
#include "krylov.hpp"

namespace ipi {
namespace tiled {

using dev::block_sum;

__device__ __forceinline__ void range_of(int64_t lb, int64_t nb, int64_t n, int64_t* b, int64_t* e) {
    *b = lb * n / nb;
    *e = (lb + 1) * n / nb;
}

// ---------------------------------------------------------------------------
// scalar finalisers (thread 0 of the last block)
// ---------------------------------------------------------------------------

// start of a GMRES cycle from residual u_0 with norm beta
__device__ inline void cycle_start(double* small, Ctrl* c, double beta) {
    small[kOffGV] = beta;
    small[kOffSC] = beta > 0.0 ? 1.0 / beta : 0.0;
    c->beta = beta;
    c->resid = beta;
    c->j = 0;
    const int conv = beta < c->target;
    c->converged = conv;
    c->active = (!conv && c->steps_total < c->max_inner) ? 1 : 0;
}

// after step j: new column j of H is complete up to H[j+1][j] = hn
__device__ inline void givens_step(double* small, Ctrl* c, int j, double hn) {
    double* H = small + kOffH;
    double* cs = small + kOffCS;
    double* sn = small + kOffSN;
    double* gv = small + kOffGV;
    double* col = H + (size_t)j * kLdH;
    col[j + 1] = hn;
    small[kOffSC + j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double r = hypot(a, b);
    const double cj = r > 0.0 ? a / r : 1.0;
    const double sj = r > 0.0 ? b / r : 0.0;
    cs[j] = cj;
    sn[j] = sj;
    col[j] = r;
    col[j + 1] = 0.0;
    const double gj = gv[j];
    gv[j] = cj * gj;
    gv[j + 1] = -sj * gj;
    const double resid = fabs(gv[j + 1]);
    c->resid = resid;
    c->j = j + 1;
    c->steps_total += 1;
    const int conv = resid < c->target;
    c->converged = conv;
    c->breakdown = hn > 0.0 ? 0 : 1;
    if (conv || c->steps_total >= c->max_inner || j + 1 >= c->restart || hn <= 0.0) c->active = 0;
}

// ---------------------------------------------------------------------------
// tiled P_pi products
// ---------------------------------------------------------------------------

// kTfqW / kTfqV: the two fused products of a TFQMR iteration (see kernels_krylov.hip)
enum Variant { kArnoldi = 0, kResid = 1, kRich = 2, kApply = 3, kTfqW = 4, kTfqV = 5 };

// partial sums each variant produces
constexpr int variant_mj(int var) { return (var == kApply || var == kTfqW) ? 2 : 1; }

// scalar slots of the short-recurrence solvers (offsets into the small buffer)
// TFQMR scalars: rho = <w, r*>, alpha, beta, tau, theta, eta (of the last
// half step; x lags by eta * d), coef = theta^2 eta / alpha for the next
// d update, the initial residual norm, sigma = <v, r*>
constexpr int kTqRho = kOffScal + 8, kTqAlpha = kOffScal + 9, kTqBeta = kOffScal + 10, kTqTau = kOffScal + 11,
              kTqTheta = kOffScal + 12, kTqEta = kOffScal + 13, kTqCoef = kOffScal + 14, kTqR0 = kOffScal + 15;
constexpr int kBiRho = kOffScal + 0, kBiAlpha = kOffScal + 1, kBiOmega = kOffScal + 2, kBiBeta = kOffScal + 3,
              kBiHalf = kOffScal + 4;

struct TileParams {
    const int* col;
    const void* val;
    const int64_t* rp;
    int k;
    int64_t S;
    double gamma;
    const double* dinv;
    int spt;
    int64_t ntiles;
    double* basis;  // arnoldi: u_0..u_j read, u_{j+1} written
    int j;
    const double* x;  // resid / rich: the vector multiplied
    const double* b;
    double* out;
    double* small;
    double* partials;
    Ctrl* ctrl;
    int pbuf;
    int flat_e;          // > 0: uniform rows streamed in chunks of flat_e values
    const double* dotA;  // apply: dot partner of the output
    int dot_self;        // apply: also <out, out>
    int fin;             // apply: 1 = BiCGStab alpha, 2 = BiCGStab omega
    int pipe;            // flat only: 0 workgroup tiles, 1 wave tiles (spt = states per wave tile)
    // TFQMR vectors (kTfqW: tx, td, tw updated, out = J q; kTfqV: tv updated
    // from out = J u and taq = J q; both dot with trs = r*)
    double* tx;
    double* td;
    double* tw;
    double* tv;
    const double* taq;
    const double* trs;
    const int32_t* band;  // wave tiles, band form: first column of each P_pi row
    int keep;             // wave tiles: load P_pi through the caches
    // wave tiles, stencil form: per P_pi row its first column and pattern,
    // the patterns' offsets (kStenMaxPatterns x k, unused patterns zero),
    // columns in adjacent pairs
    const uint32_t* sten;
    const int32_t* sten_off;
    int sten_pairs;
};

// scalars of a product's epilogue, read once per workgroup
struct EpiScal {
    double a, b, c;
};

template <int VAR>
__device__ __forceinline__ EpiScal epi_scalars(const TileParams& p) {
    EpiScal e{0.0, 0.0, 0.0};
    if (VAR == kRich) e.a = p.ctrl->omega;
    if (VAR == kTfqW) {
        e.a = p.small[kTqAlpha];
        e.b = p.small[kTqCoef];
        e.c = p.small[kTqEta];
    }
    if (VAR == kTfqV) e.a = p.small[kTqBeta];
    return e;
}

// BiCGStab scalars after v = J p (fin 1: alpha = rho / <rh, v>) or after
// t = J s (fin 2: omega = <t, s> / <t, t>)
__device__ inline void apply_finalize(const TileParams& p, const double* sums) {
    Ctrl* c = p.ctrl;
    double* sm = p.small;
    if (p.fin == 1) {
        const double den = sums[0];
        if (den == 0.0 || !isfinite(den)) {
            c->breakdown = 1;
            c->active = 0;
            return;
        }
        sm[kBiAlpha] = sm[kBiRho] / den;
    } else {
        const double ts = sums[0], tt = sums[1];
        sm[kBiOmega] = tt > 0.0 ? ts / tt : 0.0;
    }
}

// y[ls] = sum_j P_pi[s0+ls, j] x[col_j] for the tile's rows; L lanes per row
template <typename VT, int L, int VEC>
__device__ __forceinline__ void spmv_tile(const TileParams& p, const double* __restrict__ x, int64_t s0, int ns,
                                          double* __restrict__ y) {
    constexpr int G = 256 / L;
    const int grp = threadIdx.x / L;
    const int lane = threadIdx.x % L;
    const VT* __restrict__ val = static_cast<const VT*>(p.val);
    for (int ls = grp; ls < ns; ls += G) {
        const int64_t s = s0 + ls;
        int64_t b, e;
        if (p.rp) {
            b = p.rp[s];
            e = p.rp[s + 1];
        } else {
            b = s * (int64_t)p.k;
            e = b + p.k;
        }
        double acc = 0.0;
#pragma unroll 4
        for (int64_t j = b + (int64_t)lane * VEC; j < e; j += (int64_t)L * VEC) {
            double vv[VEC];
            int cc[VEC];
            dev::VecLoad<VT, VEC>::load(val, p.col, j, vv, cc);
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc = fma(vv[v], x[cc[v]], acc);
        }
        acc = dev::group_sum<L>(acc);
        if (lane == 0) y[ls] = acc;
    }
}

// Uniform rows (row s at s*k): the tile's nonzeros are one contiguous range,
// streamed in chunks of E values per thread (independent 16-byte loads, no
// row-pointer dependency); chunk sums go to LDS and each row adds its k/E
// chunks in order.
template <typename VT, int E>
__device__ __forceinline__ void spmv_tile_flat(const TileParams& p, const double* __restrict__ x, int64_t s0, int ns,
                                               double* __restrict__ y, double* __restrict__ cp) {
    const int cpr = p.k / E;
    const int nch = ns * cpr;
    const VT* __restrict__ val = static_cast<const VT*>(p.val);
    const int64_t base = s0 * (int64_t)p.k;
#pragma unroll 2
    for (int c = threadIdx.x; c < nch; c += blockDim.x) {
        double vv[E];
        int cc[E];
        dev::FlatLoad<VT, E>::load(val, p.col, base + (int64_t)c * E, vv, cc);
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) acc = fma(vv[e], x[cc[e]], acc);
        cp[c] = acc;
    }
    __syncthreads();
    for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
        double t = 0.0;
        for (int i = 0; i < cpr; ++i) t += cp[ls * cpr + i];
        y[ls] = t;
    }
}

// The per-state tail of every product variant: jx = (J_pi x)[s] from
// xv = x[s] and yv = (P_pi x)[s]; bv = b[s] where the variant reads it.
template <int VAR, int MJ>
__device__ __forceinline__ void tile_epilogue(const TileParams& p, int64_t s, double xv, double bv, double yv,
                                              double xs, int j, const EpiScal& sc, double* __restrict__ unew,
                                              double (&acc)[MJ]) {
    const double jx = xv - p.gamma * yv;  // (J_pi x)[s]
    if (VAR == kArnoldi) {
        double w = xs * jx;
        if (p.dinv) w *= p.dinv[s];
        unew[s] = w;
#pragma unroll
        for (int i = 0; i < MJ; ++i)
            if (i <= j) acc[i] = fma(p.basis[(size_t)i * p.S + s], w, acc[i]);
    } else if (VAR == kResid) {
        double r = bv - jx;
        if (p.dinv) r *= p.dinv[s];
        unew[s] = r;
        acc[0] = fma(r, r, acc[0]);
    } else if (VAR == kRich) {
        const double r = bv - jx;
        const double pr = p.dinv ? r * p.dinv[s] : r;
        unew[s] = xv + sc.a * pr;
        acc[0] = fma(r, r, acc[0]);
    } else if (VAR == kTfqW) {
        // out = J q; x += eta d; d = q + coef d; w -= alpha J q; <w, w>, <w, r*>
        const double o = p.dinv ? jx * p.dinv[s] : jx;
        unew[s] = o;
        const double dold = p.td[s];
        p.tx[s] = fma(sc.c, dold, p.tx[s]);
        p.td[s] = fma(sc.b, dold, xv);
        const double wn = fma(-sc.a, o, p.tw[s]);
        p.tw[s] = wn;
        acc[0] = fma(wn, wn, acc[0]);
        if (MJ > 1) acc[MJ > 1 ? 1 : 0] = fma(wn, p.trs[s], acc[MJ > 1 ? 1 : 0]);
    } else if (VAR == kTfqV) {
        // out = J u; v = J u + beta (J q + beta v); <v, r*>
        const double o = p.dinv ? jx * p.dinv[s] : jx;
        unew[s] = o;
        const double vn = sc.a == 0.0 ? o : fma(sc.a, fma(sc.a, p.tv[s], p.taq[s]), o);
        p.tv[s] = vn;
        acc[0] = fma(vn, p.trs[s], acc[0]);
    } else {
        const double o = p.dinv ? jx * p.dinv[s] : jx;
        unew[s] = o;
        acc[0] = fma(p.dotA[s], o, acc[0]);
        if (MJ > 1) acc[MJ > 1 ? 1 : 0] = fma(o, o, acc[MJ > 1 ? 1 : 0]);
    }
}

// Wave tiles (uniform rows): each wavefront owns a contiguous range of
// tiles of p.spt states (at most 64) with its own slice of LDS for the chunk
// sums, so no workgroup barrier separates the streaming of one wave from
// the row sums and epilogue of another.  The LDS written by the lanes of a
// wave is read back by other lanes of the same wave after a wavefront-scope
// fence.  Sums are formed in the same order as the workgroup-tile kernel
// (chunk sums in index order, then the k/E chunks of a row in order), so
// both give identical results.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Chunks a lane keeps in flight per batch: about 64 bytes of double values
// (four 16-byte loads; three and six measured slower) and 48 bytes of float
// values (three; four and more measured slower: the gathered x values take
// twice the registers of their loads), or fewer when a tile gives a lane
// only a few.
constexpr int kWaveBatchBytes64 = 64;
constexpr int kWaveBatchBytes32 = 48;
// entries of x a wave stages for a band-form tile (two per lane)
constexpr int kWaveWindow = kBandWindow;
template <typename VT, int FE>
constexpr int wave_batch_big() {
    constexpr int bytes = sizeof(VT) == 8 ? kWaveBatchBytes64 : kWaveBatchBytes32;
    return bytes / (FE * (int)sizeof(VT)) < 2 ? 2 : bytes / (FE * (int)sizeof(VT));
}

// STEN (stencil form, not with BAND): a row's columns are its word's first
// column plus its pattern's offsets (staged in LDS); the same products in the
// same order as with the columns loaded.
template <typename VT, int VAR, int MJ, int FE, bool BAND, bool KEEP, int U, bool STEN = false>
__global__ __launch_bounds__(256) void k_wave_flat(TileParams p) {
    if (VAR != kResid && p.ctrl->active == 0) return;
    extern __shared__ double wl[];
    __shared__ double red[4];
    __shared__ int soff[STEN ? kStenMaxPatterns * kStenMaxK : 1];
    if constexpr (STEN) {
        for (int i = threadIdx.x; i < kStenMaxPatterns * p.k; i += blockDim.x) soff[i] = p.sten_off[i];
        __syncthreads();
    }
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ws = p.spt;
    const int cpr = p.k / FE;
    double* __restrict__ cp = wl + (size_t)wid * (ws * cpr + 1);
    double* __restrict__ xw = wl + (size_t)4 * (ws * cpr + 1) + (size_t)wid * kWaveWindow;
    const int64_t nb = gridDim.x;
    const int64_t lb = dev::xcd_remap(blockIdx.x, nb);
    int64_t t0, t1;
    range_of(lb * 4 + wid, nb * 4, p.ntiles, &t0, &t1);
    const int64_t S = p.S;
    double acc[MJ];
#pragma unroll
    for (int i = 0; i < MJ; ++i) acc[i] = 0.0;
    const int j = p.j;
    const double* __restrict__ xin;
    double xs = 1.0;
    if (VAR == kArnoldi) {
        xin = p.basis + (size_t)j * S;
        xs = p.small[kOffSC + j];
    } else {
        xin = p.x;
    }
    double* unew = (VAR == kArnoldi) ? p.basis + (size_t)(j + 1) * S : p.out;
    const EpiScal sc = epi_scalars<VAR>(p);
    const VT* __restrict__ val = static_cast<const VT*>(p.val);
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t s0 = t * ws;
        const int ns = (int)min((int64_t)ws, S - s0);
        const int nch = ns * cpr;
        const int64_t base = s0 * (int64_t)p.k;
        // the lane's own state (clamped into the tile): its band start and
        // the entries its epilogue reads, loaded with the first batch
        const int64_t so = s0 + min(lane, ns - 1);
        int bw = 0;
        if constexpr (BAND) bw = p.band[so];
        if constexpr (STEN) bw = (int)p.sten[so];
        const double xo = xin[so];
        const double bo = (VAR == kResid || VAR == kRich) ? p.b[so] : 0.0;
        // batches of U chunks per lane: every load of a batch is issued
        // before any is used (chunks past the tile's end re-read its last
        // chunk and are not stored)
        const int nbatch = (nch + 64 * U - 1) / (64 * U);
        // band form: the tile's rows read x in one window [wlo, wlo + span)
        // of at most kWaveWindow entries (the launch checks the MDP's bound),
        // staged in the wave's LDS once per tile; the chunks read it there
        // instead of gathering from memory
        int wlo = 0;
        for (int bt = 0; bt < nbatch; ++bt) {
            double vv[U][FE];
            int cc[U][FE];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int cl = min(lane + 64 * (bt * U + u), nch - 1);
                if constexpr (BAND || STEN) dev::FlatVals<VT, FE, KEEP>::load(val, base + (int64_t)cl * FE, vv[u]);
                else dev::FlatLoad<VT, FE, KEEP>::load(val, p.col, base + (int64_t)cl * FE, vv[u], cc[u]);
            }
            if constexpr (STEN) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int cl = min(lane + 64 * (bt * U + u), nch - 1);
                    const int ls = cl / cpr;
                    const uint32_t wd = (uint32_t)__shfl(bw, ls, dev::kWave);
                    const int c0 = (int)(wd & ((1u << kStenColBits) - 1));
                    const int* o = soff + (int)(wd >> kStenColBits) * p.k + (cl - ls * cpr) * FE;
#pragma unroll
                    for (int e = 0; e < FE; ++e) cc[u][e] = c0 + o[e];
                }
            }
            if constexpr (BAND) {
                if (bt == 0) {
                    int whi = bw;
                    wlo = bw;
#pragma unroll
                    for (int off = 32; off >= 1; off >>= 1) {
                        wlo = min(wlo, __shfl_xor(wlo, off, dev::kWave));
                        whi = max(whi, __shfl_xor(whi, off, dev::kWave));
                    }
                    const int span = whi + p.k - wlo;
                    const int i0 = min(2 * lane, span - 1), i1 = min(2 * lane + 1, span - 1);
                    const double a0 = xin[wlo + i0], a1 = xin[wlo + i1];
                    xw[i0] = a0;
                    xw[i1] = a1;
                    wave_lds_sync();
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int cl = min(lane + 64 * (bt * U + u), nch - 1);
                    const int ls = cl / cpr;
                    const int c0 = __shfl(bw, ls, dev::kWave) + (cl - ls * cpr) * FE;
#pragma unroll
                    for (int e = 0; e < FE; ++e) cc[u][e] = c0 + e;
                }
            }
            double xg[U][FE];
            if constexpr (BAND) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int e = 0; e < FE; ++e) xg[u][e] = xw[cc[u][e] - wlo];
                }
            } else if (STEN && FE % 2 == 0 && p.sten_pairs) {
                // columns c and c + 1: one 16-byte load (8-byte aligned)
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int e = 0; e < FE; e += 2) {
                        dev::d2_t t;
                        __builtin_memcpy(&t, xin + cc[u][e], 16);
                        xg[u][e] = t.x;
                        xg[u][e + 1] = t.y;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int e = 0; e < FE; ++e) xg[u][e] = xin[cc[u][e]];
                }
                // keep every gather of the batch ahead of the first use
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                double x = 0.0;
#pragma unroll
                for (int e = 0; e < FE; ++e) x = fma(vv[u][e], xg[u][e], x);
                // chunks past the tile's end go to the wave's spare slot
                const int c = lane + 64 * (bt * U + u);
                cp[c < nch ? c : ws * cpr] = x;
            }
        }
        wave_lds_sync();
        if (lane < ns) {
            double yv = 0.0;
            for (int i = 0; i < cpr; ++i) yv += cp[lane * cpr + i];
            tile_epilogue<VAR, MJ>(p, so, xo, bo, yv, xs, j, sc, unew, acc);
        }
        wave_lds_sync();
    }
    const int nred = (VAR == kArnoldi) ? j + 1 : (VAR == kApply ? 1 + p.dot_self : variant_mj(VAR));
#pragma unroll
    for (int i = 0; i < MJ; ++i) {
        if (i < nred) {
            const double t = block_sum(acc[i], red);
            if (threadIdx.x == 0) p.partials[(size_t)i * nb + lb] = t;
        }
    }
}

template <typename VT, int L, int VEC, int VAR, int MJ, int FE = 0>
__global__ __launch_bounds__(256) void k_tiled(TileParams p) {
    // a restart always runs (it re-opens the cycle); the other products stop with the solve
    if (VAR != kResid && p.ctrl->active == 0) return;
    extern __shared__ double y[];
    __shared__ double red[4];
    const int64_t nb = gridDim.x;
    const int64_t lb = dev::xcd_remap(blockIdx.x, nb);
    int64_t t0, t1;
    range_of(lb, nb, p.ntiles, &t0, &t1);
    const int64_t S = p.S;
    double acc[MJ];
#pragma unroll
    for (int i = 0; i < MJ; ++i) acc[i] = 0.0;
    const int j = p.j;
    const double* xin;
    double xs = 1.0;
    if (VAR == kArnoldi) {
        xin = p.basis + (size_t)j * S;
        xs = p.small[kOffSC + j];
    } else {
        xin = p.x;
    }
    double* unew = (VAR == kArnoldi) ? p.basis + (size_t)(j + 1) * S : p.out;
    const EpiScal sc = epi_scalars<VAR>(p);
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t s0 = t * p.spt;
        const int ns = (int)min((int64_t)p.spt, S - s0);
        if constexpr (FE > 0) spmv_tile_flat<VT, FE>(p, xin, s0, ns, y, y + p.spt);
        else spmv_tile<VT, L, VEC>(p, xin, s0, ns, y);
        __syncthreads();
        for (int ls = threadIdx.x; ls < ns; ls += blockDim.x) {
            const int64_t s = s0 + ls;
            const double bv = (VAR == kResid || VAR == kRich) ? p.b[s] : 0.0;
            tile_epilogue<VAR, MJ>(p, s, xin[s], bv, y[ls], xs, j, sc, unew, acc);
        }
        __syncthreads();
    }
    // per-block partials
    const int nred = (VAR == kArnoldi) ? j + 1 : (VAR == kApply ? 1 + p.dot_self : variant_mj(VAR));
#pragma unroll
    for (int i = 0; i < MJ; ++i) {
        if (i < nred) {
            const double t = block_sum(acc[i], red);
            if (threadIdx.x == 0) p.partials[(size_t)i * nb + lb] = t;
        }
    }
}

template <typename VT, int VAR, int FE, bool BAND, bool KEEP, int U, bool STEN>
void launch_wave_flat_u(const TileParams& p, int nb, int mj, hipStream_t st) {
    // per wave: the tile's chunk sums, one spare slot and the x window
    const size_t lds = (size_t)4 * ((size_t)p.spt * (p.k / FE) + 1 + kWaveWindow) * sizeof(double);
    if constexpr (VAR != kArnoldi) {
        hipLaunchKernelGGL((k_wave_flat<VT, VAR, variant_mj(VAR), FE, BAND, KEEP, U, STEN>), dim3(nb), dim3(kBlock), lds, st, p);
    } else {
    switch (mj) {
        case 8: hipLaunchKernelGGL((k_wave_flat<VT, VAR, 8, FE, BAND, KEEP, U, STEN>), dim3(nb), dim3(kBlock), lds, st, p); break;
        case 16: hipLaunchKernelGGL((k_wave_flat<VT, VAR, 16, FE, BAND, KEEP, U, STEN>), dim3(nb), dim3(kBlock), lds, st, p); break;
        case 32: hipLaunchKernelGGL((k_wave_flat<VT, VAR, 32, FE, BAND, KEEP, U, STEN>), dim3(nb), dim3(kBlock), lds, st, p); break;
        default: hipLaunchKernelGGL((k_wave_flat<VT, VAR, 64, FE, BAND, KEEP, U, STEN>), dim3(nb), dim3(kBlock), lds, st, p); break;
    }
    }
}

template <typename VT, int VAR, int FE, bool BAND, bool KEEP, bool STEN>
void launch_wave_flat_b(const TileParams& p, int nb, int mj, hipStream_t st) {
    // a lane's chunks per tile decide the batch: the large batch when a tile
    // fills it, else two chunks, or one
    constexpr int UB = wave_batch_big<VT, FE>();
    const int per_lane = (p.spt * (p.k / FE) + 63) / 64;
    if (UB > 2 && per_lane >= UB) launch_wave_flat_u<VT, VAR, FE, BAND, KEEP, UB, STEN>(p, nb, mj, st);
    else if (per_lane >= 2) launch_wave_flat_u<VT, VAR, FE, BAND, KEEP, 2, STEN>(p, nb, mj, st);
    else launch_wave_flat_u<VT, VAR, FE, BAND, KEEP, 1, STEN>(p, nb, mj, st);
}

template <typename VT, int VAR, int FE>
void launch_wave_flat(const TileParams& p, int nb, int mj, hipStream_t st) {
    if (p.band) {
        if (p.keep) launch_wave_flat_b<VT, VAR, FE, true, true, false>(p, nb, mj, st);
        else launch_wave_flat_b<VT, VAR, FE, true, false, false>(p, nb, mj, st);
    } else if (p.sten) {
        if (p.keep) launch_wave_flat_b<VT, VAR, FE, false, true, true>(p, nb, mj, st);
        else launch_wave_flat_b<VT, VAR, FE, false, false, true>(p, nb, mj, st);
    } else {
        if (p.keep) launch_wave_flat_b<VT, VAR, FE, false, true, false>(p, nb, mj, st);
        else launch_wave_flat_b<VT, VAR, FE, false, false, false>(p, nb, mj, st);
    }
}

template <typename VT, int L, int VEC, int VAR, int FE = 0>
void launch_tiled_mj(const TileParams& p, int nb, int mj, hipStream_t st) {
    size_t lds = (size_t)p.spt * sizeof(double);
    if (FE > 0) lds += (size_t)p.spt * (p.k / (FE > 0 ? FE : 1)) * sizeof(double);
    if constexpr (VAR != kArnoldi) {
        hipLaunchKernelGGL((k_tiled<VT, L, VEC, VAR, variant_mj(VAR), FE>), dim3(nb), dim3(kBlock), lds, st, p);
    } else {
    switch (mj) {
        case 8: hipLaunchKernelGGL((k_tiled<VT, L, VEC, VAR, 8, FE>), dim3(nb), dim3(kBlock), lds, st, p); break;
        case 16: hipLaunchKernelGGL((k_tiled<VT, L, VEC, VAR, 16, FE>), dim3(nb), dim3(kBlock), lds, st, p); break;
        case 32: hipLaunchKernelGGL((k_tiled<VT, L, VEC, VAR, 32, FE>), dim3(nb), dim3(kBlock), lds, st, p); break;
        default: hipLaunchKernelGGL((k_tiled<VT, L, VEC, VAR, 64, FE>), dim3(nb), dim3(kBlock), lds, st, p); break;
    }
    }
}

// flat chunk mode (lanes unused)
template <typename VT, int VAR>
void launch_tiled_flat(const TileParams& p, int nb, int mj, hipStream_t st) {
    if (p.pipe > 0) {
        // wave tiles: chunk widths 2 (FP64 only), 4 and 8
        if constexpr (sizeof(VT) == 8) {
            if (p.flat_e == 2) {
                launch_wave_flat<VT, VAR, 2>(p, nb, mj, st);
                return;
            }
        }
        if (p.flat_e == 4) launch_wave_flat<VT, VAR, 4>(p, nb, mj, st);
        else launch_wave_flat<VT, VAR, 8>(p, nb, mj, st);
        return;
    }
    if constexpr (sizeof(VT) == 8) {
        if (p.flat_e == 2) {
            launch_tiled_mj<VT, 1, 1, VAR, 2>(p, nb, mj, st);
            return;
        }
    }
    switch (p.flat_e) {
        case 4: launch_tiled_mj<VT, 1, 1, VAR, 4>(p, nb, mj, st); break;
        case 8: launch_tiled_mj<VT, 1, 1, VAR, 8>(p, nb, mj, st); break;
        case 12: launch_tiled_mj<VT, 1, 1, VAR, 12>(p, nb, mj, st); break;
        case 16: launch_tiled_mj<VT, 1, 1, VAR, 16>(p, nb, mj, st); break;
        case 24: launch_tiled_mj<VT, 1, 1, VAR, 24>(p, nb, mj, st); break;
        case 32: launch_tiled_mj<VT, 1, 1, VAR, 32>(p, nb, mj, st); break;
        default: break;
    }
}

template <typename VT, int VEC, int VAR>
void launch_tiled_lanes(const TileParams& p, int lanes, int nb, int mj, hipStream_t st) {
    if (p.flat_e > 0) {
        launch_tiled_flat<VT, VAR>(p, nb, mj, st);
        return;
    }
    switch (lanes) {
        case 1: launch_tiled_mj<VT, 1, VEC, VAR>(p, nb, mj, st); break;
        case 2: launch_tiled_mj<VT, 2, VEC, VAR>(p, nb, mj, st); break;
        case 4: launch_tiled_mj<VT, 4, VEC, VAR>(p, nb, mj, st); break;
        case 8: launch_tiled_mj<VT, 8, VEC, VAR>(p, nb, mj, st); break;
        case 16: launch_tiled_mj<VT, 16, VEC, VAR>(p, nb, mj, st); break;
        case 32: launch_tiled_mj<VT, 32, VEC, VAR>(p, nb, mj, st); break;
        case 64: launch_tiled_mj<VT, 64, VEC, VAR>(p, nb, mj, st); break;
        default: throw Error(IPI_E_INVALID_ARG, "spmv lanes must be a power of two in [1, 64]");
    }
}

}  // namespace tiled

// per-translation-unit dispatchers (kernels_tiled_*.hip)
void tiled_arnoldi_f64(const tiled::TileParams& p, int lanes, int vec, int nb, int mj, hipStream_t st);
void tiled_arnoldi_f32(const tiled::TileParams& p, int lanes, int vec, int nb, int mj, hipStream_t st);
void tiled_other(int var, bool fp32, const tiled::TileParams& p, int lanes, int vec, int nb, hipStream_t st);
void tiled_tfqmr(int var, bool fp32, const tiled::TileParams& p, int lanes, int vec, int nb, hipStream_t st);

}  // namespace ipi
