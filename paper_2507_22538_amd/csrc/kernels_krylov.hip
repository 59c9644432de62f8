// Inner policy-evaluation kernels (Algorithm 1 steps 6-12) on the
// correction form: solve J_pi delta = b with b = TV_k - V_k and delta_0 = 0,
// so theta_i = V_k + delta_i.  J_pi = I - gamma P_pi is applied matrix-free
// (Sec. III-B.3) from the compact P_pi.
//
// Tiled product kernels (one persistent grid; each block owns a contiguous
// range of state tiles, XCD-aware):
//   arnoldi  w = J v_j written as u_{j+1}, fused with the dots <u_i, w>,
//            i <= j (classical Gram-Schmidt, one pass over each u_i)
//   resid    u_0 = b - J delta and ||u_0||^2 (restart of GMRES)
//   rich     res = b - J delta_p, delta_q = delta_p + omega res, ||res||^2
// Element-wise kernels: init of a cycle, the orthogonalisation update with
// ||w||^2 and the Givens step, a second Gram-Schmidt pass, the GMRES
// solution update, Richardson's first sweep and the final V update.
//
// Every reduction is deterministic: per-thread sums in a fixed order, a
// fixed block tree, per-block partials, and a fixed-order final sum done
// by a separate finaliser kernel (which also runs the scalar work); no
// workgroup waits for or signals another within a launch.  Inner
// stopping uses the 2-norm of the linear residual against alpha * rho_k
// (Sec. III-B.3 replaces the inf-norm test of Algorithm 1 by this norm).
#include "krylov_tiled.hpp"

namespace ipi {

namespace {

using dev::block_sum;
using tiled::range_of;
using tiled::cycle_start;
using tiled::givens_step;
using tiled::TileParams;
using tiled::kArnoldi;
using tiled::kResid;
using tiled::kRich;
using tiled::kApply;
using tiled::kTfqV;
using tiled::kTfqW;

// ---------------------------------------------------------------------------
// element-wise kernels
// ---------------------------------------------------------------------------

__global__ void k_ctrl_reset(Ctrl* c, double target, int max_inner, int restart, double omega) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->active = 1;
        c->j = 0;
        c->steps_total = 0;
        c->converged = 0;
        c->max_inner = max_inner;
        c->restart = restart;
        c->result_buf = 0;
        c->breakdown = 0;
        c->target = target;
        c->beta = 0.0;
        c->resid = 0.0;
        c->omega = omega;
    }
}

// ---------------------------------------------------------------------------
// finalise kernels: fixed-order sums of the producers' per-block partials
// (kernel boundaries make the partials visible) and the scalar steps
// ---------------------------------------------------------------------------

enum FinMode : int {
    FIN_CYCLE = 0,     // beta = ||u_0||: start a GMRES cycle
    FIN_GIVENS = 1,    // h_{j+1,j} = ||w||: Givens step j
    FIN_RICH = 2,      // Richardson sweep i >= 1 (pbuf = buffer of delta_i)
    FIN_RICH0 = 3,     // Richardson sweep 0
    FIN_BI_INIT = 4,   // BiCGStab rho_0 = <r, r>
    FIN_BI_S = 5,      // ||s||: half-step exit
    FIN_BI_ALPHA = 6,  // alpha = rho / <rh, v>
    FIN_BI_OMEGA = 7,  // omega = <t, s> / <t, t>
    FIN_BI_UPDATE = 8, // rho' = <rh, r>, ||r||: beta, stop test
    FIN_TQ_INIT = 9,   // tau_0 = ||r_0||, rho_0 = ||r_0||^2
    FIN_TQ_STEP = 10,  // half step: ||w||: theta, c, tau, eta, stop test; j = 1 (odd): also rho', beta
    FIN_TQ_SIGMA = 11, // sigma = <v, r*>: alpha = rho / sigma
    FIN_TQ_TRUE = 12   // ||D (b - J delta)||: the true residual of an unconverged end
};

// The finalisers run one workgroup of kFinThreads threads per reduced
// quantity, so that the partials of a large grid (thousands of workgroups)
// arrive in one round of loads.
constexpr int kFinThreads = 1024;

// sum of one value per thread over a kFinThreads workgroup: wave butterflies,
// then the 16 wave sums in a fixed tree
__device__ __forceinline__ double fin_block_sum(double x, double* red16) {
    x = dev::wave_sum(x);
    const int w = threadIdx.x / dev::kWave;
    if ((threadIdx.x & (dev::kWave - 1)) == 0) red16[w] = x;
    __syncthreads();
    double t[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = red16[2 * i] + red16[2 * i + 1];
    const double r = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
    __syncthreads();
    return r;
}

// fixed-order sum of nb partials: 8 independent accumulators per thread so
// the loads are in flight together, then a fixed combine and block tree
__device__ __forceinline__ double sum_slot(const double* __restrict__ part, int64_t nb, int i, double* red16) {
    const double* __restrict__ p = part + (size_t)i * nb;
    const int64_t B = kFinThreads;
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t q = threadIdx.x;
    for (; q + 7 * B < nb; q += 8 * B) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += p[q + u * B];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
        if (q + u * B < nb) a[u] += p[q + u * B];
    const double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    return fin_block_sum(s, red16);
}

__global__ __launch_bounds__(1024) void k_fin_scalar(double* small, const double* __restrict__ partials, int64_t nb,
                                                     Ctrl* c, int mode, int j, int pbuf, int always) {
    if (!always && c->active == 0) return;
    __shared__ double red[16];
    const bool two = mode == FIN_BI_OMEGA || mode == FIN_BI_UPDATE || (mode == FIN_TQ_STEP && j == 1);
    const double s0 = sum_slot(partials, nb, 0, red);
    const double s1 = two ? sum_slot(partials, nb, 1, red) : 0.0;
    if (threadIdx.x != 0) return;
    switch (mode) {
        case FIN_CYCLE: cycle_start(small, c, sqrt(s0)); break;
        case FIN_GIVENS: givens_step(small, c, j, sqrt(s0)); break;
        case FIN_RICH: {
            // j = sweeps since the previous test (>= 1); the partials are those
            // of the last of them, i.e. the residual of its input delta_p;
            // pbuf = p + 4 (1 + q) with q the buffer of its output
            const int n = j > 0 ? j : 1;
            const double r = sqrt(s0);
            c->resid = r;
            if (r < c->target) {  // delta_p already meets the forcing test
                c->converged = 1;
                c->result_buf = pbuf & 3;
                c->steps_total += n - 1;
                c->active = 0;
            } else {
                c->steps_total += n;
                c->result_buf = (pbuf >> 2) - 1;
                if (c->steps_total >= c->max_inner) c->active = 0;
            }
            break;
        }
        case FIN_RICH0: {
            const double r = sqrt(s0);
            c->resid = r;
            if (r < c->target) {  // delta_0 = 0 already meets the test
                c->converged = 1;
                c->result_buf = -1;
                c->active = 0;
            } else {
                c->steps_total = 1;
                c->result_buf = 1;
                if (c->steps_total >= c->max_inner) c->active = 0;
            }
            break;
        }
        case FIN_BI_INIT:
            small[tiled::kBiRho] = s0;
            small[tiled::kBiHalf] = 0.0;
            c->beta = sqrt(s0);
            c->resid = sqrt(s0);
            c->converged = c->resid < c->target;
            c->active = c->converged ? 0 : 1;
            break;
        case FIN_BI_S: {
            const double ns = sqrt(s0);
            if (ns < c->target) {
                small[tiled::kBiHalf] = 1.0;
                c->resid = ns;
                c->converged = 1;
                c->steps_total += 1;
                c->active = 0;
            }
            break;
        }
        case FIN_BI_ALPHA:
            if (s0 == 0.0 || !isfinite(s0)) {
                c->breakdown = 1;
                c->active = 0;
            } else {
                small[tiled::kBiAlpha] = small[tiled::kBiRho] / s0;
            }
            break;
        case FIN_BI_OMEGA: small[tiled::kBiOmega] = s1 > 0.0 ? s0 / s1 : 0.0; break;
        case FIN_BI_UPDATE: {
            const double alpha = small[tiled::kBiAlpha], omega = small[tiled::kBiOmega];
            const double rho_old = small[tiled::kBiRho];
            c->resid = sqrt(s1);
            c->steps_total += 1;
            c->converged = c->resid < c->target;
            const double beta = (rho_old != 0.0 && omega != 0.0) ? (s0 / rho_old) * (alpha / omega) : 0.0;
            small[tiled::kBiBeta] = beta;
            small[tiled::kBiRho] = s0;
            const bool brk = s0 == 0.0 || omega == 0.0 || !isfinite(beta);
            if (brk && !c->converged) c->breakdown = 1;
            if (c->converged || brk || c->steps_total >= c->max_inner) c->active = 0;
            break;
        }
        case FIN_TQ_INIT: {
            const double t = sqrt(s0);
            small[tiled::kTqTau] = t;
            small[tiled::kTqR0] = t;
            small[tiled::kTqRho] = s0;
            small[tiled::kTqTheta] = 0.0;
            small[tiled::kTqEta] = 0.0;
            small[tiled::kTqCoef] = 0.0;
            small[tiled::kTqBeta] = 0.0;
            c->beta = t;
            c->resid = t;
            c->converged = t < c->target;
            c->active = c->converged ? 0 : 1;
            break;
        }
        case FIN_TQ_STEP: {
            // quasi-residual update; ||b - J x_k|| <= sqrt(k + 1) tau_k bounds the true residual
            const double alpha = small[tiled::kTqAlpha];
            const double tau = small[tiled::kTqTau];
            const double theta = sqrt(s0) / tau;
            const double cc = 1.0 / sqrt(1.0 + theta * theta);
            const double tn = tau * theta * cc;
            const double eta = cc * cc * alpha;
            small[tiled::kTqTheta] = theta;
            small[tiled::kTqTau] = tn;
            small[tiled::kTqEta] = eta;
            small[tiled::kTqCoef] = theta * theta * eta / alpha;
            c->steps_total += 1;
            const double bound = sqrt((double)c->steps_total + 1.0) * tn;
            c->resid = bound;
            if (!isfinite(bound)) {
                c->breakdown = 1;
                c->active = 0;
                break;
            }
            if (bound < c->target) {
                c->converged = 1;
                c->active = 0;
                break;
            }
            if (c->steps_total >= c->max_inner) {
                c->active = 0;
                break;
            }
            if (j == 1) {
                const double rho_old = small[tiled::kTqRho];
                const double beta = s1 / rho_old;
                if (s1 == 0.0 || !isfinite(beta)) {
                    c->breakdown = 1;
                    c->active = 0;
                    break;
                }
                small[tiled::kTqBeta] = beta;
                small[tiled::kTqRho] = s1;
            }
            break;
        }
        case FIN_TQ_TRUE: c->resid = sqrt(s0); break;
        case FIN_TQ_SIGMA: {
            const double alpha = small[tiled::kTqRho] / s0;
            if (s0 == 0.0 || !isfinite(alpha)) {
                c->breakdown = 1;
                c->active = 0;
                break;
            }
            small[tiled::kTqAlpha] = alpha;
            small[tiled::kTqCoef] = small[tiled::kTqTheta] * small[tiled::kTqTheta] * small[tiled::kTqEta] / alpha;
            break;
        }
        default: break;
    }
}

// Hessenberg column j from the Gram-Schmidt dots: one block per i <= j.
// second: the dots of a second pass, added to the column and kept in H2.
__global__ __launch_bounds__(1024) void k_fin_hcol(double* small, const double* __restrict__ partials, int64_t nb,
                                                   const Ctrl* c, int j, int second) {
    if (c->active == 0) return;
    __shared__ double red[16];
    const int i = blockIdx.x;
    const double s = sum_slot(partials, nb, i, red);
    if (threadIdx.x == 0) {
        const double h = s * small[kOffSC + i];
        if (second) {
            small[kOffH2 + i] = h;
            small[kOffH + (size_t)j * kLdH + i] += h;
        } else {
            small[kOffH + (size_t)j * kLdH + i] = h;
        }
    }
}

// ---------------------------------------------------------------------------
// element-wise producers (partials[i * gridDim.x + block])
// ---------------------------------------------------------------------------

// u_0 = D b, partial ||u_0||^2
__global__ __launch_bounds__(256) void k_init_cycle(const double* __restrict__ b, const double* __restrict__ dinv,
                                                    double* __restrict__ u0, int64_t S, double* partials) {
    __shared__ double red[4];
    const int64_t nb = gridDim.x, lb = dev::xcd_remap(blockIdx.x, nb);
    int64_t sb, se;
    range_of(lb, nb, S, &sb, &se);
    double acc = 0.0;
    for (int64_t s = sb + threadIdx.x; s < se; s += blockDim.x) {
        double r = b[s];
        if (dinv) r *= dinv[s];
        u0[s] = r;
        acc = fma(r, r, acc);
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partials[lb] = acc;
}

// second Gram-Schmidt pass, dots <u_i, w>, i <= j
template <int MJ>
__global__ __launch_bounds__(256) void k_dots(const double* __restrict__ basis, int64_t S, int j, double* partials,
                                              const Ctrl* c) {
    if (c->active == 0) return;
    __shared__ double red[4];
    const int64_t nb = gridDim.x, lb = dev::xcd_remap(blockIdx.x, nb);
    int64_t sb, se;
    range_of(lb, nb, S, &sb, &se);
    const double* w = basis + (size_t)(j + 1) * S;
    double acc[MJ];
#pragma unroll
    for (int i = 0; i < MJ; ++i) acc[i] = 0.0;
    for (int64_t s = sb + threadIdx.x; s < se; s += blockDim.x) {
        const double ws = w[s];
#pragma unroll
        for (int i = 0; i < MJ; ++i)
            if (i <= j) acc[i] = fma(basis[(size_t)i * S + s], ws, acc[i]);
    }
#pragma unroll
    for (int i = 0; i < MJ; ++i) {
        if (i <= j) {
            const double t = block_sum(acc[i], red);
            if (threadIdx.x == 0) partials[(size_t)i * nb + lb] = t;
        }
    }
}

// w <- w - sum_i h_i v_i (h from H column j, or the second-pass
// coefficients); on the final pass also the partial ||w||^2
template <int MJ>
__global__ __launch_bounds__(256) void k_orth(double* __restrict__ basis, int64_t S, int j, int second_pass,
                                              int final_pass, const double* small, double* partials, const Ctrl* c) {
    if (c->active == 0) return;
    __shared__ double coef[MJ];
    __shared__ double red[4];
    if ((int)threadIdx.x <= j && threadIdx.x < MJ) {
        const double h = second_pass ? small[kOffH2 + threadIdx.x] : small[kOffH + (size_t)j * kLdH + threadIdx.x];
        coef[threadIdx.x] = h * small[kOffSC + threadIdx.x];
    }
    __syncthreads();
    const int64_t nb = gridDim.x, lb = dev::xcd_remap(blockIdx.x, nb);
    int64_t sb, se;
    range_of(lb, nb, S, &sb, &se);
    double* w = basis + (size_t)(j + 1) * S;
    double acc = 0.0;
    for (int64_t s = sb + threadIdx.x; s < se; s += blockDim.x) {
        double x = w[s];
#pragma unroll
        for (int i = 0; i < MJ; ++i)
            if (i <= j) x = fma(-coef[i], basis[(size_t)i * S + s], x);
        w[s] = x;
        acc = fma(x, x, acc);
    }
    if (!final_pass) return;
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partials[lb] = acc;
}

// y = H^-1 g (upper triangular, n = steps of the cycle), delta (+)= sum y_i v_i,
// Vn = V + delta
template <int MJ>
__global__ __launch_bounds__(256) void k_gmres_update(const double* __restrict__ basis, int64_t S,
                                                      const double* __restrict__ small, const Ctrl* __restrict__ c,
                                                      double* __restrict__ delta, int first,
                                                      const double* __restrict__ V, double* __restrict__ Vn) {
    __shared__ double y[MJ];
    const int n = c->j;
    if (threadIdx.x == 0) {
        const double* H = small + kOffH;
        for (int i = n - 1; i >= 0; --i) {
            double t = small[kOffGV + i];
            for (int l = i + 1; l < n; ++l) t -= H[(size_t)l * kLdH + i] * y[l];
            y[i] = t / H[(size_t)i * kLdH + i];
        }
        for (int i = 0; i < n; ++i) y[i] *= small[kOffSC + i];
    }
    __syncthreads();
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
        double d = first ? 0.0 : delta[s];
#pragma unroll
        for (int i = 0; i < MJ; ++i)
            if (i < n) d = fma(y[i], basis[(size_t)i * S + s], d);
        delta[s] = d;
        Vn[s] = V[s] + d;
    }
}

// Richardson sweep 0 (delta_0 = 0): delta_1 = omega D b; partial ||b||^2
__global__ __launch_bounds__(256) void k_rich0(const double* __restrict__ b, const double* __restrict__ dinv,
                                               double* __restrict__ dq, int64_t S, double* partials, const Ctrl* c) {
    if (c->active == 0) return;
    __shared__ double red[4];
    const int64_t nb = gridDim.x, lb = dev::xcd_remap(blockIdx.x, nb);
    int64_t sb, se;
    range_of(lb, nb, S, &sb, &se);
    const double omega = c->omega;
    double acc = 0.0;
    for (int64_t s = sb + threadIdx.x; s < se; s += blockDim.x) {
        const double r = b[s];
        dq[s] = omega * (dinv ? r * dinv[s] : r);
        acc = fma(r, r, acc);
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partials[lb] = acc;
}

// Vn = V + delta[result_buf]  (result_buf -1 means delta = 0)
__global__ __launch_bounds__(256) void k_axpy_result(const double* __restrict__ V, const double* __restrict__ d0,
                                                     const double* __restrict__ d1, const double* __restrict__ d2,
                                                     const Ctrl* __restrict__ c, double* __restrict__ Vn, int64_t S) {
    const int rb = c->result_buf;
    const double* d = rb == 0 ? d0 : (rb == 1 ? d1 : d2);
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x)
        Vn[s] = rb < 0 ? V[s] : V[s] + d[s];
}

// ---------------------------------------------------------------------------
// BiCGStab (van der Vorst) on J delta = b with left Jacobi scaling D:
//   r = D b, rh = r, p = r, rho = <rh, r>
//   loop: v = D J p; alpha = rho / <rh, v>; s = r - alpha v  (stop if small)
//         t = D J s; omega = <t, s> / <t, t>; x += alpha p + omega s;
//         r = s - omega t; rho' = <rh, r>; beta = rho'/rho * alpha/omega;
//         p = r + beta (p - omega v)
// ---------------------------------------------------------------------------

// init: r = D b, rh = r, p = r, partial ||r||^2
__global__ __launch_bounds__(256) void k_bi_init(const double* __restrict__ b, const double* __restrict__ dinv,
                                                 double* __restrict__ r, double* __restrict__ rh, double* __restrict__ p,
                                                 int64_t S, double* partials) {
    __shared__ double red[4];
    const int64_t nb = gridDim.x, lb = dev::xcd_remap(blockIdx.x, nb);
    int64_t sb, se;
    range_of(lb, nb, S, &sb, &se);
    double acc = 0.0;
    for (int64_t s = sb + threadIdx.x; s < se; s += blockDim.x) {
        const double x = dinv ? b[s] * dinv[s] : b[s];
        r[s] = x;
        rh[s] = x;
        p[s] = x;
        acc = fma(x, x, acc);
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partials[lb] = acc;
}

// s = r - alpha v, partial ||s||^2
__global__ __launch_bounds__(256) void k_bi_s(const double* __restrict__ r, const double* __restrict__ v,
                                              double* __restrict__ sv, int64_t S, const double* small,
                                              double* partials, const Ctrl* c) {
    if (c->active == 0) return;
    __shared__ double red[4];
    const int64_t nb = gridDim.x, lb = dev::xcd_remap(blockIdx.x, nb);
    int64_t sb, se;
    range_of(lb, nb, S, &sb, &se);
    const double alpha = small[tiled::kBiAlpha];
    double acc = 0.0;
    for (int64_t s = sb + threadIdx.x; s < se; s += blockDim.x) {
        const double x = fma(-alpha, v[s], r[s]);
        sv[s] = x;
        acc = fma(x, x, acc);
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partials[lb] = acc;
}

// x += alpha p + omega s; r = s - omega t; partials <rh, r>, ||r||^2
__global__ __launch_bounds__(256) void k_bi_update(double* __restrict__ x, const double* __restrict__ p,
                                                   const double* __restrict__ sv, const double* __restrict__ t,
                                                   double* __restrict__ r, const double* __restrict__ rh, int first,
                                                   int64_t S, const double* small, double* partials, const Ctrl* c) {
    if (c->active == 0) return;
    __shared__ double red[4];
    const int64_t nb = gridDim.x, lb = dev::xcd_remap(blockIdx.x, nb);
    int64_t sb, se;
    range_of(lb, nb, S, &sb, &se);
    const double alpha = small[tiled::kBiAlpha], omega = small[tiled::kBiOmega];
    double a0 = 0.0, a1 = 0.0;
    for (int64_t s = sb + threadIdx.x; s < se; s += blockDim.x) {
        const double ss = sv[s];
        const double xo = first ? 0.0 : x[s];
        x[s] = fma(omega, ss, fma(alpha, p[s], xo));
        const double rn = fma(-omega, t[s], ss);
        r[s] = rn;
        a0 = fma(rh[s], rn, a0);
        a1 = fma(rn, rn, a1);
    }
    a0 = block_sum(a0, red);
    a1 = block_sum(a1, red);
    if (threadIdx.x == 0) {
        partials[lb] = a0;
        partials[nb + lb] = a1;
    }
}

// p = r + beta (p - omega v)
__global__ __launch_bounds__(256) void k_bi_p(double* __restrict__ p, const double* __restrict__ r,
                                              const double* __restrict__ v, int64_t S, const double* small,
                                              const Ctrl* c) {
    if (c->active == 0) return;
    const double beta = small[tiled::kBiBeta], omega = small[tiled::kBiOmega];
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x)
        p[s] = fma(beta, fma(-omega, v[s], p[s]), r[s]);
}

// Safeguard: if the iteration ended with a residual above its starting
// value (BiCGStab can diverge on strongly non-normal J_pi), the correction
// is replaced by one Richardson step, delta = D b (= rh).
__global__ __launch_bounds__(256) void k_bi_final(const double* __restrict__ V, const double* __restrict__ x,
                                                  const double* __restrict__ p, const double* __restrict__ rh,
                                                  const Ctrl* __restrict__ c, int64_t S, const double* small,
                                                  double* __restrict__ Vn) {
    const bool half = small[tiled::kBiHalf] != 0.0;
    const int x_valid = (c->steps_total - (half ? 1 : 0)) >= 1;
    if (!(c->resid <= c->beta)) {
        for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x)
            Vn[s] = V[s] + rh[s];
        return;
    }
    const double alpha = small[tiled::kBiAlpha];
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
        double d = x_valid ? x[s] : 0.0;
        if (half) d = fma(alpha, p[s], d);
        Vn[s] = V[s] + d;
    }
}

// ---------------------------------------------------------------------------
// TFQMR (Freund's transpose-free QMR) on J delta = b, in the form with two
// half steps per iteration (u_m alternates between u_j and q_j = u_j -
// alpha v_j).  x lags one half step: the pending update x += eta d is folded
// into the next kernel that rewrites d, and into the final result.
// ---------------------------------------------------------------------------

// r_0 = D b; r* = w = u = r_0; d = x = 0; partial ||r_0||^2
__global__ __launch_bounds__(256) void k_tq_init(const double* __restrict__ b, const double* __restrict__ dinv,
                                                 double* __restrict__ rs, double* __restrict__ w,
                                                 double* __restrict__ u, double* __restrict__ d,
                                                 double* __restrict__ x, int64_t S, double* partials) {
    __shared__ double red[4];
    const int64_t nb = gridDim.x, lb = dev::xcd_remap(blockIdx.x, nb);
    int64_t sb, se;
    range_of(lb, nb, S, &sb, &se);
    double acc = 0.0;
    for (int64_t s = sb + threadIdx.x; s < se; s += blockDim.x) {
        const double r = dinv ? b[s] * dinv[s] : b[s];
        rs[s] = r;
        w[s] = r;
        u[s] = r;
        d[s] = 0.0;
        x[s] = 0.0;
        acc = fma(r, r, acc);
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partials[lb] = acc;
}

// even half step: x += eta d; d = u + coef d; w -= alpha J u; q = u - alpha v;
// partial ||w||^2
__global__ __launch_bounds__(256) void k_tq_even(double* __restrict__ x, double* __restrict__ d,
                                                 const double* __restrict__ u, double* __restrict__ w,
                                                 const double* __restrict__ Au, const double* __restrict__ v,
                                                 double* __restrict__ q, int64_t S, const double* small,
                                                 double* partials, const Ctrl* c) {
    if (c->active == 0) return;
    __shared__ double red[4];
    const int64_t nb = gridDim.x, lb = dev::xcd_remap(blockIdx.x, nb);
    int64_t sb, se;
    range_of(lb, nb, S, &sb, &se);
    const double alpha = small[tiled::kTqAlpha], coef = small[tiled::kTqCoef], eta = small[tiled::kTqEta];
    double acc = 0.0;
    for (int64_t s = sb + threadIdx.x; s < se; s += blockDim.x) {
        const double dold = d[s];
        const double us = u[s];
        x[s] = fma(eta, dold, x[s]);
        d[s] = fma(coef, dold, us);
        const double wn = fma(-alpha, Au[s], w[s]);
        w[s] = wn;
        q[s] = fma(-alpha, v[s], us);
        acc = fma(wn, wn, acc);
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partials[lb] = acc;
}

// u = w + beta q
__global__ __launch_bounds__(256) void k_tq_u(double* __restrict__ u, const double* __restrict__ w,
                                              const double* __restrict__ q, int64_t S, const double* small,
                                              const Ctrl* c) {
    if (c->active == 0) return;
    const double beta = small[tiled::kTqBeta];
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x)
        u[s] = fma(beta, q[s], w[s]);
}

// x += eta d: the pending half step
__global__ __launch_bounds__(256) void k_tq_commit(double* __restrict__ x, const double* __restrict__ d, int64_t S,
                                                   const double* small) {
    const double eta = small[tiled::kTqEta];
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x)
        x[s] = fma(eta, d[s], x[s]);
}

// Vn = V + x.  Safeguard: if the solve stopped without passing its test and
// its true residual (recomputed into c->resid) exceeds ||r_0||, the
// correction is replaced by one Richardson step, delta = D b (= r*).
__global__ __launch_bounds__(256) void k_tq_final(const double* __restrict__ V, const double* __restrict__ x,
                                                  const double* __restrict__ rs, const Ctrl* __restrict__ c,
                                                  int64_t S, const double* small, double* __restrict__ Vn) {
    const bool fallback = !c->converged && !(c->resid <= small[tiled::kTqR0]);
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x)
        Vn[s] = fallback ? V[s] + rs[s] : V[s] + x[s];
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------

template <int VAR>
int launch_tiled(const PpiView& P, const LaunchShape& sh, tiled::TileParams p, int mj, hipStream_t st) {
    p.col = P.col;
    p.val = P.val;
    p.rp = P.rp;
    p.k = P.k;
    p.S = P.S;
    p.gamma = P.gamma;
    p.dinv = P.dinv;
    p.flat_e = P.flat_e;
    p.spt = sh.spt;
    const bool pipe_ok = wave_tiles_ok(P, sh.spt);
    p.pipe = pipe_ok ? P.pipe : 0;
    p.band = (p.pipe == 1) ? P.band : nullptr;
    p.sten = (p.pipe == 1 && !p.band && P.sten_np > 0) ? P.sten : nullptr;
    p.sten_off = P.sten_off;
    p.sten_pairs = P.sten_pairs ? 1 : 0;
    p.keep = (p.pipe == 1 && P.keep) ? 1 : 0;
    p.ntiles = (P.S + sh.spt - 1) / sh.spt;
    int nb = sh.nb;
    if (nb > p.ntiles) nb = (int)p.ntiles;  // (wave tiles: some waves may own no tile)
    if (nb < 1) nb = 1;
    const int vec = P.fp32 ? P.vec : (P.vec > 2 ? 2 : P.vec);
    if (sh.ev0) IPI_HIP(hipEventRecord(sh.ev0, st));
    if (VAR == tiled::kArnoldi) {
        if (P.fp32) tiled_arnoldi_f32(p, sh.lanes, vec, nb, mj, st);
        else tiled_arnoldi_f64(p, sh.lanes, vec, nb, mj, st);
    } else {
        if (VAR == tiled::kTfqW || VAR == tiled::kTfqV) tiled_tfqmr(VAR, P.fp32, p, sh.lanes, vec, nb, st);
        else tiled_other(VAR, P.fp32, p, sh.lanes, vec, nb, st);
    }
    if (sh.ev1) IPI_HIP(hipEventRecord(sh.ev1, st));
    IPI_HIP(hipGetLastError());
    return nb;
}

int clamp_nb(int nb, int64_t S) {
    int64_t need = (S + kBlock - 1) / kBlock;
    if (nb > need) nb = (int)need;
    return nb < 1 ? 1 : nb;
}

void fin_scalar(double* small, const double* partials, int nb, Ctrl* c, int mode, int j, int pbuf, int always,
                hipStream_t st) {
    hipLaunchKernelGGL(k_fin_scalar, dim3(1), dim3(kFinThreads), 0, st, small, partials, (int64_t)nb, c, mode, j, pbuf,
                       always);
}

}  // namespace

int mj_bucket(int m) {
    if (m <= 8) return 8;
    if (m <= 16) return 16;
    if (m <= 32) return 32;
    return 64;
}

void k_launch_ctrl_reset(Ctrl* c, double target, int max_inner, int restart, double omega, hipStream_t st) {
    hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, st, c, target, max_inner, restart, omega);
    IPI_HIP(hipGetLastError());
}

void k_launch_init_cycle(const double* b, const double* dinv, double* u0, int64_t S, double* small, double* partials,
                         Ctrl* c, int nb, hipStream_t st) {
    nb = clamp_nb(nb, S);
    hipLaunchKernelGGL(k_init_cycle, dim3(nb), dim3(kBlock), 0, st, b, dinv, u0, S, partials);
    fin_scalar(small, partials, nb, c, FIN_CYCLE, 0, 0, 1, st);
    IPI_HIP(hipGetLastError());
}

void k_launch_resid_cycle(const PpiView& P, const LaunchShape& sh, const double* b, const double* delta, double* u0,
                          double* small, double* partials, Ctrl* c, hipStream_t st) {
    TileParams p{};
    p.x = delta;
    p.b = b;
    p.out = u0;
    p.small = small;
    p.partials = partials;
    p.ctrl = c;
    const int nb = launch_tiled<kResid>(P, sh, p, 1, st);
    fin_scalar(small, partials, nb, c, FIN_CYCLE, 0, 0, 1, st);
    IPI_HIP(hipGetLastError());
}

void k_launch_arnoldi(const PpiView& P, const LaunchShape& sh, double* basis, int j, int mj, double* small,
                      double* partials, Ctrl* c, hipStream_t st) {
    TileParams p{};
    p.basis = basis;
    p.j = j;
    p.small = small;
    p.partials = partials;
    p.ctrl = c;
    const int nb = launch_tiled<kArnoldi>(P, sh, p, mj, st);
    hipLaunchKernelGGL(k_fin_hcol, dim3(j + 1), dim3(kFinThreads), 0, st, small, (const double*)partials, (int64_t)nb,
                       (const Ctrl*)c, j, 0);
    IPI_HIP(hipGetLastError());
}

void k_launch_dots(double* basis, int64_t S, int j, int mj, double* small, double* partials, Ctrl* c, int nb,
                   hipStream_t st) {
    nb = clamp_nb(nb, S);
    switch (mj) {
        case 8: hipLaunchKernelGGL(k_dots<8>, dim3(nb), dim3(kBlock), 0, st, basis, S, j, partials, c); break;
        case 16: hipLaunchKernelGGL(k_dots<16>, dim3(nb), dim3(kBlock), 0, st, basis, S, j, partials, c); break;
        case 32: hipLaunchKernelGGL(k_dots<32>, dim3(nb), dim3(kBlock), 0, st, basis, S, j, partials, c); break;
        default: hipLaunchKernelGGL(k_dots<64>, dim3(nb), dim3(kBlock), 0, st, basis, S, j, partials, c); break;
    }
    hipLaunchKernelGGL(k_fin_hcol, dim3(j + 1), dim3(kFinThreads), 0, st, small, (const double*)partials, (int64_t)nb,
                       (const Ctrl*)c, j, 1);
    IPI_HIP(hipGetLastError());
}

void k_launch_orth(double* basis, int64_t S, int j, int mj, int second_pass, int final_pass, double* small,
                   double* partials, Ctrl* c, int nb, hipStream_t st) {
    nb = clamp_nb(nb, S);
#define ORTH(MJ)                                                                                               \
    hipLaunchKernelGGL(k_orth<MJ>, dim3(nb), dim3(kBlock), 0, st, basis, S, j, second_pass, final_pass, small, \
                       partials, c)
    switch (mj) {
        case 8: ORTH(8); break;
        case 16: ORTH(16); break;
        case 32: ORTH(32); break;
        default: ORTH(64); break;
    }
#undef ORTH
    if (final_pass) fin_scalar(small, partials, nb, c, FIN_GIVENS, j, 0, 0, st);
    IPI_HIP(hipGetLastError());
}

void k_launch_gmres_update(double* basis, int64_t S, int mj, const double* small, const Ctrl* c, double* delta,
                           int first, const double* V, double* Vn, int nb, hipStream_t st) {
    nb = clamp_nb(nb, S);
#define UPD(MJ) \
    hipLaunchKernelGGL(k_gmres_update<MJ>, dim3(nb), dim3(kBlock), 0, st, basis, S, small, c, delta, first, V, Vn)
    switch (mj) {
        case 8: UPD(8); break;
        case 16: UPD(16); break;
        case 32: UPD(32); break;
        default: UPD(64); break;
    }
#undef UPD
    IPI_HIP(hipGetLastError());
}

void k_launch_rich0(const double* b, const double* dinv, double* dq, int64_t S, double* partials, Ctrl* c, int nb,
                    double* small, hipStream_t st) {
    nb = clamp_nb(nb, S);
    hipLaunchKernelGGL(k_rich0, dim3(nb), dim3(kBlock), 0, st, b, dinv, dq, S, partials, c);
    fin_scalar(small, partials, nb, c, FIN_RICH0, 0, 0, 0, st);
    IPI_HIP(hipGetLastError());
}

void k_launch_rich(const PpiView& P, const LaunchShape& sh, const double* b, const double* dp, double* dq, int pbuf,
                   double* partials, Ctrl* c, double* small, hipStream_t st, int test_after, int obuf) {
    TileParams p{};
    p.x = dp;
    p.b = b;
    p.out = dq;
    p.partials = partials;
    p.ctrl = c;
    p.pbuf = pbuf;
    const int nb = launch_tiled<kRich>(P, sh, p, 1, st);
    if (test_after > 0) k_launch_fin_rich(small, partials, nb, c, test_after, pbuf, obuf < 0 ? 1 - pbuf : obuf, st);
    IPI_HIP(hipGetLastError());
}

void k_launch_fin_rich(double* small, const double* partials, int nb, Ctrl* c, int since, int pbuf, int obuf,
                       hipStream_t st) {
    fin_scalar(small, partials, nb, c, FIN_RICH, since, pbuf + 4 * (1 + obuf), 0, st);
}

void k_launch_axpy_result(const double* V, const double* d0, const double* d1, const double* d2, const Ctrl* c,
                          double* Vn, int64_t S, int nb, hipStream_t st) {
    hipLaunchKernelGGL(k_axpy_result, dim3(clamp_nb(nb, S)), dim3(kBlock), 0, st, V, d0, d1, d2, c, Vn, S);
    IPI_HIP(hipGetLastError());
}

void k_launch_bicgstab_iter(const PpiView& P, const LaunchShape& sh, double* x, double* r, const double* rh,
                            double* p, double* v, double* sv, double* t, int first, double* small, double* partials,
                            Ctrl* c, int nb, hipStream_t st) {
    const int64_t S = P.S;
    TileParams a{};
    a.x = p;
    a.out = v;
    a.dotA = rh;
    a.dot_self = 0;
    a.small = small;
    a.partials = partials;
    a.ctrl = c;
    int nbt = launch_tiled<kApply>(P, sh, a, 2, st);
    fin_scalar(small, partials, nbt, c, FIN_BI_ALPHA, 0, 0, 0, st);
    const int nbe = clamp_nb(nb, S);
    hipLaunchKernelGGL(k_bi_s, dim3(nbe), dim3(kBlock), 0, st, r, v, sv, S, small, partials, c);
    fin_scalar(small, partials, nbe, c, FIN_BI_S, 0, 0, 0, st);
    TileParams b2 = a;
    b2.x = sv;
    b2.out = t;
    b2.dotA = sv;
    b2.dot_self = 1;
    nbt = launch_tiled<kApply>(P, sh, b2, 2, st);
    fin_scalar(small, partials, nbt, c, FIN_BI_OMEGA, 0, 0, 0, st);
    hipLaunchKernelGGL(k_bi_update, dim3(nbe), dim3(kBlock), 0, st, x, p, sv, t, r, rh, first, S, small, partials, c);
    fin_scalar(small, partials, nbe, c, FIN_BI_UPDATE, 0, 0, 0, st);
    hipLaunchKernelGGL(k_bi_p, dim3(nbe), dim3(kBlock), 0, st, p, r, v, S, small, c);
    IPI_HIP(hipGetLastError());
}

void k_launch_bicgstab_init(const double* b, const double* dinv, double* r, double* rh, double* p, int64_t S,
                            double* small, double* partials, Ctrl* c, int nb, hipStream_t st) {
    nb = clamp_nb(nb, S);
    hipLaunchKernelGGL(k_bi_init, dim3(nb), dim3(kBlock), 0, st, b, dinv, r, rh, p, S, partials);
    fin_scalar(small, partials, nb, c, FIN_BI_INIT, 0, 0, 1, st);
    IPI_HIP(hipGetLastError());
}

void k_launch_bicgstab_final(const double* V, const double* x, const double* p, const double* rh, const Ctrl* c,
                             int64_t S, const double* small, double* Vn, int nb, hipStream_t st) {
    hipLaunchKernelGGL(k_bi_final, dim3(clamp_nb(nb, S)), dim3(kBlock), 0, st, V, x, p, rh, c, S, small, Vn);
    IPI_HIP(hipGetLastError());
}

void k_launch_tfqmr_init(const PpiView& P, const LaunchShape& sh, const double* b, const TfqmrVecs& t,
                         double* small, double* partials, Ctrl* c, int nb, hipStream_t st) {
    const int64_t S = P.S;
    const int nbe = clamp_nb(nb, S);
    hipLaunchKernelGGL(k_tq_init, dim3(nbe), dim3(kBlock), 0, st, b, P.dinv, t.rs, t.w, t.u, t.d, t.x, S, partials);
    fin_scalar(small, partials, nbe, c, FIN_TQ_INIT, 0, 0, 1, st);
    // v_0 = J u_0 (= the first J u); sigma_0 = <v_0, r*>
    TileParams a{};
    a.x = t.u;
    a.out = t.Au;
    a.tv = t.v;
    a.taq = t.Aq;
    a.trs = t.rs;
    a.small = small;
    a.partials = partials;
    a.ctrl = c;
    const int nbt = launch_tiled<kTfqV>(P, sh, a, 1, st);
    fin_scalar(small, partials, nbt, c, FIN_TQ_SIGMA, 0, 0, 0, st);
    IPI_HIP(hipGetLastError());
}

void k_launch_tfqmr_iter(const PpiView& P, const LaunchShape& sh0, const LaunchShape& sh1, const TfqmrVecs& t,
                         double* small, double* partials, Ctrl* c, int nb, hipStream_t st) {
    const int64_t S = P.S;
    const int nbe = clamp_nb(nb, S);
    // even half step (J u_j is known from the previous v update)
    hipLaunchKernelGGL(k_tq_even, dim3(nbe), dim3(kBlock), 0, st, t.x, t.d, t.u, t.w, t.Au, t.v, t.q, S, small,
                       partials, c);
    fin_scalar(small, partials, nbe, c, FIN_TQ_STEP, 0, 0, 0, st);
    // odd half step: J q_j fused with the w, d, x updates and <w, r*>
    TileParams a{};
    a.x = t.q;
    a.out = t.Aq;
    a.tx = t.x;
    a.td = t.d;
    a.tw = t.w;
    a.trs = t.rs;
    a.small = small;
    a.partials = partials;
    a.ctrl = c;
    int nbt = launch_tiled<kTfqW>(P, sh0, a, 2, st);
    fin_scalar(small, partials, nbt, c, FIN_TQ_STEP, 1, 0, 0, st);
    // u_{j+1} = w + beta q_j; v_{j+1} = J u_{j+1} + beta (J q_j + beta v_j); sigma
    hipLaunchKernelGGL(k_tq_u, dim3(nbe), dim3(kBlock), 0, st, t.u, t.w, t.q, S, small, c);
    TileParams b2{};
    b2.x = t.u;
    b2.out = t.Au;
    b2.tv = t.v;
    b2.taq = t.Aq;
    b2.trs = t.rs;
    b2.small = small;
    b2.partials = partials;
    b2.ctrl = c;
    nbt = launch_tiled<kTfqV>(P, sh1, b2, 1, st);
    fin_scalar(small, partials, nbt, c, FIN_TQ_SIGMA, 0, 0, 0, st);
    IPI_HIP(hipGetLastError());
}

void k_launch_tfqmr_final(const PpiView& P, const LaunchShape& sh, const double* b, const double* V,
                          const TfqmrVecs& t, bool check, Ctrl* c, double* small, double* partials, double* Vn, int nb,
                          hipStream_t st) {
    const int64_t S = P.S;
    const int nbe = clamp_nb(nb, S);
    hipLaunchKernelGGL(k_tq_commit, dim3(nbe), dim3(kBlock), 0, st, t.x, t.d, S, small);
    if (check) {
        // true residual D (b - J delta) into the scratch q, its norm into c->resid
        TileParams p{};
        p.x = t.x;
        p.b = b;
        p.out = t.q;
        p.small = small;
        p.partials = partials;
        p.ctrl = c;
        const int nbt = launch_tiled<kResid>(P, sh, p, 1, st);
        fin_scalar(small, partials, nbt, c, FIN_TQ_TRUE, 0, 0, 1, st);
    }
    hipLaunchKernelGGL(k_tq_final, dim3(nbe), dim3(kBlock), 0, st, V, t.x, t.rs, c, S, small, Vn);
    IPI_HIP(hipGetLastError());
}

}  // namespace ipi
