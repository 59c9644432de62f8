/*
 * Seeded synthetic MDP generators (inputs only).
 *
 * This file produces the transition tensor P in the row-stacked CSR layout
 * of the flattened-tensor equation (Sec. III-B.2: row index s*A + a,
 * 0-based), the dense stage-cost matrix g (index s*A + a) and nothing else.
 * It holds none of the method's arithmetic: no Bellman operator, no policy,
 * no linear solve.  Both the CPU oracle and the GPU library receive the
 * arrays written here.
 *
 * Randomness is counter based: every draw is splitmix64 of a key built from
 * (seed, mdp, row, j), so results do not depend on the thread count.
 *
 * Generators:
 *   ipigen_random_*   random sparse MDP: k distinct uniform columns per row
 *                     (Floyd's sampling), Dirichlet(1) probabilities, costs
 *                     U[0,1).  Row lengths uniform in [k_lo, k_hi].
 *   ipigen_birth_death  banded birth-death chain shaped like the SIS study
 *                     (Sec. IV-B): 24 columns per row in a window around s,
 *                     Binomial(23, p_a) weights.
 *   ipigen_pendulum   inverted pendulum (Sec. IV-C): forward-Euler step of
 *                     theta'' + g sin(theta) = F on an N x N (angle,velocity)
 *                     grid, bilinear interpolation onto 4 grid states.
 *   ipigen_maze       deterministic H x W grid world (Sec. IV-D).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))

/* ---- counter-based RNG: splitmix64 finaliser (Steele, Lea, Flood 2014) ---- */
static inline uint64_t sm64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

EXPORT uint64_t ipigen_key(uint64_t seed, uint64_t mdp, uint64_t row, uint64_t j) {
    return sm64(sm64(sm64(sm64(seed) ^ mdp) ^ row) ^ j);
}

/* uniform in [0,1) with 53 random bits */
static inline double u01(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }
/* uniform in (0,1] */
static inline double u01_open0(uint64_t x) { return (double)((x >> 11) + 1) * (1.0 / 9007199254740992.0); }
/* uniform integer in [0, n) by 128-bit multiply-high */
static inline uint64_t uint_below(uint64_t x, uint64_t n) {
    return (uint64_t)(((unsigned __int128)x * (unsigned __int128)n) >> 64);
}

/* stream tags (the j component of the key) */
#define TAG_LEN  0xA11CE0000ULL
#define TAG_COST 0xC0570000ULL
#define TAG_COL  0xC0100000ULL
#define TAG_PROB 0x9E0B0000ULL
#define TAG_ACT  0xAC700000ULL
#define TAG_WALL 0x3A110000ULL

/* ------------------------------------------------------------------------ */
/* random sparse                                                             */
/* ------------------------------------------------------------------------ */

static inline int32_t row_len(uint64_t seed, uint64_t mdp, uint64_t row, int32_t k_lo, int32_t k_hi) {
    if (k_hi <= k_lo) return k_lo;
    return k_lo + (int32_t)uint_below(ipigen_key(seed, mdp, row, TAG_LEN), (uint64_t)(k_hi - k_lo + 1));
}

/* Fill row_ptr (length S*A+1) for the random sparse generator; returns nnz. */
EXPORT int64_t ipigen_random_rowptr(int64_t S, int32_t A, int32_t k_lo, int32_t k_hi,
                                    uint64_t seed, uint64_t mdp, int64_t* row_ptr) {
    int64_t R = S * (int64_t)A;
    int64_t acc = 0;
    if (row_ptr) row_ptr[0] = 0;
    for (int64_t r = 0; r < R; ++r) {
        acc += row_len(seed, mdp, (uint64_t)r, k_lo, k_hi);
        if (row_ptr) row_ptr[r + 1] = acc;
    }
    return acc;
}

static void insertion_sort_i32(int32_t* a, int n) {
    for (int i = 1; i < n; ++i) {
        int32_t v = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
        a[j + 1] = v;
    }
}

/* Fill col/val/g given row_ptr from ipigen_random_rowptr.
 * Columns: k distinct values in [0,S) by Floyd's algorithm, sorted.
 * Probabilities: E_j = -ln U_j normalised by their sum (Dirichlet(1)).
 * Costs: U[0,1).  Requires k_hi <= S. */
EXPORT void ipigen_random_fill(int64_t S, int32_t A, uint64_t seed, uint64_t mdp,
                               const int64_t* row_ptr, int32_t* col, double* val, double* g) {
    int64_t R = S * (int64_t)A;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t r = 0; r < R; ++r) {
        int64_t b = row_ptr[r];
        int k = (int)(row_ptr[r + 1] - b);
        int32_t* c = col + b;
        /* Floyd: for j = S-k .. S-1 pick t in [0, j]; take j if t already taken */
        int n = 0;
        for (int64_t jj = S - k; jj < S; ++jj) {
            uint64_t t = uint_below(ipigen_key(seed, mdp, (uint64_t)r, TAG_COL + (uint64_t)(jj - (S - k))),
                                    (uint64_t)(jj + 1));
            int hit = 0;
            for (int q = 0; q < n; ++q) if ((uint64_t)c[q] == t) { hit = 1; break; }
            c[n++] = hit ? (int32_t)jj : (int32_t)t;
        }
        insertion_sort_i32(c, k);
        double sum = 0.0;
        for (int q = 0; q < k; ++q) {
            double e = -log(u01_open0(ipigen_key(seed, mdp, (uint64_t)r, TAG_PROB + (uint64_t)q)));
            val[b + q] = e;
            sum += e;
        }
        if (!(sum > 0.0)) { /* all U == 1 exactly: degenerate, use uniform weights */
            for (int q = 0; q < k; ++q) val[b + q] = 1.0 / k;
        } else {
            for (int q = 0; q < k; ++q) val[b + q] /= sum;
        }
        g[r] = u01(ipigen_key(seed, mdp, (uint64_t)r, TAG_COST));
    }
}

/* ------------------------------------------------------------------------ */
/* banded birth-death chain (SIS-shaped)                                     */
/* ------------------------------------------------------------------------ */

/* nnz = S*A*24; requires S >= 24.
 * Row (s,a): columns w0..w0+23 with w0 = clamp(s-12, 0, S-24); weights are
 * the Binomial(23, p_a) pmf, p_a = 0.55 - 0.10*a/(A-1), renormalised.
 * Cost g(s,a) = a*c_a + (s/S)*c_inf with c_a ~ U[0,1) and c_inf = A. */
EXPORT void ipigen_birth_death(int64_t S, int32_t A, uint64_t seed,
                               int64_t* row_ptr, int32_t* col, double* val, double* g) {
    enum { K = 24 };
    double* pmf = (double*)malloc(sizeof(double) * (size_t)A * K);
    double* ca = (double*)malloc(sizeof(double) * (size_t)A);
    for (int a = 0; a < A; ++a) {
        double p = (A > 1) ? 0.55 - 0.10 * (double)a / (double)(A - 1) : 0.55;
        double s = 0.0;
        for (int j = 0; j < K; ++j) {
            /* C(23,j) p^j (1-p)^(23-j) via lgamma */
            double lc = lgamma(24.0) - lgamma((double)j + 1.0) - lgamma(24.0 - (double)j);
            double v = exp(lc + j * log(p) + (23 - j) * log1p(-p));
            pmf[a * K + j] = v;
            s += v;
        }
        for (int j = 0; j < K; ++j) pmf[a * K + j] /= s;
        ca[a] = u01(ipigen_key(seed, 0, (uint64_t)a, TAG_ACT));
    }
    const double cinf = (double)A;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < S; ++s) {
        int64_t w0 = s - 12;
        if (w0 < 0) w0 = 0;
        if (w0 > S - K) w0 = S - K;
        for (int a = 0; a < A; ++a) {
            int64_t r = s * A + a;
            int64_t b = r * K;
            row_ptr[r] = b;
            for (int j = 0; j < K; ++j) {
                col[b + j] = (int32_t)(w0 + j);
                val[b + j] = pmf[a * K + j];
            }
            g[r] = (double)a * ca[a] + ((double)s / (double)S) * cinf;
        }
    }
    row_ptr[S * (int64_t)A] = S * (int64_t)A * K;
    free(pmf);
    free(ca);
}

/* ------------------------------------------------------------------------ */
/* inverted pendulum                                                         */
/* ------------------------------------------------------------------------ */

/* N x N grid, s = i*N + j, theta_i = 2*pi*i/N (periodic), v_j = -10 + 20*j/(N-1).
 * Torques F_a = fmin + (fmax-fmin)*a/(A-1).  One forward-Euler step with
 * step Ts of theta'' = F - gacc*sin(theta); theta wraps, v clamps to [-10,10].
 * Bilinear weights on (i0, i0+1 mod N) x (j0, j0+1); exactly 4 entries per
 * row (explicit zeros kept), columns sorted.
 * Cost 2[(theta-pi)^2 + v^2] + F^2 (Sec. IV-C).  Requires N >= 2. */
EXPORT void ipigen_pendulum(int64_t N, int32_t A, double fmin, double fmax, double Ts,
                            int64_t* row_ptr, int32_t* col, double* val, double* g) {
    const double two_pi = 6.283185307179586476925286766559;
    const double pi = 3.141592653589793238462643383279;
    const double gacc = 9.80665;
    const double dth = two_pi / (double)N;
    const double dv = 20.0 / (double)(N - 1);
    const int64_t S = N * N;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < S; ++s) {
        int64_t i = s / N, j = s % N;
        double th = two_pi * (double)i / (double)N;
        double v = -10.0 + 20.0 * (double)j / (double)(N - 1);
        for (int a = 0; a < A; ++a) {
            double F = (A > 1) ? fmin + (fmax - fmin) * (double)a / (double)(A - 1) : 0.5 * (fmin + fmax);
            double th2 = th + Ts * v;
            double v2 = v + Ts * (F - gacc * sin(th));
            th2 = fmod(th2, two_pi);
            if (th2 < 0) th2 += two_pi;
            if (v2 < -10.0) v2 = -10.0;
            if (v2 > 10.0) v2 = 10.0;
            double x = th2 / dth;
            double fx = floor(x);
            double wx = x - fx;
            int64_t i0 = ((int64_t)fx) % N;
            if (i0 < 0) i0 += N;
            int64_t i1 = (i0 + 1) % N;
            double y = (v2 + 10.0) / dv;
            int64_t j0 = (int64_t)floor(y);
            if (j0 < 0) j0 = 0;
            if (j0 > N - 2) j0 = N - 2;
            double wy = y - (double)j0;
            if (wy < 0) wy = 0;
            if (wy > 1) wy = 1;
            int64_t c4[4] = {i0 * N + j0, i0 * N + j0 + 1, i1 * N + j0, i1 * N + j0 + 1};
            double w4[4] = {(1 - wx) * (1 - wy), (1 - wx) * wy, wx * (1 - wy), wx * wy};
            /* sort the 4 (col, weight) pairs by column */
            for (int p = 1; p < 4; ++p) {
                int64_t cc = c4[p];
                double ww = w4[p];
                int q = p - 1;
                while (q >= 0 && c4[q] > cc) { c4[q + 1] = c4[q]; w4[q + 1] = w4[q]; --q; }
                c4[q + 1] = cc;
                w4[q + 1] = ww;
            }
            int64_t r = s * A + a;
            int64_t b = r * 4;
            row_ptr[r] = b;
            for (int p = 0; p < 4; ++p) { col[b + p] = (int32_t)c4[p]; val[b + p] = w4[p]; }
            g[r] = 2.0 * ((th - pi) * (th - pi) + v * v) + F * F;
        }
    }
    row_ptr[S * (int64_t)A] = S * (int64_t)A * 4;
}

/* ------------------------------------------------------------------------ */
/* 2D maze                                                                   */
/* ------------------------------------------------------------------------ */

/* H x W grid, s = y*W + x (row-major), A = 5: stay, north, east, south, west.
 * Cells are walls with probability wall_frac (seeded); the goal (bottom-right)
 * and the start corner are never walls.  Each (s,a) has one entry: the
 * neighbour if it is inside the grid and not a wall, else s itself.
 * Costs: goal cell -100 for every action; a blocked move (off-grid or into a
 * wall) costs wall_cost; otherwise 0.  Wall cells keep every action in place
 * at cost 0 for "stay" and wall_cost otherwise. */
EXPORT void ipigen_maze(int64_t H, int64_t W, double wall_frac, double wall_cost, uint64_t seed,
                        int64_t* row_ptr, int32_t* col, double* val, double* g, uint8_t* wall_out) {
    const int64_t S = H * W;
    const int A = 5;
    uint8_t* wall = wall_out;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < S; ++s) {
        wall[s] = (uint8_t)(u01(ipigen_key(seed, 0, (uint64_t)s, TAG_WALL)) < wall_frac);
    }
    wall[S - 1] = 0;
    wall[0] = 0;
    const int dy[5] = {0, -1, 0, 1, 0};
    const int dx[5] = {0, 0, 1, 0, -1};
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < S; ++s) {
        int64_t y = s / W, x = s % W;
        for (int a = 0; a < A; ++a) {
            int64_t r = s * A + a;
            row_ptr[r] = r;
            int64_t ny = y + dy[a], nx = x + dx[a];
            int64_t t = s;
            int blocked = 0;
            if (a != 0) {
                if (wall[s] || ny < 0 || ny >= H || nx < 0 || nx >= W || wall[ny * W + nx]) blocked = 1;
                else t = ny * W + nx;
            }
            col[r] = (int32_t)t;
            val[r] = 1.0;
            if (s == S - 1) g[r] = -100.0;
            else g[r] = blocked ? wall_cost : 0.0;
        }
    }
    row_ptr[S * A] = S * A;
}
