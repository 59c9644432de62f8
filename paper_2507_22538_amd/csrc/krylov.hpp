// Shared declarations of the inner-solve kernels (GMRES, Richardson, TFQMR,
// BiCGStab) that apply the matrix-free J_pi = I - gamma P_pi (Sec. III-B.3:
// the matrix shell) with the compact P_pi.
#pragma once

#include "internal.hpp"

namespace ipi {

// Layout of the small device buffer (doubles): Hessenberg matrix H
// (column-major, leading dimension kLdH), Givens cosines/sines, the rotated
// right-hand side g, the basis scales c_i (v_i = c_i * u_i), scratch.
constexpr int kLdH = kMaxRestart + 1;
constexpr int kOffH = 0;
constexpr int kOffCS = kOffH + kLdH * kMaxRestart;
constexpr int kOffSN = kOffCS + kMaxRestart;
constexpr int kOffGV = kOffSN + kMaxRestart;
constexpr int kOffSC = kOffGV + kLdH;
constexpr int kOffH2 = kOffSC + kLdH;  // second Gram-Schmidt pass coefficients
constexpr int kOffScal = kOffH2 + kLdH; // scalars of TFQMR / BiCGStab
constexpr int kSmallDoubles = 8192;

// P_pi as handed to the product kernels.
struct PpiView {
    const int* col;
    const void* val;       // double or float
    const int64_t* rp;     // CSR row pointers, or nullptr for uniform rows (row s at s*k)
    int k;                 // uniform row length (ELL)
    int vec;               // vector width of the loads (1 for CSR)
    bool fp32;
    int64_t S;
    double gamma;
    const double* dinv;    // Jacobi scaling D = diag(J_pi)^-1, or nullptr
    int flat_e;            // > 0: stream uniform rows in chunks of flat_e values
    int pipe = 0;          // flat schedule: 0 workgroup tiles, 1 wave tiles
    const int32_t* band = nullptr;  // band form: first column of each row (wave tiles only)
    // stencil form (wave tiles only, not with the band form): per row its
    // first column and pattern, the patterns' column offsets (sten_np x k),
    // and whether every pattern's columns come in adjacent pairs
    const uint32_t* sten = nullptr;
    const int32_t* sten_off = nullptr;
    int sten_np = 0;
    bool sten_pairs = false;
    int band_hl = 0, band_hr = 0;   // band form: a row of state s reads [s - band_hl, s + band_hr]
    int band_hl_in = 0, band_hr_in = 0;  // the same for the interior states [H, S - H),
                                         // H = max(band_hl, band_hr)
    bool keep = false;              // wave tiles: load P_pi through the caches (it fits the
                                    // last-level cache with the sweep's vectors)
    bool lds_prefetch = true;       // blocked sweeps on long rows: prefetch the next block through LDS
    bool keep_block = false;        // same for the blocked sweeps, whose workgroups re-read their
                                    // neighbours' halo rows
};

// the wave-tile schedule applies: chunk widths 2 (FP64), 4, 8; at most 64
// states and 1024 chunk slots per wave tile
inline bool wave_tiles_ok(const PpiView& P, int spt) {
    return P.flat_e > 0 && (P.flat_e == 4 || P.flat_e == 8 || (P.flat_e == 2 && !P.fp32)) && spt <= 64 &&
           (int64_t)spt * (P.k / P.flat_e) <= 1024;
}

struct LaunchShape {
    int lanes;       // lanes per row of P_pi
    int spt;         // states per tile
    int nb;          // blocks (persistent grid)
    hipEvent_t ev0 = nullptr;  // when set: recorded right before / after the product kernel
    hipEvent_t ev1 = nullptr;
};

// GMRES
void k_launch_ctrl_reset(Ctrl* c, double target, int max_inner, int restart, double omega, hipStream_t st);
void k_launch_init_cycle(const double* b, const double* dinv, double* u0, int64_t S, double* small, double* partials,
                         Ctrl* c, int nb, hipStream_t st);
void k_launch_resid_cycle(const PpiView& P, const LaunchShape& sh, const double* b, const double* delta, double* u0,
                          double* small, double* partials, Ctrl* c, hipStream_t st);
void k_launch_arnoldi(const PpiView& P, const LaunchShape& sh, double* basis, int j, int mj, double* small,
                      double* partials, Ctrl* c, hipStream_t st);
void k_launch_dots(double* basis, int64_t S, int j, int mj, double* small, double* partials, Ctrl* c, int nb,
                   hipStream_t st);
void k_launch_orth(double* basis, int64_t S, int j, int mj, int second_pass, int final_pass, double* small,
                   double* partials, Ctrl* c, int nb, hipStream_t st);
void k_launch_gmres_update(double* basis, int64_t S, int mj, const double* small, const Ctrl* c, double* delta,
                           int first, const double* V, double* Vn, int nb, hipStream_t st);

// Richardson
void k_launch_rich0(const double* b, const double* dinv, double* dq, int64_t S, double* partials, Ctrl* c, int nb,
                    double* small, hipStream_t st);
// one Richardson sweep; test_after > 0: then run the stopping test, counting
// test_after sweeps since the previous test (0: no test after this sweep)
void k_launch_rich(const PpiView& P, const LaunchShape& sh, const double* b, const double* dp, double* dq, int pbuf,
                   double* partials, Ctrl* c, double* small, hipStream_t st, int test_after = 1, int obuf = -1);
// Vn = V + delta[result_buf] over three delta buffers (result_buf -1: V)
void k_launch_axpy_result(const double* V, const double* d0, const double* d1, const double* d2, const Ctrl* c,
                          double* Vn, int64_t S, int nb, hipStream_t st);
// The stopping test after `since` sweeps: the partials hold |r|^2 of the last
// sweep's input, delta[pbuf]; the result is delta[pbuf] when it passes, else
// delta[obuf] (the last sweep's output).
void k_launch_fin_rich(double* small, const double* partials, int nb, Ctrl* c, int since, int pbuf, int obuf,
                       hipStream_t st);
// T (4, 8 or 16) Richardson sweeps in one launch for band-form P_pi whose rows
// read a short window around their state (temporal blocking; the iterates
// are those of T one-sweep launches); partials get one |r|^2 sum per
// workgroup (rich_block_grid of them) for the test on the last sweep.
bool rich_block_ok(const PpiView& P, int T);
int rich_block_grid(const PpiView& P, int T);
void k_launch_rich_block(const PpiView& P, int T, const double* b, const double* x, double* out_prev, double* out_last,
                         double* partials, Ctrl* c, hipStream_t st);

// BiCGStab
void k_launch_bicgstab_init(const double* b, const double* dinv, double* r, double* rh, double* p, int64_t S,
                            double* small, double* partials, Ctrl* c, int nb, hipStream_t st);
void k_launch_bicgstab_iter(const PpiView& P, const LaunchShape& sh, double* x, double* r, const double* rh,
                            double* p, double* v, double* sv, double* t, int first, double* small, double* partials,
                            Ctrl* c, int nb, hipStream_t st);
void k_launch_bicgstab_final(const double* V, const double* x, const double* p, const double* rh, const Ctrl* c,
                             int64_t S, const double* small, double* Vn, int nb, hipStream_t st);

// TFQMR
struct TfqmrVecs {
    double* x;   // the correction delta (lags eta * d)
    double* w;
    double* u;
    double* q;
    double* d;
    double* v;
    double* Au;  // J u_j
    double* Aq;  // J q_j
    double* rs;  // shadow r* = r_0
};
void k_launch_tfqmr_init(const PpiView& P, const LaunchShape& sh, const double* b, const TfqmrVecs& t,
                         double* small, double* partials, Ctrl* c, int nb, hipStream_t st);
// one iteration = two half steps = two J_pi products (sh0, sh1: their launch shapes / timers)
void k_launch_tfqmr_iter(const PpiView& P, const LaunchShape& sh0, const LaunchShape& sh1, const TfqmrVecs& t,
                         double* small, double* partials, Ctrl* c, int nb, hipStream_t st);
// delta = x + eta d; check: recompute the true residual of an unconverged
// end (one more product) for the safeguard; Vn = V + delta
void k_launch_tfqmr_final(const PpiView& P, const LaunchShape& sh, const double* b, const double* V,
                          const TfqmrVecs& t, bool check, Ctrl* c, double* small, double* partials, double* Vn, int nb,
                          hipStream_t st);

int mj_bucket(int m);

}  // namespace ipi
