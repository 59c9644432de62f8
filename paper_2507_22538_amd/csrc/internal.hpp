// Internal declarations shared by the translation units of libipi.so.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ipi.h"

namespace ipi {

// ---------------------------------------------------------------------------
// errors: internal code throws ipi::Error; the ABI layer converts to a status
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
    ipi_status status;
    Error(ipi_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

void set_last_error(const std::string& msg);

#define IPI_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            throw ::ipi::Error((e_ == hipErrorOutOfMemory) ? IPI_E_OOM : IPI_E_DEVICE,         \
                               std::string(#call) + ": " + hipGetErrorString(e_));             \
        }                                                                                      \
    } while (0)

#define IPI_REQUIRE(cond, status, msg)                    \
    do {                                                  \
        if (!(cond)) throw ::ipi::Error((status), (msg)); \
    } while (0)

constexpr int kBlock = 256;        // threads per workgroup (4 waves of 64)
constexpr int kMaxTileRows = 3072; // Q values held in LDS per tile of the Bellman pass (<= 48 KB)
// stencil form: at most this many column-offset patterns, and the first
// column of a row in the low kStenColBits bits of its word (the pattern in
// the bits above), so S < 2^kStenColBits
constexpr int kStenMaxPatterns = 8;
constexpr int kStenColBits = 29;
constexpr int kStenMaxK = 32;
constexpr int kMaxA = kMaxTileRows;
constexpr int kMaxRestart = 64;    // largest GMRES restart length
constexpr int kMaxSpmvTile = 4096; // states per tile of the P_pi products

// ---------------------------------------------------------------------------
// device control block of one inner solve (lives in device memory)
// ---------------------------------------------------------------------------
struct Ctrl {
    int32_t active;       // 1 while the current cycle / sweep batch continues
    int32_t j;            // Arnoldi steps done in this cycle
    int32_t steps_total;  // inner iterations done in this evaluation
    int32_t converged;    // forcing test met
    int32_t max_inner;
    int32_t restart;
    int32_t result_buf;   // Richardson: which delta buffer holds the answer
    int32_t breakdown;
    double target;        // alpha * rho_k (strict: stop when residual < target)
    double beta;          // norm of the initial residual of the cycle
    double resid;         // current 2-norm of the linear residual (estimate)
    double omega;         // Richardson scale
    uint64_t rho_bits;    // bit pattern of max |TV - V| (non-negative doubles order as integers)
    uint64_t vmax_bits;   // bit pattern of max |V|
};

// ---------------------------------------------------------------------------
// kernel configuration
// ---------------------------------------------------------------------------
struct Tuning {
    int bellman_lanes = 0;   // 0 = choose from the row length
    int bellman_spt = 0;     // states per tile
    int spmv_lanes = 0;
    int spmv_spt = 0;
    int bellman_chunk = 0;  // flat mode chunk width (0 = automatic)
    int spmv_chunk = 0;
    int spmv_schedule = 0;  // 0 automatic, 1 workgroup tiles, 2 wave tiles
    int spmv_workgroups = 0;  // 0 automatic
    int band_rows = 0;        // 0: use the band or stencil form when detected; -1: never
    int blocked_prefetch = 0; // long-row blocked sweeps: 0 LDS prefetch (persistent), -1 one block per workgroup
    int ppi_cached = 0;       // wave-tile P_pi loads: 0 cached when they fit (blocked sweeps:
                              // always), 1 always, -1 never
};

// Workspace of single-MDP solves (allocated on first solve)
struct Workspace {
    int64_t S = 0;
    int m = 0;               // GMRES restart length the basis was sized for
    int kmax = 0;
    bool fp32 = false;
    double* V = nullptr;     // current iterate
    double* TV = nullptr;    // scratch for T V
    double* b = nullptr;     // rhs TV - V of the inner solve
    double* delta = nullptr; // correction (two buffers for Richardson)
    double* delta2 = nullptr;
    double* basis = nullptr; // (m+1) x S Krylov basis (unnormalised)
    double* small = nullptr; // H, Givens, g, y, scales
    double* partials = nullptr;
    double* aux = nullptr;   // extra vectors for TFQMR / BiCGStab / Jacobi
    int naux = 0;
    double* diag = nullptr;  // Jacobi: diagonal of J_pi
    int32_t* pi = nullptr;
    int32_t* ppi_col = nullptr;
    int32_t* ppi_band = nullptr;  // first column of each P_pi row (band form)
    uint32_t* ppi_sten = nullptr; // word of each P_pi row (stencil form)
    void* ppi_val = nullptr; // double or float
    int64_t* ppi_rp = nullptr; // CSR row pointers when rows are not uniform
    int64_t* scan_tmp = nullptr;
    Ctrl* ctrl = nullptr;
    double* g_neg = nullptr; // -g for the maximisation mode (scratch-backed workspaces only)
    double* bpart = nullptr; // tile partial sums of the batched solver
    size_t bpart_n = 0;
    int nblk_red = 0;        // blocks of the reduction kernels
    size_t bytes = 0;
    // a captured GMRES cycle (the m Arnoldi steps) and the key of the
    // launch configuration it was captured for; replayed for later cycles
    hipGraphExec_t cycle_graph = nullptr;
    uint64_t cycle_key = 0;
    hipStream_t capture_stream = nullptr;  // non-blocking stream used only for capture
};

// Capture the launches `enqueue(stream)` makes into an executable graph.
// The capture runs on the workspace's private stream (never the null
// stream) in relaxed mode, so other threads may keep using HIP meanwhile.
// Capture the launches of `enqueue` into an executable graph on a private
// stream.  Returns nullptr when the capture fails (the caller then launches
// the same work one by one): device-wide synchronising calls that another
// thread makes during a capture invalidate it.  The library's own such calls
// (allocation, free, synchronous copies) hold device_sync_mutex(), which a
// capture holds too.  capture_graph replaces the workspace's cycle graph.
hipGraphExec_t capture_graph(Workspace& w, void (*enqueue)(void*, hipStream_t), void* ctx);
hipGraphExec_t capture_graph_on(hipStream_t cap, void (*enqueue)(void*, hipStream_t), void* ctx);
std::recursive_mutex& device_sync_mutex();

}  // namespace ipi

struct ipi_mdp_s {
    int64_t S = 0;
    int32_t A = 0;
    int64_t nnz = 0;
    double gamma = 0;
    int32_t k_min = 0, k_max = 0;
    bool uniform_k = false;
    bool rp32 = false;       // row_ptr stored as int32
    int vec_align = 1;       // largest v in {4,2,1} dividing every row_ptr entry
    bool borrowed = false;
    int device = 0;
    void* row_ptr = nullptr; // int32 or int64 [S*A+1]
    int32_t* col = nullptr;
    double* val = nullptr;
    float* val32 = nullptr;
    double val32_dp = 0.0;   // max over rows of sum_j |P_rj - float32(P_rj)| (0 without val32)
    float* val_lo = nullptr; // IPI_VAL_SPLIT: float32(P - val32), no FP64 values kept
    double split_dp = 0.0;   // max over rows of sum_j |P_rj - (hi_rj + lo_rj)|
    double* g = nullptr;
    double* g_neg = nullptr; // -g for the maximisation mode (lazily)
    int arch_cus = 0;
    ipi::Tuning tune;
    ipi::Workspace ws;
    size_t data_bytes = 0;
    int64_t ppi_cap = 0;     // sum over states of the longest row of the state
    // band form: when every row's k columns are consecutive integers, the
    // first column of each row (S*A entries); the flat kernels then read no
    // column indices (col stays for the other kernels).  band_dlo / band_dhi
    // bound first column - state over all rows.
    int32_t* band = nullptr;
    int band_dlo = 0, band_dhi = 0;
    // the same bounds over the rows of the interior states [H, S - H), H the
    // largest reach max(-band_dlo, band_dhi + k - 1) (equal to the global
    // ones when S <= 2 H); the blocked sweeps may use them (see rich_halos)
    int band_dlo_in = 0, band_dhi_in = 0;
    // stencil form (rows of uniform length k not in the band form): when
    // every row's columns are its first column plus one of at most
    // kStenMaxPatterns offset patterns (a grid stencil: bilinear rows c, c+1,
    // c+N, c+N+1, and the rows that wrap around a periodic axis), one 32-bit
    // word per row holds the first column and the pattern; sten_off holds the
    // patterns' offsets (kStenMaxPatterns x k, device).  The Bellman pass then
    // reads 4 bytes of indices per row instead of 4 k; col stays for the
    // other kernels.
    uint32_t* sten = nullptr;
    int32_t* sten_off = nullptr;
    int sten_np = 0;
    // every pattern's columns come in adjacent pairs (offsets 2m and 2m + 1
    // one apart: the bilinear c, c+1, c+N, c+N+1): a pair is one 16-byte load
    bool sten_pairs = false;
    void* rho_slot = nullptr;
    std::mutex mu;
};

namespace ipi {

// Lay out the solve workspace of an MDP: iterate vectors, Krylov basis of
// restart+1 vectors, compact P_pi, control block and reduction partials.
// Each buffer comes from alloc(bytes); w.bytes accumulates their sizes.
// workspace_ensure takes them from hipMalloc, ipi_solve_noalloc from a
// fixed device array.
template <class Alloc>
void workspace_layout(const ipi_mdp_s* m, int restart, int naux, bool fp32, int cus, Workspace& w, Alloc&& alloc,
                      size_t bpart_n = 0) {
    const int64_t S = m->S;
    const int mm = restart > 1 ? restart : 1;
    w.S = S;
    w.m = mm;
    w.naux = naux;
    w.fp32 = fp32;
    w.kmax = m->k_max;
    w.bytes = 0;
    auto get = [&](size_t count, size_t elem) -> void* {
        if (count == 0) count = 1;
        w.bytes += count * elem;
        return alloc(count * elem);
    };
    w.V = (double*)get(S, 8);
    w.TV = (double*)get(S, 8);
    w.b = (double*)get(S, 8);
    w.delta = (double*)get(S, 8);
    w.delta2 = (double*)get(S, 8);
    w.basis = (double*)get((size_t)(mm + 1) * S, 8);
    w.small = (double*)get(8192, 8);
    // workgroups of the product and reduction launches: enough for the state
    // count and for the nonzeros of P_pi (long rows with few states need more
    // workgroups than S / 256), at most 32 per CU
    const int64_t by_states = (S + kBlock - 1) / kBlock;
    const int64_t by_nnz = (S * (int64_t)(m->k_max > 1 ? m->k_max : 1) + 4095) / 4096;
    const int64_t want = by_states > by_nnz ? by_states : by_nnz;
    const int64_t cap = 32 * (int64_t)cus;
    w.nblk_red = (int)(want < 1 ? 1 : (want > cap ? cap : want));
    w.partials = (double*)get((size_t)w.nblk_red * (kMaxRestart + 4), 8);
    if (naux > 0) w.aux = (double*)get((size_t)naux * S, 8);
    w.diag = (double*)get(S, 8);
    w.pi = (int32_t*)get(S, 4);
    const int64_t nz = m->uniform_k ? S * (int64_t)m->k_max : m->ppi_cap;
    w.ppi_col = (int32_t*)get(nz, 4);
    if (m->band) w.ppi_band = (int32_t*)get(S, 4);
    if (m->sten) w.ppi_sten = (uint32_t*)get(S, 4);
    w.ppi_val = get(nz, fp32 ? 4 : 8);
    if (!m->uniform_k) {
        w.ppi_rp = (int64_t*)get(S + 1, 8);
        w.scan_tmp = (int64_t*)get(S / kBlock + 1024, 8);
    }
    w.ctrl = (Ctrl*)get(1, sizeof(Ctrl));
    w.bpart_n = bpart_n;
    if (bpart_n > 0) w.bpart = (double*)get(bpart_n, 8);
}

// mdp.hip
// bpart_n: doubles of tile partial sums for the batched solver (0: none)
void workspace_ensure(ipi_mdp_s* m, int restart, int naux, bool fp32, hipStream_t st, size_t bpart_n = 0);
void workspace_free(ipi_mdp_s* m);
int device_cus();

// kernels_bellman.hip
struct BellmanOut {
    double* TV;
    int32_t* pi;
    double* resid;
    uint64_t* rho_bits;
    uint64_t* vmax_bits;  // max |V[s]| (optional)
};
void launch_bellman(const ipi_mdp_s* m, const double* g, const double* V, const BellmanOut& o,
                    bool fp32, int lanes, int spt, hipStream_t st);
double bellman_alg_bytes(const ipi_mdp_s* m, bool fp32, int lanes);
bool bellman_uses_flat(const ipi_mdp_s* m, bool fp32, int lanes);
int bellman_flat_e(const ipi_mdp_s* m, bool fp32, int pref = 0);
bool flat_chunk_ok(const ipi_mdp_s* m, bool fp32, int e);
// band form in use for this MDP (detected and not disabled by tuning)
inline bool band_on(const ipi_mdp_s* m) { return m->band != nullptr && m->tune.band_rows >= 0; }
// stencil form in use (detected and not disabled by tuning: band_rows governs both)
inline bool sten_on(const ipi_mdp_s* m) { return m->sten != nullptr && m->tune.band_rows >= 0; }

// A band-form tile stages the x (or V) entries its rows read, a window of
// at most kBandWindow entries, in LDS.  For a tile of n consecutive states
// the window spans at most (n - 1) + (band_dhi - band_dlo) + k entries.
constexpr int kBandWindow = 128;
inline bool band_window_fits(const ipi_mdp_s* m, int states) {
    return (int64_t)(states - 1) + ((int64_t)m->band_dhi - m->band_dlo) + m->k_max <= kBandWindow;
}

// Bytes one P_pi sweep may stream (values, columns or band starts, vectors) and
// still find them in the last-level cache at the next sweep when loaded
// through the caches.  MI355X has 256 MB of Infinity Cache; on birth-death
// P_pi the cached loads were faster up to 262 MiB per sweep, even at
// 296 MiB and slower from 315 MiB on; on the pendulum's P_pi (columns
// loaded) 1.6% faster at 288 MiB.
constexpr double kPpiCacheBytes = 300.0 * 1024 * 1024;
int default_bellman_lanes(const ipi_mdp_s* m, bool fp32);
int default_bellman_spt(const ipi_mdp_s* m, int lanes);
int bellman_vec(const ipi_mdp_s* m, bool fp32);
int default_spmv_lanes(const ipi_mdp_s* m, bool fp32);
int default_spmv_spt(const ipi_mdp_s* m, int lanes, int flat_e);
int spmv_flat_e(const ipi_mdp_s* m, bool fp32, int lanes, int pref = 0);
int wave_tile_states(const ipi_mdp_s* m, int flat_e);
void launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t st);
void launch_rho_to_double(const uint64_t* bits, double* out, hipStream_t st);
void launch_negate(const double* x, double* y, int64_t n, hipStream_t st);

// kernels_ppi.hip: compact P_pi rows s*A + pi(s)
void launch_extract_ppi(ipi_mdp_s* m, const int32_t* pi, bool fp32, bool want_diag, hipStream_t st);
double extract_alg_bytes(const ipi_mdp_s* m, bool fp32);

// kernels_krylov.hip + solver.hip
struct SolveStats {
    int outer = 0;
    int64_t inner = 0;
    int bellman_calls = 0;
    double bellman_ms = 0, inner_ms = 0, alg_bytes = 0;
};
// noalloc: the caller has placed a complete workspace in m->ws (ipi_solve_noalloc);
// the solve then allocates nothing, creates no events and captures no graph
ipi_status solve_single(ipi_mdp_s* m, const ipi_solve_opts& o, double* V_out, int32_t* pi_out,
                        ipi_solve_info* info, hipStream_t st, bool noalloc = false);

// batch.hip: up to `capacity` independent members advanced together in
// rounds (one phase of each member's Algorithm 1 per round, all members'
// tiles in one grid); members join and leave between chunks of rounds, and
// each member's result does not depend on the others (bitwise)
class BatchEngine {
public:
    static constexpr int kRoundsPerChunk = 32;
    BatchEngine(int capacity, hipStream_t st);
    ~BatchEngine();
    BatchEngine(const BatchEngine&) = delete;
    BatchEngine& operator=(const BatchEngine&) = delete;
    int capacity() const { return cap_; }
    int active() const { return active_; }
    bool full() const { return active_ >= cap_; }
    // validates the member, sizes its workspace, writes its descriptor and a
    // fresh state into a free slot (it starts at the next chunk); the slot
    int add(ipi_mdp_s* m, const ipi_solve_opts& o, double* V_out, int32_t* pi_out);
    // one chunk of rounds; the slots whose members finished in it
    std::vector<int> step();
    // status and info of a finished member; frees its slot
    void take(int slot, ipi_status* status, ipi_solve_info* info);
    // removes a member before it finished (its outputs are not written)
    void drop(int slot);

private:
    struct Slot {
        ipi_mdp_s* m = nullptr;
        ipi_solve_opts opts{};
        double* V_out = nullptr;
        bool uniform = false, done = false, overrun = false;
        int64_t join_round = 0, max_rounds = 0;
        std::chrono::steady_clock::time_point t_join{}, t_done{};
    };
    int cap_;
    hipStream_t st_;
    char* buf_ = nullptr;  // descriptors, states, tile offsets
    size_t off_st_ = 0, off_off_ = 0;
    int grid_ = 0;
    std::vector<unsigned char> hd_, hs_;  // host copies of the descriptors and states
    std::vector<Slot> slots_;
    int active_ = 0;
    int64_t rounds_ = 0;
    bool dirty_ = false;  // tile offsets must be rescanned before the next chunk
    hipGraphExec_t graph_[4] = {};
    bool graph_tried_[4] = {};
    hipStream_t cap_stream_ = nullptr;
};
ipi_status solve_batch(int n, ipi_mdp_s* const* mdps, const ipi_solve_opts* opts, double* const* V_out,
                       int32_t* const* pi_out, ipi_solve_info* infos, ipi_status* statuses, hipStream_t st);

// autotune.hip
ipi_status autotune(ipi_mdp_s* m, bool fp32, const char* cache_path, hipStream_t st);
// the checks ipi_set_tuning applies (and a cached autotune entry must pass)
bool tuning_admissible(const ipi_mdp_s* m, const Tuning& t, std::string* why);

}  // namespace ipi
