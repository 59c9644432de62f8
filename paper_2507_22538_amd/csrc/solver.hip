// Host driver of Algorithm 1 (general inexact policy iteration) on one MDP.
//
//   k = 0, V_0 = 0 (or opts.v0)
//   loop:
//     fused Bellman pass on V_k  -> pi_{k+1} (greedy), b = T V_k - V_k,
//                                    rho_k = ||r(V_k)||_inf, max |V_k|
//     8-byte readback of rho_k; stop if rho_k <= tol, or after max_outer
//     policy evaluations (the returned V and pi come from this last pass)
//     compact P_pi (step 4), optional Jacobi diagonal (step 5)
//     inner solve of J_pi delta = b (steps 6-12, correction form), forcing
//       test ||b - J_pi delta||_2 < alpha * rho_k, at most max_inner
//       iterations; V_{k+1} = V_k + delta (step 13)
//
// Nothing crosses the host/device boundary per inner iteration: GMRES
// cycles and batches of Richardson sweeps are enqueued whole, each kernel
// exits at once when the device control block says the solve has stopped,
// and the host reads the control block once per cycle / batch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <cstdlib>

#include "device.hpp"
#include "krylov.hpp"

namespace ipi {

int default_spmv_lanes(const ipi_mdp_s* m, bool fp32) {
    const double k = m->uniform_k ? (double)m->k_max : (double)m->ppi_cap / (double)m->S;
    const int vec = m->uniform_k ? bellman_vec(m, fp32) : 1;
    int L = 1;
    while (L < 64 && (double)(2 * L) * vec * 3.0 <= k) L *= 2;
    return L;
}

// chunk width of the flat product kernel (P_pi in ELL form), 0 if not
// admissible.  Automatic choice: one 16-byte load per chunk (2 doubles or 4
// floats), so that consecutive lanes read consecutive 16-byte pieces.
int spmv_flat_e(const ipi_mdp_s* m, bool fp32, int lanes, int pref) {
    if (lanes > 0) return 0;
    if (pref <= 0 && flat_chunk_ok(m, fp32, fp32 ? 4 : 2)) return fp32 ? 4 : 2;
    const int e = bellman_flat_e(m, fp32, pref);
    return e >= 2 ? e : 0;  // rows of one entry take the lane-group kernels here
}

// states per wave tile of the flat product (at most 64 and 1024 chunk slots)
int wave_tile_states(const ipi_mdp_s* m, int flat_e) {
    const int cpr = std::max(1, m->k_max / std::max(1, flat_e));
    return std::max(1, std::min(64, 1024 / cpr));
}

int default_spmv_spt(const ipi_mdp_s* m, int lanes, int flat_e) {
    if (lanes <= 0) {
        // flat: about three chunks per thread
        const int e = std::max(1, flat_e);
        int spt = 64;
        while (spt < kMaxSpmvTile && (int64_t)(2 * spt) * (m->k_max / e) <= 3 * kBlock) spt *= 2;
        return spt;
    }
    int spt = 4 * (kBlock / lanes);
    if (spt < 256) spt = 256;
    if (spt > kMaxSpmvTile) spt = kMaxSpmvTile;
    return spt;
}

namespace {

struct Timer {
    bool on = false;
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st = nullptr;
    void init(bool enable, hipStream_t s) {
        on = enable;
        st = s;
        if (on) {
            IPI_HIP(hipEventCreate(&a));
            IPI_HIP(hipEventCreate(&b));
        }
    }
    void start() {
        if (on) IPI_HIP(hipEventRecord(a, st));
    }
    void stop() {
        if (on) IPI_HIP(hipEventRecord(b, st));
    }
    double ms() {  // after a synchronisation of the stream
        if (!on) return 0.0;
        float t = 0.f;
        IPI_HIP(hipEventSynchronize(b));
        IPI_HIP(hipEventElapsedTime(&t, a, b));
        return (double)t;
    }
    ~Timer() {
        if (a) hipEventDestroy(a);
        if (b) hipEventDestroy(b);
    }
};

double bits_to_double(uint64_t u) {
    double d;
    std::memcpy(&d, &u, 8);
    return d;
}

// Pool of event pairs timing product launches between two host
// synchronisations (profile mode).  Every `stride`-th pair is recorded, so
// the events themselves barely slow the solve (profile 1: every 16th;
// profile 2: every one).  A pair may bracket several back-to-back launches
// (`count`), which spreads the cost of recording the events over them.
struct ProductTimer {
    bool on = false;
    int stride = 1;
    std::vector<hipEvent_t> ev;
    std::vector<int64_t> at;  // launch index (since the last collect) of each pair
    std::vector<double> own;  // bytes of the pair's launches, or < 0 (the caller's share)
    std::vector<int> cnt;     // launches the pair brackets
    std::vector<int> kind;    // sweeps of a blocked Richardson launch, else 0
    size_t used = 0;
    int64_t seq = 0;
    int64_t calls = 0;
    double ms = 0.0, bytes = 0.0;
    // the timed blocked launches by sweeps per launch (4, 8, 16)
    int64_t kcalls[3] = {0, 0, 0};
    double kms[3] = {0.0, 0.0, 0.0}, kbytes[3] = {0.0, 0.0, 0.0};
    static int kslot(int k) { return k == 16 ? 2 : (k == 8 ? 1 : (k == 4 ? 0 : -1)); }
    void init(bool enable, int every) {
        on = enable;
        stride = every < 1 ? 1 : every;
    }
    // event pair for the next launch (or nulls when off or not sampled);
    // `index` (>= 0) replaces the running launch count in collect's test,
    // `bytes` (>= 0) gives the launches their own byte count and `count` is
    // the number of launches the pair brackets; `sweeps` marks a blocked
    // Richardson launch of that many sweeps
    void next(LaunchShape& sh, int64_t index = -1, double bytes = -1.0, int count = 1, int sweeps = 0) {
        sh.ev0 = nullptr;
        sh.ev1 = nullptr;
        if (!on) return;
        const int64_t i = seq++;
        if (i % stride) return;
        if (used + 2 > ev.size()) {
            for (int q = 0; q < 64; ++q) {
                hipEvent_t e;
                IPI_HIP(hipEventCreate(&e));
                ev.push_back(e);
            }
        }
        sh.ev0 = ev[used];
        sh.ev1 = ev[used + 1];
        at.push_back(index >= 0 ? index : i);
        own.push_back(bytes);
        cnt.push_back(count);
        kind.push_back(sweeps);
        used += 2;
    }
    // after the stream was synchronised: accumulate the timed launches among
    // the first `ran` (those that did work), each with its share of the bytes
    void collect(int64_t ran, double bytes_per_call) { collect_total(ran, bytes_per_call * (double)ran); }
    void collect_total(int64_t ran, double total_bytes) {
        if (!on) return;
        const double per = ran > 0 ? total_bytes / (double)ran : 0.0;
        const size_t pairs = used / 2;
        for (size_t q = 0; q < pairs; ++q) {
            if (at[q] >= ran) continue;
            float t = 0.f;
            IPI_HIP(hipEventElapsedTime(&t, ev[2 * q], ev[2 * q + 1]));
            const double b = own[q] >= 0.0 ? own[q] : per * cnt[q];
            ms += t;
            calls += cnt[q];
            bytes += b;
            const int ks = kslot(kind[q]);
            if (ks >= 0) {
                kcalls[ks] += cnt[q];
                kms[ks] += t;
                kbytes[ks] += b;
            }
        }
        used = 0;
        seq = 0;
        at.clear();
        own.clear();
        cnt.clear();
        kind.clear();
    }
    ~ProductTimer() {
        for (auto e : ev) hipEventDestroy(e);
    }
};

struct InnerCtx {
    ProductTimer* pt = nullptr;
    ipi_mdp_s* m;
    const ipi_solve_opts* o;
    bool fp32;
    PpiView P;
    LaunchShape sh;
    hipStream_t st;
    bool graphs = true;  // GMRES cycles may be captured into a HIP graph
    int64_t block_launches = 0;  // Richardson launches that ran 4, 8 or 16 sweeps (temporal blocking)
    int block_sweeps = 0;        // the most sweeps one of them ran
    double ppi_bytes;  // bytes of one P_pi product's matrix stream
};

// the m Arnoldi steps of one GMRES cycle (each exits at once after the stop)
struct CycleArgs {
    InnerCtx* c;
    int m, mj, nb;
};

void enqueue_cycle(void* ctx, hipStream_t st) {
    const CycleArgs& a = *static_cast<const CycleArgs*>(ctx);
    InnerCtx& c = *a.c;
    Workspace& w = c.m->ws;
    const int64_t S = c.m->S;
    for (int j = 0; j < a.m; ++j) {
        LaunchShape sh = c.sh;
        c.pt->next(sh);
        k_launch_arnoldi(c.P, sh, w.basis, j, a.mj, w.small, w.partials, w.ctrl, st);
        if (c.o->reorth >= 2) {
            k_launch_orth(w.basis, S, j, a.mj, 0, 0, w.small, w.partials, w.ctrl, a.nb, st);
            k_launch_dots(w.basis, S, j, a.mj, w.small, w.partials, w.ctrl, a.nb, st);
            k_launch_orth(w.basis, S, j, a.mj, 1, 1, w.small, w.partials, w.ctrl, a.nb, st);
        } else {
            k_launch_orth(w.basis, S, j, a.mj, 0, 1, w.small, w.partials, w.ctrl, a.nb, st);
        }
    }
}

// key of everything a captured cycle bakes into its launches
uint64_t cycle_key(const InnerCtx& c, int m) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
    mix((uint64_t)m);
    mix((uint64_t)c.o->reorth);
    mix((uint64_t)c.fp32);
    mix((uint64_t)c.P.flat_e);
    mix((uint64_t)c.P.pipe);
    mix((uint64_t)c.P.vec);
    mix((uint64_t)(uintptr_t)c.P.dinv);
    mix((uint64_t)(uintptr_t)c.P.col);
    mix((uint64_t)(uintptr_t)c.P.val);
    mix((uint64_t)(uintptr_t)c.P.rp);
    mix((uint64_t)(uintptr_t)c.P.band);
    mix((uint64_t)c.sh.lanes);
    mix((uint64_t)c.sh.spt);
    mix((uint64_t)c.sh.nb);
    mix((uint64_t)(uintptr_t)c.m->ws.basis);
    return h;
}

// one GMRES(m) solve of J delta = b, writes Vn = V + delta.  Without
// profiling, the m Arnoldi steps of a cycle are captured once into a HIP
// graph and replayed for every cycle (the launches of a cycle are the same
// each time; the steps past the stop exit at once).
int64_t inner_gmres(InnerCtx& c, const double* V, double* Vn, double target, double* bytes, double* resid) {
    Workspace& w = c.m->ws;
    const int64_t S = c.m->S;
    const int m = c.o->gmres_restart;
    const int mj = mj_bucket(m);
    const int nb = w.nblk_red;
    const double vecb = 8.0 * (double)S;
    k_launch_ctrl_reset(w.ctrl, target, c.o->max_inner, m, 0.0, c.st);
    k_launch_init_cycle(w.b, c.P.dinv, w.basis, S, w.small, w.partials, w.ctrl, nb, c.st);
    *bytes += 2 * vecb + (c.P.dinv ? vecb : 0);
    bool first = true;
    Ctrl h{};
    int64_t steps_before = 0;
    CycleArgs ca{&c, m, mj, nb};
    bool graph = !c.pt->on && c.graphs;
    for (;;) {
        if (graph) {
            const uint64_t key = cycle_key(c, m);
            if (!w.cycle_graph || w.cycle_key != key) {
                w.cycle_graph = capture_graph(w, enqueue_cycle, &ca);
                w.cycle_key = key;
                graph = w.cycle_graph != nullptr;
            }
        }
        if (graph) {
            IPI_HIP(hipGraphLaunch(w.cycle_graph, c.st));
        } else {
            enqueue_cycle(&ca, c.st);
        }
        k_launch_gmres_update(w.basis, S, mj, w.small, w.ctrl, w.delta, first ? 1 : 0, V, Vn, nb, c.st);
        IPI_HIP(hipMemcpyAsync(&h, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c.st));
        IPI_HIP(hipStreamSynchronize(c.st));
        // algorithmic bytes of the steps that ran
        const int n = h.j;
        {
            // arnoldi product step j: P_pi stream, u_0..u_j read, u_{j+1} written
            double tb = 0.0;
            for (int j = 0; j < n; ++j) tb += c.ppi_bytes + (j + 2) * vecb + (c.P.dinv ? vecb : 0);
            c.pt->collect_total(n, tb);
        }
        for (int j = 0; j < n; ++j) {
            // arnoldi: P_pi stream + basis u_0..u_j + write u_{j+1}; orth: u_0..u_{j+1} read, u_{j+1} write
            *bytes += c.ppi_bytes + (j + 1) * vecb + vecb + (c.P.dinv ? vecb : 0);
            *bytes += (j + 2) * vecb + vecb;
            if (c.o->reorth >= 2) *bytes += (j + 2) * vecb + (j + 2) * vecb + vecb;
        }
        *bytes += n * vecb + (first ? 0 : vecb) + 3 * vecb;  // update: basis, delta, V read; delta, Vn write
        const bool progressed = first || h.steps_total > steps_before;
        steps_before = h.steps_total;
        *resid = h.resid;
        first = false;
        if (h.converged || h.steps_total >= c.o->max_inner) break;
        if (!progressed) throw Error(IPI_E_NUMERICAL, "GMRES restart made no progress");
        // restart from the true residual b - J delta
        k_launch_resid_cycle(c.P, c.sh, w.b, w.delta, w.basis, w.small, w.partials, w.ctrl, c.st);
        *bytes += c.ppi_bytes + 3 * vecb + (c.P.dinv ? vecb : 0);
    }
    return steps_before;
}

// Richardson: delta_{i+1} = delta_i + omega D (b - J delta_i)
int64_t inner_richardson(InnerCtx& c, const double* V, double* Vn, double target, double* bytes, double* resid) {
    Workspace& w = c.m->ws;
    const int64_t S = c.m->S;
    const int nb = w.nblk_red;
    const double vecb = 8.0 * (double)S;
    k_launch_ctrl_reset(w.ctrl, target, c.o->max_inner, 1, c.o->richardson_scale, c.st);
    // three delta buffers (the Krylov basis is unused by Richardson): a
    // blocked launch reads one and writes the last two iterates to the others
    double* d[3] = {w.delta, w.delta2, w.basis};
    const bool blocked = c.o->richardson_block != 0;
    const bool b16 = rich_block_ok(c.P, 16);  // 16 sweeps between tests late in long solves
    int64_t i = 0;
    int cur = 1;  // buffer of the current iterate (sweep 0 writes delta_1 to d[1])
    Ctrl h{};
    const int64_t maxi = c.o->max_inner;
    // sweeps that did work, and their algorithmic bytes, in launch order
    std::vector<std::pair<int64_t, double>> work;  // (first sweep index, bytes)
    std::vector<std::pair<int64_t, int>> blocks;    // (first sweep index, sweeps) of each blocked launch
    const double sweep_bytes = c.ppi_bytes + 3 * vecb + (c.P.dinv ? vecb : 0);
    const double block_bytes = c.ppi_bytes + 4 * vecb + (c.P.dinv ? vecb : 0);
    for (;;) {
        // sweeps per host check: a small first batch (VI-like solves stop early),
        // then 64 (launches past the stop exit at once).  The stopping test runs
        // after every sweep for the first 16, then after every 4th, then every
        // 8th sweep, and from sweep 1024 on after every 16th when 16 sweeps fit
        // one blocked launch of this P_pi (always at the end of a batch and at
        // the cap); the schedule depends on P_pi only, so the blocked and the
        // one-sweep paths test at the same sweeps.  A long solve does at most
        // 15 sweeps more than the first one whose residual passes; the iterate
        // returned is always one that passed.
        const int64_t want = i < 16 ? 16 : 64;
        const int64_t batch = std::max<int64_t>(1, std::min<int64_t>(maxi - i, want));
        int64_t q = 0;
        while (q < batch) {
            if (i == 0) {
                k_launch_rich0(w.b, c.P.dinv, d[1], S, w.partials, w.ctrl, nb, w.small, c.st);
                work.push_back({0, 2 * vecb});
                cur = 1;
                ++q;
                ++i;
                continue;
            }
            // the sweeps up to and including the next stopping test
            int n = 0;
            for (;;) {
                const int64_t ii = i + n, qq = q + n;
                ++n;
                const int every = ii < 16 ? 1 : (ii < 256 ? 4 : (ii < 1024 || !b16 ? 8 : 16));
                if (n >= every || qq == batch - 1 || ii == maxi - 1) break;
            }
            const int o1 = (cur + 1) % 3, o2 = (cur + 2) % 3;
            if (blocked && (n == 4 || n == 8 || n == 16) && rich_block_ok(c.P, n) &&
                rich_block_grid(c.P, n) <= (int64_t)w.nblk_red * (kMaxRestart + 4)) {
                LaunchShape sh = c.sh;
                c.pt->next(sh, i, block_bytes, 1, n);
                if (sh.ev0) IPI_HIP(hipEventRecord(sh.ev0, c.st));
                k_launch_rich_block(c.P, n, w.b, d[cur], d[o1], d[o2], w.partials, w.ctrl, c.st);
                if (sh.ev1) IPI_HIP(hipEventRecord(sh.ev1, c.st));
                k_launch_fin_rich(w.small, w.partials, rich_block_grid(c.P, n), w.ctrl, n, o1, o2, c.st);
                work.push_back({i, block_bytes});
                blocks.push_back({i, n});
                cur = o2;
            } else {
                // one event pair around the group's n back-to-back product
                // launches (the stopping test's kernel follows the last)
                LaunchShape grp = c.sh;
                c.pt->next(grp, i, n * sweep_bytes, n);
                for (int u = 0; u < n; ++u) {
                    const int nx = (cur + 1) % 3;
                    LaunchShape sh = c.sh;
                    sh.ev0 = u == 0 ? grp.ev0 : nullptr;
                    sh.ev1 = u == n - 1 ? grp.ev1 : nullptr;
                    k_launch_rich(c.P, sh, w.b, d[cur], d[nx], cur, w.partials, w.ctrl, w.small, c.st,
                                  u == n - 1 ? n : 0, nx);
                    work.push_back({i + u, sweep_bytes});
                    cur = nx;
                }
            }
            q += n;
            i += n;
        }
        IPI_HIP(hipMemcpyAsync(&h, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c.st));
        IPI_HIP(hipStreamSynchronize(c.st));
        // product launches that did work in this batch: those whose first
        // sweep index is below the number of sweeps that ran (sweep 0 has none)
        const int64_t ran_total = h.converged ? h.steps_total + 1 : h.steps_total;
        c.pt->collect_total(ran_total, 0.0);
        if (!h.active || i >= maxi) break;
        if (h.steps_total < i) throw Error(IPI_E_NUMERICAL, "Richardson sweeps stopped without a verdict");
    }
    k_launch_axpy_result(V, d[0], d[1], d[2], w.ctrl, Vn, S, nb, c.st);
    // launches that ran: their first sweep index is below the sweeps that ran
    const int64_t ran = h.converged ? h.steps_total + 1 : h.steps_total;
    for (const auto& e : work)
        if (e.first < ran) *bytes += e.second;
    for (const auto& b : blocks) {
        if (b.first >= ran) continue;
        c.block_launches += 1;
        c.block_sweeps = std::max(c.block_sweeps, b.second);
    }
    *bytes += 3 * vecb;
    *resid = h.resid;
    return h.steps_total;
}

// BiCGStab on J delta = b (two P_pi products per iteration, no restarts)
int64_t inner_bicgstab(InnerCtx& c, const double* V, double* Vn, double target, double* bytes, double* resid) {
    Workspace& w = c.m->ws;
    const int64_t S = c.m->S;
    const int nb = w.nblk_red;
    const double vecb = 8.0 * (double)S;
    double* r = w.aux;
    double* rh = w.aux + S;
    double* p = w.aux + 2 * S;
    double* v = w.aux + 3 * S;
    double* sv = w.aux + 4 * S;
    double* t = w.aux + 5 * S;
    k_launch_ctrl_reset(w.ctrl, target, c.o->max_inner, 1, 0.0, c.st);
    k_launch_bicgstab_init(w.b, c.P.dinv, r, rh, p, S, w.small, w.partials, w.ctrl, nb, c.st);
    *bytes += 4 * vecb + (c.P.dinv ? vecb : 0);
    int64_t i = 0;
    Ctrl h{};
    const int64_t maxi = c.o->max_inner;
    for (;;) {
        const int64_t batch = std::min<int64_t>(maxi - i, 8);
        for (int64_t q = 0; q < batch; ++q, ++i)
            k_launch_bicgstab_iter(c.P, c.sh, w.delta, r, rh, p, v, sv, t, i == 0 ? 1 : 0, w.small, w.partials,
                                   w.ctrl, nb, c.st);
        IPI_HIP(hipMemcpyAsync(&h, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c.st));
        IPI_HIP(hipStreamSynchronize(c.st));
        if (!h.active || i >= maxi) break;
        if (h.steps_total < i) throw Error(IPI_E_NUMERICAL, "BiCGStab stopped without a verdict");
    }
    k_launch_bicgstab_final(V, w.delta, p, rh, w.ctrl, S, w.small, Vn, nb, c.st);
    // per iteration: two products (P_pi stream, gathered input, dot partner, output)
    // and the vector updates (s: 3, x/r update: 7, p: 4 vectors)
    const double dvec = c.P.dinv ? 2 * vecb : 0.0;
    *bytes += (double)h.steps_total * (2 * (c.ppi_bytes + 3 * vecb) + dvec + 14 * vecb);
    *bytes += 3 * vecb;
    *resid = h.resid;
    return h.steps_total;
}

// TFQMR on J delta = b; max_inner counts half steps (one J_pi product each)
int64_t inner_tfqmr(InnerCtx& c, const double* V, double* Vn, double target, double* bytes, double* resid) {
    Workspace& w = c.m->ws;
    const int64_t S = c.m->S;
    const int nb = w.nblk_red;
    const double vecb = 8.0 * (double)S;
    TfqmrVecs t;
    t.x = w.delta;
    t.w = w.aux;
    t.u = w.aux + S;
    t.q = w.aux + 2 * S;
    t.d = w.aux + 3 * S;
    t.v = w.aux + 4 * S;
    t.Au = w.aux + 5 * S;
    t.Aq = w.aux + 6 * S;
    t.rs = w.aux + 7 * S;
    k_launch_ctrl_reset(w.ctrl, target, c.o->max_inner, 1, 0.0, c.st);
    {
        LaunchShape sh = c.sh;
        c.pt->next(sh);
        k_launch_tfqmr_init(c.P, sh, w.b, t, w.small, w.partials, w.ctrl, nb, c.st);
    }
    const double dvec = c.P.dinv ? vecb : 0.0;
    *bytes += 6 * vecb + dvec;                        // init: b read, 5 vectors written
    int64_t launched = 0;                             // half steps launched
    Ctrl h{};
    const int64_t maxi = c.o->max_inner;
    for (;;) {
        const int64_t iters = std::max<int64_t>(1, std::min<int64_t>((maxi - launched + 1) / 2, 8));
        for (int64_t q = 0; q < iters; ++q) {
            LaunchShape sh0 = c.sh, sh1 = c.sh;
            c.pt->next(sh0);
            c.pt->next(sh1);
            k_launch_tfqmr_iter(c.P, sh0, sh1, t, w.small, w.partials, w.ctrl, nb, c.st);
            launched += 2;
        }
        IPI_HIP(hipMemcpyAsync(&h, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c.st));
        IPI_HIP(hipStreamSynchronize(c.st));
        if (!h.active || launched >= maxi) break;
        if (h.steps_total < launched) throw Error(IPI_E_NUMERICAL, "TFQMR stopped without a verdict");
    }
    // products that did work, in launch order: J u_0, then J q_j and J u_{j+1}
    // per iteration; after k half steps that is k of them (none if r_0 passed)
    const int64_t k = h.steps_total;
    const int64_t products = k > 0 ? k : (h.converged ? 0 : 1);
    c.pt->collect_total(products, (double)products * (c.ppi_bytes + 2 * vecb));
    const bool check = !h.converged;
    k_launch_tfqmr_final(c.P, c.sh, w.b, V, t, check, w.ctrl, w.small, w.partials, Vn, nb, c.st);
    if (check) {
        IPI_HIP(hipMemcpyAsync(&h, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c.st));
        IPI_HIP(hipStreamSynchronize(c.st));
        *bytes += c.ppi_bytes + 3 * vecb + dvec;
    }
    // per iteration: even step 10 vectors; odd product (P_pi, q gathered and
    // read, x d w r* read, Aq x d w written); u update 3; v product (P_pi, u,
    // Aq, v, r* read, Au v written)
    *bytes += (double)(k / 2) * (2 * c.ppi_bytes + 28 * vecb + 2 * dvec) + (k % 2) * 10 * vecb;
    *bytes += c.ppi_bytes + 5 * vecb + dvec;          // J u_0
    *bytes += 5 * vecb;                                // commit x += eta d; Vn = V + x
    *resid = h.resid;
    return k;
}

}  // namespace

ipi_status solve_single(ipi_mdp_s* m, const ipi_solve_opts& o, double* V_out, int32_t* pi_out,
                        ipi_solve_info* info, hipStream_t st, bool noalloc) {
    IPI_REQUIRE(o.atol >= 0.0 && std::isfinite(o.atol), IPI_E_INVALID_ARG, "atol must be >= 0");
    IPI_REQUIRE(o.rtol_cert >= 0.0 && std::isfinite(o.rtol_cert), IPI_E_INVALID_ARG, "rtol_cert must be >= 0");
    IPI_REQUIRE(o.alpha > 0.0 && o.alpha < 1.0, IPI_E_INVALID_ARG, "alpha must lie in (0, 1)");
    IPI_REQUIRE(o.max_outer >= 1 && o.max_inner >= 1, IPI_E_INVALID_ARG, "iteration caps must be >= 1");
    IPI_REQUIRE(o.inner == IPI_INNER_GMRES || o.inner == IPI_INNER_RICHARDSON || o.inner == IPI_INNER_BICGSTAB ||
                    o.inner == IPI_INNER_TFQMR,
                IPI_E_INVALID_ARG, "inner solver must be gmres, richardson, tfqmr or bicgstab");
    IPI_REQUIRE(o.pc == IPI_PC_NONE || o.pc == IPI_PC_JACOBI, IPI_E_INVALID_ARG, "pc_type must be none or jacobi");
    IPI_REQUIRE(o.gmres_restart >= 1 && o.gmres_restart <= kMaxRestart, IPI_E_INVALID_ARG,
                "gmres restart must lie in [1, 64]");
    IPI_REQUIRE(o.precision == IPI_FP64 || o.precision == IPI_FP32_MIXED || o.precision == IPI_FP32_INNER,
                IPI_E_INVALID_ARG, "bad precision");
    IPI_REQUIRE(o.reorth == 1 || o.reorth == 2, IPI_E_INVALID_ARG, "Gram-Schmidt passes must be 1 or 2");
    IPI_REQUIRE(o.mode == IPI_MINCOST || o.mode == IPI_MAXREWARD, IPI_E_INVALID_ARG, "bad mode");
    IPI_REQUIRE(o.richardson_scale > 0.0 && std::isfinite(o.richardson_scale), IPI_E_INVALID_ARG,
                "richardson scale must be > 0");
    // fp32_mixed: the Bellman pass and the inner products read float32 P values;
    // fp32_inner: only the inner products (a float32 P_pi formed from the FP64 values)
    const bool fp32 = o.precision != IPI_FP64;  // inner products on float32 P_pi
    const bool outer32 = o.precision == IPI_FP32_MIXED;
    IPI_REQUIRE(!outer32 || m->val32, IPI_E_INVALID_ARG,
                "fp32_mixed precision needs an MDP created with IPI_VAL_FP32");
    IPI_REQUIRE(outer32 || m->val || (m->val_lo && o.precision == IPI_FP32_INNER), IPI_E_INVALID_ARG,
                "fp64 needs the FP64 values of P, fp32_inner the FP64 or the split values (IPI_VAL_SPLIT)");

    const auto t_wall0 = std::chrono::steady_clock::now();
    const int restart = o.inner == IPI_INNER_GMRES ? o.gmres_restart : 1;
    const int naux = o.inner == IPI_INNER_BICGSTAB ? 6 : (o.inner == IPI_INNER_TFQMR ? 8 : 0);
    if (!noalloc) workspace_ensure(m, restart, naux, fp32, st);
    Workspace& w = m->ws;
    IPI_REQUIRE(w.S == m->S && w.m >= restart && w.naux >= naux && w.fp32 == fp32 && w.ppi_val, IPI_E_INVALID_ARG,
                "solve workspace does not fit the options");
    const int64_t S = m->S;

    // maximisation of rewards = minimisation of the negated costs
    const double* g = m->g;
    if (o.mode == IPI_MAXREWARD && noalloc) {
        IPI_REQUIRE(w.g_neg, IPI_E_INVALID_ARG, "maximisation needs room for -g in the workspace");
        launch_negate(m->g, w.g_neg, S * (int64_t)m->A, st);
        g = w.g_neg;
    } else if (o.mode == IPI_MAXREWARD) {
        if (!m->g_neg) {
            std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
            IPI_HIP(hipMalloc(&m->g_neg, (size_t)S * m->A * sizeof(double)));
            launch_negate(m->g, m->g_neg, S * (int64_t)m->A, st);
        }
        g = m->g_neg;
    }
    double* V = w.V;
    double* Vn = w.TV;
    if (o.v0) {
        if (o.mode == IPI_MAXREWARD) launch_negate(o.v0, V, S, st);
        else IPI_HIP(hipMemcpyAsync(V, o.v0, S * sizeof(double), hipMemcpyDeviceToDevice, st));
    } else {
        launch_fill_u64(reinterpret_cast<uint64_t*>(V), S, 0, st);
    }

    ProductTimer ptimer;
    ptimer.init(o.profile != 0 && !noalloc, o.profile >= 2 ? 1 : 16);
    InnerCtx ic;
    ic.pt = &ptimer;
    ic.m = m;
    ic.o = &o;
    ic.fp32 = fp32;
    ic.st = st;
    ic.graphs = !noalloc;
    ic.P.col = w.ppi_col;
    ic.P.val = w.ppi_val;
    ic.P.rp = m->uniform_k ? nullptr : w.ppi_rp;
    ic.P.k = m->k_max;
    ic.P.vec = m->uniform_k ? bellman_vec(m, fp32) : 1;
    ic.P.fp32 = fp32;
    ic.P.S = S;
    ic.P.gamma = m->gamma;
    ic.P.dinv = o.pc == IPI_PC_JACOBI ? w.diag : nullptr;
    ic.P.flat_e = m->uniform_k ? spmv_flat_e(m, fp32, m->tune.spmv_lanes, m->tune.spmv_chunk) : 0;
    // flat products default to wave tiles (schedule 2); 1 selects workgroup tiles
    ic.P.pipe = (ic.P.flat_e > 0 && m->tune.spmv_schedule != 1) ? 1 : 0;
    ic.sh.lanes = m->tune.spmv_lanes > 0 ? m->tune.spmv_lanes : default_spmv_lanes(m, fp32);
    if (m->tune.spmv_spt) ic.sh.spt = m->tune.spmv_spt;
    else if (ic.P.pipe) ic.sh.spt = wave_tile_states(m, ic.P.flat_e);
    else ic.sh.spt = default_spmv_spt(m, ic.P.flat_e ? 0 : ic.sh.lanes, ic.P.flat_e);
    if (ic.P.flat_e > 0)  // tile output plus chunk sums must fit in 64 KiB of LDS
        while (ic.sh.spt > 64 && (int64_t)ic.sh.spt * (1 + m->k_max / ic.P.flat_e) * 8 > 65536) ic.sh.spt /= 2;
    ic.sh.nb = m->tune.spmv_workgroups > 0 ? std::min(m->tune.spmv_workgroups, w.nblk_red) : w.nblk_red;
    {
        const double bv = fp32 ? 4.0 : 8.0;
        const double kk = m->uniform_k ? (double)m->k_max : (double)m->ppi_cap / (double)S;
        // band form (wave tiles only, the tile's x window within its LDS
        // slice): one first column per row instead of k columns
        const bool band = band_on(m) && w.ppi_band && ic.P.pipe == 1 && wave_tiles_ok(ic.P, ic.sh.spt) &&
                          band_window_fits(m, ic.sh.spt);
        ic.P.band = band ? w.ppi_band : nullptr;
        // stencil form (wave tiles, rows that are not bands): one word per
        // row instead of k columns
        const bool sten = !band && sten_on(m) && w.ppi_sten && ic.P.pipe == 1 && wave_tiles_ok(ic.P, ic.sh.spt);
        ic.P.sten = sten ? w.ppi_sten : nullptr;
        ic.P.sten_off = m->sten_off;
        ic.P.sten_np = m->sten_np;
        ic.P.sten_pairs = m->sten_pairs;
        ic.P.band_hl = std::max(0, -m->band_dlo);
        ic.P.band_hr = std::max(0, m->band_dhi + m->k_max - 1);
        ic.P.band_hl_in = std::max(0, -m->band_dlo_in);
        ic.P.band_hr_in = std::max(0, m->band_dhi_in + m->k_max - 1);
        ic.ppi_bytes = band || sten ? (double)S * kk * bv + 4.0 * S
                            : (double)S * kk * (bv + 4.0) + (m->uniform_k ? 0.0 : 8.0 * (S + 1));
        // a sweep reads x and b (and D) and writes its output
        const double sweep = ic.ppi_bytes + 8.0 * S * (3 + (ic.P.dinv ? 1 : 0));
        const bool wave = ic.P.pipe == 1 && wave_tiles_ok(ic.P, ic.sh.spt);
        ic.P.keep = wave && (m->tune.ppi_cached > 0 || (m->tune.ppi_cached == 0 && sweep <= kPpiCacheBytes));
        ic.P.keep_block = band && m->tune.ppi_cached >= 0;
        ic.P.lds_prefetch = m->tune.blocked_prefetch == 0;
    }
    const int blanes = m->tune.bellman_lanes;
    const int bspt = m->tune.bellman_spt;

    Timer t_all, t_bell, t_inner;
    t_all.init(!noalloc, st);
    t_bell.init(o.profile != 0 && !noalloc, st);
    t_inner.init(o.profile != 0 && !noalloc, st);
    t_all.start();

    static const bool trace = std::getenv("IPI_TRACE") != nullptr;
    SolveStats stats;
    const double bell_bytes =
        bellman_alg_bytes(m, outer32, blanes) - 8.0 * S;  // T V itself is not written here
    ipi_status status = IPI_E_NOT_CONVERGED;
    double rho = 0.0, inner_resid = 0.0, vmax_last = 0.0;
    uint64_t hb[2];
    for (int k = 0;; ++k) {
        launch_fill_u64(&w.ctrl->rho_bits, 2, 0, st);  // rho_bits and vmax_bits
        BellmanOut bo{nullptr, w.pi, w.b, &w.ctrl->rho_bits, &w.ctrl->vmax_bits};
        t_bell.start();
        launch_bellman(m, g, V, bo, outer32, blanes, bspt, st);
        t_bell.stop();
        IPI_HIP(hipMemcpyAsync(hb, &w.ctrl->rho_bits, 16, hipMemcpyDeviceToHost, st));
        IPI_HIP(hipStreamSynchronize(st));
        stats.bellman_calls++;
        stats.alg_bytes += bell_bytes;
        stats.bellman_ms += t_bell.ms();
        rho = bits_to_double(hb[0]);
        const double vmax = bits_to_double(hb[1]);
        vmax_last = vmax;
        if (!std::isfinite(rho) || !std::isfinite(vmax)) {
            status = IPI_E_NUMERICAL;
            set_last_error("non-finite Bellman residual");
            break;
        }
        const bool stop = rho <= o.atol || (o.rtol_cert > 0.0 && rho <= o.rtol_cert * (1.0 - m->gamma) * vmax);
        if (trace)
            std::fprintf(stderr, "[ipi] outer %d rho %.6e |V| %.6e inner_total %lld last_inner_resid %.3e\n", k, rho,
                         vmax, (long long)stats.inner, inner_resid);
        if (stop) {
            status = IPI_OK;
            break;
        }
        if (k >= o.max_outer) {
            status = IPI_E_NOT_CONVERGED;
            set_last_error("outer iteration cap reached");
            break;
        }
        t_inner.start();
        launch_extract_ppi(m, w.pi, fp32, o.pc == IPI_PC_JACOBI, st);
        stats.alg_bytes += extract_alg_bytes(m, fp32);
        const double target = o.alpha * rho;
        int64_t steps = 0;
        if (o.inner == IPI_INNER_GMRES) steps = inner_gmres(ic, V, Vn, target, &stats.alg_bytes, &inner_resid);
        else if (o.inner == IPI_INNER_BICGSTAB)
            steps = inner_bicgstab(ic, V, Vn, target, &stats.alg_bytes, &inner_resid);
        else if (o.inner == IPI_INNER_TFQMR)
            steps = inner_tfqmr(ic, V, Vn, target, &stats.alg_bytes, &inner_resid);
        else steps = inner_richardson(ic, V, Vn, target, &stats.alg_bytes, &inner_resid);
        t_inner.stop();
        stats.inner += steps;
        stats.outer++;
        std::swap(V, Vn);
        stats.inner_ms += t_inner.ms();
    }
    // the residual of the returned V on the FP64 values: the last pass's,
    // except in fp32_mixed, where one FP64 pass (its policy goes to scratch)
    // states how far V is from the V* of the MDP as given.  Without FP64
    // values the bound uses the largest row perturbation of the float32
    // copy: ||T64 V - T32 V||_inf <= gamma dP ||V||_inf.
    // With split values the FP64 pass reads hi + lo, within split_dp of P per
    // row: ||T V - T_split V||_inf <= gamma split_dp ||V||_inf.
    double rho64 = rho;
    double err_bound = rho / (1.0 - m->gamma);
    const double split_term = m->val_lo ? m->gamma * m->split_dp * vmax_last : 0.0;
    if (!outer32) err_bound = (rho + split_term) / (1.0 - m->gamma);
    if (outer32 && status != IPI_E_NUMERICAL) {
        rho64 = std::numeric_limits<double>::quiet_NaN();
        err_bound = (rho + m->gamma * m->val32_dp * vmax_last) / (1.0 - m->gamma);
        if (m->val || m->val_lo) {
            launch_fill_u64(&w.ctrl->rho_bits, 2, 0, st);
            BellmanOut bo{nullptr, reinterpret_cast<int32_t*>(w.delta), nullptr, &w.ctrl->rho_bits, nullptr};
            launch_bellman(m, g, V, bo, false, blanes, bspt, st);
            IPI_HIP(hipMemcpyAsync(hb, &w.ctrl->rho_bits, 8, hipMemcpyDeviceToHost, st));
            IPI_HIP(hipStreamSynchronize(st));
            rho64 = bits_to_double(hb[0]);
            err_bound = (rho64 + split_term) / (1.0 - m->gamma);
            stats.alg_bytes += bellman_alg_bytes(m, false, blanes) - 16.0 * S;  // no TV, no resid written
        }
    }
    // outputs: V (negated back in maximisation mode) and the greedy policy of the last pass
    if (o.mode == IPI_MAXREWARD) launch_negate(V, V_out, S, st);
    else IPI_HIP(hipMemcpyAsync(V_out, V, S * sizeof(double), hipMemcpyDeviceToDevice, st));
    IPI_HIP(hipMemcpyAsync(pi_out, w.pi, S * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    t_all.stop();
    IPI_HIP(hipStreamSynchronize(st));
    // keep the workspace's V pointer pair consistent for the next solve
    if (V != w.V) std::swap(w.V, w.TV);
    // without events (noalloc) the time is the host's, from entry to the final synchronisation
    const double dev_ms =
        noalloc ? std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_wall0).count()
                : t_all.ms();
    if (info) {
        info->outer_iters = stats.outer;
        info->converged = status == IPI_OK ? 1 : 0;
        info->inner_iters = stats.inner;
        info->final_rho = rho;
        info->device_ms = dev_ms;
        info->alg_bytes = stats.alg_bytes;
        info->precision = o.precision;
        info->inner = o.inner;
        info->bellman_calls = stats.bellman_calls;
        info->ppi_cached = (ic.P.keep ? 1 : 0) | (ic.P.keep_block ? 2 : 0);
        info->bellman_ms = stats.bellman_ms;
        info->bellman_bytes = bell_bytes;
        info->inner_ms = stats.inner_ms;
        info->inner_resid = inner_resid;
        info->product_calls = ptimer.calls;
        info->product_ms = ptimer.ms;
        info->product_bytes = ptimer.bytes;
        info->fp64_rho = rho64;
        info->block_launches = ic.block_launches;
        info->block_sweeps = ic.block_sweeps;
        const int ks = ProductTimer::kslot(ic.block_sweeps);
        info->block_calls = ks >= 0 ? ptimer.kcalls[ks] : 0;
        info->block_ms = ks >= 0 ? ptimer.kms[ks] : 0.0;
        info->block_bytes = ks >= 0 ? ptimer.kbytes[ks] : 0.0;
        info->err_bound = err_bound;
    }
    return status;
}

}  // namespace ipi
