// Autotuner for the two streaming kernels of the solve: the fused Bellman
// pass and the P_pi product (timed through the Richardson sweep kernel,
// which streams P_pi once plus three vectors).  For each admissible
// (lanes per row, states per tile) it times a few launches with HIP events
// and keeps the fastest.  Results are cached in a JSON file keyed by the
// GPU architecture, the precision and the MDP's shape class (exact action
// count and shortest / longest row, state count rounded to a power of two),
// so the choice depends only on the shape, never on what else is being
// solved.  A cached entry is used only if it passes the same checks as
// ipi_set_tuning for this MDP; otherwise it is dropped and re-tuned.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "device.hpp"
#include "krylov.hpp"

namespace ipi {

namespace {

int pow2_round(double x) {
    if (x <= 1.0) return 1;
    return 1 << (int)std::lround(std::log2(x));
}

std::string arch_name() {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

std::string shape_key(const ipi_mdp_s* m, bool fp32) {
    std::ostringstream os;
    os << arch_name() << "|" << (fp32 ? "fp32_mixed" : "fp64") << "|k" << m->k_min << "-" << m->k_max << "|A"
       << m->A << "|S" << pow2_round((double)m->S) << "|vec" << m->vec_align << "|rp" << (m->rp32 ? 4 : 8)
       << "|u" << (m->uniform_k ? 1 : 0) << "|band" << (band_on(m) ? 1 : 0) << "|st" << (sten_on(m) ? 1 : 0);
    return os.str();
}

// tiny JSON reader/writer for {"key": [bl, bspt, sl, sspt, bchunk, schunk, ssched], ...}
std::map<std::string, Tuning> read_cache(const char* path) {
    std::map<std::string, Tuning> out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t i = 0;
    while (true) {
        const size_t a = s.find('"', i);
        if (a == std::string::npos) break;
        const size_t b = s.find('"', a + 1);
        if (b == std::string::npos) break;
        const std::string key = s.substr(a + 1, b - a - 1);
        const size_t lb = s.find('[', b);
        const size_t rb = s.find(']', lb);
        if (lb == std::string::npos || rb == std::string::npos) break;
        Tuning t;
        if (std::sscanf(s.substr(lb + 1, rb - lb - 1).c_str(), "%d,%d,%d,%d,%d,%d,%d", &t.bellman_lanes, &t.bellman_spt,
                        &t.spmv_lanes, &t.spmv_spt, &t.bellman_chunk, &t.spmv_chunk, &t.spmv_schedule) == 7)
            out[key] = t;
        i = rb + 1;
    }
    return out;
}

void write_cache(const char* path, const std::map<std::string, Tuning>& c) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << "{\n";
        size_t n = 0;
        for (const auto& kv : c) {
            f << "  \"" << kv.first << "\": [" << kv.second.bellman_lanes << ", " << kv.second.bellman_spt << ", "
              << kv.second.spmv_lanes << ", " << kv.second.spmv_spt << ", " << kv.second.bellman_chunk << ", "
              << kv.second.spmv_chunk << ", " << kv.second.spmv_schedule << "]" << (++n < c.size() ? "," : "")
              << "\n";
        }
        f << "}\n";
    }
    std::rename(tmp.c_str(), path);
}

template <typename F>
double time_ms(F&& launch, hipStream_t st, int reps) {
    hipEvent_t a, b;
    IPI_HIP(hipEventCreate(&a));
    IPI_HIP(hipEventCreate(&b));
    launch();  // warm
    IPI_HIP(hipEventRecord(a, st));
    for (int r = 0; r < reps; ++r) launch();
    IPI_HIP(hipEventRecord(b, st));
    IPI_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    IPI_HIP(hipEventElapsedTime(&ms, a, b));
    hipEventDestroy(a);
    hipEventDestroy(b);
    return (double)ms / reps;
}

}  // namespace

bool tuning_admissible(const ipi_mdp_s* m, const Tuning& t, std::string* why) {
    auto no = [&](const char* msg) {
        if (why) *why = msg;
        return false;
    };
    auto pow2_in = [](int x, int lo, int hi) { return x >= lo && x <= hi && (x & (x - 1)) == 0; };
    if (!((t.bellman_lanes >= -3 && t.bellman_lanes <= 0) || pow2_in(t.bellman_lanes, 1, 64)))
        return no("bellman_lanes must be -3, -2, -1, 0 or a power of two in [1, 64]");
    if (!(t.spmv_lanes == 0 || t.spmv_lanes == -1 || pow2_in(t.spmv_lanes, 1, 64)))
        return no("spmv_lanes must be -1, 0 or a power of two in [1, 64]");
    if (!(t.bellman_spt >= 0 && (int64_t)t.bellman_spt * m->A <= kMaxTileRows))
        return no("bellman_states_per_tile * A must be <= 3072");
    if (!(t.spmv_spt >= 0 && t.spmv_spt <= kMaxSpmvTile)) return no("spmv_states_per_tile must be <= 4096");
    if (!(t.bellman_chunk >= 0 && t.bellman_chunk <= 32 && t.spmv_chunk >= 0 && t.spmv_chunk <= 32))
        return no("chunk widths must lie in [0, 32]");
    if (!(t.spmv_schedule >= 0 && t.spmv_schedule <= 2)) return no("spmv_schedule must lie in [0, 2]");
    if (t.spmv_workgroups < 0) return no("spmv_workgroups must be >= 0");
    if (!(t.band_rows == 0 || t.band_rows == -1)) return no("band_rows must be 0 or -1");
    if (!(t.ppi_cached >= -1 && t.ppi_cached <= 1)) return no("ppi_cached must be -1, 0 or 1");
    if (!(t.blocked_prefetch == 0 || t.blocked_prefetch == -1)) return no("blocked_prefetch must be 0 or -1");
    return true;
}

ipi_status autotune(ipi_mdp_s* m, bool fp32, const char* cache_path, hipStream_t st) {
    IPI_REQUIRE(!fp32 || m->val32, IPI_E_INVALID_ARG, "fp32_mixed tuning needs IPI_VAL_FP32");
    IPI_REQUIRE(fp32 || m->val, IPI_E_INVALID_ARG, "fp64 tuning needs the FP64 values of P");
    const std::string key = shape_key(m, fp32);
    std::map<std::string, Tuning> cache;
    if (cache_path) {
        cache = read_cache(cache_path);
        auto it = cache.find(key);
        if (it != cache.end()) {
            // the cached launch shapes; the fields the cache does not hold
            // (band form, cached loads, grid size) keep the caller's settings
            const Tuning& c = it->second;
            Tuning t = m->tune;
            t.bellman_lanes = c.bellman_lanes;
            t.bellman_spt = c.bellman_spt;
            t.spmv_lanes = c.spmv_lanes;
            t.spmv_spt = c.spmv_spt;
            t.bellman_chunk = c.bellman_chunk;
            t.spmv_chunk = c.spmv_chunk;
            t.spmv_schedule = c.spmv_schedule;
            const bool chunks_ok = (t.bellman_chunk == 0 || flat_chunk_ok(m, fp32, t.bellman_chunk) ||
                                    (m->uniform_k && m->k_max == 1 && t.bellman_chunk == 1)) &&
                                   (t.spmv_chunk == 0 || flat_chunk_ok(m, fp32, t.spmv_chunk));
            if (tuning_admissible(m, t, nullptr) && chunks_ok) {
                m->tune = t;
                return IPI_OK;
            }
            cache.erase(it);  // not valid for this MDP (a corrupt or edited entry): tune again
        }
    }
    workspace_ensure(m, 1, 0, fp32, st);
    Workspace& w = m->ws;
    const int64_t S = m->S;
    launch_fill_u64(reinterpret_cast<uint64_t*>(w.V), S, 0, st);
    // repetitions so that each measurement covers at least ~2 ms of work
    const double bb = bellman_alg_bytes(m, fp32, 1);
    const int reps = std::max(3, std::min(50, (int)(2e-3 * 5e12 / std::max(bb, 1.0))));

    Tuning best = m->tune;
    double best_ms = 1e300;
    // lanes -1 = flat chunk streaming (uniform rows only), for every admissible chunk width
    // (-3 / -2: the same on wave / workgroup tiles)
    const int lanes_list[] = {-1, -3, -2, 1, 2, 4, 8, 16, 32, 64};
    const int chunk_list[] = {2, 4, 8, 12, 16, 24, 32};
    std::vector<int> widths;
    for (int e : chunk_list)
        if (flat_chunk_ok(m, fp32, e)) widths.push_back(e);
    if (widths.empty() && m->uniform_k && m->k_max == 1) widths.push_back(1);  // rows of one entry
    const Tuning saved = m->tune;
    for (int L : lanes_list) {
        const std::vector<int> es = L < 0 ? widths : std::vector<int>{0};
        for (int fe : es) {
            if (L == -3 && fe * (fp32 ? 4 : 8) != 16) continue;  // wave tiles take 16-byte chunks only
            m->tune.bellman_chunk = fe;
            for (int spt = 1; spt <= 1024; spt *= 2) {
                if ((int64_t)spt * m->A > kMaxTileRows) break;
                if (L < 0) {
                    const int64_t chunks = (int64_t)spt * m->A * (m->k_max / fe);
                    if (chunks > 4096) break;
                    if (chunks < kBlock / 2 && (int64_t)(2 * spt) * m->A <= kMaxTileRows) continue;
                } else {
                    const int groups = kBlock / L;
                    if ((int64_t)spt * m->A < groups / 4 && (int64_t)(2 * spt) * m->A <= kMaxTileRows) continue;
                    if ((int64_t)spt * m->A > 16 * groups) continue;
                }
                BellmanOut bo{nullptr, w.pi, w.b, nullptr, nullptr};
                const double ms = time_ms([&] { launch_bellman(m, m->g, w.V, bo, fp32, L, spt, st); }, st, reps);
                if (ms < best_ms) {
                    best_ms = ms;
                    best.bellman_lanes = L;
                    best.bellman_spt = spt;
                    best.bellman_chunk = fe;
                }
            }
        }
    }
    m->tune = saved;
    m->tune.bellman_chunk = best.bellman_chunk;
    // P_pi of the greedy policy for V = 0, then the product kernel
    BellmanOut bo{nullptr, w.pi, w.b, nullptr, nullptr};
    launch_bellman(m, m->g, w.V, bo, fp32, best.bellman_lanes, best.bellman_spt, st);
    launch_extract_ppi(m, w.pi, fp32, false, st);
    PpiView P;
    P.col = w.ppi_col;
    P.val = w.ppi_val;
    P.rp = m->uniform_k ? nullptr : w.ppi_rp;
    P.k = m->k_max;
    P.vec = m->uniform_k ? bellman_vec(m, fp32) : 1;
    P.fp32 = fp32;
    P.S = S;
    P.gamma = m->gamma;
    P.dinv = nullptr;
    P.flat_e = 0;
    k_launch_ctrl_reset(w.ctrl, 0.0, 1 << 30, 1, 1.0, st);  // target 0: the sweeps never stop early
    best_ms = 1e300;
    for (int L : lanes_list) {
        if (L < -1) continue;  // Bellman-only schedules
        const std::vector<int> es = L < 0 ? widths : std::vector<int>{0};
        for (int sfe : es) {
            P.flat_e = sfe;
            // workgroup tiles (schedule 1), then for flat rows wave tiles (schedule 2)
            for (int sched = 1; sched <= (L < 0 ? 2 : 1); ++sched) {
                P.pipe = sched == 2 ? 1 : 0;
                const int lo = sched == 2 ? 8 : 64, hi = sched == 2 ? 64 : kMaxSpmvTile;
                for (int spt = lo; spt <= hi; spt *= 2) {
                    if (L > 0 && spt < kBlock / L / 2) continue;
                    if (sched == 1 && L < 0 && (int64_t)spt * (m->k_max / sfe) > 8 * kBlock) break;
                    if (sched == 2 && (int64_t)spt * (m->k_max / sfe) > 1024) break;
                    LaunchShape sh{L < 0 ? 1 : L, spt, w.nblk_red};
                    const double ms = time_ms([&] {
                        k_launch_rich(P, sh, w.b, w.delta, w.delta2, 0, w.partials, w.ctrl, w.small, st);
                    }, st, reps);
                    if (ms < best_ms) {
                        best_ms = ms;
                        best.spmv_lanes = L;
                        best.spmv_spt = spt;
                        best.spmv_chunk = sfe;
                        best.spmv_schedule = L < 0 ? sched : 0;
                    }
                }
            }
        }
    }
    IPI_HIP(hipStreamSynchronize(st));
    m->tune = best;
    if (cache_path) {
        cache[key] = best;
        write_cache(cache_path, cache);
    }
    return IPI_OK;
}

}  // namespace ipi
