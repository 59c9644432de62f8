// MDP residency: validation, upload to HBM (row_ptr narrowed to int32 when
// nnz < 2^31, optional float32 value copy), derived shape facts, and the
// solve workspace.  Everything is allocated once here or on the first solve,
// never inside the iteration loops.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

namespace ipi {

namespace {

// Run f(begin, end) over [0, n) on up to 16 host threads.
template <typename F>
void host_parallel(int64_t n, F&& f) {
    unsigned nt = std::thread::hardware_concurrency();
    if (nt == 0) nt = 1;
    if (nt > 16) nt = 16;
    if (n < (int64_t)1 << 16) nt = 1;
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        int64_t b = t * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        th.emplace_back([&f, b, e] { f(b, e); });
    }
    for (auto& x : th) x.join();
}

struct ShapeFacts {
    int32_t kmin = 0, kmax = 0;
    int vec = 4;
    int64_t ppi_cap = 0;  // sum over states of the longest row of the state
};

// Host-side checks of the tuple of Sec. II on host arrays.
ShapeFacts validate_host(int64_t S, int32_t A, int64_t nnz, const int64_t* rp, const int32_t* col,
                         const double* val, const double* g, bool check, double rs_tol_abs) {
    const int64_t R = S * (int64_t)A;
    IPI_REQUIRE(rp[0] == 0, IPI_E_INVALID_ARG, "row_ptr[0] must be 0");
    IPI_REQUIRE(rp[R] == nnz, IPI_E_INVALID_ARG, "row_ptr[S*A] must equal nnz");
    std::mutex mu;
    ShapeFacts out;
    out.kmin = INT32_MAX;
    out.kmax = 0;
    std::string err;
    ipi_status est = IPI_OK;
    host_parallel(S, [&](int64_t sb, int64_t se) {
        int32_t kmin = INT32_MAX, kmax = 0;
        int64_t orv = 0, cap = 0;
        std::string lerr;
        ipi_status lst = IPI_OK;
        for (int64_t s = sb; s < se && lst == IPI_OK; ++s) {
            int64_t smax = 0;
            for (int a = 0; a < A; ++a) {
                const int64_t r = s * A + a;
                const int64_t b = rp[r], e = rp[r + 1];
                if (e < b || b < 0 || e > nnz) {
                    lst = IPI_E_INVALID_ARG;
                    lerr = "row_ptr is not non-decreasing within [0, nnz] at row " + std::to_string(r);
                    break;
                }
                const int64_t len = e - b;
                kmin = std::min<int64_t>(kmin, len);
                kmax = std::max<int64_t>(kmax, len);
                smax = std::max(smax, len);
                orv |= b;
                if (!check) continue;
                double sum = 0.0;
                int32_t prev = -1;
                for (int64_t j = b; j < e; ++j) {
                    const int32_t c = col[j];
                    const double v = val[j];
                    if (c < 0 || c >= S || c <= prev) {
                        lst = IPI_E_INVALID_ARG;
                        lerr = "column index out of range or not strictly ascending in row " + std::to_string(r);
                        break;
                    }
                    prev = c;
                    if (!(v >= 0.0) || !std::isfinite(v)) {
                        lst = IPI_E_NOT_STOCHASTIC;
                        lerr = "negative or non-finite probability in row " + std::to_string(r);
                        break;
                    }
                    sum += v;
                }
                if (lst != IPI_OK) break;
                const double tol = rs_tol_abs > 0 ? rs_tol_abs : 1e-12 * std::max<double>(1.0, (double)len);
                if (!(std::fabs(sum - 1.0) <= tol)) {
                    lst = IPI_E_NOT_STOCHASTIC;
                    lerr = "row " + std::to_string(r) + " of P sums to " + std::to_string(sum) + ", not 1";
                    break;
                }
                if (!std::isfinite(g[r])) {
                    lst = IPI_E_INVALID_ARG;
                    lerr = "non-finite stage cost at row " + std::to_string(r);
                    break;
                }
            }
            cap += smax;
        }
        std::lock_guard<std::mutex> lk(mu);
        if (lst != IPI_OK && est == IPI_OK) {
            est = lst;
            err = lerr;
        }
        out.kmin = std::min(out.kmin, kmin);
        out.kmax = std::max(out.kmax, kmax);
        out.ppi_cap += cap;
        if (orv & 3) out.vec = std::min(out.vec, (orv & 1) ? 1 : 2);
    });
    if (est != IPI_OK) throw Error(est, err);
    if (nnz & 3) out.vec = std::min(out.vec, (nnz & 1) ? 1 : 2);
    return out;
}

// ---- device-side validation for device inputs ----------------------------
struct DevFacts {
    uint32_t err;      // bit 0 structure, bit 1 stochastic, bit 2 cost
    int32_t kmin;
    int32_t kmax;
    uint32_t orbits;   // OR of all row_ptr values (low bits give the vector alignment)
    unsigned long long cap;
};

__global__ void k_validate(int64_t S, int A, int64_t nnz, const int64_t* rp, const int* col, const double* val,
                           const double* g, int check, double rs_tol_abs, DevFacts* f) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
        int64_t smax = 0;
        uint32_t err = 0;
        int32_t kmin = INT32_MAX, kmax = 0;
        uint32_t orb = 0;
        for (int a = 0; a < A; ++a) {
            const int64_t r = s * A + a;
            const int64_t b = rp[r], e = rp[r + 1];
            if (e < b || b < 0 || e > nnz) {
                err |= 1;
                break;
            }
            const int64_t len = e - b;
            kmin = min((int64_t)kmin, len);
            kmax = max((int64_t)kmax, len);
            smax = max(smax, len);
            orb |= (uint32_t)(b & 3);
            if (!check) continue;
            double sum = 0.0;
            int prev = -1;
            for (int64_t j = b; j < e; ++j) {
                const int c = col[j];
                const double v = val[j];
                if (c < 0 || c >= S || c <= prev) err |= 1;
                prev = c;
                if (!(v >= 0.0) || isinf(v)) err |= 2;
                sum += v;
            }
            const double tol = rs_tol_abs > 0 ? rs_tol_abs : 1e-12 * fmax(1.0, (double)len);
            if (!(fabs(sum - 1.0) <= tol)) err |= 2;
            if (isnan(g[r]) || isinf(g[r])) err |= 4;
        }
        if (err) atomicOr(&f->err, err);
        atomicMin(&f->kmin, kmin);
        atomicMax(&f->kmax, kmax);
        if (orb) atomicOr(&f->orbits, orb);
        atomicAdd(&f->cap, (unsigned long long)smax);
    }
}

__global__ void k_narrow_rowptr(const int64_t* in, int32_t* out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int32_t)in[i];
}

// band form: first column of each row of length k, and whether every row's
// columns are consecutive integers (any entry that is not clears flags[0]).
// One thread per nonzero, so the column stream is read coalesced.  flags[1]
// and flags[2] receive the min and max of first column - state over all rows
// (one atomic per workgroup).
__global__ void k_band_detect(const int* __restrict__ col, int64_t R, int k, int A, int32_t* __restrict__ band,
                              int* __restrict__ flags) {
    const int64_t n = R * (int64_t)k;
    int dlo = INT_MAX, dhi = INT_MIN;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = j / k;
        const int e = (int)(j - r * k);
        const int c0 = col[r * k];
        if (e == 0) {
            band[r] = c0;
            const int d = (int)((int64_t)c0 - r / A);
            dlo = min(dlo, d);
            dhi = max(dhi, d);
        }
        if (col[j] != c0 + e) flags[0] = 0;
    }
    __shared__ int lo[kBlock], hi[kBlock];
    lo[threadIdx.x] = dlo;
    hi[threadIdx.x] = dhi;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            lo[threadIdx.x] = min(lo[threadIdx.x], lo[threadIdx.x + h]);
            hi[threadIdx.x] = max(hi[threadIdx.x], hi[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMin(flags + 1, lo[0]);
        atomicMax(flags + 2, hi[0]);
    }
}

// stencil form: each row's pattern among the np known ones (the offsets of
// its columns from its first), written with its first column into the row's
// word; the lowest index of a row that matches none goes to *unmatched (one
// atomic per workgroup)
__global__ void k_sten_match(const int* __restrict__ col, int64_t R, int k, const int32_t* __restrict__ off, int np,
                             uint32_t* __restrict__ sten, unsigned long long* __restrict__ unmatched) {
    unsigned long long first = ~0ull;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < R; r += (int64_t)gridDim.x * blockDim.x) {
        const int* c = col + r * k;
        const int c0 = c[0];
        int found = -1;
        for (int q = 0; q < np && found < 0; ++q) {
            bool ok = true;
            for (int j = 1; j < k && ok; ++j) ok = c[j] - c0 == off[q * k + j];
            if (ok) found = q;
        }
        if (found >= 0) sten[r] = (uint32_t)c0 | ((uint32_t)found << kStenColBits);
        else if ((unsigned long long)r < first) first = (unsigned long long)r;
    }
    __shared__ unsigned long long lo[kBlock];
    lo[threadIdx.x] = first;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) lo[threadIdx.x] = min(lo[threadIdx.x], lo[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && lo[0] != ~0ull) atomicMin(unmatched, lo[0]);
}

// band form: min / max of first column - state over the rows of the states
// in [H, S - H) (the interior, away from the edges where a band window is
// clamped to [0, S) and reaches further); one atomic per workgroup
__global__ void k_band_interior(const int32_t* __restrict__ band, int64_t S, int A, int64_t H,
                                int* __restrict__ out) {
    int dlo = INT_MAX, dhi = INT_MIN;
    const int64_t r0 = H * (int64_t)A, r1 = (S - H) * (int64_t)A;
    for (int64_t r = r0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < r1; r += (int64_t)gridDim.x * blockDim.x) {
        const int d = (int)((int64_t)band[r] - r / A);
        dlo = min(dlo, d);
        dhi = max(dhi, d);
    }
    __shared__ int lo[kBlock], hi[kBlock];
    lo[threadIdx.x] = dlo;
    hi[threadIdx.x] = dhi;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            lo[threadIdx.x] = min(lo[threadIdx.x], lo[threadIdx.x + h]);
            hi[threadIdx.x] = max(hi[threadIdx.x], hi[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMin(out, lo[0]);
        atomicMax(out + 1, hi[0]);
    }
}

// float32 copy of P's values, one thread per row, and the largest row
// perturbation max_r sum_j |P_rj - float32(P_rj)| (it bounds how far the
// float32-rounded MDP's V* moves: gamma * dP * ||V*||_inf / (1 - gamma))
template <typename PT>
__global__ __launch_bounds__(256) void k_to_f32_rows(const PT* __restrict__ row_ptr, const double* __restrict__ in,
                                                     float* __restrict__ out, int64_t R, uint64_t* __restrict__ dp) {
    double worst = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < R; r += (int64_t)gridDim.x * blockDim.x) {
        double sum = 0.0;
        for (int64_t j = row_ptr[r]; j < (int64_t)row_ptr[r + 1]; ++j) {
            const double v = in[j];
            const float f = (float)v;
            out[j] = f;
            sum += fabs(v - (double)f);
        }
        worst = fmax(worst, sum);
    }
    worst = dev::wave_max(worst);
    if ((threadIdx.x & (dev::kWave - 1)) == 0) dev::atomic_max_nonneg(dp, worst);
}

// IPI_VAL_SPLIT: hi = float32(P) and lo = float32(P - hi) (P - hi is exact
// in FP64), one thread per row, with the largest row perturbations of hi
// alone (dp[0]) and of hi + lo rounded once to FP64 (dp[1]).
template <typename PT>
__global__ __launch_bounds__(256) void k_split_rows(const PT* __restrict__ row_ptr, const double* __restrict__ in,
                                                    float* __restrict__ hi, float* __restrict__ lo, int64_t R,
                                                    uint64_t* __restrict__ dp) {
    double w32 = 0.0, wsp = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < R; r += (int64_t)gridDim.x * blockDim.x) {
        double s32 = 0.0, ssp = 0.0;
        for (int64_t j = row_ptr[r]; j < (int64_t)row_ptr[r + 1]; ++j) {
            const double v = in[j];
            const float h = (float)v;
            const float l = (float)(v - (double)h);
            hi[j] = h;
            lo[j] = l;
            s32 += fabs(v - (double)h);
            ssp += fabs(v - ((double)h + (double)l));
        }
        w32 = fmax(w32, s32);
        wsp = fmax(wsp, ssp);
    }
    w32 = dev::wave_max(w32);
    wsp = dev::wave_max(wsp);
    if ((threadIdx.x & (dev::kWave - 1)) == 0) {
        dev::atomic_max_nonneg(dp, w32);
        dev::atomic_max_nonneg(dp + 1, wsp);
    }
}

unsigned grid_for(int64_t n, int cap = 16384) {
    int64_t nb = (n + kBlock - 1) / kBlock;
    if (nb > cap) nb = cap;
    if (nb < 1) nb = 1;
    return (unsigned)nb;
}

template <typename T>
T* dmalloc(size_t count, size_t* acc) {
    void* p = nullptr;
    if (count == 0) count = 1;
    IPI_HIP(hipMalloc(&p, count * sizeof(T)));
    if (acc) *acc += count * sizeof(T);
    return (T*)p;
}

// Uploads of host arrays through two pinned staging buffers: host threads
// copy the next 64 MB piece into one buffer while the other is in flight on
// the DMA engine.  From ordinary (pageable) host memory hipMemcpy measured
// 26 GB/s on MI355X hosts; this pipeline 55 GB/s, the pinned DMA rate (57).
// Arrays under 16 MB take a plain copy.  An upload takes a stager (two
// buffers, two events) from a process-wide pool for its duration, so
// concurrent uploads (the serving loop's workers) each have their own.  The
// call returns when the data is on the device, as a copy from pageable
// memory does.
struct Stager {
    char* buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
};
constexpr size_t kStagePiece = (size_t)64 << 20;
constexpr size_t kStageMin = (size_t)16 << 20;
std::mutex g_stage_mu;
std::vector<Stager*> g_stage_free;

Stager* stager_get() {
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        if (!g_stage_free.empty()) {
            Stager* sg = g_stage_free.back();
            g_stage_free.pop_back();
            return sg;
        }
    }
    auto* sg = new Stager();
    try {
        std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
        for (int i = 0; i < 2; ++i) {
            IPI_HIP(hipHostMalloc((void**)&sg->buf[i], kStagePiece, 0));
            IPI_HIP(hipEventCreateWithFlags(&sg->ev[i], hipEventDisableTiming));
        }
    } catch (...) {
        for (int i = 0; i < 2; ++i) {
            if (sg->buf[i]) hipHostFree(sg->buf[i]);
            if (sg->ev[i]) hipEventDestroy(sg->ev[i]);
        }
        delete sg;
        throw;
    }
    return sg;
}

void host_copy(char* dst, const char* src, size_t n) {
    const unsigned hw = std::thread::hardware_concurrency();
    const unsigned nt = (unsigned)std::min<size_t>(std::max(1u, std::min(8u, hw)), std::max<size_t>(1, n >> 22));
    if (nt <= 1) {
        std::memcpy(dst, src, n);
        return;
    }
    std::vector<std::thread> th;
    const size_t per = (n + nt - 1) / nt;
    for (unsigned t = 1; t < nt; ++t) {
        const size_t a = t * per, b = std::min(n, a + per);
        if (a < b) th.emplace_back([=] { std::memcpy(dst + a, src + a, b - a); });
    }
    std::memcpy(dst, src, std::min(n, per));
    for (auto& x : th) x.join();
}

void upload_h2d(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes < kStageMin) {
        IPI_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
        return;
    }
    Stager* sg = stager_get();
    bool used[2] = {false, false};
    // the buffers go back to the pool only with their copies done, also
    // when a call below fails
    struct Back {
        Stager* sg;
        bool* used;
        ~Back() {
            for (int i = 0; i < 2; ++i)
                if (used[i]) hipEventSynchronize(sg->ev[i]);
            std::lock_guard<std::mutex> lk(g_stage_mu);
            g_stage_free.push_back(sg);
        }
    } back{sg, used};
    int b = 0;
    for (size_t off = 0; off < bytes; off += kStagePiece) {
        const size_t n = std::min(kStagePiece, bytes - off);
        if (used[b]) IPI_HIP(hipEventSynchronize(sg->ev[b]));
        host_copy(sg->buf[b], static_cast<const char*>(src) + off, n);
        IPI_HIP(hipMemcpyAsync(static_cast<char*>(dst) + off, sg->buf[b], n, hipMemcpyHostToDevice, st));
        IPI_HIP(hipEventRecord(sg->ev[b], st));
        used[b] = true;
        b ^= 1;
    }
}

void free_data(ipi_mdp_s* m) {
    if (!m->borrowed) {
        hipFree(m->row_ptr);
        hipFree(m->col);
        hipFree(m->val);
        hipFree(m->g);
    } else if (m->rp32) {
        hipFree(m->row_ptr);
    }
    hipFree(m->val32);
    hipFree(m->val_lo);
    m->val_lo = nullptr;
    m->split_dp = 0.0;
    hipFree(m->band);
    m->band = nullptr;
    hipFree(m->sten);
    hipFree(m->sten_off);
    m->sten = nullptr;
    m->sten_off = nullptr;
    m->sten_np = 0;
    m->sten_pairs = false;
    hipFree(m->g_neg);
    hipFree(m->rho_slot);
    m->rho_slot = nullptr;
    m->row_ptr = nullptr;
    m->col = nullptr;
    m->val = nullptr;
    m->g = nullptr;
    m->val32 = nullptr;
    m->g_neg = nullptr;
}

// Stencil form.  The patterns of the first rows (at most 4096) are read on the
// host; more than kStenMaxPatterns of them there, or a row longer than
// kStenMaxK, rules the form out at once (random columns: one copy of 4096
// rows).  Otherwise every row is matched on the device; a row that matches
// none adds its pattern, up to kStenMaxPatterns, and the pass repeats.  The
// words and the offsets are kept only when every row matches.
void detect_stencil(ipi_mdp_s* m, hipStream_t st, size_t* bytes) {
    const int k = m->k_max;
    const int64_t R = m->S * (int64_t)m->A;
    if (!m->uniform_k || k < 2 || k > kStenMaxK || m->S >= ((int64_t)1 << kStenColBits)) return;
    std::vector<std::vector<int32_t>> pats;
    auto add = [&](const int32_t* c) {
        std::vector<int32_t> o(k);
        for (int j = 0; j < k; ++j) o[j] = c[j] - c[0];
        for (const auto& q : pats)
            if (q == o) return true;
        if ((int)pats.size() == kStenMaxPatterns) return false;
        pats.push_back(o);
        return true;
    };
    const int64_t rs = std::min<int64_t>(R, 4096);
    std::vector<int32_t> hc((size_t)rs * k);
    IPI_HIP(hipMemcpyAsync(hc.data(), m->col, hc.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    IPI_HIP(hipStreamSynchronize(st));
    for (int64_t r = 0; r < rs; ++r)
        if (!add(&hc[(size_t)r * k])) return;
    uint32_t* sten = dmalloc<uint32_t>(R, bytes);
    int32_t* off = dmalloc<int32_t>((size_t)kStenMaxPatterns * k, bytes);
    unsigned long long* um = dmalloc<unsigned long long>(1, nullptr);
    auto drop = [&]() {
        hipFree(sten);
        hipFree(off);
        hipFree(um);
        *bytes -= (size_t)R * sizeof(uint32_t) + (size_t)kStenMaxPatterns * k * sizeof(int32_t);
    };
    try {
    for (;;) {
        std::vector<int32_t> flat((size_t)kStenMaxPatterns * k, 0);
        for (size_t q = 0; q < pats.size(); ++q) std::copy(pats[q].begin(), pats[q].end(), flat.begin() + q * k);
        const unsigned long long none = ~0ull;
        unsigned long long first = 0;
        IPI_HIP(hipMemcpyAsync(off, flat.data(), flat.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
        IPI_HIP(hipMemcpyAsync(um, &none, sizeof(none), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_sten_match, dim3(grid_for(R)), dim3(kBlock), 0, st, m->col, R, k, off, (int)pats.size(),
                           sten, um);
        IPI_HIP(hipGetLastError());
        IPI_HIP(hipMemcpyAsync(&first, um, sizeof(first), hipMemcpyDeviceToHost, st));
        IPI_HIP(hipStreamSynchronize(st));
        if (first == none) break;
        std::vector<int32_t> c(k);
        IPI_HIP(hipMemcpyAsync(c.data(), m->col + (int64_t)first * k, k * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        IPI_HIP(hipStreamSynchronize(st));
        if (!add(c.data())) {
            drop();
            return;
        }
    }
    } catch (...) {
        drop();
        throw;
    }
    hipFree(um);
    m->sten = sten;
    m->sten_off = off;
    m->sten_np = (int)pats.size();
    bool pairs = k % 2 == 0;
    for (const auto& q : pats)
        for (int j = 0; j + 1 < k; j += 2) pairs = pairs && q[j + 1] == q[j] + 1;
    m->sten_pairs = pairs;
}

}  // namespace

// Host checks of a request before it is queued (the serving loop).
void validate_host_arrays(int64_t S, int32_t A, int64_t nnz, const int64_t* rp, const int32_t* col, const double* val,
                          const double* g, double gamma, uint32_t flags, int32_t* kmax) {
    IPI_REQUIRE(S >= 1 && S < ((int64_t)1 << 31), IPI_E_INVALID_ARG, "S must lie in [1, 2^31)");
    IPI_REQUIRE(A >= 1 && A <= kMaxA, IPI_E_INVALID_ARG, "A must lie in [1, 3072]");
    IPI_REQUIRE(nnz >= S * (int64_t)A, IPI_E_INVALID_ARG, "every row of P needs at least one entry (nnz >= S*A)");
    IPI_REQUIRE(rp && col && val && g, IPI_E_INVALID_ARG, "null input array");
    IPI_REQUIRE(gamma > 0.0 && gamma < 1.0, IPI_E_INVALID_ARG, "gamma must lie in (0, 1)");
    const ShapeFacts f = validate_host(S, A, nnz, rp, col, val, g, !(flags & IPI_NO_VALIDATE),
                                       (flags & IPI_FP32_ORIGIN) ? 1e-6 : 0.0);
    if (kmax) *kmax = f.kmax;
}

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipGetDevice(&dev);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

// Host side of the same conversion (host inputs kept in float32 only).
double host_to_f32_rows(const int64_t* rp, const double* val, float* out, int64_t R) {
    std::mutex mu;
    double worst = 0.0;
    host_parallel(R, [&](int64_t b, int64_t e) {
        double w = 0.0;
        for (int64_t r = b; r < e; ++r) {
            double sum = 0.0;
            for (int64_t j = rp[r]; j < rp[r + 1]; ++j) {
                const float f = (float)val[j];
                out[j] = f;
                sum += std::fabs(val[j] - (double)f);
            }
            w = std::max(w, sum);
        }
        std::lock_guard<std::mutex> lk(mu);
        worst = std::max(worst, w);
    });
    return worst;
}

ipi_mdp_s* create_mdp(int64_t S, int32_t A, int64_t nnz, const int64_t* row_ptr, const int32_t* col,
                      const double* val, const double* g, double gamma, uint32_t flags, hipStream_t st) {
    std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
    IPI_REQUIRE(S >= 1, IPI_E_INVALID_ARG, "S must be >= 1");
    IPI_REQUIRE(S < ((int64_t)1 << 31), IPI_E_INVALID_ARG, "S must be < 2^31 (int32 columns)");
    IPI_REQUIRE(A >= 1 && A <= kMaxA, IPI_E_INVALID_ARG, "A must lie in [1, 3072]");
    IPI_REQUIRE(nnz >= S * (int64_t)A, IPI_E_INVALID_ARG, "every row of P needs at least one entry (nnz >= S*A)");
    IPI_REQUIRE(row_ptr && col && val && g, IPI_E_INVALID_ARG, "null input array");
    IPI_REQUIRE(gamma > 0.0 && gamma < 1.0, IPI_E_INVALID_ARG, "gamma must lie in (0, 1)");
    const bool dev_in = flags & IPI_DEVICE_PTRS;
    const bool borrow = flags & IPI_BORROW;
    const bool only32 = flags & IPI_VAL_FP32_ONLY;
    const bool split = flags & IPI_VAL_SPLIT;
    IPI_REQUIRE(!borrow || dev_in, IPI_E_INVALID_ARG, "IPI_BORROW needs IPI_DEVICE_PTRS");
    IPI_REQUIRE(!(split && only32), IPI_E_INVALID_ARG, "IPI_VAL_SPLIT and IPI_VAL_FP32_ONLY exclude each other");
    const bool check = !(flags & IPI_NO_VALIDATE);
    const double rs_tol = (flags & IPI_FP32_ORIGIN) ? 1e-6 : 0.0;
    const int64_t R = S * (int64_t)A;

    ShapeFacts facts;
    if (!dev_in) facts = validate_host(S, A, nnz, row_ptr, col, val, g, check, rs_tol);

    auto* m = new ipi_mdp_s();
    m->S = S;
    m->A = A;
    m->nnz = nnz;
    m->gamma = gamma;
    m->borrowed = borrow;
    hipGetDevice(&m->device);
    try {
        size_t bytes = 0;
        m->rp32 = nnz < ((int64_t)1 << 31) && !borrow;
        if (dev_in) {
            if (borrow) {
                m->row_ptr = (void*)row_ptr;
                m->col = (int32_t*)col;
                m->val = (double*)val;
                m->g = (double*)g;
            } else {
                m->col = dmalloc<int32_t>(nnz, &bytes);
                m->val = dmalloc<double>(nnz, &bytes);
                m->g = dmalloc<double>(R, &bytes);
                IPI_HIP(hipMemcpyAsync(m->col, col, nnz * 4, hipMemcpyDeviceToDevice, st));
                IPI_HIP(hipMemcpyAsync(m->val, val, nnz * 8, hipMemcpyDeviceToDevice, st));
                IPI_HIP(hipMemcpyAsync(m->g, g, R * 8, hipMemcpyDeviceToDevice, st));
            }
            DevFacts* df = nullptr;
            IPI_HIP(hipMalloc(&df, sizeof(DevFacts)));
            DevFacts init{0, INT32_MAX, 0, 0, 0};
            IPI_HIP(hipMemcpyAsync(df, &init, sizeof(init), hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_validate, dim3(grid_for(S)), dim3(kBlock), 0, st, S, A, nnz, row_ptr,
                               (const int*)col, val, g, check ? 1 : 0, rs_tol, df);
            DevFacts hf;
            IPI_HIP(hipMemcpyAsync(&hf, df, sizeof(hf), hipMemcpyDeviceToHost, st));
            IPI_HIP(hipStreamSynchronize(st));
            hipFree(df);
            int64_t last = 0, first = 0;
            IPI_HIP(hipMemcpy(&first, row_ptr, 8, hipMemcpyDeviceToHost));
            IPI_HIP(hipMemcpy(&last, row_ptr + R, 8, hipMemcpyDeviceToHost));
            IPI_REQUIRE(first == 0 && last == nnz, IPI_E_INVALID_ARG, "row_ptr must start at 0 and end at nnz");
            if (hf.err & 1) throw Error(IPI_E_INVALID_ARG, "malformed CSR structure (row_ptr or column indices)");
            if (hf.err & 2) throw Error(IPI_E_NOT_STOCHASTIC, "a row of P is negative, non-finite or does not sum to 1");
            if (hf.err & 4) throw Error(IPI_E_INVALID_ARG, "non-finite stage cost");
            facts.kmin = hf.kmin;
            facts.kmax = hf.kmax;
            facts.ppi_cap = (int64_t)hf.cap;
            facts.vec = (hf.orbits & 1) ? 1 : ((hf.orbits & 2) ? 2 : 4);
            if (nnz & 3) facts.vec = std::min(facts.vec, (nnz & 1) ? 1 : 2);
            if (m->rp32) {
                m->row_ptr = dmalloc<int32_t>(R + 1, &bytes);
                hipLaunchKernelGGL(k_narrow_rowptr, dim3(grid_for(R + 1)), dim3(kBlock), 0, st, row_ptr,
                                   (int32_t*)m->row_ptr, R + 1);
            } else if (!borrow) {
                m->row_ptr = dmalloc<int64_t>(R + 1, &bytes);
                IPI_HIP(hipMemcpyAsync(m->row_ptr, row_ptr, (R + 1) * 8, hipMemcpyDeviceToDevice, st));
            }
        } else {
            m->col = dmalloc<int32_t>(nnz, &bytes);
            if (!only32) m->val = dmalloc<double>(nnz, &bytes);
            m->g = dmalloc<double>(R, &bytes);
            if (m->rp32) {
                std::vector<int32_t> rp32((size_t)R + 1);
                host_parallel(R + 1, [&](int64_t b, int64_t e) {
                    for (int64_t i = b; i < e; ++i) rp32[i] = (int32_t)row_ptr[i];
                });
                m->row_ptr = dmalloc<int32_t>(R + 1, &bytes);
                upload_h2d(m->row_ptr, rp32.data(), (R + 1) * 4, st);
                IPI_HIP(hipStreamSynchronize(st));
            } else {
                m->row_ptr = dmalloc<int64_t>(R + 1, &bytes);
                upload_h2d(m->row_ptr, row_ptr, (R + 1) * 8, st);
            }
            upload_h2d(m->col, col, nnz * 4, st);
            if (only32) {
                // float32 values only: converted here, the FP64 ones never uploaded
                std::vector<float> v32((size_t)nnz);
                m->val32_dp = host_to_f32_rows(row_ptr, val, v32.data(), R);
                m->val32 = dmalloc<float>(nnz, &bytes);
                upload_h2d(m->val32, v32.data(), nnz * 4, st);
                IPI_HIP(hipStreamSynchronize(st));
            } else {
                upload_h2d(m->val, val, nnz * 8, st);
            }
            upload_h2d(m->g, g, R * 8, st);
        }
        if (split) {
            // float32 hi and lo made from the FP64 values, which are then released
            // (borrowed ones stay the caller's)
            m->val32 = dmalloc<float>(nnz, &bytes);
            m->val_lo = dmalloc<float>(nnz, &bytes);
            uint64_t* dp = dmalloc<uint64_t>(2, nullptr);
            IPI_HIP(hipMemsetAsync(dp, 0, 16, st));
            const int64_t nb = std::min<int64_t>(grid_for(R), 4096);
            if (m->rp32)
                hipLaunchKernelGGL(k_split_rows<int32_t>, dim3((unsigned)nb), dim3(kBlock), 0, st,
                                   (const int32_t*)m->row_ptr, m->val, m->val32, m->val_lo, R, dp);
            else
                hipLaunchKernelGGL(k_split_rows<int64_t>, dim3((unsigned)nb), dim3(kBlock), 0, st,
                                   (const int64_t*)m->row_ptr, m->val, m->val32, m->val_lo, R, dp);
            uint64_t hb[2] = {0, 0};
            IPI_HIP(hipMemcpyAsync(hb, dp, 16, hipMemcpyDeviceToHost, st));
            IPI_HIP(hipStreamSynchronize(st));
            hipFree(dp);
            std::memcpy(&m->val32_dp, &hb[0], 8);
            std::memcpy(&m->split_dp, &hb[1], 8);
            if (!borrow) {
                hipFree(m->val);
                bytes -= (size_t)nnz * sizeof(double);
            }
            m->val = nullptr;
        }
        if ((flags & (IPI_VAL_FP32 | IPI_VAL_FP32_ONLY)) && !m->val32) {
            m->val32 = dmalloc<float>(nnz, &bytes);
            uint64_t* dp = dmalloc<uint64_t>(1, nullptr);
            IPI_HIP(hipMemsetAsync(dp, 0, 8, st));
            const int64_t nb = std::min<int64_t>(grid_for(R), 4096);
            if (m->rp32)
                hipLaunchKernelGGL(k_to_f32_rows<int32_t>, dim3((unsigned)nb), dim3(kBlock), 0, st,
                                   (const int32_t*)m->row_ptr, m->val, m->val32, R, dp);
            else
                hipLaunchKernelGGL(k_to_f32_rows<int64_t>, dim3((unsigned)nb), dim3(kBlock), 0, st,
                                   (const int64_t*)m->row_ptr, m->val, m->val32, R, dp);
            uint64_t hb = 0;
            IPI_HIP(hipMemcpyAsync(&hb, dp, 8, hipMemcpyDeviceToHost, st));
            IPI_HIP(hipStreamSynchronize(st));
            hipFree(dp);
            std::memcpy(&m->val32_dp, &hb, 8);
            if (only32) {
                // the FP64 values are not kept (borrowed ones stay the caller's)
                if (!borrow) {
                    hipFree(m->val);
                    bytes -= (size_t)nnz * sizeof(double);
                }
                m->val = nullptr;
            }
        }
        IPI_HIP(hipGetLastError());
        IPI_HIP(hipStreamSynchronize(st));
        m->k_min = facts.kmin;
        m->k_max = facts.kmax;
        m->uniform_k = facts.kmin == facts.kmax;
        m->vec_align = facts.vec;
        // vector loads need 16-byte aligned value/column arrays (borrowed arrays may not be)
        if (((uintptr_t)m->col | (uintptr_t)m->val) & 15) m->vec_align = 1;
        m->data_bytes = bytes;
        m->ws.kmax = facts.kmax;
        m->ws.S = 0;
        m->ppi_cap = facts.ppi_cap;
        m->arch_cus = device_cus();
        if (m->uniform_k && m->k_max >= 2) {
            const int64_t R = S * (int64_t)A;
            int32_t* band = dmalloc<int32_t>(R, &bytes);
            int* flags = dmalloc<int>(3, &bytes);
            const int init[3] = {1, INT_MAX, INT_MIN};
            IPI_HIP(hipMemcpyAsync(flags, init, sizeof(init), hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_band_detect, dim3(grid_for(R * (int64_t)m->k_max)), dim3(kBlock), 0, st, m->col, R,
                               m->k_max, A, band, flags);
            int hf[3] = {0, 0, 0};
            IPI_HIP(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st));
            IPI_HIP(hipStreamSynchronize(st));
            hipFree(flags);
            bytes -= 3 * sizeof(int);
            if (hf[0]) {
                m->band = band;
                m->band_dlo = hf[1];
                m->band_dhi = hf[2];
                // the same bounds over the interior states only
                const int64_t H = std::max<int64_t>(0, std::max<int64_t>(-(int64_t)hf[1], (int64_t)hf[2] + m->k_max - 1));
                m->band_dlo_in = hf[1];
                m->band_dhi_in = hf[2];
                if (S > 2 * H) {
                    int* io = dmalloc<int>(2, nullptr);
                    const int init_io[2] = {INT_MAX, INT_MIN};
                    IPI_HIP(hipMemcpyAsync(io, init_io, sizeof(init_io), hipMemcpyHostToDevice, st));
                    hipLaunchKernelGGL(k_band_interior, dim3(grid_for((S - 2 * H) * (int64_t)A)), dim3(kBlock), 0, st,
                                       band, S, A, H, io);
                    int hio[2] = {0, 0};
                    IPI_HIP(hipMemcpyAsync(hio, io, sizeof(hio), hipMemcpyDeviceToHost, st));
                    IPI_HIP(hipStreamSynchronize(st));
                    hipFree(io);
                    m->band_dlo_in = hio[0];
                    m->band_dhi_in = hio[1];
                }
            } else {
                hipFree(band);
                bytes -= (size_t)R * sizeof(int32_t);
                detect_stencil(m, st, &bytes);
            }
            m->data_bytes = bytes;
        }
    } catch (...) {
        free_data(m);
        delete m;
        throw;
    }
    return m;
}

void destroy_mdp(ipi_mdp_s* m) {
    if (!m) return;
    std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(m->device);
    hipDeviceSynchronize();
    workspace_free(m);
    free_data(m);
    hipSetDevice(cur);
    delete m;
}

// Release an MDP whose work the caller has already waited for: no
// device-wide synchronisation (the serving loop waits for its own stream).
void release_mdp(ipi_mdp_s* m) {
    if (!m) return;
    std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
    workspace_free(m);
    free_data(m);
    delete m;
}

void workspace_free(ipi_mdp_s* m) {
    Workspace& w = m->ws;
    void* ptrs[] = {w.V, w.TV, w.b, w.delta, w.delta2, w.basis, w.small, w.partials, w.aux, w.diag,
                    w.pi, w.ppi_col, w.ppi_band, w.ppi_sten, w.ppi_val, w.ppi_rp, w.scan_tmp, w.ctrl, w.bpart};
    for (void* p : ptrs) hipFree(p);
    if (w.cycle_graph) hipGraphExecDestroy(w.cycle_graph);
    if (w.capture_stream) hipStreamDestroy(w.capture_stream);
    int kmax = w.kmax;
    w = Workspace();
    w.kmax = kmax;
}

hipGraphExec_t capture_graph(Workspace& w, void (*enqueue)(void*, hipStream_t), void* ctx) {
    std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
    if (w.cycle_graph) hipGraphExecDestroy(w.cycle_graph);
    w.cycle_graph = nullptr;
    if (!w.capture_stream) IPI_HIP(hipStreamCreateWithFlags(&w.capture_stream, hipStreamNonBlocking));
    return capture_graph_on(w.capture_stream, enqueue, ctx);
}

std::recursive_mutex& device_sync_mutex() {
    static std::recursive_mutex mu;
    return mu;
}

hipGraphExec_t capture_graph_on(hipStream_t cap, void (*enqueue)(void*, hipStream_t), void* ctx) {
    std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    std::string why;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        try {
            enqueue(ctx, cap);
        } catch (const Error& err) {
            why = err.what();
        }
        e = hipStreamEndCapture(cap, &g);
        if (e == hipSuccess && why.empty()) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (g) hipGraphDestroy(g);
    }
    if (e != hipSuccess || !why.empty()) {
        if (why.empty()) why = hipGetErrorString(e);
        if (ex) hipGraphExecDestroy(ex);
        ex = nullptr;
        (void)hipGetLastError();  // the failure is handled: launch eagerly
        if (std::getenv("IPI_TRACE")) std::fprintf(stderr, "[ipi] graph capture failed (%s); launching eagerly\n", why.c_str());
    }
    return ex;
}

// Allocate (or grow) the solve workspace: iterate vectors, Krylov basis of
// restart+1 vectors, compact P_pi, control block and reduction partials.
void workspace_ensure(ipi_mdp_s* m, int restart, int naux, bool fp32, hipStream_t st, size_t bpart_n) {
    std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
    Workspace& w = m->ws;
    if (w.S == m->S && w.m >= restart && w.naux >= naux && w.ppi_val && w.fp32 == fp32 && w.bpart_n >= bpart_n)
        return;
    // each buffer is stored in w as soon as it is allocated, so a failure
    // part way leaves only buffers the next workspace_free releases
    workspace_free(m);
    workspace_layout(
        m, restart, naux, fp32, device_cus(), w,
        [](size_t bytes) {
            void* p = nullptr;
            IPI_HIP(hipMalloc(&p, bytes));
            return p;
        },
        bpart_n);
    IPI_HIP(hipMemsetAsync(w.ctrl, 0, sizeof(Ctrl), st));
    IPI_HIP(hipMemsetAsync(w.small, 0, 8192 * sizeof(double), st));
}

}  // namespace ipi
