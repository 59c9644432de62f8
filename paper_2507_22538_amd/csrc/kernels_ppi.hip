// Compact P_pi (Algorithm 1 step 4: the transition matrix of the greedy
// policy).  Row s of P_pi is row s*A + pi(s) of the row-stacked P
// (Sec. III-B.2: the row-stacked layout makes this a row access).
//
// Uniform row length k: P_pi is stored ELL-like (row s at s*k, no row
// pointers) and the copy is one thread per entry.  Otherwise the row
// lengths are scanned (three-pass exclusive scan, int64) into CSR row
// pointers and each row is copied by one thread.
//
// The Jacobi diagonal 1 - gamma*P(s,s,pi(s)) is produced on request.
#include "device.hpp"
#include "internal.hpp"

namespace ipi {

namespace {

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__global__ void k_scan_set_last(int64_t* p) { *p = 0; }

// VI: value type of P, VO: of P_pi (float32 P_pi from FP64 P rounds to nearest,
// as the float32 copy of P does)
template <typename PT, typename VI, typename VO>
__global__ __launch_bounds__(256) void k_extract_ell(const PT* __restrict__ row_ptr, const int* __restrict__ col,
                                                     const VI* __restrict__ val, const int32_t* __restrict__ pi,
                                                     int A, int k, int64_t S, int* __restrict__ ocol,
                                                     VO* __restrict__ oval) {
    const int64_t n = S * (int64_t)k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = e / k;
        const int j = (int)(e - s * k);
        const int64_t src = (int64_t)row_ptr[s * A + pi[s]] + j;
        ocol[e] = col[src];
        oval[e] = (VO)val[src];
    }
}

template <typename PT>
__global__ __launch_bounds__(256) void k_row_lengths(const PT* __restrict__ row_ptr, const int32_t* __restrict__ pi,
                                                     int A, int64_t S, int64_t* __restrict__ len_out) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = s * A + pi[s];
        len_out[s] = (int64_t)row_ptr[r + 1] - (int64_t)row_ptr[r];
    }
}

// exclusive scan, pass 1: per-tile scan in place, tile totals out
__global__ __launch_bounds__(256) void k_scan_tiles(int64_t* __restrict__ x, int64_t n, int64_t* __restrict__ tot) {
    __shared__ int64_t sh[kBlock];
    const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * (int64_t)kScanItems;
    int64_t v[kScanItems];
    int64_t run = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        const int64_t t = idx < n ? x[idx] : 0;
        v[i] = run;  // exclusive within the thread
        run += t;
    }
    sh[threadIdx.x] = run;
    __syncthreads();
    // Hillis-Steele inclusive scan of the thread totals
    for (int off = 1; off < kBlock; off <<= 1) {
        int64_t add = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const int64_t excl = threadIdx.x ? sh[threadIdx.x - 1] : 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        if (idx < n) x[idx] = v[i] + excl;
    }
    if (threadIdx.x == kBlock - 1) tot[blockIdx.x] = sh[kBlock - 1];
}

// pass 2: exclusive scan of the tile totals (one block, sequential chunks)
__global__ __launch_bounds__(256) void k_scan_totals(int64_t* __restrict__ tot, int64_t nt, int64_t* __restrict__ grand) {
    __shared__ int64_t sh[kBlock];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nt; b0 += kBlock) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t t = i < nt ? tot[i] : 0;
        sh[threadIdx.x] = t;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            int64_t add = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nt) tot[i] = carry + sh[threadIdx.x] - t;
        __syncthreads();
        if (threadIdx.x == 0) carry += sh[kBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *grand = carry;
}

// pass 3: add the tile offsets
__global__ __launch_bounds__(256) void k_scan_add(int64_t* __restrict__ x, int64_t n, const int64_t* __restrict__ tot) {
    const int64_t base = blockIdx.x * (int64_t)kScanTile;
    const int64_t off = tot[blockIdx.x];
    for (int i = threadIdx.x; i < kScanTile; i += kBlock) {
        const int64_t idx = base + i;
        if (idx < n) x[idx] += off;
    }
}

template <typename PT, typename VI, typename VO>
__global__ __launch_bounds__(256) void k_extract_csr(const PT* __restrict__ row_ptr, const int* __restrict__ col,
                                                     const VI* __restrict__ val, const int32_t* __restrict__ pi,
                                                     int A, int64_t S, const int64_t* __restrict__ orp,
                                                     int* __restrict__ ocol, VO* __restrict__ oval) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = s * A + pi[s];
        const int64_t b = row_ptr[r], e = row_ptr[r + 1];
        int64_t d = orp[s];
        for (int64_t j = b; j < e; ++j, ++d) {
            ocol[d] = col[j];
            oval[d] = (VO)val[j];
        }
    }
}

// Jacobi diagonal of J_pi: 1 - gamma * P_pi(s, s)
template <typename VT>
__global__ __launch_bounds__(256) void k_diag(const int* __restrict__ ocol, const VT* __restrict__ oval,
                                              const int64_t* __restrict__ orp, int k, int64_t S, double gamma,
                                              double* __restrict__ dinv) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = orp ? orp[s] : s * (int64_t)k;
        const int64_t e = orp ? orp[s + 1] : b + k;
        double p = 0.0;
        for (int64_t j = b; j < e; ++j)
            if (ocol[j] == (int)s) p += (double)oval[j];
        dinv[s] = 1.0 / (1.0 - gamma * p);
    }
}

// band form: first column of each P_pi row
__global__ __launch_bounds__(256) void k_extract_band(const int32_t* __restrict__ band,
                                                      const int32_t* __restrict__ pi, int A, int64_t S,
                                                      int32_t* __restrict__ out) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x)
        out[s] = band[s * A + pi[s]];
}

// stencil form: the word (first column and pattern) of each P_pi row
__global__ __launch_bounds__(256) void k_extract_sten(const uint32_t* __restrict__ sten,
                                                      const int32_t* __restrict__ pi, int A, int64_t S,
                                                      uint32_t* __restrict__ out) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x)
        out[s] = sten[s * A + pi[s]];
}

unsigned grid_for(int64_t n, int cap = 16384) {
    int64_t nb = (n + kBlock - 1) / kBlock;
    if (nb > cap) nb = cap;
    if (nb < 1) nb = 1;
    return (unsigned)nb;
}

template <typename PT, typename VI, typename VT>
void extract_typed(ipi_mdp_s* m, const int32_t* pi, const VI* val, bool want_diag, hipStream_t st) {
    Workspace& w = m->ws;
    const PT* rp = (const PT*)m->row_ptr;
    VT* oval = (VT*)w.ppi_val;
    const int64_t S = m->S;
    if (m->uniform_k) {
        const int k = m->k_max;
        hipLaunchKernelGGL((k_extract_ell<PT, VI, VT>), dim3(grid_for(S * (int64_t)k, 65536)), dim3(kBlock), 0, st, rp,
                           m->col, val, pi, m->A, k, S, w.ppi_col, oval);
        if (m->band && w.ppi_band)
            hipLaunchKernelGGL(k_extract_band, dim3(grid_for(S)), dim3(kBlock), 0, st, m->band, pi, m->A, S,
                               w.ppi_band);
        if (m->sten && w.ppi_sten)
            hipLaunchKernelGGL(k_extract_sten, dim3(grid_for(S)), dim3(kBlock), 0, st, m->sten, pi, m->A, S,
                               w.ppi_sten);
        if (want_diag)
            hipLaunchKernelGGL((k_diag<VT>), dim3(grid_for(S)), dim3(kBlock), 0, st, w.ppi_col, oval,
                               (const int64_t*)nullptr, k, S, m->gamma, w.diag);
    } else {
        // lengths into ppi_rp[0..S), exclusive scan over S+1 entries (last = total)
        hipLaunchKernelGGL((k_row_lengths<PT>), dim3(grid_for(S)), dim3(kBlock), 0, st, rp, pi, m->A, S, w.ppi_rp);
        const int64_t n = S + 1;
        const int64_t nt = (n + kScanTile - 1) / kScanTile;
        // entry S is a zero length (written here) so the exclusive scan leaves the total there
        hipLaunchKernelGGL(k_scan_set_last, dim3(1), dim3(1), 0, st, w.ppi_rp + S);
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(kBlock), 0, st, w.ppi_rp, n, w.scan_tmp);
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kBlock), 0, st, w.scan_tmp, nt, w.scan_tmp + nt);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nt), dim3(kBlock), 0, st, w.ppi_rp, n, w.scan_tmp);
        hipLaunchKernelGGL((k_extract_csr<PT, VI, VT>), dim3(grid_for(S)), dim3(kBlock), 0, st, rp, m->col, val, pi,
                           m->A, S, w.ppi_rp, w.ppi_col, oval);
        if (want_diag)
            hipLaunchKernelGGL((k_diag<VT>), dim3(grid_for(S)), dim3(kBlock), 0, st, w.ppi_col, oval,
                               (const int64_t*)w.ppi_rp, 0, S, m->gamma, w.diag);
    }
    IPI_HIP(hipGetLastError());
}

}  // namespace

// A float32 P_pi comes from the float32 copy of P when the MDP holds one,
// else from the FP64 values (rounded to nearest: the same floats).
void launch_extract_ppi(ipi_mdp_s* m, const int32_t* pi, bool fp32, bool want_diag, hipStream_t st) {
    if (fp32 && m->val32) {
        if (m->rp32) extract_typed<int32_t, float, float>(m, pi, m->val32, want_diag, st);
        else extract_typed<int64_t, float, float>(m, pi, m->val32, want_diag, st);
    } else if (fp32) {
        IPI_REQUIRE(m->val, IPI_E_INVALID_ARG, "the MDP holds no P values");
        if (m->rp32) extract_typed<int32_t, double, float>(m, pi, m->val, want_diag, st);
        else extract_typed<int64_t, double, float>(m, pi, m->val, want_diag, st);
    } else {
        IPI_REQUIRE(m->val, IPI_E_INVALID_ARG, "fp64 P_pi needs the FP64 values of P");
        if (m->rp32) extract_typed<int32_t, double, double>(m, pi, m->val, want_diag, st);
        else extract_typed<int64_t, double, double>(m, pi, m->val, want_diag, st);
    }
}

double extract_alg_bytes(const ipi_mdp_s* m, bool fp32) {
    const double bv = fp32 ? 4.0 : 8.0;
    const double bin = (fp32 && m->val32) ? 4.0 : 8.0;  // values read from P
    const double bp = m->rp32 ? 4.0 : 8.0;
    const double S = (double)m->S;
    // pi read, one row pointer per state (two for CSR + output pointers), the rows read and written
    const double kavg = m->uniform_k ? (double)m->k_max : (double)m->ppi_cap / S;
    double b = 4.0 * S + S * kavg * (bin + bv + 8.0);
    b += m->uniform_k ? bp * S : (2.0 * bp * S + 3.0 * 8.0 * S);
    if (m->band && m->uniform_k) b += 12.0 * S;  // band form: pi and the row's first column read, one written
    if (m->sten && m->uniform_k) b += 12.0 * S;  // stencil form: pi and the row's word read, one written
    return b;
}

}  // namespace ipi
