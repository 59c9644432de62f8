// extern "C" entry points of libipi.so: argument checks, error capture,
// option parsing (Table 1 names).  No exception crosses this boundary.
#include <cerrno>
#include <cmath>
#include <cstdlib>
#include <string>

#include "internal.hpp"

namespace ipi {
ipi_mdp_s* create_mdp(int64_t S, int32_t A, int64_t nnz, const int64_t* row_ptr, const int32_t* col,
                      const double* val, const double* g, double gamma, uint32_t flags, hipStream_t st);
void destroy_mdp(ipi_mdp_s* m);

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace ipi

using namespace ipi;

#define IPI_GUARD_BEGIN try {
#define IPI_GUARD_END                                          \
    }                                                          \
    catch (const ipi::Error& e) {                              \
        set_last_error(e.what());                              \
        return e.status;                                       \
    }                                                          \
    catch (const std::bad_alloc&) {                            \
        set_last_error("host allocation failed");              \
        return IPI_E_OOM;                                      \
    }                                                          \
    catch (const std::exception& e) {                          \
        set_last_error(e.what());                              \
        return IPI_E_DEVICE;                                   \
    }

extern "C" {

const char* ipi_last_error(void) { return g_last_error.c_str(); }

const char* ipi_version(void) { return "ipi-mi355x 0.1.0 (gfx950)"; }

ipi_status ipi_mdp_create_csr(int64_t S, int32_t A, int64_t nnz, const int64_t* row_ptr, const int32_t* col,
                              const double* val, const double* g, double gamma, uint32_t flags, void* stream,
                              ipi_mdp_t* out) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(out != nullptr, IPI_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    *out = create_mdp(S, A, nnz, row_ptr, col, val, g, gamma, flags, (hipStream_t)stream);
    set_last_error("");
    return IPI_OK;
    IPI_GUARD_END
}

ipi_status ipi_mdp_destroy(ipi_mdp_t mdp) {
    IPI_GUARD_BEGIN
    destroy_mdp(mdp);
    return IPI_OK;
    IPI_GUARD_END
}

ipi_status ipi_mdp_describe(ipi_mdp_t m, ipi_mdp_desc* out) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(m && out, IPI_E_INVALID_ARG, "NULL argument");
    out->S = m->S;
    out->A = m->A;
    out->nnz = m->nnz;
    out->k_min = m->k_min;
    out->k_max = m->k_max;
    out->uniform_k = m->uniform_k ? 1 : 0;
    out->row_ptr_bytes = m->rp32 ? 4 : 8;
    out->has_fp32 = m->val32 ? 1 : 0;
    out->band = m->band ? 1 : 0;
    out->gamma = m->gamma;
    out->device_bytes = (int64_t)(m->data_bytes + m->ws.bytes);
    out->has_fp64 = m->val ? 1 : 0;
    out->fp32_row_perturbation = m->val32_dp;
    out->stencil_patterns = m->sten_np;
    out->stencil_pairs = m->sten_pairs ? 1 : 0;
    out->has_split = m->val_lo ? 1 : 0;
    out->split_row_perturbation = m->split_dp;
    return IPI_OK;
    IPI_GUARD_END
}

void ipi_opts_default(ipi_solve_opts* o) {
    if (!o) return;
    o->atol = 1e-8;
    o->rtol_cert = 0.0;
    o->alpha = 1e-4;
    o->max_outer = 1000;
    o->max_inner = 1000;
    o->inner = IPI_INNER_GMRES;
    o->pc = IPI_PC_NONE;
    o->richardson_scale = 1.0;
    o->gmres_restart = 30;
    o->precision = IPI_FP64;
    o->reorth = 1;
    o->mode = IPI_MINCOST;
    o->profile = 0;
    o->v0 = nullptr;
    o->richardson_block = 1;
}

static bool parse_double(const char* s, double* out) {
    if (!s || !*s) return false;
    char* end = nullptr;
    errno = 0;
    double v = std::strtod(s, &end);
    if (errno || !end || *end) return false;
    *out = v;
    return true;
}

static bool parse_int(const char* s, int32_t* out) {
    if (!s || !*s) return false;
    char* end = nullptr;
    errno = 0;
    long v = std::strtol(s, &end, 10);
    if (errno || !end || *end || v < INT32_MIN || v > INT32_MAX) return false;
    *out = (int32_t)v;
    return true;
}

ipi_status ipi_opts_set(ipi_solve_opts* o, const char* name, const char* value) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(o && name && value, IPI_E_INVALID_ARG, "NULL argument");
    std::string n(name);
    while (!n.empty() && n[0] == '-') n.erase(0, 1);
    std::string v(value);
    double d = 0;
    int32_t i = 0;
    auto bad = [&]() { throw Error(IPI_E_INVALID_ARG, "bad value '" + v + "' for option -" + n); };
    if (n == "atol_pi") {
        if (!parse_double(value, &d) || !(d >= 0.0) || !std::isfinite(d)) bad();
        o->atol = d;
    } else if (n == "rtol_cert") {
        if (!parse_double(value, &d) || !(d >= 0.0) || !std::isfinite(d)) bad();
        o->rtol_cert = d;
    } else if (n == "alpha") {
        if (!parse_double(value, &d) || !(d > 0.0 && d < 1.0)) bad();
        o->alpha = d;
    } else if (n == "max_iter_pi") {
        if (!parse_int(value, &i) || i < 1) bad();
        o->max_outer = i;
    } else if (n == "max_iter_ksp" || n == "ksp_max_it") {
        if (!parse_int(value, &i) || i < 1) bad();
        o->max_inner = i;
    } else if (n == "ksp_type") {
        if (v == "gmres") o->inner = IPI_INNER_GMRES;
        else if (v == "richardson") o->inner = IPI_INNER_RICHARDSON;
        else if (v == "tfqmr") o->inner = IPI_INNER_TFQMR;
        else if (v == "bcgs" || v == "bicgstab") o->inner = IPI_INNER_BICGSTAB;
        else bad();
    } else if (n == "pc_type") {
        if (v == "none") o->pc = IPI_PC_NONE;
        else if (v == "jacobi") o->pc = IPI_PC_JACOBI;
        else bad();
    } else if (n == "ksp_richardson_scale") {
        if (!parse_double(value, &d) || !(d > 0.0) || !std::isfinite(d)) bad();
        o->richardson_scale = d;
    } else if (n == "ksp_gmres_restart") {
        if (!parse_int(value, &i) || i < 1 || i > kMaxRestart) bad();
        o->gmres_restart = i;
    } else if (n == "precision") {
        if (v == "fp64" || v == "double") o->precision = IPI_FP64;
        else if (v == "fp32_mixed" || v == "mixed") o->precision = IPI_FP32_MIXED;
        else if (v == "fp32_inner") o->precision = IPI_FP32_INNER;
        else bad();
    } else if (n == "ksp_gmres_cgs_passes") {
        if (!parse_int(value, &i) || i < 1 || i > 2) bad();
        o->reorth = i;
    } else if (n == "mode") {
        if (v == "MINCOST" || v == "mincost") o->mode = IPI_MINCOST;
        else if (v == "MAXREWARD" || v == "maxreward") o->mode = IPI_MAXREWARD;
        else bad();
    } else if (n == "ksp_richardson_block") {
        if (!parse_int(value, &i) || i < 0 || i > 1) bad();
        o->richardson_block = i;
    } else if (n == "profile") {
        if (!parse_int(value, &i) || i < 0 || i > 2) bad();
        o->profile = i;
    } else {
        throw Error(IPI_E_INVALID_ARG, "unknown option -" + n);
    }
    return IPI_OK;
    IPI_GUARD_END
}

ipi_status ipi_bellman(ipi_mdp_t m, const double* V, double* TV, int32_t* pi, double* resid, double* rho,
                       int32_t precision, void* stream) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(m && V && TV && pi, IPI_E_INVALID_ARG, "NULL argument");
    IPI_REQUIRE(precision == IPI_FP64 || precision == IPI_FP32_MIXED, IPI_E_INVALID_ARG, "bad precision");
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(m->mu);
    const bool fp32 = precision == IPI_FP32_MIXED;
    uint64_t* bits = nullptr;
    if (rho) {
        // the MDP keeps one 8-byte slot for the device-wide max
        if (!m->rho_slot) {
            std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
            IPI_HIP(hipMalloc(&m->rho_slot, 16));
        }
        bits = (uint64_t*)m->rho_slot;
        launch_fill_u64(bits, 1, 0, st);
    }
    BellmanOut o{TV, pi, resid, bits, nullptr};
    launch_bellman(m, m->g, V, o, fp32, m->tune.bellman_lanes, m->tune.bellman_spt, st);
    if (rho) launch_rho_to_double(bits, rho, st);
    return IPI_OK;
    IPI_GUARD_END
}

ipi_status ipi_solve(ipi_mdp_t m, const ipi_solve_opts* opts, double* V_out, int32_t* pi_out, ipi_solve_info* info,
                     void* stream) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(m && opts && V_out && pi_out, IPI_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(m->mu);
    return solve_single(m, *opts, V_out, pi_out, info, (hipStream_t)stream);
    IPI_GUARD_END
}

ipi_status ipi_solve_batch(int32_t n, const ipi_mdp_t* mdps, const ipi_solve_opts* opts, double* const* V_out,
                           int32_t* const* pi_out, ipi_solve_info* infos, ipi_status* statuses, void* stream) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(n >= 0, IPI_E_INVALID_ARG, "n must be >= 0");
    if (n == 0) return IPI_OK;
    IPI_REQUIRE(mdps && opts && V_out && pi_out && statuses, IPI_E_INVALID_ARG, "NULL argument");
    for (int i = 0; i < n; ++i) IPI_REQUIRE(mdps[i] && V_out[i] && pi_out[i], IPI_E_INVALID_ARG, "NULL member");
    return solve_batch(n, mdps, opts, V_out, pi_out, infos, statuses, (hipStream_t)stream);
    IPI_GUARD_END
}

ipi_status ipi_get_tuning(ipi_mdp_t m, ipi_tuning* out) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(m && out, IPI_E_INVALID_ARG, "NULL argument");
    out->bellman_lanes = m->tune.bellman_lanes;
    out->bellman_states_per_tile = m->tune.bellman_spt;
    out->spmv_lanes = m->tune.spmv_lanes;
    out->spmv_states_per_tile = m->tune.spmv_spt;
    out->bellman_chunk = m->tune.bellman_chunk;
    out->spmv_chunk = m->tune.spmv_chunk;
    out->spmv_schedule = m->tune.spmv_schedule;
    out->spmv_workgroups = m->tune.spmv_workgroups;
    out->band_rows = m->tune.band_rows;
    out->ppi_cached = m->tune.ppi_cached;
    out->blocked_prefetch = m->tune.blocked_prefetch;
    return IPI_OK;
    IPI_GUARD_END
}

ipi_status ipi_set_tuning(ipi_mdp_t m, const ipi_tuning* t) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(m && t, IPI_E_INVALID_ARG, "NULL argument");
    Tuning n = m->tune;
    n.bellman_lanes = t->bellman_lanes;
    n.bellman_spt = t->bellman_states_per_tile;
    n.spmv_lanes = t->spmv_lanes;
    n.spmv_spt = t->spmv_states_per_tile;
    n.bellman_chunk = t->bellman_chunk;
    n.spmv_chunk = t->spmv_chunk;
    n.spmv_schedule = t->spmv_schedule;
    n.spmv_workgroups = t->spmv_workgroups;
    n.band_rows = t->band_rows;
    n.ppi_cached = t->ppi_cached;
    n.blocked_prefetch = t->blocked_prefetch;
    std::string why;
    IPI_REQUIRE(tuning_admissible(m, n, &why), IPI_E_INVALID_ARG, why);
    m->tune = n;
    return IPI_OK;
    IPI_GUARD_END
}

ipi_status ipi_autotune(ipi_mdp_t m, int32_t precision, const char* cache_path, void* stream) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(m, IPI_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(m->mu);
    return autotune(m, precision == IPI_FP32_MIXED, cache_path, (hipStream_t)stream);
    IPI_GUARD_END
}

int64_t ipi_footprint_bytes(int64_t S, int32_t A, int64_t nnz, int32_t k_max, const ipi_solve_opts* opts) {
    if (S <= 0 || A <= 0 || nnz < 0 || k_max < 0) return -1;
    const bool mixed = opts && opts->precision == IPI_FP32_MIXED;
    const bool inner32 = opts && opts->precision != IPI_FP64;
    const int m = opts ? opts->gmres_restart : 30;
    const double R = (double)S * A;
    const double bp = nnz < ((int64_t)1 << 31) ? 4.0 : 8.0;
    double b = nnz * (8.0 + 4.0) + (R + 1) * bp + 8.0 * R;  // P (f64 values kept) + row_ptr + g
    if (mixed) b += nnz * 4.0;                               // float32 value copy
    b += S * (5 * 8.0 + 4.0 + 8.0);                          // V, TV, b, delta x2, pi, diag
    b += (double)S * k_max * ((inner32 ? 4.0 : 8.0) + 4.0) + 8.0 * (S + 1);  // compact P_pi
    b += 8.0 * (m + 1) * S;                                  // Krylov basis
    if (opts && (opts->inner == IPI_INNER_TFQMR || opts->inner == IPI_INNER_BICGSTAB)) b += 8.0 * 8 * S;
    return (int64_t)b + (1 << 20);
}

}  // extern "C"
