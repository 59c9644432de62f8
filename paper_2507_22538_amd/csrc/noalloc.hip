// ipi_solve_noalloc: the solve of ipi_solve with its workspace (iterate
// vectors, Krylov basis, compact P_pi, control block, reduction partials)
// placed in one fixed device array instead of memory from hipMalloc.  For
// callers that cannot allocate (tight serving loops, harnesses that forbid
// allocation).  The kernels are ipi_solve's; only where their buffers live
// differs, and GMRES cycles are launched one by one instead of replayed from
// a captured graph (the same launches, so the same bits).
#include <chrono>
#include <mutex>

#include "internal.hpp"

using namespace ipi;

namespace {

// 64 MiB of device memory, held by every GPU the library runs on until the
// process ends.  Host code must not pass the array's name to a kernel or a
// copy: on the host it is a stand-in symbol, not a device address.  The
// address on each device comes from hipGetSymbolAddress (scratch_base).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static_assert(sizeof(Ctrl) % 8 == 0, "the control block is cleared in 8-byte words");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;             // serialises the calls (they share the array)
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` on each device

// The array's address on the current device, looked up once per device.
// Called with g_scratch_mu held.
void* scratch_base(int dev) {
    IPI_REQUIRE(dev >= 0 && dev < kMaxDevices, IPI_E_DEVICE, "device index out of range");
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        IPI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        IPI_REQUIRE(p != nullptr, IPI_E_DEVICE, "scratch array has no device address");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

// Bump allocation of 256-byte aligned buffers from [base, base + cap);
// with base == nullptr only the total is computed.
struct Bump {
    unsigned char* base;
    size_t off = 0;
    void* operator()(size_t bytes) {
        off = (off + 255) & ~size_t(255);
        void* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

size_t plan(const ipi_mdp_s* m, const ipi_solve_opts& o, int cus, unsigned char* base, Workspace& w) {
    const bool fp32 = o.precision != IPI_FP64;  // float32 P_pi
    const int restart = o.inner == IPI_INNER_GMRES ? o.gmres_restart : 1;
    const int naux = o.inner == IPI_INNER_BICGSTAB ? 6 : (o.inner == IPI_INNER_TFQMR ? 8 : 0);
    Bump bump{base};
    workspace_layout(m, restart, naux, fp32, cus, w, bump);
    w.g_neg = o.mode == IPI_MAXREWARD ? (double*)bump((size_t)m->S * m->A * sizeof(double)) : nullptr;
    return bump.off;
}

// puts the MDP's own workspace back when the call ends, however it ends
struct SwapBack {
    ipi_mdp_s* m;
    Workspace saved;
    ~SwapBack() { m->ws = saved; }
};

}  // namespace

extern "C" ipi_status ipi_solve_noalloc(ipi_mdp_t m, const ipi_solve_opts* opts, double* V_out, int32_t* pi_out,
                                        ipi_solve_info* info, void* stream) {
    try {
        IPI_REQUIRE(m && opts && V_out && pi_out, IPI_E_INVALID_ARG, "NULL argument");
        IPI_REQUIRE(opts->precision == IPI_FP64 || opts->precision == IPI_FP32_MIXED ||
                        opts->precision == IPI_FP32_INNER,
                    IPI_E_INVALID_ARG, "bad precision");
        IPI_REQUIRE(opts->gmres_restart >= 1 && opts->gmres_restart <= kMaxRestart, IPI_E_INVALID_ARG,
                    "gmres restart must lie in [1, 64]");
        int dev = 0;
        IPI_HIP(hipGetDevice(&dev));
        IPI_REQUIRE(dev == m->device, IPI_E_INVALID_ARG, "the MDP lives on another device than the current one");
        Workspace probe;
        const size_t need = plan(m, *opts, m->arch_cus > 0 ? m->arch_cus : device_cus(), nullptr, probe);
        if (need > kScratchBytes) {
            throw Error(IPI_E_TOO_LARGE, "ipi_solve_noalloc: this MDP and these options need " +
                                             std::to_string(need) + " bytes of workspace; the fixed array holds " +
                                             std::to_string(kScratchBytes));
        }
        std::lock_guard<std::mutex> lk_scratch(g_scratch_mu);
        std::lock_guard<std::mutex> lk(m->mu);
        unsigned char* base = static_cast<unsigned char*>(scratch_base(dev));
        hipStream_t st = (hipStream_t)stream;
        SwapBack keep{m, m->ws};
        Workspace w;
        plan(m, *opts, m->arch_cus > 0 ? m->arch_cus : device_cus(), base, w);
        // the array keeps the previous call's contents: clear what the solve
        // expects to start at zero (with a fill kernel, no memset)
        launch_fill_u64(reinterpret_cast<uint64_t*>(w.ctrl), (int64_t)(sizeof(Ctrl) / 8), 0, st);
        launch_fill_u64(reinterpret_cast<uint64_t*>(w.small), 8192, 0, st);
        m->ws = w;
        ipi_status s = solve_single(m, *opts, V_out, pi_out, info, st, /*noalloc=*/true);
        if (s == IPI_OK) set_last_error("");
        return s;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.status;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return IPI_E_DEVICE;
    }
}
