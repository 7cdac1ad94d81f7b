// Plan-free FP64 solve for callers that cannot allocate device memory: the
// tables of a plan (twiddles, eigenvalues, z geometry, interface factors) and
// its workspace (spectrum, partial sums, scalars, flags) are carved out of one
// static device array per GPU, filled on each call from kernel arguments, and
// the solve runs the same passes as psv_solve with the built-in launch shapes.
// Nothing here calls hipMalloc, hipFree, a host allocator or hipMemsetAsync.
#include <algorithm>
#include <mutex>

#include "internal.hpp"
#include "pass_yz.hpp"

namespace psv {
namespace {

constexpr size_t STATIC_BYTES = PSV_STATIC_SCRATCH_BYTES;

// One array per GPU, alive until the process ends. Its name is a host-side
// stand-in: host code uses the per-device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[STATIC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char* g_addr[MAX_DEVICES] = {};

// Device address of the array on the current device, looked up once per
// device (with that device current) and kept.
unsigned char* scratch_address() {
    int dev = 0;
    PSV_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) fail(PSV_ERR_HIP, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void* ptr = nullptr;
        PSV_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) fail(PSV_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_addr[dev] = static_cast<unsigned char*>(ptr);
    }
    return g_addr[dev];
}

// Table values travel as kernel arguments, PUT_N doubles per launch.
constexpr int PUT_N = 256;
struct PutChunk {
    int n;
    double v[PUT_N];
};

__global__ void __launch_bounds__(PUT_N) k_put(double* __restrict__ dst, PutChunk c) {
    if ((int)threadIdx.x < c.n) dst[threadIdx.x] = c.v[threadIdx.x];
}

// Writes n doubles to dst: value(i) for i < n, in launches of PUT_N.
template <typename F>
void put(double* dst, int n, F value, hipStream_t s) {
    PutChunk c;
    for (int i0 = 0; i0 < n; i0 += PUT_N) {
        c.n = std::min(PUT_N, n - i0);
        for (int i = 0; i < c.n; ++i) c.v[i] = value(i0 + i);
        hipLaunchKernelGGL(k_put, dim3(1), dim3(PUT_N), 0, s, dst + i0, c);
    }
    PSV_HIP(hipGetLastError());
}

// Byte offsets of the tables and workspace inside the array (256-byte aligned).
struct Layout {
    size_t twx, twy, lamx, lamy, za, zb, zc, inv_h, inv_g, h, g, vol, inv_vol;
    size_t ifc, spec, partials, scal, flags, total;
};

int static_partials(const Plan& p) { return std::max(8192, 2 * p.ny * p.nz + 64); }

Layout layout(const Plan& p, int kc) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) & ~size_t(255);
        return at;
    };
    const size_t d = sizeof(double);
    L.twx = take(p.nx * sizeof(double2));
    L.twy = take(p.ny * sizeof(double2));
    L.lamx = take(p.mx * d);
    L.lamy = take(p.ny * d);
    L.za = take(p.nz * d);
    L.zb = take(p.nz * d);
    L.zc = take(p.nz * d);
    L.inv_h = take(p.nz * d);
    L.inv_g = take((p.nz + 1) * d);
    L.h = take(p.nz * d);
    L.g = take((p.nz + 1) * d);
    L.vol = take(p.nz * d);
    L.inv_vol = take(p.nz * d);
    L.ifc = take(ifc_table_bytes(p, kc));
    L.spec = take(p.nspec() * sizeof(double2));
    L.partials = take(static_partials(p) * d);
    L.scal = take(S_NSCAL * d);
    L.flags = take(F_NFLAG * sizeof(int));
    L.total = off;
    return L;
}

}  // namespace

void solve_static(const psv_grid& grid, const psv_opts& o, const double* f, const double* rho,
                  double rho0, const double* p_prev, double* p_out, int n_steps, hipStream_t s) {
    if (o.precision != PSV_FP64) fail(PSV_ERR_INVALID_ARG, "the static-scratch solve runs FP64 only");
    if (o.autotune != 0) fail(PSV_ERR_INVALID_ARG, "the static-scratch solve takes autotune = 0");
    if (o.check_inputs != 0) fail(PSV_ERR_INVALID_ARG, "the static-scratch solve takes check_inputs = 0");
    Plan P;
    plan_geometry(P, grid, o);
    // the spectrum alone: rejected before any device work
    if (P.nspec() * sizeof(double2) > STATIC_BYTES)
        fail(PSV_ERR_UNSUPPORTED_SIZE, "grid too large for the static scratch array (64 MiB)");
    const int kc = builtin_shape(P);
    const Layout L = layout(P, kc);
    if (L.total > STATIC_BYTES)
        fail(PSV_ERR_UNSUPPORTED_SIZE, "tables and workspace exceed the static scratch array (64 MiB)");
    unsigned char* base = scratch_address();
    P.lp.kc = kc;
    P.t.twx64 = reinterpret_cast<double2*>(base + L.twx);
    P.t.twy64 = reinterpret_cast<double2*>(base + L.twy);
    P.t.lamx = reinterpret_cast<double*>(base + L.lamx);
    P.t.lamy = reinterpret_cast<double*>(base + L.lamy);
    P.t.za = reinterpret_cast<double*>(base + L.za);
    P.t.zb = reinterpret_cast<double*>(base + L.zb);
    P.t.zc = reinterpret_cast<double*>(base + L.zc);
    P.t.inv_h = reinterpret_cast<double*>(base + L.inv_h);
    P.t.inv_g = reinterpret_cast<double*>(base + L.inv_g);
    P.t.h = reinterpret_cast<double*>(base + L.h);
    P.t.g = reinterpret_cast<double*>(base + L.g);
    P.t.vol = reinterpret_cast<double*>(base + L.vol);
    P.t.inv_vol = reinterpret_cast<double*>(base + L.inv_vol);
    P.ifc_tab = base + L.ifc;
    P.ifc_tab_bytes = ifc_table_bytes(P, kc);
    P.spec = base + L.spec;
    P.partials = reinterpret_cast<double*>(base + L.partials);
    P.n_partials = static_partials(P);
    P.scal = reinterpret_cast<double*>(base + L.scal);
    P.flags = reinterpret_cast<int*>(base + L.flags);

    // tables, from the same per-element expressions as a plan's
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const double dx = P.dx, dy = P.dy;
    put(reinterpret_cast<double*>(P.t.twx64), 2 * nx, [&](int i) {
        double re, im;
        twiddle(i / 2, nx, &re, &im);
        return (i & 1) ? im : re;
    }, s);
    put(reinterpret_cast<double*>(P.t.twy64), 2 * ny, [&](int i) {
        double re, im;
        twiddle(i / 2, ny, &re, &im);
        return (i & 1) ? im : re;
    }, s);
    put(P.t.lamx, P.mx, [&](int m) { return periodic_eigenvalue(m, nx, dx); }, s);
    put(P.t.lamy, ny, [&](int n) { return periodic_eigenvalue(n, ny, dy); }, s);
    const psv_grid& g = grid;
    put(P.t.za, nz, [&](int k) { return z_coef(g, k, dx, dy).a; }, s);
    put(P.t.zb, nz, [&](int k) { return z_coef(g, k, dx, dy).b; }, s);
    put(P.t.zc, nz, [&](int k) { return z_coef(g, k, dx, dy).c; }, s);
    put(P.t.inv_h, nz, [&](int k) { return z_coef(g, k, dx, dy).inv_h; }, s);
    put(P.t.inv_g, nz + 1, [&](int k) { return z_coef(g, k, dx, dy).inv_g; }, s);
    put(P.t.h, nz, [&](int k) { return z_coef(g, k, dx, dy).h; }, s);
    put(P.t.g, nz + 1, [&](int k) { return z_coef(g, k, dx, dy).g; }, s);
    put(P.t.vol, nz, [&](int k) { return z_coef(g, k, dx, dy).vol; }, s);
    put(P.t.inv_vol, nz, [&](int k) { return z_coef(g, k, dx, dy).inv_vol; }, s);
    launch_ifc_table(P, s);
    // the array keeps the previous call's contents: clear the scalars and flags
    launch_fill(P.scal, S_NSCAL, 0.0, s);
    launch_fill(reinterpret_cast<double*>(P.flags), F_NFLAG * sizeof(int) / sizeof(double), 0.0, s);

    // the passes of psv_solve (FP64, no relative residual)
    const bool method1 = o.method == PSV_SPLIT_RHO0;
    FwdArgs a{};
    a.f = f;
    a.rho = rho;
    a.rho0 = P.scal + S_RHO0;
    if (method1) {
        if (rho0 > 0.0)
            launch_set_scalar(P.scal + S_RHO0, rho0, s);
        else
            launch_min_reduce(P, rho, P.scal + S_RHO0, P.flags + F_ARGMIN, s);
        if (!p_prev) {
            launch_fill(p_out, P.ncell(), 0.0, s);
            p_prev = p_out;
        }
    }
    a.mode = method1 ? FWD_METHOD1 : FWD_CONST;
    const double inv_scale = 2.0 / ((double)nx * ny);
    for (int step = 0; step < n_steps; ++step) {
        a.pprev = (step == 0) ? p_prev : p_out;
        launch_fwd_x(P, false, a, s);
        launch_z_solve(P, false, P.scal + S_RHS_MEAN, nullptr, s);
        launch_inv_x(P, false, INV_STORE, p_out, inv_scale, nullptr, s);
    }
}

}  // namespace psv
