// Plan construction: grid validation, FP64 host tables (z geometry and the
// wall-normal tridiagonal coefficients, eigenvalues of the periodic second
// differences, FFT twiddles) and the device workspace.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>

#include "pass_x.hpp"
#include "pass_yz.hpp"

namespace psv {

[[noreturn]] void fail(psv_status s, const std::string& msg) { throw Error{s, msg}; }

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        std::ostringstream os;
        os << what << ": " << hipGetErrorString(e);
        fail(e == hipErrorOutOfMemory ? PSV_ERR_OOM : PSV_ERR_HIP, os.str());
    }
}

static bool is_23_smooth(int n) {
    if (n <= 0) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

Radices make_radices(int n) {
    Radices r{};
    r.n = n;
    int a = 0, b = 0, m = n;
    while (m % 2 == 0) { m /= 2; ++a; }
    while (m % 3 == 0) { m /= 3; ++b; }
    while (a >= 3) { r.r[r.count++] = 8; a -= 3; }
    if (a == 2) r.r[r.count++] = 4;
    if (a == 1) r.r[r.count++] = 2;
    while (b-- > 0) r.r[r.count++] = 3;
    return r;
}

// Host-side checks of a grid; no device access.
void validate_grid(const psv_grid* g) {
    if (!g) fail(PSV_ERR_INVALID_ARG, "grid is NULL");
    if (g->bc_z != PSV_BC_WALL_NEUMANN) fail(PSV_ERR_INVALID_ARG, "unknown z boundary condition");
    if (g->nz < 2) fail(PSV_ERR_INVALID_ARG, "nz must be >= 2");
    if (g->nz > 2048) fail(PSV_ERR_UNSUPPORTED_SIZE, "nz must be <= 2048");
    // ny = 1 is a two-dimensional x-z problem (one periodic cell in y: no y fluxes)
    auto size_ok = [](int n) { return n >= 4 && n <= 1024 && !(n & 1) && is_23_smooth(n); };
    if (!size_ok(g->nx) || !(g->ny == 1 || size_ok(g->ny)))
        fail(PSV_ERR_UNSUPPORTED_SIZE,
             "nx and ny must be even, of the form 2^a 3^b, in [4, 1024] (or ny = 1)");
    if (!(g->lx > 0) || !(g->ly > 0) || !(g->lz > 0) || !std::isfinite(g->lx) ||
        !std::isfinite(g->ly) || !std::isfinite(g->lz))
        fail(PSV_ERR_INVALID_ARG, "domain lengths must be positive and finite");
    const double ncell = (double)g->nx * g->ny * g->nz;
    if (ncell >= 2147483647.0) fail(PSV_ERR_UNSUPPORTED_SIZE, "nx*ny*nz must be < 2^31");
    if (g->zf) {
        if (g->zf[0] != 0.0) fail(PSV_ERR_INVALID_ARG, "zf[0] must be 0");
        if (std::fabs(g->zf[g->nz] - g->lz) > 1e-12 * g->lz) fail(PSV_ERR_INVALID_ARG, "zf[nz] must equal lz");
        for (int k = 0; k < g->nz; ++k) {
            if (!(g->zf[k + 1] > g->zf[k]) || !std::isfinite(g->zf[k + 1]))
                fail(PSV_ERR_INVALID_ARG, "zf must be finite and strictly increasing");
        }
    }
}

void validate_opts(const psv_opts* o) {
    if (!o) return;
    if (o->precision != PSV_FP64 && o->precision != PSV_MIXED) fail(PSV_ERR_INVALID_ARG, "bad precision");
    if (o->method != PSV_CONST && o->method != PSV_SPLIT_RHO0) fail(PSV_ERR_INVALID_ARG, "bad method");
    if (o->max_refine > 64) fail(PSV_ERR_INVALID_ARG, "max_refine must be <= 64");
    if (!(o->tol >= 0.0) && !(o->tol < 0.0)) fail(PSV_ERR_INVALID_ARG, "tol is NaN");
    if (o->check_inputs != 0 && o->check_inputs != 1) fail(PSV_ERR_INVALID_ARG, "check_inputs must be 0 or 1");
    if (o->autotune < 0 || o->autotune > 2) fail(PSV_ERR_INVALID_ARG, "autotune must be 0..2");
    if (o->batch_executor < 0 || o->batch_executor > 2)
        fail(PSV_ERR_INVALID_ARG, "batch_executor must be 0..2");
    if (o->chunk_rows != 0 && o->chunk_rows != 4 && o->chunk_rows != 8 && o->chunk_rows != 16)
        fail(PSV_ERR_INVALID_ARG, "chunk_rows must be 0, 4, 8 or 16");
    if (o->x_stencil < 0 || o->x_stencil > 2) fail(PSV_ERR_INVALID_ARG, "x_stencil must be 0..2");
}

void default_opts(psv_opts* o) {
    std::memset(o, 0, sizeof(*o));
    o->precision = PSV_FP64;
    o->method = PSV_SPLIT_RHO0;
    o->tol = 1e-10;
    o->max_refine = 4;
    o->check_inputs = 0;
    o->autotune = 0;
    o->batch_executor = 0;
    o->chunk_rows = 0;
    o->x_stencil = 0;
}

// ---- per-element tables: plan_init and the plan-free solve evaluate the
// same expressions, so both hold the same bits.

// exp(-2 pi i t / n): cosl/sinl of the angle in extended precision, rounded
// to double, with exact values on the four axes.
void twiddle(int t, int n, double* re, double* im) {
    if ((4 * t) % n == 0) {
        const int q = (4 * t) / n;
        *re = (q == 0) ? 1.0 : (q == 2 ? -1.0 : 0.0);
        *im = (q == 1) ? -1.0 : (q == 3 ? 1.0 : 0.0);
        return;
    }
    const long double two_pi = 6.283185307179586476925286766559005768L;
    const long double a = two_pi * (long double)t / (long double)n;
    *re = (double)cosl(a);
    *im = (double)-sinl(a);
}

// eigenvalue of the periodic second difference: -4 sin^2(pi m / n) / d^2
double periodic_eigenvalue(int m, int n, double d) {
    const long double pi_l = 3.141592653589793238462643383279502884L;
    const long double s = sinl(pi_l * m / n);
    return (double)(-4.0L * s * s / ((long double)d * d));
}

// z face k (0 .. nz): the caller's positions, or uniform spacing lz / nz
double grid_face(const psv_grid& g, int k) {
    if (k <= 0) return 0.0;
    if (k >= g.nz) return g.lz;
    return g.zf ? g.zf[k] : g.lz * (double)k / g.nz;
}

static double cell_centre(const psv_grid& g, int k) {
    return 0.5 * (grid_face(g, k) + grid_face(g, k + 1));
}

// z geometry and wall-normal operator at index k (cell k for k < nz; the
// face arrays g and inv_g run to k = nz): a_k x_{k-1} + b_k x_k + c_k x_{k+1}
// is the flux-form second difference with zero flux through both walls.
ZCoef z_coef(const psv_grid& g, int k, double dx, double dy) {
    ZCoef z{};
    const int nz = g.nz;
    if (k >= 1 && k <= nz - 1) {
        z.g = cell_centre(g, k) - cell_centre(g, k - 1);
        z.inv_g = 1.0 / z.g;
    }
    if (k >= nz) return z;
    z.h = grid_face(g, k + 1) - grid_face(g, k);
    if (k > 0) z.a = 1.0 / (z.h * z.g);
    if (k + 1 < nz) z.c = 1.0 / (z.h * (cell_centre(g, k + 1) - cell_centre(g, k)));
    z.b = -(z.a + z.c);
    z.inv_h = 1.0 / z.h;
    z.vol = dx * dy * z.h;
    z.inv_vol = 1.0 / z.vol;
    return z;
}

template <typename T>
static T* upload(const std::vector<T>& v) {
    T* d = nullptr;
    PSV_HIP(hipMalloc(&d, v.size() * sizeof(T)));
    PSV_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
}

void plan_geometry(Plan& p, const psv_grid& g, const psv_opts& o) {
    p.grid = g;
    p.grid.zf = nullptr;  // the caller's array is not retained
    p.opts = o;
    if (p.opts.tol <= 0.0) p.opts.tol = 1e-10;
    if (p.opts.max_refine <= 0) p.opts.max_refine = 4;
    p.nx = g.nx;
    p.ny = g.ny;
    p.nz = g.nz;
    p.mx = g.nx / 2 + 1;
    p.dx = g.lx / g.nx;
    p.dy = g.ly / g.ny;
    p.rad_xh = make_radices(p.nx / 2);
    p.rad_y = make_radices(p.ny);
}

// Built-in launch shapes of the current device: x lines per block bounded by
// the LDS a block may take (FP64 worst case, leaving 2 KiB for static shared
// arrays), the caller's stencil variant, and the chunk rows of the z
// partition (returned, not yet set): the largest of 16, 8, 4 whose y tile
// takes at most 48 KiB of LDS (three blocks per CU), else the largest that
// fits a block at all.
int builtin_shape(Plan& p) {
    PSV_HIP(hipGetDevice(&p.device));
    int lds_max = 0;
    PSV_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p.device));
    const size_t budget = (size_t)std::min(lds_max, 64 * 1024) - 2048;
    p.lp.lbx = 1;
    while (p.lp.lbx * 2 <= 16 && p.ny % (p.lp.lbx * 2) == 0 && x_lds_max(p.nx, p.lp.lbx * 2) <= budget)
        p.lp.lbx *= 2;
    // one line per block may take up to the whole LDS (nx = 1024)
    if (x_lds_max(p.nx, p.lp.lbx) > (size_t)std::min(lds_max, LDS_MAX_BLOCK))
        fail(PSV_ERR_UNSUPPORTED_SIZE, "line length exceeds the LDS budget");
    p.lp.lbx_inv = p.lp.lbx;
    p.lp.xstage = p.opts.x_stencil == 2 ? 0 : 1;
    const size_t csz = p.opts.precision == PSV_MIXED ? sizeof(float2) : sizeof(double2);
    int kc = p.opts.chunk_rows;
    if (kc && !kc_fits(p, kc))
        fail(PSV_ERR_UNSUPPORTED_SIZE, "the y tile of chunk_rows planes exceeds the LDS of a block");
    for (int c : {16, 8, 4})
        if (!kc && yz_lds(p.ny, c, csz) <= 48 * 1024) kc = c;
    if (!kc)
        for (int c : {16, 8, 4})
            if (!kc && kc_fits(p, c)) kc = c;
    if (!kc) fail(PSV_ERR_UNSUPPORTED_SIZE, "y lines exceed the LDS of a block");
    return kc;
}

void plan_init(Plan& p, const psv_grid& g, const psv_opts& o, bool alloc_ws) {
    plan_geometry(p, g, o);
    const int nz = g.nz;
    p.zf.resize(nz + 1);
    for (int k = 0; k <= nz; ++k) p.zf[k] = grid_face(g, k);
    p.h.resize(nz);
    p.zcen.resize(nz);
    p.g.assign(nz + 1, 0.0);
    std::vector<double> a(nz), b(nz), c(nz), inv_h(nz), inv_g(nz + 1), vol(nz), inv_vol(nz);
    for (int k = 0; k <= nz; ++k) {
        const ZCoef z = z_coef(g, k, p.dx, p.dy);
        p.g[k] = z.g;
        inv_g[k] = z.inv_g;
        if (k == nz) break;
        p.h[k] = z.h;
        p.zcen[k] = cell_centre(g, k);
        a[k] = z.a;
        b[k] = z.b;
        c[k] = z.c;
        inv_h[k] = z.inv_h;
        vol[k] = z.vol;
        inv_vol[k] = z.inv_vol;
    }
    std::vector<double> lamx(p.mx), lamy(p.ny);
    for (int m = 0; m < p.mx; ++m) lamx[m] = periodic_eigenvalue(m, p.nx, p.dx);
    for (int n = 0; n < p.ny; ++n) lamy[n] = periodic_eigenvalue(n, p.ny, p.dy);
    std::vector<double2> tx64(p.nx), ty64(p.ny);
    std::vector<float2> tx32(p.nx), ty32(p.ny);
    for (int t = 0; t < p.nx; ++t) {
        twiddle(t, p.nx, &tx64[t].x, &tx64[t].y);
        tx32[t] = float2{(float)tx64[t].x, (float)tx64[t].y};
    }
    for (int t = 0; t < p.ny; ++t) {
        twiddle(t, p.ny, &ty64[t].x, &ty64[t].y);
        ty32[t] = float2{(float)ty64[t].x, (float)ty64[t].y};
    }
    const int kc = builtin_shape(p);
    p.t.twx64 = upload(tx64);
    p.t.twx32 = upload(tx32);
    p.t.twy64 = upload(ty64);
    p.t.twy32 = upload(ty32);
    p.t.lamx = upload(lamx);
    p.t.lamy = upload(lamy);
    p.t.za = upload(a);
    p.t.zb = upload(b);
    p.t.zc = upload(c);
    p.t.inv_h = upload(inv_h);
    p.t.inv_g = upload(inv_g);
    p.t.h = upload(p.h);
    p.t.g = upload(p.g);
    p.t.vol = upload(vol);
    p.t.inv_vol = upload(inv_vol);
    plan_set_kc(p, kc);
    // per-block partial sums: 2 per forward-x block, or the reductions' 1.5 * 1024
    // two per forward-x block at any lines-per-block (the autotuner may pick 1)
    p.n_partials = std::max(8192, 2 * p.ny * p.nz + 64);
    PSV_HIP(hipMalloc(&p.partials, p.n_partials * sizeof(double)));
    PSV_HIP(hipMalloc(&p.scal, S_NSCAL * sizeof(double)));
    PSV_HIP(hipMalloc(&p.flags, F_NFLAG * sizeof(int)));
    PSV_HIP(hipMemset(p.scal, 0, S_NSCAL * sizeof(double)));
    PSV_HIP(hipMemset(p.flags, 0, F_NFLAG * sizeof(int)));
    PSV_HIP(hipHostMalloc(&p.host_scal, S_NSCAL * sizeof(double)));
    PSV_HIP(hipHostMalloc(&p.host_flags, F_NFLAG * sizeof(int)));
    const size_t nspec = p.nspec(), ncell = p.ncell();
    p.ws_bytes = nspec * sizeof(double2) + 2 * ncell * sizeof(double);
    if (alloc_ws) {
        PSV_HIP(hipMalloc(&p.spec, nspec * sizeof(double2)));
        PSV_HIP(hipMalloc(&p.r_ws, 2 * ncell * sizeof(double)));
        p.own_ws = true;
        if (p.opts.autotune >= 1) autotune_plan(p);
    }
}

void plan_free(Plan& p) {
    void* ptrs[] = {p.t.twx64, p.t.twx32, p.t.twy64, p.t.twy32, p.t.lamx, p.t.lamy, p.t.za,
                    p.t.zb, p.t.zc, p.t.inv_h, p.t.inv_g, p.t.h, p.t.g, p.t.vol, p.t.inv_vol,
                    p.partials, p.scal, p.flags, p.ifc_tab};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (p.own_ws) {
        if (p.spec) (void)hipFree(p.spec);
        if (p.r_ws) (void)hipFree(p.r_ws);
    }
    if (p.host_scal) (void)hipHostFree(p.host_scal);
    if (p.host_flags) (void)hipHostFree(p.host_flags);
    p = Plan{};
}

}  // namespace psv
