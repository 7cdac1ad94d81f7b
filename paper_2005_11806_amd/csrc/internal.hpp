// Host-side internals of libpsv: the plan, launch parameters and the kernel
// launchers implemented in the .hip translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "psv.h"
#include "device_common.hpp"

namespace psv {

// Error carrying a psv_status; caught at the C-ABI boundary.
struct Error {
    psv_status status;
    std::string msg;
};

[[noreturn]] void fail(psv_status s, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define PSV_HIP(call) ::psv::hip_check((call), #call)

// LDS a block may take on gfx950 (160 KiB), less room for static arrays
constexpr int LDS_MAX_BLOCK = 152 * 1024;

// Lets `kernel` take more than 64 KiB of dynamic LDS; a no-op below that.
template <typename K>
void allow_lds(K kernel, size_t bytes) {
    if (bytes > 65536)
        hip_check(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes),
                  "hipFuncSetAttribute");
}

// Radix sequence of a 2^a 3^b length (8s, then 4 / 2, then 3s).
Radices make_radices(int n);

// Assembly modes of the forward x pass.
enum FwdMode : int {
    FWD_CONST = 0,    // r = f * scale[k] (scale may be null)
    FWD_METHOD1 = 1,  // r = rho0 f + D((1 - rho0/rho_f) G p_prev)
    FWD_RESID = 2,    // r = r_in - mean - L p (refinement residual), norm partials
    FWD_METHOD3 = 3   // r = rho (f - D(rho_f^-1 G p)) (Method III correction; p may be
                      // null, read as 0), partials of sum |f - D(rho_f^-1 G p)|
};
// Store modes of the inverse x pass.
enum InvMode : int {
    INV_STORE = 0,  // p = x
    INV_ADD = 1,    // p += x
    INV_SCALE = 2   // p = x * vol[k]
};

// Device-resident scalars of a plan (offsets into Plan::scal).
enum Scalar : int {
    S_RHO0 = 0,
    S_RHS_MEAN = 1,
    S_RES2 = 2,
    S_R2 = 3,
    S_RELRES = 4,
    S_GRAD_RHO0 = 5,
    S_MEAN2 = 6,       // mean removed by a refinement solve (discarded)
    S_EPS = 7,         // Method III: sum |f - D(rho_f^-1 G p)| of the current iterate
    S_EPS0 = 8,        // Method III: the same for p = 0 (u = u*)
    S_FMEAN = 9,       // converged solve: volume-weighted mean of the right-hand side
    S_UNIT = 10,       // the constant 1 (weight of the implicit adjoint's face products)
    S_RHOMAX = 11,     // max rho (Method II weight)
    S_OMEGA = 12,      // Method II weight: harmonic mean of min rho and max rho
    S_HIST = 16,       // mixed refinement: relres after the FP32 solve and after each sweep
    S_NHIST = PSV_RELRES_HISTORY,
    S_NSCAL = 32
};
enum Flag : int { F_DONE = 0, F_ARGMIN = 1, F_STEPS = 2, F_CONV = 3, F_NFLAG = 8 };

struct DevTables {
    // twiddles exp(-2 pi i t / n)
    double2* twx64 = nullptr;
    float2* twx32 = nullptr;
    double2* twy64 = nullptr;
    float2* twy32 = nullptr;
    double* lamx = nullptr;  // [mx]
    double* lamy = nullptr;  // [ny]
    double* za = nullptr;    // [nz] tridiagonal sub-diagonal
    double* zb = nullptr;    // [nz] diagonal
    double* zc = nullptr;    // [nz] super-diagonal
    double* inv_h = nullptr; // [nz]
    double* inv_g = nullptr; // [nz+1], face k between cells k-1 and k (walls: 0)
    double* h = nullptr;     // [nz]
    double* g = nullptr;     // [nz+1] centre gaps (g[0] = g[nz] = 0)
    double* vol = nullptr;   // [nz]
    double* inv_vol = nullptr;
};

struct Launch {
    int lbx = 8;      // lines per block, forward x pass (and both x passes of batches)
    int kc = 8;       // planes per y tile = rows per chunk of the z partition
    int lbx_inv = 8;  // lines per block, inverse x pass of a plan
    int xstage = 1;   // forward x pass of a plan: stencil rows staged in LDS (1) or read directly (0)
    int xorder = 1;   // forward x pass of a plan: tiles in line windows (1) or plane ranges (0) per XCD
};

// Launch-shape autotuning (autotune.cpp): times candidate shapes per pass on
// synthetic data in the plan's workspace, checks the tuned solve against the
// default shapes, and caches the choice per (arch, grid, precision, method).
struct Plan;
void autotune_plan(Plan& p);

// Optional per-kernel timing: a pair of hipEvents around every launch on the
// launch stream, summed per kernel name when the summary is read.
struct TraceRec {
    const char* name;
    hipEvent_t a, b;
};
struct Trace {
    bool on = false;
    std::vector<TraceRec> recs;
    std::vector<hipEvent_t> pool;
    size_t next = 0;
    hipEvent_t get();
    void release_all();
};

struct Plan;
class TraceScope {
public:
    TraceScope(const Plan& p, const char* name, hipStream_t s);
    ~TraceScope();
    TraceScope(const TraceScope&) = delete;
    TraceScope& operator=(const TraceScope&) = delete;

private:
    Trace* t_;
    hipStream_t s_;
    size_t idx_;
};

struct Plan {
    mutable Trace trace;
    psv_grid grid{};
    psv_opts opts{};
    int nx = 0, ny = 0, nz = 0, mx = 0;
    double dx = 0, dy = 0;
    std::vector<double> zf, h, zcen, g;
    Radices rad_xh{}, rad_y{};  // complex half-length x, full y
    DevTables t;
    Launch lp;
    int device = 0;
    // workspace
    void* spec = nullptr;      // spectrum [nz][mx][ny] complex, FP64 or FP32
    void* ifc_tab = nullptr;   // interface factors of the z partition (plan's precision)
    size_t ifc_tab_bytes = 0;
    double* r_ws = nullptr;    // FP64 right-hand side [N]
    double* partials = nullptr;
    int n_partials = 0;
    double* scal = nullptr;    // [S_NSCAL]
    int* flags = nullptr;      // [F_NFLAG]
    double* host_scal = nullptr;  // pinned mirror
    int* host_flags = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = true;
    size_t ncell() const { return (size_t)nx * ny * nz; }
    size_t nspec() const { return (size_t)mx * ny * nz; }
};

// Builds host tables and uploads them; allocates workspace when alloc_ws.
void plan_init(Plan& p, const psv_grid& g, const psv_opts& o, bool alloc_ws);
void plan_free(Plan& p);
// Sizes, spacings and radix sequences of a plan (no device access).
void plan_geometry(Plan& p, const psv_grid& g, const psv_opts& o);
// Built-in launch shapes on the current device (sets p.device and p.lp
// except kc, which it returns).
int builtin_shape(Plan& p);

// Table entries, one at a time (the plan and the plan-free solve evaluate
// the same expressions): FFT twiddle exp(-2 pi i t / n), eigenvalue
// -4 sin^2(pi m / n) / d^2 of the periodic second difference, z face k, and
// the z geometry and wall-normal operator at index k (g and inv_g are face
// arrays of nz + 1 entries; the other fields are zero at k = nz).
void twiddle(int t, int n, double* re, double* im);
double periodic_eigenvalue(int m, int n, double d);
double grid_face(const psv_grid& g, int k);
struct ZCoef {
    double h, g, a, b, c, inv_h, inv_g, vol, inv_vol;
};
ZCoef z_coef(const psv_grid& g, int k, double dx, double dy);

// ---- launchers (kernels in *.hip) ----
struct FwdArgs {
    int mode;
    const double* f;
    const double* rho;
    const double* pprev;  // METHOD1: previous pressure; RESID: current p
    const double* r_in;   // RESID: stored RHS
    const double* scale;  // CONST, METHOD3: per-k scale of f, or null
    double* r_out;        // optional: store the assembled RHS
    const double* rho0;   // device scalar; METHOD3: constant weight instead of rho (or null)
    const double* mean;   // RESID, METHOD3: device scalar removed from r (or f); METHOD3 may pass null
    double* partials;     // RESID: 2 per block
    double* partials_abs; // METHOD3: sum |f - D(rho_f^-1 G p)| per block
    const int* done;      // skip when *done != 0 (may be null)
    int max_blocks;       // > 0: at most this many blocks (FP32 RESID only)
};
void launch_fwd_x(const Plan& p, bool fp32, const FwdArgs& a, hipStream_t s);
// y passes with the chunk elimination (forward) or back substitution
// (inverse) of the z solve, the interface pass between them, and the three
// in order; mean_out receives the volume-weighted mean of the RHS.
void launch_yz(const Plan& p, bool fp32, bool inverse, const int* done, hipStream_t s);
void launch_interface(const Plan& p, bool fp32, double* mean_out, const int* done, hipStream_t s);
void launch_z_solve(const Plan& p, bool fp32, double* mean_out, const int* done, hipStream_t s);
// Chunk rows of the z partition: whether kc fits, and setting it (recomputes
// the interface factor table, synchronising).
bool kc_fits(const Plan& p, int kc);
void plan_set_kc(Plan& p, int kc);
// Bytes of the interface factor table at chunk rows kc, and the kernel that
// fills p.ifc_tab for p.lp.kc on stream s.
size_t ifc_table_bytes(const Plan& p, int kc);
void launch_ifc_table(const Plan& p, hipStream_t s);
// max_blocks > 0 (honoured by the FP32 INV_ADD pass): at most that many
// blocks (a multiple of 8), each looping over tiles, for launches that
// usually find *done set and return (a full grid still dispatches every
// block)
void launch_inv_x(const Plan& p, bool fp32, int mode, double* out, double scale_all,
                  const int* done, hipStream_t s, int max_blocks = 0);

// Method II weight 2 a b / (a + b) of a = min rho, b = max rho into scal[S_OMEGA]
// (also leaves them in scal[S_RHO0] and scal[S_RHOMAX]).
void launch_harmonic_weight(const Plan& p, const double* rho, hipStream_t s);
void launch_min_reduce(const Plan& p, const double* x, double* out_scalar, int* argmin_out,
                       hipStream_t s);
void launch_norm_finalize(const Plan& p, int nblocks, double tol, hipStream_t s);
// Mixed refinement on the device: reset clears flags[F_DONE], F_STEPS, F_CONV
// and the relres history; check (skipped once F_DONE is set) turns the
// residual pass's partials into relres, records it as history entry `sweep`,
// and sets F_DONE and F_CONV when relres <= tol, F_DONE alone when sweep ==
// max_refine or relres is not finite, else counts a sweep in F_STEPS.
void launch_refine_reset(const Plan& p, hipStream_t s);
void launch_refine_check(const Plan& p, int nblocks, int sweep, int max_refine, double tol,
                         hipStream_t s);
void launch_residual(const Plan& p, const double* r, const double* p_sol, const double* mean,
                     hipStream_t s);
// Blocks of the forward x pass (also the number of per-block partial sums it writes).
int fwd_x_blocks(const Plan& p);
void launch_set_scalar(double* dst, double v, hipStream_t s);
void launch_density(const Plan& p, const double* phi, const double* rg, double rl, double* out,
                    hipStream_t s);
void launch_divergence(const Plan& p, const double* ux, const double* uy, const double* uz,
                       double* out, hipStream_t s);
// out = scale (D u - target); target may be null
void launch_divergence_rhs(const Plan& p, const double* ux, const double* uy, const double* uz,
                           const double* target, double scale, double* out, hipStream_t s);
// Method III correction u = u* - dt rho_f^-1 G p on the faces
void launch_correct_velocity(const Plan& p, const double* ux, const double* uy, const double* uz,
                             const double* pr, const double* rho, double dt, double* ox,
                             double* oy, double* oz, hipStream_t s);
// out = sum of partials[0 .. nblocks)
void launch_sum_partials(const Plan& p, const double* partials, int nblocks, double* out,
                         hipStream_t s);
// Method III loop control on the device: clear the loop flags; after each
// forward pass, eps = dt * sum(partials) goes to S_EPS (S_EPS0 without a
// pressure iterate); flags[F_DONE] is set once eps <= eps_t (F_CONV too) or
// once max_iter solves were launched, else flags[F_STEPS] counts the solve
// that follows. Nothing changes once F_DONE is set.
void launch_m3_reset(const Plan& p, hipStream_t s);
void launch_m3_check(const Plan& p, const double* partials, int nblocks, double dt, double eps_t,
                     bool has_p, int max_iter, hipStream_t s);
void launch_adjoint_faces(const Plan& p, const double* x, const double* f, const double* rho,
                          const double* pprev, const double* rho0, double* grad_f,
                          double* grad_rho, double* grad_p, double* partials, hipStream_t s);
void launch_adjoint_finalize(const Plan& p, int nblocks, double* grad_rho, int add_argmin,
                             hipStream_t s);
int adjoint_blocks(const Plan& p);
void launch_scale_vol(const Plan& p, const double* x, double* out, hipStream_t s);
// volume-weighted mean of r (times the per-k scale, if given)
void launch_vmean(const Plan& p, const double* r, double* out_scalar, hipStream_t s,
                  const double* scale = nullptr);
void launch_fill(double* x, size_t n, double v, hipStream_t s);
// volume-weighted mean from the forward pass's per-block sums of vol * r
void launch_mean_finalize(const Plan& p, int nblocks, double* out_scalar, hipStream_t s);
void launch_scan_inputs(const Plan& p, const double* x, int positive, int* bad, hipStream_t s);

}  // namespace psv
