// C-ABI entry points of libpsv (declared in include/psv.h). Every entry point
// validates on the host first, then enqueues the kernel sequence of the
// eigenexpansion solve on the caller's stream. Exceptions never cross the ABI.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <initializer_list>
#include <string>

#include "internal.hpp"
#include "pass_x.hpp"

namespace psv {
void validate_grid(const psv_grid* g);
void validate_opts(const psv_opts* o);
void default_opts(psv_opts* o);
std::string trace_summary(Plan& p);
void trace_free(Plan& p);
psv_batch* batch_new();
void batch_delete(psv_batch* b);
void batch_create(psv_batch& B, int n, const psv_grid* grids, const psv_opts& o);
int batch_size(const psv_batch& B);
int batch_method(const psv_batch& B);
bool batch_fp32(const psv_batch& B);
void batch_set_io(psv_batch& B, int p, const double* f, const double* rho, const double* pprev,
                  double* pout, double rho0, bool want_r);
void batch_solve(psv_batch& B, hipStream_t s, bool check);
bool batch_infos(psv_batch& B, hipStream_t s, psv_info* infos);
void solve_static(const psv_grid& grid, const psv_opts& o, const double* f, const double* rho,
                  double rho0, const double* p_prev, double* p_out, int n_steps, hipStream_t s);
}  // namespace psv

struct psv_plan {
    psv::Plan p;
};

namespace {

thread_local std::string g_last_error;

psv_status ok() { return PSV_OK; }

psv_status record(psv_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

template <typename F>
psv_status guarded(F&& fn) {
    try {
        fn();
        return ok();
    } catch (const psv::Error& e) {
        return record(e.status, e.msg);
    } catch (const std::bad_alloc&) {
        return record(PSV_ERR_OOM, "host allocation failed");
    } catch (...) {
        return record(PSV_ERR_HIP, "unexpected internal error");
    }
}

void need(bool cond, const char* msg) {
    if (!cond) psv::fail(PSV_ERR_INVALID_ARG, msg);
}

// The passes read and write fields as pairs of doubles (16-byte accesses).
void need_aligned(std::initializer_list<const void*> ptrs) {
    for (const void* q : ptrs)
        need((reinterpret_cast<uintptr_t>(q) & 15) == 0,
             "field pointers must be 16-byte aligned");
}

using psv::Plan;

void sync_read(const Plan& P, hipStream_t s) {
    PSV_HIP(hipMemcpyAsync(P.host_scal, P.scal, psv::S_NSCAL * sizeof(double), hipMemcpyDeviceToHost, s));
    PSV_HIP(hipMemcpyAsync(P.host_flags, P.flags, psv::F_NFLAG * sizeof(int), hipMemcpyDeviceToHost, s));
    PSV_HIP(hipStreamSynchronize(s));
}

// Data-dependent input checks (synchronising); flags[F_STEPS] is used as scratch.
void check_field(const Plan& P, const double* x, bool positive, const char* name, hipStream_t s) {
    if (!x) return;
    int* bad = P.flags + psv::F_STEPS;
    PSV_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
    psv::launch_scan_inputs(P, x, positive ? 1 : 0, bad, s);
    sync_read(P, s);
    const int b = P.host_flags[psv::F_STEPS];
    if (b & 1) psv::fail(PSV_ERR_NONFINITE, std::string(name) + " holds NaN or Inf");
    if (b & 2) psv::fail(PSV_ERR_INVALID_ARG, std::string(name) + " must be > 0 everywhere");
}

// One constant-coefficient solve of the system assembled by `a` (CONST or
// METHOD1), written to `out`. FP64: five passes (x, y with the z chunk
// elimination, z interface, y with the back substitution, inverse x).
// MIXED: the same passes in FP32, then refinement sweeps until relres <= tol:
// each sweep's fused pass forms the FP64 residual, its norm and the FP32 x
// transform of the residual at once; a one-block check turns the norm into
// relres and sets the device flags; the correction passes (z solve, inverse
// x accumulating into out) are gated by the done flag. With host_checks the
// host reads the flags after each check and stops enqueueing at convergence;
// without, max_refine sweeps are enqueued and nothing waits on the host.
// relres is left in scal[S_RELRES] when it was computed.
struct CoreResult {
    int steps = 0;
    bool converged = true;
    bool have_relres = false;
};

CoreResult solve_core(Plan& P, psv::FwdArgs a, double* out, bool want_relres, bool host_checks,
                      hipStream_t s) {
    using namespace psv;
    const bool mixed = P.opts.precision == PSV_MIXED;
    const double inv_scale = 2.0 / ((double)P.nx * P.ny);
    CoreResult res;
    a.r_out = (mixed || want_relres) ? P.r_ws : nullptr;
    a.done = nullptr;
    // MIXED: the mean removed by the projection is taken in FP64 from the
    // assembly pass; the one the FP32 (0,0) column yields is discarded.
    a.partials = mixed ? P.partials : nullptr;
    launch_fwd_x(P, mixed, a, s);
    if (mixed) launch_mean_finalize(P, fwd_x_blocks(P), P.scal + S_RHS_MEAN, s);
    launch_z_solve(P, mixed, P.scal + (mixed ? S_MEAN2 : S_RHS_MEAN), nullptr, s);
    launch_inv_x(P, mixed, INV_STORE, out, inv_scale, nullptr, s);
    if (!mixed) {
        if (want_relres) {
            launch_residual(P, P.r_ws, out, P.scal + S_RHS_MEAN, s);
            res.have_relres = true;
        }
        return res;
    }
    const int* done = P.flags + F_DONE;
    FwdArgs ra{};
    ra.mode = FWD_RESID;
    ra.r_in = P.r_ws;
    ra.pprev = out;
    ra.mean = P.scal + S_RHS_MEAN;
    ra.partials = P.partials;
    ra.done = done;
    const int maxr = P.opts.max_refine;
    launch_refine_reset(P, s);
    res.have_relres = true;
    // One refinement sweep usually converges: the x passes that follow its
    // check (and, without host checks, return at once) run on a capped grid,
    // as dispatching every tile's block costs more than the pass's early exit
    constexpr int SPARE_BLOCKS = 1024;
    for (int sweep = 0;; ++sweep) {
        ra.max_blocks = sweep >= 2 ? SPARE_BLOCKS : 0;
        launch_fwd_x(P, true, ra, s);
        launch_refine_check(P, fwd_x_blocks(P), sweep, maxr, P.opts.tol, s);
        if (host_checks) {
            sync_read(P, s);
            if (P.host_flags[F_DONE]) break;
        }
        if (sweep == maxr) break;
        launch_z_solve(P, true, P.scal + S_MEAN2, done, s);
        launch_inv_x(P, true, INV_ADD, out, inv_scale, done, s, sweep >= 1 ? SPARE_BLOCKS : 0);
    }
    if (host_checks) {
        res.steps = P.host_flags[F_STEPS];
        res.converged = P.host_flags[F_CONV] != 0;
    }
    return res;
}

}  // namespace

extern "C" {

void psv_opts_default(psv_opts* opts) {
    if (opts) psv::default_opts(opts);
}

psv_status psv_grid_validate(const psv_grid* grid) {
    return guarded([&] { psv::validate_grid(grid); });
}

psv_status psv_plan_create(const psv_grid* grid, const psv_opts* opts, psv_plan** out) {
    return guarded([&] {
        need(out != nullptr, "out is NULL");
        *out = nullptr;
        psv::validate_grid(grid);
        psv::validate_opts(opts);
        psv_opts o;
        if (opts)
            o = *opts;
        else
            psv::default_opts(&o);
        auto* pl = new psv_plan();
        try {
            psv::plan_init(pl->p, *grid, o, true);
        } catch (...) {
            psv::plan_free(pl->p);
            delete pl;
            throw;
        }
        *out = pl;
    });
}

psv_status psv_plan_workspace_size(const psv_plan* plan, size_t* bytes) {
    return guarded([&] {
        need(plan && bytes, "plan and bytes must be non-NULL");
        *bytes = plan->p.ws_bytes;
    });
}

psv_status psv_plan_shape(const psv_plan* plan, int* lines_x, int* chunk_rows) {
    return guarded([&] {
        need(plan != nullptr, "plan is NULL");
        if (lines_x) *lines_x = plan->p.lp.lbx;
        if (chunk_rows) *chunk_rows = plan->p.lp.kc;
    });
}

psv_status psv_plan_get_shape(const psv_plan* plan, psv_shape* shape) {
    return guarded([&] {
        need(plan != nullptr && shape != nullptr, "plan and shape must be non-NULL");
        const psv::Launch& l = plan->p.lp;
        shape->lines_x = l.lbx;
        shape->lines_x_inv = l.lbx_inv;
        shape->chunk_rows = l.kc;
        shape->x_staged = l.xstage;
        shape->x_order = l.xorder;
    });
}

psv_status psv_plan_set_shape(psv_plan* plan, const psv_shape* shape) {
    return guarded([&] {
        need(plan != nullptr && shape != nullptr, "plan and shape must be non-NULL");
        Plan& P = plan->p;
        const psv_shape& h = *shape;
        for (int lb : {h.lines_x, h.lines_x_inv})
            need(lb >= 1 && lb <= 64 && P.ny % lb == 0, "lines per x block must divide ny (1..64)");
        need(h.chunk_rows == 4 || h.chunk_rows == 8 || h.chunk_rows == 16, "chunk_rows must be 4, 8 or 16");
        need(h.x_staged == 0 || h.x_staged == 1, "x_staged must be 0 or 1");
        need(h.x_order == 0 || h.x_order == 1, "x_order must be 0 or 1");
        if (!psv::kc_fits(P, h.chunk_rows))
            psv::fail(PSV_ERR_UNSUPPORTED_SIZE, "the y tile of chunk_rows planes exceeds the LDS of a block");
        for (int lb : {h.lines_x, h.lines_x_inv})
            if (psv::x_lds_max(P.nx, lb) > (size_t)psv::LDS_MAX_BLOCK)
                psv::fail(PSV_ERR_UNSUPPORTED_SIZE, "an x tile of that many lines exceeds the LDS of a block");
        psv::Launch l = P.lp;
        l.lbx = h.lines_x;
        l.lbx_inv = h.lines_x_inv;
        l.xstage = h.x_staged;
        l.xorder = h.x_order;
        PSV_HIP(hipSetDevice(P.device));
        if (h.chunk_rows != P.lp.kc) psv::plan_set_kc(P, h.chunk_rows);
        l.kc = P.lp.kc;
        P.lp = l;
    });
}

psv_status psv_plan_destroy(psv_plan* plan) {
    return guarded([&] {
        if (!plan) return;
        psv::trace_free(plan->p);
        psv::plan_free(plan->p);
        delete plan;
    });
}

psv_status psv_solve(psv_plan* plan, const double* f, const double* rho, double rho0,
                     const double* p_prev, double* p_out, int32_t n_steps, void* stream,
                     psv_info* info) {
    return guarded([&] {
        need(plan != nullptr, "plan is NULL");
        need(f != nullptr, "f is NULL");
        need(p_out != nullptr, "p_out is NULL");
        need(n_steps >= 1, "n_steps must be >= 1");
        need(std::isfinite(rho0), "rho0 must be finite");
        need_aligned({f, rho, p_prev, p_out});
        Plan& P = plan->p;
        const bool method1 = P.opts.method == PSV_SPLIT_RHO0;
        if (method1)
            need(rho != nullptr, "rho is required by Method I");
        else
            need(n_steps == 1, "the constant-coefficient solve takes n_steps = 1");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        PSV_HIP(hipSetDevice(P.device));
        if (P.opts.check_inputs) {
            check_field(P, f, false, "f", s);
            if (method1) check_field(P, rho, true, "rho", s);
            if (method1) check_field(P, p_prev, false, "p_prev", s);
        }
        psv::FwdArgs a{};
        a.f = f;
        a.rho = rho;
        a.rho0 = P.scal + psv::S_RHO0;
        if (method1) {
            if (rho0 > 0.0)
                psv::launch_set_scalar(P.scal + psv::S_RHO0, rho0, s);
            else
                psv::launch_min_reduce(P, rho, P.scal + psv::S_RHO0, P.flags + psv::F_ARGMIN, s);
            if (P.opts.check_inputs && rho0 > 0.0) {
                psv::launch_min_reduce(P, rho, P.scal + psv::S_MEAN2, nullptr, s);
                sync_read(P, s);
                if (rho0 > P.host_scal[psv::S_MEAN2])
                    psv::fail(PSV_ERR_INVALID_ARG, "rho0 exceeds min(rho): the splitting does not contract");
            }
            if (!p_prev) {
                psv::launch_fill(p_out, P.ncell(), 0.0, s);
                p_prev = p_out;
            }
        } else {
            psv::launch_set_scalar(P.scal + psv::S_RHO0, 0.0, s);
        }
        a.mode = method1 ? psv::FWD_METHOD1 : psv::FWD_CONST;
        CoreResult cr;
        int total_steps = 0;
        auto fill_info = [&] {
            sync_read(P, s);
            info->refine_steps = total_steps;
            info->relres = cr.have_relres ? P.host_scal[psv::S_RELRES] : NAN;
            info->rhs_mean_removed = P.host_scal[psv::S_RHS_MEAN];
            info->rho0_used = P.host_scal[psv::S_RHO0];
            const bool mixed = P.opts.precision == PSV_MIXED;
            for (int i = 0; i < PSV_RELRES_HISTORY; ++i)
                info->relres_sweep[i] = mixed ? P.host_scal[psv::S_HIST + i] : NAN;
            if (!mixed && cr.have_relres) info->relres_sweep[0] = info->relres;
        };
        for (int step = 0; step < n_steps; ++step) {
            a.pprev = (step == 0) ? p_prev : p_out;
            const bool last = step + 1 == n_steps;
            cr = solve_core(P, a, p_out, last && info != nullptr, info != nullptr, s);
            total_steps += cr.steps;
            if (!cr.converged) {
                if (info) fill_info();
                psv::fail(PSV_ERR_NOT_CONVERGED, "mixed-precision refinement reached max_refine");
            }
        }
        if (info) fill_info();
    });
}

psv_status psv_solve_adjoint(psv_plan* plan, const double* w, const double* f, const double* rho,
                             double rho0, const double* p_prev, double* grad_f, double* grad_rho,
                             double* grad_p_prev, double* grad_rho0_host, void* stream) {
    return guarded([&] {
        need(plan != nullptr, "plan is NULL");
        need(w != nullptr, "w is NULL");
        need(std::isfinite(rho0), "rho0 must be finite");
        need_aligned({w, f, rho, p_prev, grad_f, grad_rho, grad_p_prev});
        Plan& P = plan->p;
        const bool method1 = P.opts.method == PSV_SPLIT_RHO0;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        PSV_HIP(hipSetDevice(P.device));
        double* x = P.r_ws + P.ncell();  // S(V^-1 w)
        psv::FwdArgs a{};
        a.mode = psv::FWD_CONST;
        a.f = w;
        a.scale = P.t.inv_vol;
        CoreResult cr = solve_core(P, a, x, false, true, s);
        if (!cr.converged) psv::fail(PSV_ERR_NOT_CONVERGED, "mixed-precision refinement reached max_refine");
        if (!method1) {
            if (grad_f) psv::launch_scale_vol(P, x, grad_f, s);
            return;
        }
        need(rho != nullptr && p_prev != nullptr, "Method I adjoint needs rho and p_prev");
        const bool want_r0 = grad_rho0_host != nullptr || (rho0 <= 0.0 && grad_rho != nullptr);
        if (want_r0) need(f != nullptr, "f is required for the rho0 derivative");
        if (rho0 > 0.0)
            psv::launch_set_scalar(P.scal + psv::S_RHO0, rho0, s);
        else
            psv::launch_min_reduce(P, rho, P.scal + psv::S_RHO0, P.flags + psv::F_ARGMIN, s);
        psv::launch_adjoint_faces(P, x, f, rho, p_prev, P.scal + psv::S_RHO0, grad_f, grad_rho,
                                  grad_p_prev, P.partials, s);
        psv::launch_adjoint_finalize(P, psv::adjoint_blocks(P), grad_rho,
                                     (rho0 <= 0.0 && f != nullptr) ? 1 : 0, s);
        if (grad_rho0_host) {
            sync_read(P, s);
            *grad_rho0_host = P.host_scal[psv::S_GRAD_RHO0];
        }
    });
}

static void loop_info(Plan& P, hipStream_t s, bool from_init, psv_m3_info* info) {
    if (!info) return;
    sync_read(P, s);
    info->iterations = P.host_flags[psv::F_STEPS];
    info->converged = P.host_flags[psv::F_CONV];
    info->eps = P.host_scal[psv::S_EPS];
    info->eps_start = from_init ? NAN : P.host_scal[psv::S_EPS0];
}

// The pressure-form loop shared by Method III and the converged solve: each
// iteration assembles q = f*scale - mean - D(rho_f^-1 G p) and omega q
// (omega = rho, or the constant *a.rho0), tests eps_scale * sum|q| against
// eps_t on the device before the next solve, and adds S[omega q] to p. The
// residual of each iterate is tested before the next solve; launches after
// convergence (or after max_iter solves) return at once. The host looks at
// the flag every few iterations. a.f, a.rho, a.scale, a.mean and a.rho0 come
// from the caller.
static void residual_loop(Plan& P, bool fp32, psv::FwdArgs a, double eps_scale, double eps_t,
                          int max_iter, const double* p_init, double* p_out, hipStream_t s) {
    const size_t n = P.ncell();
    bool has_p = p_init != nullptr;
    if (has_p && p_init != p_out)
        PSV_HIP(hipMemcpyAsync(p_out, p_init, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    const int nb = psv::fwd_x_blocks(P);
    double* qpart = P.partials + nb;  // sum |q| per block
    const double inv_scale = 2.0 / ((double)P.nx * P.ny);
    const int* done = P.flags + psv::F_DONE;
    // Iterations launched between two looks at the flag: a few at first, then
    // as many as the contraction seen between the last two looks predicts to
    // reach eps_t (plus one), at most MAX_BATCH; with eps_t = 0 the loop runs
    // to max_iter.
    constexpr int FIRST_BATCH = 4, MAX_BATCH = 32;
    a.mode = psv::FWD_METHOD3;
    a.partials_abs = qpart;
    a.done = done;
    psv::launch_m3_reset(P, s);
    int batch = eps_t > 0.0 ? FIRST_BATCH : MAX_BATCH;
    double prev_eps = 0.0;
    int prev_steps = -1;
    // max_iter solves and one last residual test need at most max_iter + 1 launches
    for (int launched = 0;;) {
        batch = std::max(1, std::min(batch, max_iter + 1 - launched));
        for (int b = 0; b < batch; ++b, ++launched) {
            a.pprev = has_p ? p_out : nullptr;
            psv::launch_fwd_x(P, fp32, a, s);
            psv::launch_m3_check(P, qpart, nb, eps_scale, eps_t, has_p, max_iter, s);
            psv::launch_z_solve(P, fp32, P.scal + psv::S_MEAN2, done, s);
            psv::launch_inv_x(P, fp32, has_p ? psv::INV_ADD : psv::INV_STORE, p_out, inv_scale,
                              done, s);
            has_p = true;
        }
        sync_read(P, s);
        if (P.host_flags[psv::F_DONE]) break;
        const double eps = P.host_scal[psv::S_EPS];
        if (!std::isfinite(eps)) psv::fail(PSV_ERR_NONFINITE, "iteration residual is not finite");
        if (launched >= max_iter + 1) psv::fail(PSV_ERR_HIP, "iteration loop control failed");
        const int steps = P.host_flags[psv::F_STEPS];
        batch = eps_t > 0.0 ? FIRST_BATCH : MAX_BATCH;
        if (eps_t > 0.0 && prev_steps >= 0 && steps > prev_steps && eps > 0.0 && eps < prev_eps) {
            const double rate = std::pow(eps / prev_eps, 1.0 / (steps - prev_steps));
            const double need = std::log(eps_t / eps) / std::log(rate);
            batch = (int)std::min<double>(MAX_BATCH, std::max(1.0, std::ceil(need) + 1.0));
        }
        prev_eps = eps;
        prev_steps = steps;
    }
}

psv_status psv_solve_method3(psv_plan* plan, const double* ux, const double* uy, const double* uz,
                             const double* div_target, const double* rho, double dt, double eps_t,
                             int32_t max_iter, const double* p_init, double* p_out,
                             double* ux_out, double* uy_out, double* uz_out, void* stream,
                             psv_m3_info* info) {
    return guarded([&] {
        need(plan != nullptr, "plan is NULL");
        need(ux && uy && uz, "u* face arrays must be non-NULL");
        need(div_target != nullptr, "div_target is NULL");
        need(rho != nullptr, "rho is NULL");
        need(p_out != nullptr, "p_out is NULL");
        need(std::isfinite(dt) && dt > 0.0, "dt must be positive and finite");
        need(std::isfinite(eps_t) && eps_t >= 0.0, "eps_t must be >= 0 and finite");
        need(max_iter >= 1 && max_iter <= 100000, "max_iter must be in [1, 100000]");
        need_aligned({ux, uy, uz, div_target, rho, p_init, p_out, ux_out, uy_out, uz_out});
        const bool want_u = ux_out && uy_out && uz_out;
        need(want_u || (!ux_out && !uy_out && !uz_out), "give all three velocity outputs or none");
        if (want_u)
            need(ux_out != ux && uy_out != uy && uz_out != uz, "velocity outputs must not alias u*");
        Plan& P = plan->p;
        const bool fp32 = P.opts.precision == PSV_MIXED;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        PSV_HIP(hipSetDevice(P.device));
        if (P.opts.check_inputs) {
            check_field(P, rho, true, "rho", s);
            check_field(P, div_target, false, "div_target", s);
            check_field(P, ux, false, "ux", s);
            check_field(P, uy, false, "uy", s);
        }
        // f = (D u* - div_target) / dt, the loop-invariant part (Algorithm 1)
        double* f = P.r_ws;
        psv::launch_divergence_rhs(P, ux, uy, uz, div_target, 1.0 / dt, f, s);
        psv::FwdArgs a{};
        a.f = f;
        a.rho = rho;
        residual_loop(P, fp32, a, dt, eps_t, max_iter, p_init, p_out, s);
        if (want_u) psv::launch_correct_velocity(P, ux, uy, uz, p_out, rho, dt, ux_out, uy_out, uz_out, s);
        loop_info(P, s, p_init != nullptr, info);
    });
}

// Shared set-up of the converged solve and its adjoint: the mean of f*scale
// is removed inside the loop, and the Method-I weight is min rho.
static void converged_loop(Plan& P, const double* f, const double* scale, const double* rho,
                           int32_t iteration, double eps_t, int32_t max_iter, const double* p_init,
                           double* p_out, hipStream_t s) {
    const bool fp32 = P.opts.precision == PSV_MIXED;
    psv::FwdArgs a{};
    a.f = f;
    a.scale = scale;
    a.rho = rho;
    a.mean = P.scal + psv::S_FMEAN;
    psv::launch_vmean(P, f, P.scal + psv::S_FMEAN, s, scale);
    if (iteration == PSV_ITER_METHOD1) {
        psv::launch_min_reduce(P, rho, P.scal + psv::S_RHO0, P.flags + psv::F_ARGMIN, s);
        a.rho0 = P.scal + psv::S_RHO0;
    } else if (iteration == PSV_ITER_METHOD2) {
        psv::launch_harmonic_weight(P, rho, s);
        a.rho0 = P.scal + psv::S_OMEGA;
    }
    residual_loop(P, fp32, a, 1.0, eps_t, max_iter, p_init, p_out, s);
}

static void need_loop_args(int32_t iteration, double eps_t, int32_t max_iter) {
    need(iteration == PSV_ITER_METHOD1 || iteration == PSV_ITER_METHOD2 ||
             iteration == PSV_ITER_METHOD3,
         "iteration must be PSV_ITER_METHOD1, PSV_ITER_METHOD2 or PSV_ITER_METHOD3");
    need(std::isfinite(eps_t) && eps_t >= 0.0, "eps_t must be >= 0 and finite");
    need(max_iter >= 1 && max_iter <= 100000, "max_iter must be in [1, 100000]");
}

psv_status psv_solve_converged(psv_plan* plan, const double* f, const double* rho,
                               int32_t iteration, double eps_t, int32_t max_iter,
                               const double* p_init, double* p_out, void* stream,
                               psv_m3_info* info) {
    return guarded([&] {
        need(plan != nullptr, "plan is NULL");
        need(f && rho && p_out, "f, rho and p_out must be non-NULL");
        need(p_out != f && p_out != rho, "p_out must not alias f or rho");
        need_aligned({f, rho, p_init, p_out});
        need_loop_args(iteration, eps_t, max_iter);
        Plan& P = plan->p;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        PSV_HIP(hipSetDevice(P.device));
        if (P.opts.check_inputs) {
            check_field(P, f, false, "f", s);
            check_field(P, rho, true, "rho", s);
            check_field(P, p_init, false, "p_init", s);
        }
        converged_loop(P, f, nullptr, rho, iteration, eps_t, max_iter, p_init, p_out, s);
        loop_info(P, s, p_init != nullptr, info);
    });
}

psv_status psv_solve_converged_adjoint(psv_plan* plan, const double* w, const double* rho,
                                       const double* p, int32_t iteration, double eps_t,
                                       int32_t max_iter, double* grad_f, double* grad_rho,
                                       void* stream, psv_m3_info* info) {
    return guarded([&] {
        need(plan != nullptr, "plan is NULL");
        need(w && rho, "w and rho must be non-NULL");
        need(grad_rho == nullptr || p != nullptr, "grad_rho needs the converged pressure p");
        for (const double* out : {static_cast<const double*>(grad_f), static_cast<const double*>(grad_rho)})
            need(out == nullptr || (out != rho && out != p), "gradients must not alias rho or p");
        need(grad_f == nullptr || grad_f != grad_rho, "grad_f and grad_rho must differ");
        need_aligned({w, rho, p, grad_f, grad_rho});
        need_loop_args(iteration, eps_t, max_iter);
        Plan& P = plan->p;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        PSV_HIP(hipSetDevice(P.device));
        if (P.opts.check_inputs) {
            check_field(P, w, false, "w", s);
            check_field(P, rho, true, "rho", s);
            check_field(P, p, false, "p", s);
        }
        // lambda = A^+ (V^-1 w): the same converged solve on the scaled seed
        double* lam = P.r_ws + P.ncell();
        converged_loop(P, w, P.t.inv_vol, rho, iteration, eps_t, max_iter, nullptr, lam, s);
        if (grad_f || grad_rho) {
            // face products (D^T V lambda)(G p) / (2 rho_f^2) with unit weight; grad_f = V lambda
            psv::launch_set_scalar(P.scal + psv::S_UNIT, 1.0, s);
            psv::launch_adjoint_faces(P, lam, nullptr, rho, p ? p : lam, P.scal + psv::S_UNIT,
                                      grad_f, grad_rho, nullptr, P.partials, s);
        }
        loop_info(P, s, false, info);
    });
}

psv_status psv_solve_static(const psv_grid* grid, const psv_opts* opts, const double* f,
                            const double* rho, double rho0, const double* p_prev, double* p_out,
                            int32_t n_steps, void* stream) {
    return guarded([&] {
        psv::validate_grid(grid);
        psv::validate_opts(opts);
        psv_opts o;
        if (opts)
            o = *opts;
        else
            psv::default_opts(&o);
        need(f != nullptr, "f is NULL");
        need(p_out != nullptr, "p_out is NULL");
        need(n_steps >= 1, "n_steps must be >= 1");
        need(std::isfinite(rho0), "rho0 must be finite");
        need_aligned({f, rho, p_prev, p_out});
        if (o.method == PSV_SPLIT_RHO0)
            need(rho != nullptr, "rho is required by Method I");
        else
            need(n_steps == 1, "the constant-coefficient solve takes n_steps = 1");
        psv::solve_static(*grid, o, f, rho, rho0, p_prev, p_out, n_steps,
                          reinterpret_cast<hipStream_t>(stream));
    });
}

psv_status psv_density_from_colour(const psv_plan* plan, const double* phi, const double* rho_gas,
                                   double rho_liq, double* rho_out, void* stream) {
    return guarded([&] {
        need(plan && phi && rho_gas && rho_out, "plan, phi, rho_gas and rho_out must be non-NULL");
        need(std::isfinite(rho_liq) && rho_liq > 0.0, "rho_liq must be positive and finite");
        need_aligned({phi, rho_gas, rho_out});
        PSV_HIP(hipSetDevice(plan->p.device));
        psv::launch_density(plan->p, phi, rho_gas, rho_liq, rho_out, reinterpret_cast<hipStream_t>(stream));
    });
}

psv_status psv_divergence(const psv_plan* plan, const double* ux, const double* uy,
                          const double* uz, double* div_out, void* stream) {
    return guarded([&] {
        need(plan && ux && uy && uz && div_out, "all pointers must be non-NULL");
        need_aligned({ux, uy, uz, div_out});
        PSV_HIP(hipSetDevice(plan->p.device));
        psv::launch_divergence(plan->p, ux, uy, uz, div_out, reinterpret_cast<hipStream_t>(stream));
    });
}

psv_status psv_relres(psv_plan* plan, const double* r, const double* p, void* stream,
                      double* relres) {
    return guarded([&] {
        need(plan && r && p && relres, "all pointers must be non-NULL");
        need_aligned({r, p});
        Plan& P = plan->p;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        PSV_HIP(hipSetDevice(P.device));
        psv::launch_vmean(P, r, P.scal + psv::S_MEAN2, s);
        psv::launch_residual(P, r, p, P.scal + psv::S_MEAN2, s);
        sync_read(P, s);
        *relres = P.host_scal[psv::S_RELRES];
    });
}

psv_status psv_batch_create(int32_t n, const psv_grid* grids, const psv_opts* opts,
                            psv_batch** out) {
    return guarded([&] {
        need(out != nullptr, "out is NULL");
        *out = nullptr;
        need(n >= 1 && n <= 65536, "n must be in [1, 65536]");
        need(grids != nullptr, "grids is NULL");
        for (int p = 0; p < n; ++p) psv::validate_grid(&grids[p]);
        psv::validate_opts(opts);
        psv_opts o;
        if (opts)
            o = *opts;
        else
            psv::default_opts(&o);
        if (o.tol <= 0.0) o.tol = 1e-10;
        if (o.max_refine <= 0) o.max_refine = 4;
        psv_batch* b = psv::batch_new();
        try {
            psv::batch_create(*b, n, grids, o);
        } catch (...) {
            psv::batch_delete(b);
            throw;
        }
        *out = b;
    });
}

psv_status psv_batch_solve(psv_batch* batch, const double* const* f, const double* const* rho,
                           const double* rho0, const double* const* p_prev, double* const* p_out,
                           void* stream, psv_info* infos) {
    return guarded([&] {
        need(batch != nullptr, "batch is NULL");
        need(f != nullptr && p_out != nullptr, "f and p_out are required");
        const int n = psv::batch_size(*batch);
        const bool method1 = psv::batch_method(*batch) == PSV_SPLIT_RHO0;
        const bool fp32 = psv::batch_fp32(*batch);
        for (int p = 0; p < n; ++p) {
            need(f[p] != nullptr && p_out[p] != nullptr, "f[p] and p_out[p] must be non-NULL");
            need_aligned({f[p], p_out[p], rho ? rho[p] : nullptr, p_prev ? p_prev[p] : nullptr});
            if (method1) {
                need(rho != nullptr && rho[p] != nullptr, "rho[p] is required by Method I");
                need(p_prev != nullptr && p_prev[p] != nullptr, "p_prev[p] is required by Method I");
                need(p_prev[p] != p_out[p], "batched solves need p_prev[p] != p_out[p]");
            }
            if (rho0) need(std::isfinite(rho0[p]), "rho0 must be finite");
        }
        for (int p = 0; p < n; ++p)
            psv::batch_set_io(*batch, p, f[p], method1 ? rho[p] : nullptr,
                              method1 ? p_prev[p] : nullptr, p_out[p], rho0 ? rho0[p] : 0.0,
                              fp32 || infos != nullptr);
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        psv::batch_solve(*batch, s, fp32 || infos != nullptr);
        if (infos) {
            const bool ok = psv::batch_infos(*batch, s, infos);
            if (!ok) psv::fail(PSV_ERR_NOT_CONVERGED, "a batched problem did not reach tol");
        }
    });
}

psv_status psv_batch_destroy(psv_batch* batch) {
    return guarded([&] {
        if (batch) psv::batch_delete(batch);
    });
}

psv_status psv_trace_enable(psv_plan* plan, int32_t enable) {
    return guarded([&] {
        need(plan != nullptr, "plan is NULL");
        plan->p.trace.on = enable != 0;
    });
}

psv_status psv_trace_summary(psv_plan* plan, char* buf, size_t len, size_t* needed) {
    return guarded([&] {
        need(plan != nullptr, "plan is NULL");
        need(buf != nullptr || len == 0, "buf is NULL");
        const std::string s = psv::trace_summary(plan->p);
        if (needed) *needed = s.size() + 1;
        if (len > 0) {
            const size_t n = std::min(len - 1, s.size());
            std::memcpy(buf, s.data(), n);
            buf[n] = '\0';
        }
    });
}

const char* psv_status_string(psv_status s) {
    switch (s) {
        case PSV_OK: return "PSV_OK";
        case PSV_ERR_INVALID_ARG: return "PSV_ERR_INVALID_ARG";
        case PSV_ERR_UNSUPPORTED_SIZE: return "PSV_ERR_UNSUPPORTED_SIZE";
        case PSV_ERR_HIP: return "PSV_ERR_HIP";
        case PSV_ERR_NONFINITE: return "PSV_ERR_NONFINITE";
        case PSV_ERR_NOT_CONVERGED: return "PSV_ERR_NOT_CONVERGED";
        case PSV_ERR_OOM: return "PSV_ERR_OOM";
    }
    return "PSV_ERR_UNKNOWN";
}

const char* psv_last_error_message(void) { return g_last_error.c_str(); }

}  // extern "C"
