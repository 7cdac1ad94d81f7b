// Per-pass kernels of the x direction (tile bodies in pass_x.hpp): one block
// per tile, remapped so each XCD walks a contiguous range of tiles (of planes,
// or for the forward pass of lines through all planes).
#include <algorithm>

#include "pass_x.hpp"

namespace psv {
namespace {

template <typename TC, typename TS, int MODE, int N, bool STAGE>
__global__ void __launch_bounds__(256) k_fwd_x(XGeom g, Stencil st, FwdArgs a,
                                                const c2<TC>* __restrict__ tw_g,
                                                c2<TS>* __restrict__ spec) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[16];
    if (a.done && *a.done) return;
    const int b = g.win ? xcd_windows(blockIdx.x, g.win, g.tiles) : xcd_remap(blockIdx.x, gridDim.x);
    fwd_x_tile<TC, TS, MODE, N, STAGE>(g, st, a, tw_g, spec, b, smem_raw, red);
}

// The same on a capped grid (a multiple of 8 blocks): block v takes tiles v,
// v + gridDim.x, ..., whose XCD is v % 8 as for the full grid. For launches
// that usually find *done set (the refinement sweeps after the first); the
// loop keeps more registers live (129 VGPRs against 70 for the FP32
// refinement residual), so a pass that does run takes longer than on the
// full grid.
template <typename TC, typename TS, int MODE, int N, bool STAGE>
__global__ void __launch_bounds__(256) k_fwd_x_capped(XGeom g, Stencil st, FwdArgs a,
                                                       const c2<TC>* __restrict__ tw_g,
                                                       c2<TS>* __restrict__ spec) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[16];
    if (a.done && *a.done) return;
    const int nt = g.tiles * g.nz;
    for (int v = blockIdx.x; v < nt; v += gridDim.x) {
        const int b = g.win ? xcd_windows(v, g.win, g.tiles) : xcd_remap(v, nt);
        fwd_x_tile<TC, TS, MODE, N, STAGE>(g, st, a, tw_g, spec, b, smem_raw, red);
        if (v + (int)gridDim.x < nt) __syncthreads();  // the next tile reuses the LDS
    }
}

template <typename TC, typename TS, int MODE, int N>
__global__ void __launch_bounds__(256) k_inv_x(XGeom g, const c2<TC>* __restrict__ tw_g,
                                                const c2<TS>* __restrict__ spec,
                                                double* __restrict__ out,
                                                const double* __restrict__ vol, double scale,
                                                const int* done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (done && *done) return;
    inv_x_tile<TC, TS, MODE, N>(g, tw_g, spec, out, vol, scale, xcd_remap(blockIdx.x, gridDim.x),
                                smem_raw);
}

// capped grid, as k_fwd_x_capped
template <typename TC, typename TS, int MODE, int N>
__global__ void __launch_bounds__(256) k_inv_x_capped(XGeom g, const c2<TC>* __restrict__ tw_g,
                                                       const c2<TS>* __restrict__ spec,
                                                       double* __restrict__ out,
                                                       const double* __restrict__ vol, double scale,
                                                       const int* done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (done && *done) return;
    const int nt = g.tiles * g.nz;
    for (int v = blockIdx.x; v < nt; v += gridDim.x) {
        inv_x_tile<TC, TS, MODE, N>(g, tw_g, spec, out, vol, scale, xcd_remap(v, nt), smem_raw);
        if (v + (int)gridDim.x < nt) __syncthreads();
    }
}

// Blocks of an x pass over nt tiles: all of them, or at most max_blocks > 0
// rounded down to a multiple of 8 (the kernels loop over the tiles)
inline int x_grid(int nt, int max_blocks) {
    if (max_blocks <= 0 || nt <= max_blocks) return nt;
    return std::max(8, max_blocks / 8 * 8);
}

// x-line lengths with a compile-time FFT (M = nx/2); others use the runtime one
#define PSV_X_SIZES(X) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(512)

template <typename TC, typename TS, int MODE, int N, bool STAGE>
void fwd_launch_s(const Plan& p, const XGeom& g, const Stencil& st, const FwdArgs& a,
                  const c2<TC>* tw, hipStream_t s) {
    const size_t lds = fwd_x_lds(g, sizeof(c2<TC>), MODE);
    allow_lds(k_fwd_x<TC, TS, MODE, N, STAGE>, lds);
    const int nt = g.tiles * p.nz, grid = x_grid(nt, a.max_blocks);
    // capped grids only for the FP32 refinement residual, the one pass that
    // is launched capped
    if constexpr (MODE == FWD_RESID && sizeof(TC) == 4) {
        if (grid < nt) {
            allow_lds(k_fwd_x_capped<TC, TS, MODE, N, STAGE>, lds);
            hipLaunchKernelGGL((k_fwd_x_capped<TC, TS, MODE, N, STAGE>), dim3(grid), dim3(256), lds, s,
                               g, st, a, tw, reinterpret_cast<c2<TS>*>(p.spec));
            return;
        }
    }
    hipLaunchKernelGGL((k_fwd_x<TC, TS, MODE, N, STAGE>), dim3(nt), dim3(256), lds, s,
                       g, st, a, tw, reinterpret_cast<c2<TS>*>(p.spec));
}

// the constant-coefficient copy has no stencil: one variant
template <typename TC, typename TS, int MODE, int N>
void fwd_launch(const Plan& p, const XGeom& g, const Stencil& st, const FwdArgs& a,
                const c2<TC>* tw, hipStream_t s) {
    if (MODE == FWD_CONST || g.stage)
        fwd_launch_s<TC, TS, MODE, N, true>(p, g, st, a, tw, s);
    else
        fwd_launch_s<TC, TS, MODE, N, MODE == FWD_CONST>(p, g, st, a, tw, s);
}

template <typename TC, typename TS, int MODE>
void fwd_impl(const Plan& p, const FwdArgs& a, hipStream_t s) {
    XGeom g = make_xgeom(p);
    Stencil st{p.t.inv_h, p.t.inv_g, p.t.vol};
    const c2<TC>* tw;
    if constexpr (sizeof(TC) == 8) tw = p.t.twx64; else tw = p.t.twx32;
    static const char* names[2][4] = {
        {"fwd_x_const_fp64", "fwd_x_method1_fp64", "fwd_x_resid_fp64", "fwd_x_method3_fp64"},
        {"fwd_x_const_fp32", "fwd_x_method1_fp32", "fwd_x_resid_fp32", "fwd_x_method3_fp32"}};
    TraceScope ts(p, names[sizeof(TC) == 4][MODE], s);
    switch (g.M) {
#define PSV_CASE(n) case n: fwd_launch<TC, TS, MODE, n>(p, g, st, a, tw, s); break;
        PSV_X_SIZES(PSV_CASE)
#undef PSV_CASE
        default: fwd_launch<TC, TS, MODE, 0>(p, g, st, a, tw, s); break;
    }
    PSV_HIP(hipGetLastError());
}

template <typename TC, typename TS, int MODE, int N>
void inv_launch(const Plan& p, const XGeom& g, const c2<TC>* tw, double* out, double scale,
                const int* done, hipStream_t s, int max_blocks) {
    const size_t lds = inv_x_lds(g, sizeof(c2<TC>));
    allow_lds(k_inv_x<TC, TS, MODE, N>, lds);
    const int nt = g.tiles * p.nz, grid = x_grid(nt, max_blocks);
    if constexpr (MODE == INV_ADD && sizeof(TC) == 4) {  // the refinement's correction
        if (grid < nt) {
            allow_lds(k_inv_x_capped<TC, TS, MODE, N>, lds);
            hipLaunchKernelGGL((k_inv_x_capped<TC, TS, MODE, N>), dim3(grid), dim3(256), lds, s, g, tw,
                               reinterpret_cast<const c2<TS>*>(p.spec), out, p.t.vol, scale, done);
            return;
        }
    }
    hipLaunchKernelGGL((k_inv_x<TC, TS, MODE, N>), dim3(nt), dim3(256), lds, s, g, tw,
                       reinterpret_cast<const c2<TS>*>(p.spec), out, p.t.vol, scale, done);
}

template <typename TC, typename TS, int MODE>
void inv_impl(const Plan& p, double* out, double scale, const int* done, hipStream_t s,
              int max_blocks) {
    XGeom g = make_xgeom(p, true);
    const c2<TC>* tw;
    if constexpr (sizeof(TC) == 8) tw = p.t.twx64; else tw = p.t.twx32;
    static const char* names[2][3] = {{"inv_x_store_fp64", "inv_x_add_fp64", "inv_x_scale_fp64"},
                                      {"inv_x_store_fp32", "inv_x_add_fp32", "inv_x_scale_fp32"}};
    TraceScope ts(p, names[sizeof(TC) == 4][MODE], s);
    switch (g.M) {
#define PSV_CASE(n) case n: inv_launch<TC, TS, MODE, n>(p, g, tw, out, scale, done, s, max_blocks); break;
        PSV_X_SIZES(PSV_CASE)
#undef PSV_CASE
        default: inv_launch<TC, TS, MODE, 0>(p, g, tw, out, scale, done, s, max_blocks); break;
    }
    PSV_HIP(hipGetLastError());
}

}  // namespace

int fwd_x_blocks(const Plan& p) { return (p.ny / p.lp.lbx) * p.nz; }

void launch_fwd_x(const Plan& p, bool fp32, const FwdArgs& a, hipStream_t s) {
    if (fp32) {
        switch (a.mode) {
            case FWD_CONST: fwd_impl<float, float, FWD_CONST>(p, a, s); break;
            case FWD_METHOD1: fwd_impl<float, float, FWD_METHOD1>(p, a, s); break;
            case FWD_METHOD3: fwd_impl<float, float, FWD_METHOD3>(p, a, s); break;
            default: fwd_impl<float, float, FWD_RESID>(p, a, s); break;
        }
    } else {
        switch (a.mode) {
            case FWD_CONST: fwd_impl<double, double, FWD_CONST>(p, a, s); break;
            case FWD_METHOD1: fwd_impl<double, double, FWD_METHOD1>(p, a, s); break;
            case FWD_METHOD3: fwd_impl<double, double, FWD_METHOD3>(p, a, s); break;
            default: fwd_impl<double, double, FWD_RESID>(p, a, s); break;
        }
    }
}

void launch_inv_x(const Plan& p, bool fp32, int mode, double* out, double scale_all,
                  const int* done, hipStream_t s, int max_blocks) {
    if (fp32) {
        switch (mode) {
            case INV_STORE: inv_impl<float, float, INV_STORE>(p, out, scale_all, done, s, max_blocks); break;
            case INV_ADD: inv_impl<float, float, INV_ADD>(p, out, scale_all, done, s, max_blocks); break;
            default: inv_impl<float, float, INV_SCALE>(p, out, scale_all, done, s, max_blocks); break;
        }
    } else {
        switch (mode) {
            case INV_STORE: inv_impl<double, double, INV_STORE>(p, out, scale_all, done, s, max_blocks); break;
            case INV_ADD: inv_impl<double, double, INV_ADD>(p, out, scale_all, done, s, max_blocks); break;
            default: inv_impl<double, double, INV_SCALE>(p, out, scale_all, done, s, max_blocks); break;
        }
    }
}

}  // namespace psv
