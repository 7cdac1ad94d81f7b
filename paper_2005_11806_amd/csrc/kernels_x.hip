// Per-pass kernels of the x direction (tile bodies in pass_x.hpp): one block
// per tile, remapped so each XCD walks a contiguous range of tiles (of planes,
// or for the forward pass of lines through all planes).
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

// x-line lengths with a compile-time FFT (M = nx/2); others use the runtime one
#define PSV_X_SIZES(X) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(512)

template <typename TC, typename TS, int MODE, int N, bool STAGE>
void fwd_launch_s(const Plan& p, const XGeom& g, const Stencil& st, const FwdArgs& a,
                  const c2<TC>* tw, hipStream_t s) {
    const size_t lds = fwd_x_lds(g, sizeof(c2<TC>));
    allow_lds(k_fwd_x<TC, TS, MODE, N, STAGE>, lds);
    hipLaunchKernelGGL((k_fwd_x<TC, TS, MODE, N, STAGE>), dim3(g.tiles * p.nz), dim3(256), lds, s,
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
                const int* done, hipStream_t s) {
    const size_t lds = inv_x_lds(g, sizeof(c2<TC>));
    allow_lds(k_inv_x<TC, TS, MODE, N>, lds);
    hipLaunchKernelGGL((k_inv_x<TC, TS, MODE, N>), dim3(g.tiles * p.nz), dim3(256), lds, s, g, tw,
                       reinterpret_cast<const c2<TS>*>(p.spec), out, p.t.vol, scale, done);
}

template <typename TC, typename TS, int MODE>
void inv_impl(const Plan& p, double* out, double scale, const int* done, hipStream_t s) {
    XGeom g = make_xgeom(p, true);
    const c2<TC>* tw;
    if constexpr (sizeof(TC) == 8) tw = p.t.twx64; else tw = p.t.twx32;
    static const char* names[2][3] = {{"inv_x_store_fp64", "inv_x_add_fp64", "inv_x_scale_fp64"},
                                      {"inv_x_store_fp32", "inv_x_add_fp32", "inv_x_scale_fp32"}};
    TraceScope ts(p, names[sizeof(TC) == 4][MODE], s);
    switch (g.M) {
#define PSV_CASE(n) case n: inv_launch<TC, TS, MODE, n>(p, g, tw, out, scale, done, s); break;
        PSV_X_SIZES(PSV_CASE)
#undef PSV_CASE
        default: inv_launch<TC, TS, MODE, 0>(p, g, tw, out, scale, done, s); break;
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
                  const int* done, hipStream_t s) {
    if (fp32) {
        switch (mode) {
            case INV_STORE: inv_impl<float, float, INV_STORE>(p, out, scale_all, done, s); break;
            case INV_ADD: inv_impl<float, float, INV_ADD>(p, out, scale_all, done, s); break;
            default: inv_impl<float, float, INV_SCALE>(p, out, scale_all, done, s); break;
        }
    } else {
        switch (mode) {
            case INV_STORE: inv_impl<double, double, INV_STORE>(p, out, scale_all, done, s); break;
            case INV_ADD: inv_impl<double, double, INV_ADD>(p, out, scale_all, done, s); break;
            default: inv_impl<double, double, INV_SCALE>(p, out, scale_all, done, s); break;
        }
    }
}

}  // namespace psv
