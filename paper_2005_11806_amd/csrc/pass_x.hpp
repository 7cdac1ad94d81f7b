// x-direction passes of the eigenexpansion solve (Sec. 3.3.1) as block-level
// tile functions, shared by the per-pass kernels and the persistent batch
// kernel:
//  * forward: right-hand-side assembly (Method I, Eq. poisson_me1, a scaled
//    copy, or a refinement residual) fused with the real FFT along x; the
//    half spectrum goes to layout A [k][m][j];
//  * inverse: real inverse FFT along x from layout A and the store of p.
// A tile is `lb` consecutive x-lines (j0 .. j0+lb-1) of one z-plane k; the
// block has 256 threads.
#pragma once

#include "internal.hpp"

namespace psv {

struct XGeom {
    int nx, ny, nz, mx, M, lb, tiles;  // tiles = ny / lb
    double inv_dx, inv_dy;
    Radices rad;
};

struct Stencil {
    const double* inv_h;
    const double* inv_g;
    const double* vol;
};

// LDS bytes of the x tiles for complex element size csz
inline size_t fwd_x_lds(const XGeom& g, size_t csz) { return ((size_t)2 * g.lb * g.M + 2 * g.M) * csz; }
inline size_t inv_x_lds(const XGeom& g, size_t csz) {
    return ((size_t)g.lb * (2 * g.M + 1) + 2 * g.M) * csz;
}

// Blocks are dispatched round-robin over the 8 XCDs; remap so that each XCD
// walks a contiguous range of (plane, tile) indices and the neighbouring
// lines/planes read by the stencil stay in its L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, i = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// Method-I right-hand side at one cell (Eq. poisson_me1):
//   rho0 f + sum over faces of (1 - rho0/rho_f) (grad p)_f, differenced,
// with beta_f = 1 - 2 rho0 / (rho_L + rho_R); wall faces carry no flux.
__device__ __forceinline__ double method1_cell(const double* __restrict__ f,
                                               const double* __restrict__ rho,
                                               const double* __restrict__ pp, double rho0,
                                               int i, int j, int k, const XGeom& g,
                                               const Stencil& st) {
    const size_t plane = (size_t)g.nx * g.ny;
    const size_t row = (size_t)k * plane + (size_t)j * g.nx;
    const size_t c = row + i;
    const int ie = (i + 1 == g.nx) ? 0 : i + 1;
    const int iw = (i == 0) ? g.nx - 1 : i - 1;
    const int jn = (j + 1 == g.ny) ? 0 : j + 1;
    const int js = (j == 0) ? g.ny - 1 : j - 1;
    const double pc = pp[c], rc = rho[c];
    const double two_r0 = 2.0 * rho0;
    double acc;
    {
        const double pe = pp[row + ie], pw = pp[row + iw];
        const double re = rho[row + ie], rw = rho[row + iw];
        const double fe = (re + rc - two_r0) / (re + rc) * (pe - pc);
        const double fw = (rw + rc - two_r0) / (rw + rc) * (pc - pw);
        acc = (fe - fw) * (g.inv_dx * g.inv_dx);
    }
    {
        const size_t cn = (size_t)k * plane + (size_t)jn * g.nx + i;
        const size_t cs = (size_t)k * plane + (size_t)js * g.nx + i;
        const double pn = pp[cn], ps = pp[cs];
        const double rn = rho[cn], rs = rho[cs];
        const double fn = (rn + rc - two_r0) / (rn + rc) * (pn - pc);
        const double fs = (rs + rc - two_r0) / (rs + rc) * (pc - ps);
        acc += (fn - fs) * (g.inv_dy * g.inv_dy);
    }
    {
        double ft = 0.0, fb = 0.0;
        if (k + 1 < g.nz) {
            const size_t ct = c + plane;
            const double rt = rho[ct];
            ft = (rt + rc - two_r0) / (rt + rc) * (pp[ct] - pc) * st.inv_g[k + 1];
        }
        if (k > 0) {
            const size_t cb = c - plane;
            const double rb = rho[cb];
            fb = (rb + rc - two_r0) / (rb + rc) * (pc - pp[cb]) * st.inv_g[k];
        }
        acc += (ft - fb) * st.inv_h[k];
    }
    return acc + rho0 * f[c];
}

// 7-point L p at one cell (flux form in z; zero wall flux).
__device__ __forceinline__ double lap_cell(const double* __restrict__ p, int i, int j, int k,
                                           const XGeom& g, const Stencil& st) {
    const size_t plane = (size_t)g.nx * g.ny;
    const size_t row = (size_t)k * plane + (size_t)j * g.nx;
    const size_t c = row + i;
    const int ie = (i + 1 == g.nx) ? 0 : i + 1;
    const int iw = (i == 0) ? g.nx - 1 : i - 1;
    const int jn = (j + 1 == g.ny) ? 0 : j + 1;
    const int js = (j == 0) ? g.ny - 1 : j - 1;
    const double pc = p[c];
    double acc = ((p[row + ie] - pc) - (pc - p[row + iw])) * (g.inv_dx * g.inv_dx);
    acc += ((p[(size_t)k * plane + (size_t)jn * g.nx + i] - pc) -
            (pc - p[(size_t)k * plane + (size_t)js * g.nx + i])) * (g.inv_dy * g.inv_dy);
    const double ft = (k + 1 < g.nz) ? (p[c + plane] - pc) * st.inv_g[k + 1] : 0.0;
    const double fb = (k > 0) ? (pc - p[c - plane]) * st.inv_g[k] : 0.0;
    return acc + (ft - fb) * st.inv_h[k];
}

// Forward tile b. N = nx/2 as a compile-time constant, or 0 (runtime length).
// Partial sums (when requested) go to a.partials at slot b: one value
// (vol * sum r) for CONST/METHOD1, two (sum res^2, sum r~^2) for RESID.
template <typename TC, typename TS, int MODE, int N>
__device__ __forceinline__ void fwd_x_tile(const XGeom& g, const Stencil& st, const FwdArgs& a,
                                           const c2<TC>* __restrict__ tw_g,
                                           c2<TS>* __restrict__ spec, int b, unsigned char* smem,
                                           double* red) {
    using C = c2<TC>;
    const int k = b / g.tiles;
    const int j0 = (b - k * g.tiles) * g.lb;
    const int M = N ? N : g.M;
    C* buf0 = reinterpret_cast<C*>(smem);
    C* buf1 = buf0 + g.lb * M;
    C* tw = buf1 + g.lb * M;  // exp(-2 pi i t / nx), t < nx
    for (int t = threadIdx.x; t < 2 * M; t += 256) tw[t] = tw_g[t];
    TC* rbuf = reinterpret_cast<TC*>(buf0);

    const double rho0 = (MODE == FWD_METHOD1) ? *a.rho0 : 0.0;
    const double mean = (MODE == FWD_RESID) ? *a.mean : 0.0;
    const double sc = (MODE == FWD_CONST && a.scale) ? a.scale[k] : 1.0;
    double res2 = 0.0, r2 = 0.0, rsum = 0.0;
    const int ncell = g.lb * g.nx;
    for (int t = threadIdx.x; t < ncell; t += 256) {
        const int line = t / g.nx;
        const int i = t - line * g.nx;
        const int j = j0 + line;
        const size_t c = ((size_t)k * g.ny + j) * g.nx + i;
        double r;
        if (MODE == FWD_CONST) {
            r = a.f[c] * sc;
        } else if (MODE == FWD_METHOD1) {
            r = method1_cell(a.f, a.rho, a.pprev, rho0, i, j, k, g, st);
        } else {
            const double rp = a.r_in[c] - mean;
            r = rp - lap_cell(a.pprev, i, j, k, g, st);
            res2 += r * r;
            r2 += rp * rp;
        }
        if (a.r_out) a.r_out[c] = r;
        rsum += r;
        rbuf[line * g.nx + i] = (TC)r;  // z_n = r_{2n} + i r_{2n+1}
    }
    if (MODE != FWD_RESID && a.partials) {
        // FP64 volume-weighted sum of the right-hand side (its mean is the
        // compatibility projection; the FP32 spectrum is too coarse for it)
        const double s1 = block_sum(rsum, red);
        if (threadIdx.x == 0) a.partials[b] = s1 * st.vol[k];
    }
    if (MODE == FWD_RESID) {
        const double s1 = block_sum(res2, red);
        __syncthreads();
        const double s2 = block_sum(r2, red);
        if (threadIdx.x == 0) {
            a.partials[2 * b] = s1;
            a.partials[2 * b + 1] = s2;
        }
    }
    __syncthreads();
    C* Z = lds_fft_n<N, -1, 2>(buf0, buf1, M, g.lb, M, g.rad, tw);
    // Split the half-length transform into the real-input spectrum:
    //   E_m = (Z_m + conj Z_{M-m}) / 2, O_m = (Z_m - conj Z_{M-m}) / (2i),
    //   X_m = E_m + exp(-2 pi i m / nx) O_m, m = 0..M.
    const int nout = (M + 1) * g.lb;
    const size_t plane_s = (size_t)g.mx * g.ny;
    for (int t = threadIdx.x; t < nout; t += 256) {
        const int m = t / g.lb;
        const int line = t - m * g.lb;
        const C zm = Z[line * M + (m == M ? 0 : m)];
        const C zc = cconj(Z[line * M + (m == 0 ? 0 : M - m)]);
        const C e = C{(TC)0.5 * (zm.x + zc.x), (TC)0.5 * (zm.y + zc.y)};
        const C o = C{(TC)0.5 * (zm.y - zc.y), (TC)-0.5 * (zm.x - zc.x)};
        const C x = cadd(e, cmul(tw[m], o));
        spec[(size_t)k * plane_s + (size_t)m * g.ny + j0 + line] = cconv<c2<TS>>(x);
    }
}

// Inverse tile b: p = scale * x (STORE), p += scale * x (ADD) or
// p = scale * vol[k] * x (SCALE).
template <typename TC, typename TS, int MODE, int N>
__device__ __forceinline__ void inv_x_tile(const XGeom& g, const c2<TC>* __restrict__ tw_g,
                                           const c2<TS>* __restrict__ spec,
                                           double* __restrict__ out,
                                           const double* __restrict__ vol, double scale, int b,
                                           unsigned char* smem) {
    using C = c2<TC>;
    const int k = b / g.tiles;
    const int j0 = (b - k * g.tiles) * g.lb;
    const int M = N ? N : g.M;
    C* buf0 = reinterpret_cast<C*>(smem);
    C* xb = buf0 + g.lb * M;  // lb x (M+1), later reused as the FFT's second buffer
    C* tw = xb + g.lb * (M + 1);
    for (int t = threadIdx.x; t < 2 * M; t += 256) tw[t] = tw_g[t];
    const size_t plane_s = (size_t)g.mx * g.ny;
    const int nin = (M + 1) * g.lb;
    for (int t = threadIdx.x; t < nin; t += 256) {
        const int m = t / g.lb;
        const int line = t - m * g.lb;
        C x = cconv<C>(spec[(size_t)k * plane_s + (size_t)m * g.ny + j0 + line]);
        if (m == 0 || m == M) x.y = (TC)0;  // a real field has real DC and Nyquist bins
        xb[line * (M + 1) + m] = x;
    }
    __syncthreads();
    // Z_m = E_m + i O_m with E_m = (X_m + conj X_{M-m}) / 2 and
    // O_m = (X_m - conj X_{M-m}) exp(+2 pi i m / nx) / 2, m = 0..M-1.
    const int nzz = M * g.lb;
    for (int t = threadIdx.x; t < nzz; t += 256) {
        const int line = t / M;
        const int m = t - line * M;
        const C xm = xb[line * (M + 1) + m];
        const C xc = cconj(xb[line * (M + 1) + (M - m)]);
        const C e = C{(TC)0.5 * (xm.x + xc.x), (TC)0.5 * (xm.y + xc.y)};
        const C d = C{(TC)0.5 * (xm.x - xc.x), (TC)0.5 * (xm.y - xc.y)};
        const C o = cmul(d, cconj(tw[m]));
        buf0[line * M + m] = C{e.x - o.y, e.y + o.x};
    }
    __syncthreads();
    C* z = lds_fft_n<N, +1, 2>(buf0, xb, M, g.lb, M, g.rad, tw);
    const double s = (MODE == INV_SCALE) ? scale * vol[k] : scale;
    const int ncell = g.lb * g.nx;
    for (int t = threadIdx.x; t < ncell; t += 256) {
        const int line = t / g.nx;
        const int i = t - line * g.nx;
        const C v = z[line * M + (i >> 1)];
        const double x = (double)((i & 1) ? v.y : v.x) * s;
        const size_t c = ((size_t)k * g.ny + j0 + line) * g.nx + i;
        if (MODE == INV_ADD)
            out[c] += x;
        else
            out[c] = x;
    }
}

inline XGeom make_xgeom(const Plan& p) {
    XGeom g;
    g.nx = p.nx;
    g.ny = p.ny;
    g.nz = p.nz;
    g.mx = p.mx;
    g.M = p.nx / 2;
    g.lb = p.lp.lbx;
    g.tiles = p.ny / p.lp.lbx;
    g.inv_dx = 1.0 / p.dx;
    g.inv_dy = 1.0 / p.dy;
    g.rad = p.rad_xh;
    return g;
}

}  // namespace psv
