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

#include <type_traits>

#include "internal.hpp"

namespace psv {

struct XGeom {
    int nx, ny, nz, mx, M, lb, tiles;  // tiles = ny / lb
    int stage;                         // forward tile: stencil rows staged in LDS (1) or not (0)
    int win;                           // forward pass: tiles per XCD line window, 0 = plane ranges
    double inv_dx, inv_dy;
    Radices rad;
};

struct Stencil {
    const double* inv_h;
    const double* inv_g;
    const double* vol;
};

// FFT buffers of the x tiles hold lb lines of M elements in the layout
// XLayout<N>: one pad element after every 8 for the compile-time lengths (the
// radix scatter of a Stockham stage then spreads over the LDS banks), plain
// for runtime lengths. Either way a buffer spans xbuf_span(lb M) elements.
template <int N>
using XLayout = std::conditional_t<(N > 0), Pad8, NoPad>;
__host__ __device__ inline int xbuf_span(int n) { return n + (n >> 3) + 1; }

// LDS bytes of the x tiles for complex element size csz. Forward: FFT buffer,
// twiddles, then the second FFT buffer, which with `stage` shares its space
// with the staged rows (lb + 2 rows, FP64) of the `fields` stencil fields:
// p and rho (2), p alone for a residual (1), none for a copy (0). Inverse:
// FFT buffer, the staged half spectrum (lb x (M+1), reused as the second
// FFT buffer), twiddles.
inline size_t fwd_x_lds_n(int nx, int lb, size_t csz, bool stage = true, int fields = 2) {
    const size_t M = nx / 2;
    const size_t rows = stage ? (size_t)fields * (lb + 2) * nx * sizeof(double) : 0;
    const size_t buf = (size_t)xbuf_span(lb * (int)M) * csz;
    return buf + 2 * M * csz + 16 + (rows > buf ? rows : buf);
}
__host__ __device__ inline int inv_x_stage_span(int M, int lb) {
    const int a = lb * (M + 1), b = xbuf_span(lb * M);
    return a > b ? a : b;
}
inline size_t inv_x_lds_n(int nx, int lb, size_t csz) {
    const int M = nx / 2;
    return ((size_t)xbuf_span(lb * M) + inv_x_stage_span(M, lb) + 2 * (size_t)M) * csz;
}
// mode: the forward pass's FwdMode (the default sizes for Method I, the most)
inline size_t fwd_x_lds(const XGeom& g, size_t csz, int mode = FWD_METHOD1) {
    const int fields = mode == FWD_CONST ? 0 : (mode == FWD_RESID ? 1 : 2);
    return fwd_x_lds_n(g.nx, g.lb, csz, g.stage != 0, fields);
}
inline size_t inv_x_lds(const XGeom& g, size_t csz) { return inv_x_lds_n(g.nx, g.lb, csz); }
// the larger of the two at FP64 (forward with staged rows), for choosing lines
// per block
inline size_t x_lds_max(int nx, int lb) {
    const size_t a = fwd_x_lds_n(nx, lb, 16), b = inv_x_lds_n(nx, lb, 16);
    return a > b ? a : b;
}

// (1 - rho0/rho_f) (p_R - p_L) across the face between cells L and R, with
// rho_f = (rho_L + rho_R)/2, i.e. (s - 2 rho0)/s with s = rho_L + rho_R.
__device__ __forceinline__ double bflux(double rl, double rr, double pl, double pr, double two_r0) {
    const double s = rl + rr;
    return (s - two_r0) * rcp_nr1(s) * (pr - pl);
}

// rho_f^-1 (p_R - p_L) across the face between cells L and R,
// rho_f = (rho_L + rho_R)/2.
__device__ __forceinline__ double gflux(double rl, double rr, double pl, double pr) {
    return 2.0 * rcp_nr1(rl + rr) * (pr - pl);
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
template <typename TC, typename TS, int MODE, int N, bool STAGE = true>
__device__ __forceinline__ void fwd_x_tile(const XGeom& g, const Stencil& st, const FwdArgs& a,
                                           const c2<TC>* __restrict__ tw_g,
                                           c2<TS>* __restrict__ spec, int b, unsigned char* smem,
                                           double* red) {
    using C = c2<TC>;
    const int k = b / g.tiles;
    const int j0 = (b - k * g.tiles) * g.lb;
    const int M = N ? N : g.M;
    const int nx = 2 * M;
    const int lb = g.lb;
    using P = XLayout<N>;
    C* buf0 = reinterpret_cast<C*>(smem);
    C* tw = buf0 + xbuf_span(lb * M);  // exp(-2 pi i t / nx), t < nx
    // second FFT buffer, 16-byte aligned (FP32 buffers may end on an 8-byte
    // boundary); with STAGE it first holds the p and rho rows j0-1 .. j0+lb
    const size_t off = ((reinterpret_cast<size_t>(tw + 2 * M) - reinterpret_cast<size_t>(smem)) + 15) & ~size_t(15);
    C* buf1 = reinterpret_cast<C*>(smem + off);
    double2* pt = reinterpret_cast<double2*>(smem + off);  // staged p rows (periodic in y)
    double2* rt = pt + (lb + 2) * M;                        // staged rho rows
    const size_t plane = (size_t)nx * g.ny;

    const double rho0 = (MODE == FWD_METHOD1) ? *a.rho0 : 0.0;
    const double two_r0 = 2.0 * rho0;
    const double mean = (MODE == FWD_RESID || (MODE == FWD_METHOD3 && a.mean)) ? *a.mean : 0.0;
    const double sc = ((MODE == FWD_CONST || MODE == FWD_METHOD3) && a.scale) ? a.scale[k] : 1.0;
    // Method III weights the residual by the cell density; a constant weight
    // (min rho) gives the Method-I iteration in the same pressure form
    const bool const_w = MODE == FWD_METHOD3 && a.rho0 != nullptr;
    const double omega = const_w ? *a.rho0 : 0.0;
    const double idx2 = g.inv_dx * g.inv_dx, idy2 = g.inv_dy * g.inv_dy;
    const bool has_t = k + 1 < g.nz, has_b = k > 0;
    const double igt = has_t ? st.inv_g[k + 1] : 0.0, igb = has_b ? st.inv_g[k] : 0.0;
    const double ih = st.inv_h[k];
    double res2 = 0.0, r2 = 0.0, rsum = 0.0, qabs = 0.0;
    // Method III without a pressure iterate reads p as 0
    const bool has_p = MODE != FWD_METHOD3 || a.pprev != nullptr;
    // One thread per pair of cells (2n, 2n+1): exactly the packed input
    // z_n = r_{2n} + i r_{2n+1} of the half-length transform. The global
    // operands of a thread's next PF pairs are loaded into registers together:
    // with STAGE, f (or r_in) and p, rho on the planes k +- 1, issued before
    // the rows j0-1 .. j0+lb of p and rho are staged in LDS for the in-plane
    // neighbours, so the two loads overlap; without, every operand (the pair,
    // its y and z neighbour pairs and, unless the neighbouring lanes hold them,
    // its two x neighbours), where the caches serve the rows that neighbouring
    // pairs and tiles share. The autotuner picks the faster of the two per grid.
    struct Pre {
        double2 f, pc, pn, ps, ptz, pbz, rc, rn, rs, rtz, rbz;
        double pw, pe, rw, re;
    };
    constexpr int PF = (MODE == FWD_CONST || STAGE) ? 2 : 1;
    // Without staging, the x neighbours of a pair (cell 2n-1 is the .y of pair
    // n-1, cell 2n+2 the .x of pair n+1) come from the neighbouring lanes
    // where a wave holds whole lines (N divides 64: groups of N lanes, wrapping
    // periodically) or 64 consecutive pairs of one line (64 divides N: only a
    // wave's first and last lanes load theirs). Pairs map to lanes in order, so
    // lane exchanges replace two loads per field.
    constexpr bool XLANE = !STAGE && N > 0 && (64 % N == 0 || N % 64 == 0);
    constexpr int XG = (N > 0 && N < 64) ? N : 64;  // lanes per exchange group
    const double* pd = a.pprev;
    const double* rd = a.rho;
    const int npair = lb * M;
    const double2* fg = reinterpret_cast<const double2*>(MODE == FWD_RESID ? a.r_in : a.f);
    const double2* pg = reinterpret_cast<const double2*>(a.pprev);
    const double2* rg = reinterpret_cast<const double2*>(a.rho);
    auto pair_index = [&](int t) {
        const int line = t / M;
        return (((size_t)k * g.ny + j0 + line) * nx) / 2 + (t - line * M);  // double2 index
    };
    auto prefetch = [&](int t0, Pre* pre) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int t = t0 + u * 256;
            Pre& q = pre[u];
            q.pc = q.pn = q.ps = q.ptz = q.pbz = double2{0.0, 0.0};
            q.rc = q.rn = q.rs = q.rtz = q.rbz = double2{1.0, 1.0};
            q.pw = q.pe = 0.0;
            q.rw = q.re = 1.0;
            if (t < npair) {
                const size_t c2 = pair_index(t);
                q.f = fg[c2];
                if (MODE != FWD_CONST && STAGE) {
                    if (has_p) {
                        if (has_t) q.ptz = pg[c2 + plane / 2];
                        if (has_b) q.pbz = pg[c2 - plane / 2];
                    }
                    if (MODE == FWD_METHOD1 || MODE == FWD_METHOD3) {
                        if (has_t) q.rtz = rg[c2 + plane / 2];
                        if (has_b) q.rbz = rg[c2 - plane / 2];
                    }
                } else if (MODE != FWD_CONST) {
                    const int line = t / M, n = t - line * M, j = j0 + line;
                    // neighbour pairs in y (periodic) and cells in x (periodic in the line)
                    const size_t cn = c2 + (size_t)((j + 1 == g.ny) ? -(g.ny - 1) * M : M);
                    const size_t cs = c2 - (size_t)((j == 0) ? -(g.ny - 1) * M : M);
                    const size_t xw = 2 * c2 + (n == 0 ? nx - 1 : -1);
                    const size_t xe = 2 * c2 + (n + 1 == M ? 2 - nx : 2);
                    const int lane = t & 63;
                    const bool ld_w = !XLANE || (N > 64 && lane == 0);
                    const bool ld_e = !XLANE || (N > 64 && lane == 63);
                    if (has_p) {
                        q.pc = pg[c2];
                        q.pn = pg[cn];
                        q.ps = pg[cs];
                        if (ld_w) q.pw = pd[xw];
                        if (ld_e) q.pe = pd[xe];
                        if (has_t) q.ptz = pg[c2 + plane / 2];
                        if (has_b) q.pbz = pg[c2 - plane / 2];
                    }
                    if (MODE == FWD_METHOD1 || MODE == FWD_METHOD3) {
                        q.rc = rg[c2];
                        q.rn = rg[cn];
                        q.rs = rg[cs];
                        if (ld_w) q.rw = rd[xw];
                        if (ld_e) q.re = rd[xe];
                        if (has_t) q.rtz = rg[c2 + plane / 2];
                        if (has_b) q.rbz = rg[c2 - plane / 2];
                    }
                }
            }
        }
    };
    Pre cur[PF];
    prefetch(threadIdx.x, cur);
    // The twiddles and (with STAGE) the rows j0-1 .. j0+lb of p and rho
    // (periodic in y; p reads as 0 without an iterate) go to LDS. Compile-time
    // lengths: the rows (FP64 at either spectrum precision) and FP64 twiddles
    // by direct-to-LDS loads, in 64-entry chunks (one per wave instruction),
    // the waves taking every fourth chunk, nothing passing through registers;
    // FP32 twiddles (8-byte entries whose LDS slot is only 8-byte aligned)
    // wait in registers meanwhile. Runtime lengths: through registers, every
    // load of a thread issued before its LDS writes (a p element and the rho
    // element at the same place share their address).
    {
        constexpr bool ROWS = MODE != FWD_CONST && STAGE;
        constexpr bool RHO = MODE == FWD_METHOD1 || MODE == FWD_METHOD3;
        constexpr bool DMA = N > 0;
        const int nst = ROWS ? (lb + 2) * M : 0;
        const size_t kbase = (size_t)k * g.ny * M;
        auto row_j = [&](int rr) {
            int j = j0 - 1 + rr;
            j += (j < 0) ? g.ny : 0;
            j -= (j >= g.ny) ? g.ny : 0;
            return j;
        };
        if constexpr (DMA) {
            constexpr bool TWD = std::is_same<TC, double>::value;  // twiddles by direct loads
            constexpr int TWP = (2 * N + 255) / 256;
            C twr[TWD ? 1 : TWP];
            if constexpr (!TWD) {
#pragma unroll
                for (int j = 0; j < TWP; ++j) {
                    const int t = (int)threadIdx.x + 256 * j;
                    twr[j] = tw_g[t < 2 * N ? t : 0];
                }
            }
            constexpr int CPR = (N + 63) / 64;                 // chunks per row
            constexpr int CTW = TWD ? (2 * N + 63) / 64 : 0;  // chunks of twiddles
            const int prow = ROWS && has_p ? lb + 2 : 0;
            const int nrow = prow + (ROWS && RHO ? lb + 2 : 0);
            const int nch = nrow * CPR + CTW;
            const int lane = (int)threadIdx.x & 63;
            // the chunk arithmetic is the same on every lane of a wave: scalar
            const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
            for (int c = wave; c < nch; c += 4) {
                if (c < nrow * CPR) {
                    const int row = c / CPR, part = c - row * CPR;
                    const bool rho_row = row >= prow;
                    const int rr = rho_row ? row - prow : row;
                    const size_t sb = kbase + (size_t)row_j(rr) * M + part * 64;
                    double2* dst = (rho_row ? rt : pt) + rr * M + part * 64;
                    if (part * 64 + lane < M) lds_dma16((rho_row ? rg : pg) + sb + lane, dst);
                } else if constexpr (TWD) {
                    const int e = (c - nrow * CPR) * 64;
                    if (e + lane < 2 * M) lds_dma16(tw_g + e + lane, tw + e);
                }
            }
            if constexpr (!TWD) {
#pragma unroll
                for (int j = 0; j < TWP; ++j) {
                    const int t = (int)threadIdx.x + 256 * j;
                    if (t < 2 * N) tw[t] = twr[j];
                }
            }
            if (ROWS && !has_p)
                for (int t = threadIdx.x; t < nst; t += 256) pt[t] = double2{0.0, 0.0};
            lds_dma_wait();
        } else {
            constexpr int TWP = N > 0 ? (2 * N + 255) / 256 : 1;
            C twr[TWP];
            if constexpr (N > 0) {
#pragma unroll
                for (int j = 0; j < TWP; ++j) {
                    const int t = (int)threadIdx.x + 256 * j;
                    twr[j] = tw_g[t < 2 * N ? t : 0];
                }
            }
            auto src = [&](int t) {
                const int rr = t / M;
                return kbase + (size_t)row_j(rr) * M + (t - rr * M);
            };
            if constexpr (ROWS && RHO) {
                struct PR {
                    double2 p, r;
                };
                const double2* pv = has_p ? pg : rg;  // a valid array where p is absent
                block_copy<4, PR>(
                    nst,
                    [&](int t) {
                        const size_t i = src(t);
                        return PR{pv[i], rg[i]};
                    },
                    [&](int t, PR v) {
                        pt[t] = has_p ? v.p : double2{0.0, 0.0};
                        rt[t] = v.r;
                    });
            } else if constexpr (ROWS) {
                block_copy<4, double2>(nst, [&](int t) { return pg[src(t)]; },
                                       [&](int t, double2 v) { pt[t] = v; });
            }
            if constexpr (N > 0) {
#pragma unroll
                for (int j = 0; j < TWP; ++j) {
                    const int t = (int)threadIdx.x + 256 * j;
                    if (t < 2 * N) tw[t] = twr[j];
                }
            } else {
                block_copy<2, C>(2 * M, [&](int t) { return tw_g[t]; }, [&](int t, C v) { tw[t] = v; });
            }
        }
        __syncthreads();
    }
    // x neighbours by lane exchange: every lane of a group takes part (whole
    // groups are active together, as npair is a multiple of XG)
    auto x_nb = [&](const double2& c, double w_loaded, double e_loaded, double& w, double& e) {
        if constexpr (XLANE) {
            const int lane = threadIdx.x & 63;
            const int g0 = lane & ~(XG - 1), li = lane & (XG - 1);
            const double wl = __shfl(c.y, g0 + ((li + XG - 1) & (XG - 1)), 64);
            const double el = __shfl(c.x, g0 + ((li + 1) & (XG - 1)), 64);
            w = (N > 64 && lane == 0) ? w_loaded : wl;
            e = (N > 64 && lane == 63) ? e_loaded : el;
        } else {
            w = w_loaded;
            e = e_loaded;
        }
    };
    // The west face of pair n is the east face of pair n-1 (same operands in
    // the same order): with lane exchange it comes from the west lane (the
    // first lane of a 64-pair segment of a longer line evaluates its own).
    auto west_face = [&](double fe, auto own) -> double {
        if constexpr (XLANE) {
            const int lane = threadIdx.x & 63;
            const int g0 = lane & ~(XG - 1), li = lane & (XG - 1);
            const double w = __shfl(fe, g0 + ((li + XG - 1) & (XG - 1)), 64);
            if constexpr (N > 64) return lane == 0 ? own() : w;
            return w;
        } else {
            return own();
        }
    };
    // in-plane neighbours of pair n of a line: from the staged rows or the registers
    auto p_nb = [&](const Pre& q, int line, int n, double2& pc, double2& pn, double2& ps, double& pw,
                    double& pe) {
        if constexpr (STAGE) {
            const double2* Pr = pt + (line + 1) * M;
            pc = Pr[n];
            pn = Pr[n + M];
            ps = Pr[n - M];
            pw = Pr[n == 0 ? M - 1 : n - 1].y;
            pe = Pr[n + 1 == M ? 0 : n + 1].x;
        } else {
            pc = q.pc;
            pn = q.pn;
            ps = q.ps;
            x_nb(pc, q.pw, q.pe, pw, pe);
        }
    };
    auto r_nb = [&](const Pre& q, int line, int n, double2& rc, double2& rn, double2& rs, double& rw,
                    double& re) {
        if constexpr (STAGE) {
            const double2* Rr = rt + (line + 1) * M;
            rc = Rr[n];
            rn = Rr[n + M];
            rs = Rr[n - M];
            rw = Rr[n == 0 ? M - 1 : n - 1].y;
            re = Rr[n + 1 == M ? 0 : n + 1].x;
        } else {
            rc = q.rc;
            rn = q.rn;
            rs = q.rs;
            x_nb(rc, q.rw, q.re, rw, re);
        }
    };
    for (int t0 = threadIdx.x; t0 < npair; t0 += PF * 256) {
        if (t0 != (int)threadIdx.x) prefetch(t0, cur);
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int t = t0 + u * 256;
            if (t >= npair) break;
            const int line = t / M;
            const int n = t - line * M;
            const size_t c2 = pair_index(t);
            const Pre& q = cur[u];
            double v0, v1;
            if (MODE == FWD_CONST) {
                v0 = q.f.x * sc;
                v1 = q.f.y * sc;
            } else {
                double2 pc, pn, ps;
                double pw, pe;
                p_nb(q, line, n, pc, pn, ps, pw, pe);
                const double2 ptz = q.ptz, pbz = q.pbz;
                if (MODE == FWD_METHOD1) {
                    double2 rc, rn, rs;
                    double rw, re;
                    r_nb(q, line, n, rc, rn, rs, rw, re);
                    const double2 rtz = q.rtz, rbz = q.rbz;
                    // x faces: west of 2n, between the pair, east of 2n+1
                    const double fm = bflux(rc.x, rc.y, pc.x, pc.y, two_r0);
                    const double fe = bflux(rc.y, re, pc.y, pe, two_r0);
                    const double fw = west_face(fe, [&] { return bflux(rw, rc.x, pw, pc.x, two_r0); });
                    double d0 = (fm - fw) * idx2, d1 = (fe - fm) * idx2;
                    d0 += (bflux(rc.x, rn.x, pc.x, pn.x, two_r0) - bflux(rs.x, rc.x, ps.x, pc.x, two_r0)) * idy2;
                    d1 += (bflux(rc.y, rn.y, pc.y, pn.y, two_r0) - bflux(rs.y, rc.y, ps.y, pc.y, two_r0)) * idy2;
                    const double t0z = has_t ? bflux(rc.x, rtz.x, pc.x, ptz.x, two_r0) * igt : 0.0;
                    const double t1z = has_t ? bflux(rc.y, rtz.y, pc.y, ptz.y, two_r0) * igt : 0.0;
                    const double b0z = has_b ? bflux(rbz.x, rc.x, pbz.x, pc.x, two_r0) * igb : 0.0;
                    const double b1z = has_b ? bflux(rbz.y, rc.y, pbz.y, pc.y, two_r0) * igb : 0.0;
                    d0 += (t0z - b0z) * ih;
                    d1 += (t1z - b1z) * ih;
                    v0 = d0 + rho0 * q.f.x;
                    v1 = d1 + rho0 * q.f.y;
                } else if (MODE == FWD_METHOD3) {
                    // q = f - D(rho_f^-1 G p), r = rho q (cell density, Eq. new_poisson in
                    // pressure form)
                    double2 rc, rn, rs;
                    double rw, re;
                    r_nb(q, line, n, rc, rn, rs, rw, re);
                    const double2 rtz = q.rtz, rbz = q.rbz;
                    const double fm = gflux(rc.x, rc.y, pc.x, pc.y);
                    const double fe = gflux(rc.y, re, pc.y, pe);
                    const double fw = west_face(fe, [&] { return gflux(rw, rc.x, pw, pc.x); });
                    double d0 = (fm - fw) * idx2, d1 = (fe - fm) * idx2;
                    d0 += (gflux(rc.x, rn.x, pc.x, pn.x) - gflux(rs.x, rc.x, ps.x, pc.x)) * idy2;
                    d1 += (gflux(rc.y, rn.y, pc.y, pn.y) - gflux(rs.y, rc.y, ps.y, pc.y)) * idy2;
                    const double t0z = has_t ? gflux(rc.x, rtz.x, pc.x, ptz.x) * igt : 0.0;
                    const double t1z = has_t ? gflux(rc.y, rtz.y, pc.y, ptz.y) * igt : 0.0;
                    const double b0z = has_b ? gflux(rbz.x, rc.x, pbz.x, pc.x) * igb : 0.0;
                    const double b1z = has_b ? gflux(rbz.y, rc.y, pbz.y, pc.y) * igb : 0.0;
                    d0 += (t0z - b0z) * ih;
                    d1 += (t1z - b1z) * ih;
                    const double q0 = (q.f.x * sc - mean) - d0, q1 = (q.f.y * sc - mean) - d1;
                    qabs += fabs(q0) + fabs(q1);
                    v0 = (const_w ? omega : rc.x) * q0;
                    v1 = (const_w ? omega : rc.y) * q1;
                } else {  // residual r - mean - L p
                    double l0 = ((pc.y - pc.x) - (pc.x - pw)) * idx2;
                    double l1 = ((pe - pc.y) - (pc.y - pc.x)) * idx2;
                    l0 += ((pn.x - pc.x) - (pc.x - ps.x)) * idy2;
                    l1 += ((pn.y - pc.y) - (pc.y - ps.y)) * idy2;
                    l0 += ((has_t ? (ptz.x - pc.x) * igt : 0.0) - (has_b ? (pc.x - pbz.x) * igb : 0.0)) * ih;
                    l1 += ((has_t ? (ptz.y - pc.y) * igt : 0.0) - (has_b ? (pc.y - pbz.y) * igb : 0.0)) * ih;
                    const double rp0 = q.f.x - mean, rp1 = q.f.y - mean;
                    v0 = rp0 - l0;
                    v1 = rp1 - l1;
                    res2 += v0 * v0 + v1 * v1;
                    r2 += rp0 * rp0 + rp1 * rp1;
                }
            }
            if (a.r_out) reinterpret_cast<double2*>(a.r_out)[c2] = double2{v0, v1};
            rsum += v0 + v1;
            buf0[P::at(line * M + n)] = C{(TC)v0, (TC)v1};
        }
    }
    if (MODE == FWD_METHOD3 && a.partials_abs) {
        const double s1 = block_sum(qabs, red);
        if (threadIdx.x == 0) a.partials_abs[b] = s1;
        __syncthreads();
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
    C* Z = lds_fft_n<N, -1, 2, P>(buf0, buf1, M, g.lb, M, g.rad, tw);
    // Split the half-length transform into the real-input spectrum:
    //   E_m = (Z_m + conj Z_{M-m}) / 2, O_m = (Z_m - conj Z_{M-m}) / (2i),
    //   X_m = E_m + exp(-2 pi i m / nx) O_m, m = 0..M.
    const int nout = (M + 1) * g.lb;
    const size_t plane_s = (size_t)g.mx * g.ny;
    for (int t = threadIdx.x; t < nout; t += 256) {
        const int m = t / g.lb;
        const int line = t - m * g.lb;
        const C zm = Z[P::at(line * M + (m == M ? 0 : m))];
        const C zc = cconj(Z[P::at(line * M + (m == 0 ? 0 : M - m))]);
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
    using P = XLayout<N>;
    C* buf0 = reinterpret_cast<C*>(smem);
    C* xb = buf0 + xbuf_span(g.lb * M);  // lb x (M+1), later reused as the FFT's second buffer
    C* tw = xb + inv_x_stage_span(M, g.lb);
    const size_t plane_s = (size_t)g.mx * g.ny;
    const int nin = (M + 1) * g.lb;
    const c2<TS>* sk = spec + (size_t)k * plane_s + j0;
    // Both branches stage the bins and the twiddles, then split the
    // half-length transform's input: Z_m = E_m + i O_m with
    // E_m = (X_m + conj X_{M-m}) / 2, O_m = (X_m - conj X_{M-m}) exp(+2 pi i m / nx) / 2,
    // m = 0..M-1.
    // FP64 compile-time lengths: the bins (in their load order t = m lb +
    // line) and the twiddles by direct-to-LDS loads, 64 entries per wave
    // instruction; the split reads bin m of line l at xb[m lb + l] and clears
    // the imaginary parts of the DC and Nyquist bins itself.
    constexpr bool DMA = std::is_same<TC, double>::value && std::is_same<TS, double>::value && N > 0;
    if constexpr (DMA) {
        const int lane = (int)threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
        const int cin = (nin + 63) / 64, nch = cin + (2 * M + 63) / 64;
        for (int c = wave; c < nch; c += 4) {
            if (c < cin) {
                const int t = c * 64 + lane;
                const int m = t / g.lb;
                if (t < nin) lds_dma16(sk + (size_t)m * g.ny + (t - m * g.lb), xb + c * 64);
            } else {
                const int e = (c - cin) * 64;
                if (e + lane < 2 * M) lds_dma16(tw_g + e + lane, tw + e);
            }
        }
        lds_dma_wait();
        __syncthreads();
        const int nzz = M * g.lb;
        for (int t = threadIdx.x; t < nzz; t += 256) {
            const int line = t / M;
            const int m = t - line * M;
            C xm = xb[m * g.lb + line];
            C xc = cconj(xb[(M - m) * g.lb + line]);
            if (m == 0) xm.y = xc.y = (TC)0;  // real DC (m = 0) and Nyquist (M - m = M) bins
            const C e = C{(TC)0.5 * (xm.x + xc.x), (TC)0.5 * (xm.y + xc.y)};
            const C d = C{(TC)0.5 * (xm.x - xc.x), (TC)0.5 * (xm.y - xc.y)};
            const C o = cmul(d, cconj(tw[m]));
            buf0[P::at(line * M + m)] = C{e.x - o.y, e.y + o.x};
        }
    } else {
        // one index space: the lb lines' M + 1 bins, then the 2 M twiddles
        block_copy<4, C>(
            nin + 2 * M,
            [&](int t) {
                const int m = t / g.lb;
                return t < nin ? cconv<C>(sk[(size_t)m * g.ny + (t - m * g.lb)]) : tw_g[t - nin];
            },
            [&](int t, C x) {
                if (t < nin) {
                    const int m = t / g.lb;
                    if (m == 0 || m == M) x.y = (TC)0;  // a real field has real DC and Nyquist bins
                    xb[(t - m * g.lb) * (M + 1) + m] = x;
                } else {
                    tw[t - nin] = x;
                }
            });
        __syncthreads();
        const int nzz = M * g.lb;
        for (int t = threadIdx.x; t < nzz; t += 256) {
            const int line = t / M;
            const int m = t - line * M;
            const C xm = xb[line * (M + 1) + m];
            const C xc = cconj(xb[line * (M + 1) + (M - m)]);
            const C e = C{(TC)0.5 * (xm.x + xc.x), (TC)0.5 * (xm.y + xc.y)};
            const C d = C{(TC)0.5 * (xm.x - xc.x), (TC)0.5 * (xm.y - xc.y)};
            const C o = cmul(d, cconj(tw[m]));
            buf0[P::at(line * M + m)] = C{e.x - o.y, e.y + o.x};
        }
    }
    __syncthreads();
    C* z = lds_fft_n<N, +1, 2, P>(buf0, xb, M, g.lb, M, g.rad, tw);
    const double s = (MODE == INV_SCALE) ? scale * vol[k] : scale;
    // z_n = x_{2n} + i x_{2n+1}: one 16-byte store per pair of cells
    double2* out2 = reinterpret_cast<double2*>(out);
    const int npair = g.lb * M;
    for (int t = threadIdx.x; t < npair; t += 256) {
        const int line = t / M;
        const int n = t - line * M;
        const C v = z[P::at(t)];
        const size_t c2 = (((size_t)k * g.ny + j0 + line) * (2 * M)) / 2 + n;
        double2 x{(double)v.x * s, (double)v.y * s};
        if (MODE == INV_ADD) {
            const double2 o = out2[c2];
            x.x += o.x;
            x.y += o.y;
        }
        st_stream(out2 + c2, x);
    }
}

// Geometry of the x tiles; `inverse` selects the inverse pass's lines per block.
inline XGeom make_xgeom(const Plan& p, bool inverse = false) {
    XGeom g;
    g.nx = p.nx;
    g.ny = p.ny;
    g.nz = p.nz;
    g.mx = p.mx;
    g.M = p.nx / 2;
    g.lb = inverse ? p.lp.lbx_inv : p.lp.lbx;
    g.tiles = p.ny / g.lb;
    g.stage = p.lp.xstage;
    g.win = (!inverse && p.lp.xorder && g.tiles % 8 == 0) ? g.tiles / 8 : 0;
    g.inv_dx = 1.0 / p.dx;
    g.inv_dy = 1.0 / p.dy;
    g.rad = p.rad_xh;
    return g;
}

}  // namespace psv
