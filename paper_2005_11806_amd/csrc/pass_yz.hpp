// y and z passes of the eigenexpansion solve (Sec. 3.3.1) as block-level
// tile functions (256 threads), shared by the per-pass kernels and the
// persistent batch kernel.
//
// The spectrum keeps one layout, [k][m][n] (plane k, x wavenumber m, y
// wavenumber n; y lines contiguous), through every pass. For every
// wavenumber pair (m, n) != (0, 0) the wall-normal system
//     a_k x_{k-1} + (b_k + lx[m] + ly[n]) x_k + c_k x_{k+1} = R_k
// is solved by a partition method whose chunks are the y tiles themselves:
//  * forward y tile: kc consecutive planes of one m, all n: the FFT along y
//    of its kc lines, then, per n, the local elimination of the chunk's rows
//    (forward sweep, and a backward sweep that reduces row 0), leaving
//      row 0:      A x_{last of previous chunk} + x_first + C x_last = d_0
//      row i:      aa_i x_first + x_i + cc_i x_{i+1} = d_i   (0 < i < kc-1)
//      row kc-1:   aa x_first + x_last + cc x_{first of next chunk} = d_{kc-1}
//    written back in place;
//  * interface pass: per pair, the 2 nc rows (first, last) of its nc chunks
//    form a tridiagonal system with unit diagonal, solved with the Thomas
//    factors precomputed per plan (they do not depend on the data), its two
//    sweeps as affine scans over up to 8 lanes per pair; its tile 0 solves
//    the singular (0, 0) pair in FP64: projection of the right-hand side
//    (removal of its volume-weighted mean), flux integration from the bottom
//    wall, gauge sum_k h_k x_k = 0;
//  * inverse y tile: back substitution of the interior rows from x_first and
//    x_last, then the inverse FFT along y, in place.
// The elimination coefficients of every row are recomputed where they are
// needed (one division per row), so the z solve adds no pass over the
// spectrum: only the interface rows are read and written once more.
#pragma once

#include <type_traits>

#include "internal.hpp"

namespace psv {

// y-line lengths with a compile-time FFT (in place in one LDS buffer); other
// lengths use the runtime FFT, which ping-pongs between two buffers
#define PSV_YZ_SIZES(X) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(512)
inline bool yz_compiled(int ny) {
    switch (ny) {
#define PSV_CASE(n) case n:
        PSV_YZ_SIZES(PSV_CASE)
#undef PSV_CASE
        return true;
        default: return false;
    }
}

// LDS of a y tile: kc lines (padded by one element per 8 for a compile-time
// length; two plain buffers of them for a runtime length) and the twiddles
inline size_t yz_lds(int ny, int kc, size_t csz) {
    const size_t lines = yz_compiled(ny) ? (size_t)kc * ny + (size_t)kc * ny / 8 : (size_t)2 * kc * ny;
    return (lines + ny) * csz;
}

// LDS layout of the tile's lines: padded for the compile-time lengths (all
// multiples of 8), plain for the runtime FFT
template <int N>
using YzLayout = std::conditional_t<(N > 0), Pad8, NoPad>;

struct ZArgs {
    int nz, mx, ny;
    int kc;          // rows per chunk = planes per y tile (4, 8 or 16)
    int nc;          // chunks per column, ceil(nz / kc)
    double nxny_lz;  // nx * ny * lz
    double lz;
    const double* za;
    const double* zb;
    const double* zc;
    const double* lamx;
    const double* lamy;
    const double* h;
    const double* g;  // centre gaps, g[k] between cells k-1 and k
    double* rhs_mean;
    const void* tab;  // interface factors (layout: ifc_tab_index), in the spectrum's precision
};

// Row k of the system with eigenvalue sum lam; rows k >= nz pad the last
// chunk as identity rows.
struct ZRow {
    double a, b, c;
};
__device__ __forceinline__ ZRow zrow(const ZArgs& z, int k, double lam) {
    if (k < z.nz) return ZRow{z.za[k], z.zb[k] + lam, z.zc[k]};
    return ZRow{0.0, 1.0, 0.0};
}

// Forward elimination of chunk row i given the reduced row i-1: row i
// becomes aa x_first + x_i + cc x_{i+1} = d (for i = 0, aa couples to the
// previous chunk's last unknown). Returns the pivot reciprocal.
template <typename T>
__device__ __forceinline__ double chunk_fwd(int i, const ZRow& w, T aa_prev, T cc_prev, T& aa,
                                            T& cc) {
    double r;
    if (i < 2) {
        r = rcp_nr(w.b);
        aa = (T)(w.a * r);
    } else {
        r = rcp_nr(w.b - w.a * (double)cc_prev);
        aa = (T)(-w.a * (double)aa_prev * r);
    }
    cc = (T)(w.c * r);
    return r;
}

template <typename T>
__device__ __forceinline__ c2<T> chunk_fwd_rhs(int i, const ZRow& w, double r, c2<T> d, c2<T> dp) {
    if (i < 2) return c2<T>{(T)(d.x * r), (T)(d.y * r)};
    return c2<T>{(T)((d.x - w.a * dp.x) * r), (T)((d.y - w.a * dp.y) * r)};
}

// One backward step over interior row i: with row i+1 in the form
// ab x_first + x_{i+1} + cb x_last = db, row i takes the same form.
template <typename T>
__device__ __forceinline__ void chunk_bwd(T aa, T cc, T& ab, T& cb) {
    ab = aa - cc * ab;
    cb = -cc * cb;
}
template <typename T>
__device__ __forceinline__ c2<T> chunk_bwd_rhs(c2<T> d, T cc, c2<T> db) {
    return c2<T>{d.x - cc * db.x, d.y - cc * db.y};
}
template <typename T>
__device__ __forceinline__ T chunk_row0_pivot(T cc0, T ab1) {
    return (T)1 / ((T)1 - cc0 * ab1);
}

// Local elimination of one system's chunk (rows col[i * stride], i < KC, in
// LDS), in registers: forward sweep, and the backward sweep that reduces row
// 0; rows 1..KC-1 keep their forward-swept right-hand sides.
template <typename T, int KC>
__device__ __forceinline__ void chunk_eliminate(const ZArgs& z, int k0, double lam, c2<T>* col,
                                                int stride) {
    using C = c2<T>;
    C d[KC];
    T aa[KC], cc[KC];
#pragma unroll
    for (int i = 0; i < KC; ++i) d[i] = col[i * stride];
    C dp{(T)0, (T)0};
    T ap = (T)0, cp = (T)0;
#pragma unroll
    for (int i = 0; i < KC; ++i) {
        const ZRow row = zrow(z, k0 + i, lam);
        const double r = chunk_fwd<T>(i, row, ap, cp, aa[i], cc[i]);
        d[i] = chunk_fwd_rhs<T>(i, row, r, d[i], dp);
        dp = d[i];
        ap = aa[i];
        cp = cc[i];
    }
    if constexpr (KC >= 3) {
        C db = d[KC - 2];
        T ab = aa[KC - 2], cb = cc[KC - 2];
#pragma unroll
        for (int i = KC - 3; i >= 1; --i) {
            db = chunk_bwd_rhs<T>(d[i], cc[i], db);
            chunk_bwd<T>(aa[i], cc[i], ab, cb);
        }
        const T r0 = chunk_row0_pivot<T>(cc[0], ab);
        d[0] = C{(d[0].x - cc[0] * db.x) * r0, (d[0].y - cc[0] * db.y) * r0};
    }
#pragma unroll
    for (int i = 0; i < KC; ++i) col[i * stride] = d[i];
}

// Back substitution of one system's chunk: rows 0 and KC-1 hold x_first and
// x_last, rows 1..KC-2 the forward-swept d_i; x_i = d_i - aa_i x_first -
// cc_i x_{i+1}, from i = KC-2 down. Rows i >= nl are padding (x = 0).
template <typename T, int KC>
__device__ __forceinline__ void chunk_substitute(const ZArgs& z, int k0, int nl, double lam,
                                                 c2<T>* col, int stride) {
    using C = c2<T>;
    if constexpr (KC >= 3) {
        C d[KC];
        T aa[KC], cc[KC];
#pragma unroll
        for (int i = 0; i < KC; ++i) d[i] = i < nl ? col[i * stride] : C{(T)0, (T)0};
        T ap = (T)0, cp = (T)0;
#pragma unroll
        for (int i = 0; i < KC - 1; ++i) {
            (void)chunk_fwd<T>(i, zrow(z, k0 + i, lam), ap, cp, aa[i], cc[i]);
            ap = aa[i];
            cp = cc[i];
        }
        const C xf = d[0];
        C xn = d[KC - 1];
#pragma unroll
        for (int i = KC - 2; i >= 1; --i) {
            xn = i < nl ? C{d[i].x - aa[i] * xf.x - cc[i] * xn.x, d[i].y - aa[i] * xf.y - cc[i] * xn.y}
                        : C{(T)0, (T)0};
            d[i] = xn;
        }
#pragma unroll
        for (int i = 1; i < KC - 1; ++i)
            if (i < nl) col[i * stride] = d[i];
    }
}

// FFT of the tile's lines: in place for a compile-time length N, else the
// runtime routine with the second buffer; returns the buffer with the result.
template <typename T, int N, int KC, int DIR>
__device__ __forceinline__ c2<T>* yz_fft(c2<T>* buf, int ny, int nlines, const Radices& rad,
                                         const c2<T>* tw) {
    if constexpr (N > 0) {
        fft_inplace<N, 0, DIR, 1, KC, YzLayout<N>>(buf, tw);
        return buf;
    } else {
        return lds_fft<DIR>(buf, buf + KC * ny, ny, nlines, ny, rad, tw, ny);
    }
}

// Stages the tile's lines (planes [k0, k0 + nl) of wavenumber m; rows past
// nl read as 0) and the twiddles into LDS.
template <typename T, int N, int KC>
__device__ __forceinline__ void yz_load(const ZArgs& z, const c2<T>* __restrict__ base, size_t SP,
                                        int nl, const c2<T>* __restrict__ tw_g, c2<T>* buf,
                                        c2<T>* tw) {
    using C = c2<T>;
    using P = YzLayout<N>;
    const int ny = N ? N : z.ny;
    // one index space: the KC lines, then the ny twiddles; rows past nl
    // load row 0 and are stored as 0
    const int nel = KC * ny;
    constexpr int G = N > 0 ? ((KC + 1) * N + 255) / 256 < 16 ? ((KC + 1) * N + 255) / 256 : 16 : 8;
    block_copy<G, C>(
        nel + ny,
        [&](int e) {
            const int i = e / ny, n = e - i * ny;
            return e < nel ? base[(size_t)(i < nl ? i : 0) * SP + n] : tw_g[e - nel];
        },
        [&](int e, C v) {
            if (e < nel)
                buf[P::at(e)] = e / ny < nl ? v : C{(T)0, (T)0};
            else
                tw[e - nel] = v;
        });
    __syncthreads();
}

// Number of buffer elements the tile's KC lines take in their layout.
template <int N, int KC>
__device__ __forceinline__ int yz_span(int ny) {
    return N ? KC * N + KC * N / 8 : KC * ny;
}

// Forward y tile b = c mx + m (chunk c, wavenumber m): FFT along y of planes
// [c KC, c KC + KC) and the local elimination of every system (m, n).
// N = ny as a compile-time constant, or 0 for the runtime-length FFT.
template <typename T, int N, int KC>
__device__ __forceinline__ void yz_fwd_tile(const ZArgs& z, const Radices& rad,
                                            c2<T>* __restrict__ spec, const c2<T>* __restrict__ tw_g,
                                            int b, unsigned char* smem) {
    using C = c2<T>;
    using P = YzLayout<N>;
    const int ny = N ? N : z.ny;
    C* buf = reinterpret_cast<C*>(smem);
    C* tw = buf + (N ? yz_span<N, KC>(ny) : 2 * KC * ny);  // exp(-2 pi i t / ny), t < ny
    const int c = b / z.mx, m = b - c * z.mx;
    const int k0 = c * KC;
    const int nl = min(KC, z.nz - k0);
    const size_t SP = (size_t)z.mx * ny;
    C* base = spec + (size_t)k0 * SP + (size_t)m * ny;
    yz_load<T, N, KC>(z, base, SP, nl, tw_g, buf, tw);
    C* d = yz_fft<T, N, KC, -1>(buf, ny, KC, rad, tw);
    for (int n = threadIdx.x; n < ny; n += 256) {
        if (m == 0 && n == 0) continue;  // the (0,0) pair is solved apart
        chunk_eliminate<T, KC>(z, k0, z.lamx[m] + z.lamy[n], d + P::at(n), P::at(ny));
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nl * ny; e += 256) {
        const int i = e / ny, n = e - i * ny;
        base[(size_t)i * SP + n] = d[P::at(e)];
    }
}

// Inverse y tile b = c mx + m: x_first and x_last of every system sit in rows
// 0 and KC-1 (written by the interface pass), the interior rows hold the
// forward-swept d_i; back substitution, then the inverse FFT along y.
template <typename T, int N, int KC>
__device__ __forceinline__ void yz_inv_tile(const ZArgs& z, const Radices& rad,
                                            c2<T>* __restrict__ spec, const c2<T>* __restrict__ tw_g,
                                            int b, unsigned char* smem) {
    using C = c2<T>;
    using P = YzLayout<N>;
    const int ny = N ? N : z.ny;
    C* buf = reinterpret_cast<C*>(smem);
    C* tw = buf + (N ? yz_span<N, KC>(ny) : 2 * KC * ny);
    const int c = b / z.mx, m = b - c * z.mx;
    const int k0 = c * KC;
    const int nl = min(KC, z.nz - k0);
    const size_t SP = (size_t)z.mx * ny;
    C* base = spec + (size_t)k0 * SP + (size_t)m * ny;
    yz_load<T, N, KC>(z, base, SP, nl, tw_g, buf, tw);
    for (int n = threadIdx.x; n < ny; n += 256) {
        if (m == 0 && n == 0) continue;
        chunk_substitute<T, KC>(z, k0, nl, z.lamx[m] + z.lamy[n], buf + P::at(n), P::at(ny));
    }
    __syncthreads();
    C* r = yz_fft<T, N, KC, +1>(buf, ny, nl, rad, tw);
    for (int e = threadIdx.x; e < nl * ny; e += 256) {
        const int i = e / ny, n = e - i * ny;
        base[(size_t)i * SP + n] = r[P::at(e)];
    }
}

// Calls f with the compile-time chunk rows matching kc (4, 8 or 16).
template <typename F>
__device__ __forceinline__ void with_kc(int kc, F&& f) {
    if (kc == 4)
        f(std::integral_constant<int, 4>{});
    else if (kc == 8)
        f(std::integral_constant<int, 8>{});
    else
        f(std::integral_constant<int, 16>{});
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// exclusive prefix sum over the 64 lanes
__device__ __forceinline__ double wave_excl_scan(double v) {
    const int lane = threadIdx.x & 63;
    double inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const double t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    return inc - v;
}

// (0,0) column (entry k at col[k * stride]), FP64, as a tile of its own: the
// block (any multiple of 64 threads) stages the real parts, h and g in LDS
// (one global round trip), then one wave solves from there; lane l owns rows [l C, (l+1) C). With
// r~_k = r_k - mean (mean = sum_k h_k r_k / lz, the projection), the flux
// through face k is phi_{k-1} = sum_{j<k} h_j r~_j and
// x_k = sum_{j<=k} g_j phi_{j-1} (x_0 = 0); then the gauge removes
// sum_k h_k x_k / lz.
inline size_t zero_mode_lds(int nz) { return ((size_t)3 * nz + 1) * sizeof(double); }

template <typename TS>
__device__ __forceinline__ void zero_mode_tile(const ZArgs& z, c2<TS>* col, size_t stride,
                                               unsigned char* smem) {
    double* r = reinterpret_cast<double*>(smem);
    double* hh = r + z.nz;
    double* gg = hh + z.nz;  // [nz + 1]
    for (int k = threadIdx.x; k < z.nz; k += blockDim.x) {
        r[k] = (double)col[(size_t)k * stride].x;
        hh[k] = z.h[k];
    }
    for (int k = threadIdx.x; k <= z.nz; k += blockDim.x) gg[k] = z.g[k];
    __syncthreads();
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    const int C = (z.nz + 63) / 64;
    const int k0 = min(lane * C, z.nz), k1 = min(k0 + C, z.nz);
    double s = 0.0;
    for (int k = k0; k < k1; ++k) s += hh[k] * r[k];
    s = wave_sum(s);
    const double mean = s / z.lz;
    if (lane == 0) *z.rhs_mean = s / z.nxny_lz;
    double t = 0.0;
    for (int k = k0; k < k1; ++k) t += hh[k] * (r[k] - mean);
    const double phi0 = wave_excl_scan(t);
    double u = 0.0, phi = phi0;
    for (int k = k0; k < k1; ++k) {
        if (k > 0) u += gg[k] * phi;
        phi += hh[k] * (r[k] - mean);
    }
    const double x0 = wave_excl_scan(u);
    double hx = 0.0, x = x0;
    phi = phi0;
    for (int k = k0; k < k1; ++k) {
        if (k > 0) x += gg[k] * phi;
        phi += hh[k] * (r[k] - mean);
        hx += hh[k] * x;
    }
    const double shift = wave_sum(hx) / z.lz;
    using T = decltype(c2<TS>::x);
    x = x0;
    phi = phi0;
    for (int k = k0; k < k1; ++k) {
        if (k > 0) x += gg[k] * phi;
        phi += hh[k] * (r[k] - mean);
        col[(size_t)k * stride] = c2<TS>{(T)(x - shift), (T)0};
    }
}

// plane of interface row r: first (even r) or last (odd r) row of chunk r/2
__device__ __forceinline__ int ifc_plane(const ZArgs& z, int r) {
    return (r >> 1) * z.kc + ((r & 1) ? z.kc - 1 : 0);
}

constexpr int IFC_THREADS = 256;  // threads per interface tile

// Lanes per interface system: up to 8 (so that a wave's access to one row
// covers 8 consecutive pairs, whole 128-byte lines of FP64 spectrum), as few
// as leave at most two rows per lane; more than 8 only to keep the rows per
// lane <= 16 (R > 128, i.e. nz / kc > 64).
__host__ __device__ inline int ifc_lanes(int R) {
    int L = 1;
    while (L < 8 && 2 * L < R) L *= 2;
    while (L < 64 && 16 * L < R) L *= 2;
    return L;
}

// Interface systems of one wavenumber pair: R = 2 nc rows on L lanes of a
// wave, Q consecutive rows per lane, spw = 64 / L systems per wave; W waves
// cover the S = mx ny pairs.
struct IfcShape {
    int R, L, Q, spw, W;
};
__host__ __device__ inline IfcShape ifc_shape(int nc, int S) {
    IfcShape h;
    h.R = 2 * nc;
    h.L = ifc_lanes(h.R);
    h.Q = (h.R + h.L - 1) / h.L;
    h.spw = 64 / h.L;
    h.W = (S + h.spw - 1) / h.spw;
    return h;
}

// Factor table layout, wave-blocked: for the wave of systems [w spw, (w+1)
// spw), row slot j < Q and component c (0: -A_r / den_r, 1: -c'_r (0 on the
// last row), 2: 1 / den_r), 64 consecutive entries, one per lane
// (lane = g spw + s - w spw for row r = g Q + j). Each table load of a wave
// is then one contiguous 64-entry access. Slots of no row (s >= S or
// r >= R) are loaded and discarded.
__host__ __device__ inline size_t ifc_tab_index(const IfcShape& h, int s, int r, int c) {
    const int w = s / h.spw, g = r / h.Q, j = r - g * h.Q;
    return (((size_t)w * h.Q + j) * 3 + c) * 64 + g * h.spw + (s - w * h.spw);
}
__host__ __device__ inline size_t ifc_tab_entries(const IfcShape& h) {
    return (size_t)h.W * h.Q * 3 * 64;
}

// One interface system on L lanes of a wave, Q <= QM consecutive rows per
// lane (rows g Q .. g Q + Q - 1 on the lane of group g). With the plan-time
// Thomas factors both sweeps are first-order affine recurrences,
//   forward   d'_r = -(A_r I_r) d'_{r-1} + I_r D_r,         d'_{-1} = 0,
//   backward  x_r  = -c'_r x_{r+1} + d'_r,                    x_R = 0, c'_{R-1} = 0,
// so each lane composes the maps of its rows, the L lanes of a system combine
// theirs by a log2(L)-step scan over the wave (shuffles), and every lane then
// applies its rows from the value coming in. One load and one store per row.
// Padding slots (j >= Q, r >= R) are identity maps in both directions; lanes
// with no system (s = 0, the zero mode, or s >= S) carry identity maps
// through the shuffles and store nothing.
template <typename T, int QM>
__device__ __forceinline__ void ifc_scan(const ZArgs& z, c2<T>* __restrict__ spec, int b) {
    using C = c2<T>;
    const int S = z.mx * z.ny;
    const IfcShape h = ifc_shape(z.nc, S);
    const int R = h.R, L = h.L, Q = h.Q, spw = h.spw;
    const int lane = (int)threadIdx.x & 63;
    const int g = lane / spw;
    // the wave's first system, and its block of the factor table (the last
    // tile's waves past S read the last block and discard it)
    const int sw = __builtin_amdgcn_readfirstlane((b - 1) * (IFC_THREADS / L) +
                                                  ((int)threadIdx.x >> 6) * spw);
    const int s = sw + (lane - g * spw);
    const bool act = s < S && s != 0;
    const int r0 = g * Q;
    const T* tw = reinterpret_cast<const T*>(z.tab) +
                  (size_t)min(sw / spw, h.W - 1) * Q * 3 * 64 + lane;
    // 32-bit element offsets (every index here is below nx ny nz < 2^31)
    const unsigned us = (unsigned)s, uS = (unsigned)S;
    T al[QM], cm[QM];  // forward -A_r I_r, backward -c'_r (identity 1 on padding)
    C d[QM];           // I_r D_r, then d'_r (0 on padding)
    // Every slot is loaded unconditionally (slots j >= Q read slot 0; the
    // right-hand side of a slot without a row reads spectrum element s0 of
    // plane 0) and masked afterwards, so that all 4 QM loads of a lane are
    // in flight together; loads under per-row branches would each wait.
    const unsigned s0 = act ? us : 1u;
#pragma unroll
    for (int j = 0; j < QM; ++j) {
        const int r = r0 + j;
        const bool row = act && j < Q && r < R;
        const bool rhs = row && ifc_plane(z, r) < z.nz;
        const T* tj = tw + (size_t)(j < Q ? j : 0) * 3 * 64;
        const unsigned od = rhs ? (unsigned)ifc_plane(z, r) * uS + us : s0;
        const T A = ld_stream(tj), Cc = ld_stream(tj + 64), I = ld_stream(tj + 128);
        const C D = spec[od];
        al[j] = row ? A : (T)1;
        cm[j] = row ? Cc : (T)1;
        d[j] = rhs ? C{I * D.x, I * D.y} : C{(T)0, (T)0};
    }
    // forward: this lane's map d'_{r0-1} -> d'_{r0+Q-1}, then an inclusive scan
    T fa = (T)1;
    C fb{(T)0, (T)0};
#pragma unroll
    for (int j = 0; j < QM; ++j) {
        fa = al[j] * fa;
        fb = C{al[j] * fb.x + d[j].x, al[j] * fb.y + d[j].y};
    }
    for (int off = 1; off < L; off *= 2) {
        const int src = (lane - off * spw) & 63;
        const T pa = __shfl(fa, src, 64);
        const T px = __shfl(fb.x, src, 64), py = __shfl(fb.y, src, 64);
        if (g >= off) {
            fb = C{fa * px + fb.x, fa * py + fb.y};
            fa = fa * pa;
        }
    }
    // d'_{r0-1} is the scanned value of the previous group (0 for g = 0)
    const int prev = (lane - spw) & 63, next = (lane + spw) & 63;
    C v{__shfl(fb.x, prev, 64), __shfl(fb.y, prev, 64)};
    if (g == 0) v = C{(T)0, (T)0};
#pragma unroll
    for (int j = 0; j < QM; ++j) {
        v = C{al[j] * v.x + d[j].x, al[j] * v.y + d[j].y};
        if (act && j < Q && r0 + j < R) d[j] = v;
    }
    // backward: this lane's map x_{r0+Q} -> x_{r0}, then a suffix scan
    T ba = (T)1;
    C bb{(T)0, (T)0};
#pragma unroll
    for (int j = QM - 1; j >= 0; --j) {
        ba = cm[j] * ba;
        bb = C{cm[j] * bb.x + d[j].x, cm[j] * bb.y + d[j].y};
    }
    for (int off = 1; off < L; off *= 2) {
        const int src = (lane + off * spw) & 63;
        const T pa = __shfl(ba, src, 64);
        const T px = __shfl(bb.x, src, 64), py = __shfl(bb.y, src, 64);
        if (g + off < L) {
            bb = C{ba * px + bb.x, ba * py + bb.y};
            ba = ba * pa;
        }
    }
    C x{__shfl(bb.x, next, 64), __shfl(bb.y, next, 64)};
    if (g == L - 1) x = C{(T)0, (T)0};
#pragma unroll
    for (int j = QM - 1; j >= 0; --j) {
        x = C{cm[j] * x.x + d[j].x, cm[j] * x.y + d[j].y};
        const int r = r0 + j;
        if (act && j < Q && r < R && ifc_plane(z, r) < z.nz)
            spec[(unsigned)ifc_plane(z, r) * uS + us] = x;
    }
}

// Register rows per lane for R interface rows: 2, 4, 8 or 16 (nz / kc <= 512).
__host__ __device__ inline int ifc_qmax(int R) {
    const int q = (R + ifc_lanes(R) - 1) / ifc_lanes(R);
    return q <= 2 ? 2 : (q <= 4 ? 4 : (q <= 8 ? 8 : 16));
}

// Interface tile b: tile 0 is the (0,0) column; tile b >= 1 solves the
// interface systems of pairs [(b-1) P, b P), P = IFC_THREADS / L. Needs
// blockDim.x == IFC_THREADS and QM == ifc_qmax(2 nc) (QM = 0: chosen here).
template <typename T, int QM = 0>
__device__ __forceinline__ void ifc_tile(const ZArgs& z, c2<T>* __restrict__ spec, int b,
                                         unsigned char* smem) {
    if (b == 0) {
        zero_mode_tile<T>(z, spec, (size_t)z.mx * z.ny, smem);
        return;
    }
    if constexpr (QM > 0) {
        ifc_scan<T, QM>(z, spec, b);
    } else {
        const int q = ifc_qmax(2 * z.nc);
        if (q == 2)
            ifc_scan<T, 2>(z, spec, b);
        else if (q == 4)
            ifc_scan<T, 4>(z, spec, b);
        else if (q == 8)
            ifc_scan<T, 8>(z, spec, b);
        else
            ifc_scan<T, 16>(z, spec, b);
    }
}

// Interface factors of pair s (plan time; thread per pair, kc <= 64 rows of
// scratch per thread in LDS at [i][thread]): the coefficients (A, C) of the
// first and last row of every chunk, from the same sweeps as the y tiles,
// then the Thomas factors c'_r = C_r / den_r, 1/den_r with
// den_r = 1 - A_r c'_{r-1} (den_0 = 1), stored as the maps of the interface
// scans: -A_r / den_r, -c'_r, 1 / den_r. Computed in FP64 whatever the
// spectrum's precision and stored in it: for the near-singular low
// wavenumber pairs den_r is a difference of nearly equal terms, and an FP32
// recurrence would spoil the corrections of the mixed refinement (256x256x512
// tanh grid: relres 1.8e-10 after one sweep, against 1.1e-11 with the FP64
// table).
template <typename T>
__device__ __forceinline__ void ifc_table_pair(const ZArgs& z, int s, T* tab, c2<double>* scratch,
                                               int sstride) {
    using C = c2<double>;
    const int S = z.mx * z.ny;
    const IfcShape h = ifc_shape(z.nc, S);
    const int m = s / z.ny, n = s - m * z.ny;
    const double lam = z.lamx[m] + z.lamy[n];
    const int kc = z.kc;
    double cprev = 0.0;
    for (int c = 0; c < z.nc; ++c) {
        const int k0 = c * kc;
        double aa = 0.0, cc = 0.0;
        for (int i = 0; i < kc; ++i) {
            const ZRow row = zrow(z, k0 + i, lam);
            double na, ncc;
            (void)chunk_fwd<double>(i, row, aa, cc, na, ncc);
            scratch[i * sstride] = C{na, ncc};
            aa = na;
            cc = ncc;
        }
        const C w0 = scratch[0];
        const C wl = scratch[(kc - 1) * sstride];
        double A0 = w0.x, C0 = w0.y;
        if (kc >= 3) {
            double ab = scratch[(kc - 2) * sstride].x, cb = scratch[(kc - 2) * sstride].y;
            for (int i = kc - 3; i >= 1; --i) {
                const C wi = scratch[i * sstride];
                chunk_bwd<double>(wi.x, wi.y, ab, cb);
            }
            const double r0 = chunk_row0_pivot<double>(w0.y, ab);
            A0 = w0.x * r0;
            C0 = -w0.y * cb * r0;
        }
        const double rowA[2] = {A0, wl.x};
        const double rowC[2] = {C0, wl.y};
        for (int e = 0; e < 2; ++e) {
            const int r = 2 * c + e;
            const double inv = r == 0 ? 1.0 : 1.0 / (1.0 - rowA[e] * cprev);
            cprev = rowC[e] * inv;
            tab[ifc_tab_index(h, s, r, 0)] = (T)(-rowA[e] * inv);
            tab[ifc_tab_index(h, s, r, 1)] = (T)(r < h.R - 1 ? -cprev : 0.0);
            tab[ifc_tab_index(h, s, r, 2)] = (T)inv;
        }
    }
}

inline ZArgs make_zargs(const Plan& p, double* mean_out) {
    ZArgs z;
    z.nz = p.nz;
    z.mx = p.mx;
    z.ny = p.ny;
    z.kc = p.lp.kc;
    z.nc = (p.nz + p.lp.kc - 1) / p.lp.kc;
    z.lz = p.grid.lz;
    z.nxny_lz = (double)p.nx * p.ny * p.grid.lz;
    z.za = p.t.za;
    z.zb = p.t.zb;
    z.zc = p.t.zc;
    z.lamx = p.t.lamx;
    z.lamy = p.t.lamy;
    z.h = p.t.h;
    z.g = p.t.g;
    z.rhs_mean = mean_out;
    z.tab = p.ifc_tab;
    return z;
}

inline int yz_tiles(const Plan& p) { return p.mx * ((p.nz + p.lp.kc - 1) / p.lp.kc); }
inline int ifc_tiles(const Plan& p) {
    const int per = IFC_THREADS / ifc_lanes(2 * ((p.nz + p.lp.kc - 1) / p.lp.kc));
    return 1 + (p.mx * p.ny + per - 1) / per;
}
inline size_t ifc_lds(const Plan& p) { return zero_mode_lds(p.nz); }

}  // namespace psv
