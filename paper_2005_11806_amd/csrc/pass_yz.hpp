// y and z passes of the eigenexpansion solve (Sec. 3.3.1) as block-level
// tile functions (256 threads), shared by the per-pass kernels and the
// persistent batch kernel.
//
// Spectrum layouts: A = [k][m][n] (written and read by the x passes, y lines
// contiguous) and B = [m][n][k] (one wall-normal system per contiguous column).
//  * forward y tile: FFT along y of the lines of A, stored transposed into B
//    (a tile is one m and kb consecutive planes, so every store run is kb
//    consecutive k);
//  * z tile: one tridiagonal solve per wavenumber pair (m, n) != (0, 0),
//      a_k x_{k-1} + (b_k + lx[m] + ly[n]) x_k + c_k x_{k+1} = R_k,
//    by a partition method in registers: P lanes per system each own L
//    consecutive rows, eliminate them to two interface rows, the 2P-row
//    interface system is solved by parallel cyclic reduction over wave
//    shuffles, then the interior rows are recovered;
//  * the singular (0, 0) pair in FP64: projection of the right-hand side
//    (removal of its volume-weighted mean), flux integration from the bottom
//    wall, gauge sum_k h_k x_k = 0;
//  * inverse y tile: B back to A with the inverse FFT along y.
#pragma once

#include "internal.hpp"

namespace psv {

inline size_t fft_y_lds(int ny, int kb, size_t csz) { return ((size_t)2 * kb * (ny + 1) + ny) * csz; }

// N = ny as a compile-time constant, or 0 for the runtime-length FFT.
template <typename TS, typename TC, int DIR, int N>
__device__ __forceinline__ void fft_y_tile(int ny_rt, int nz, int mx, int kb, const Radices& rad,
                                           const c2<TS>* __restrict__ in, c2<TS>* __restrict__ out,
                                           const c2<TC>* __restrict__ tw_g, int b,
                                           unsigned char* smem) {
    using C = c2<TC>;
    const int ny = N ? N : ny_rt;
    const int ls = ny + 1;  // padded line stride: transposed LDS accesses hit distinct banks
    C* buf0 = reinterpret_cast<C*>(smem);
    C* buf1 = buf0 + kb * ls;
    C* tw = buf1 + kb * ls;  // exp(-2 pi i t / ny), t < ny
    for (int t = threadIdx.x; t < ny; t += 256) tw[t] = tw_g[t];
    const int kchunks = (nz + kb - 1) / kb;
    const int m = b / kchunks;
    const int k0 = (b - m * kchunks) * kb;
    const int nl = min(kb, nz - k0);
    const int n_el = nl * ny;
    if (DIR < 0) {  // A -> LDS: nl contiguous lines of ny
        for (int t = threadIdx.x; t < n_el; t += 256) {
            const int q = t / ny, n = t - q * ny;
            buf0[q * ls + n] = cconv<C>(in[((size_t)(k0 + q) * mx + m) * ny + n]);
        }
    } else {  // B -> LDS: runs of nl consecutive k per n
        for (int t = threadIdx.x; t < n_el; t += 256) {
            const int n = t / nl, q = t - n * nl;
            buf0[q * ls + n] = cconv<C>(in[((size_t)m * ny + n) * nz + k0 + q]);
        }
    }
    __syncthreads();
    C* r = lds_fft_n<N, DIR, 1>(buf0, buf1, ny, nl, ls, rad, tw);
    if (DIR < 0) {  // LDS -> B
        for (int t = threadIdx.x; t < n_el; t += 256) {
            const int n = t / nl, q = t - n * nl;
            out[((size_t)m * ny + n) * nz + k0 + q] = cconv<c2<TS>>(r[q * ls + n]);
        }
    } else {  // LDS -> A
        for (int t = threadIdx.x; t < n_el; t += 256) {
            const int q = t / ny, n = t - q * ny;
            out[((size_t)(k0 + q) * mx + m) * ny + n] = cconv<c2<TS>>(r[q * ls + n]);
        }
    }
}

struct ZArgs {
    int nz, mx, ny;
    int P;           // lanes per system (power of 2, <= 64)
    float rcp_nz;    // 1/nz, for splitting staged element indices
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
};

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

// (0,0) column (contiguous in layout B), FP64, by one wave; lane l owns rows
// [l C, (l+1) C). With r~_k = r_k - mean (mean = sum_k h_k r_k / lz, the
// projection), the flux through face k is phi_{k-1} = sum_{j<k} h_j r~_j and
// x_k = sum_{j<=k} g_j phi_{j-1} (x_0 = 0); then the gauge removes
// sum_k h_k x_k / lz.
template <typename TS>
__device__ __forceinline__ void zero_mode_wave(const ZArgs& z, c2<TS>* colg) {
    const int lane = threadIdx.x & 63;
    const int C = (z.nz + 63) / 64;
    const int k0 = min(lane * C, z.nz), k1 = min(k0 + C, z.nz);
    double s = 0.0;
    for (int k = k0; k < k1; ++k) s += z.h[k] * (double)colg[k].x;
    s = wave_sum(s);
    const double mean = s / z.lz;
    if (lane == 0) *z.rhs_mean = s / z.nxny_lz;
    double t = 0.0;
    for (int k = k0; k < k1; ++k) t += z.h[k] * ((double)colg[k].x - mean);
    const double phi0 = wave_excl_scan(t);
    double u = 0.0, phi = phi0;
    for (int k = k0; k < k1; ++k) {
        if (k > 0) u += z.g[k] * phi;
        phi += z.h[k] * ((double)colg[k].x - mean);
    }
    const double x0 = wave_excl_scan(u);
    double hx = 0.0, x = x0;
    phi = phi0;
    for (int k = k0; k < k1; ++k) {
        if (k > 0) x += z.g[k] * phi;
        phi += z.h[k] * ((double)colg[k].x - mean);
        hx += z.h[k] * x;
    }
    const double shift = wave_sum(hx) / z.lz;
    // every lane has read its rows above; the writes below touch only them
    using T = decltype(c2<TS>::x);
    x = x0;
    phi = phi0;
    for (int k = k0; k < k1; ++k) {
        if (k > 0) x += z.g[k] * phi;
        phi += z.h[k] * ((double)colg[k].x - mean);
        colg[k] = c2<TS>{(T)(x - shift), (T)0};
    }
}

__device__ __forceinline__ double shfl_v(double v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ float shfl_v(float v, int src) { return __shfl(v, src, 64); }

// LDS of a tridiagonal tile: columns staged with one pad entry per partition
// (rows per lane L <= 8; longer chains read their rows from global memory)
template <typename T>
inline size_t tri_lds(int L) { return L <= 8 ? (size_t)256 * (L + 1) * sizeof(c2<T>) : 0; }

// Tridiagonal tile b: systems [b * 256/P, (b+1) * 256/P), whose columns are
// contiguous in layout B. For L <= 8 the block copies them to LDS with
// coalesced 16-byte loads (partition p of a system at offset p (L+1)), each
// lane then takes its L rows from there, and the solved columns go back the
// same way. Tile 0's first wave also solves the (0,0) column.
template <typename T, int L>
__device__ __forceinline__ void tri_tile(const ZArgs& z, c2<T>* __restrict__ spec, int b,
                                         unsigned char* smem) {
    using C = c2<T>;
    constexpr bool STAGE = L <= 8;
    const int S = z.mx * z.ny;
    if (b == 0 && threadIdx.x < 64) zero_mode_wave<T>(z, spec);
    const int P = z.P;
    const int lane = threadIdx.x & 63;
    const int p = lane & (P - 1);
    const int gbase = lane - p;  // first lane of this system's group
    const int sys_per_block = 256 / P;
    const int s0 = b * sys_per_block;
    const int sl = (int)(threadIdx.x / P);  // system within the tile
    const int s = s0 + sl;
    const bool active = (s < S) && (s != 0);
    const int k0 = p * L;
    C* colp = spec + (size_t)(active ? s : 0) * z.nz;
    C* lds = reinterpret_cast<C*>(smem);
    const int sstride = P * (L + 1);
    const int cnt = min(sys_per_block, S - s0) * z.nz;
    C d[L];
    T aa[L], cc[L];
    if constexpr (STAGE) {
        const C* src = spec + (size_t)s0 * z.nz;
        for (int e = threadIdx.x; e < cnt; e += 256) {
            // (system, row) of element e; the float estimate is off by at most one
            int q = (int)((float)e * z.rcp_nz);
            int r = e - q * z.nz;
            if (r < 0) { --q; r += z.nz; } else if (r >= z.nz) { ++q; r -= z.nz; }
            lds[q * sstride + (r / L) * (L + 1) + (r % L)] = src[e];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const int k = k0 + i;
            d[i] = (active && k < z.nz) ? lds[sl * sstride + p * (L + 1) + i] : C{(T)0, (T)0};
        }
    } else {
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const int k = k0 + i;
            d[i] = (active && k < z.nz) ? colp[k] : C{(T)0, (T)0};
        }
    }
    double lam = 0.0;
    if (active) {
        const int m = s / z.ny;
        lam = z.lamx[m] + z.lamy[s - m * z.ny];
    }
    // forward elimination: rows end as aa_i x_first + x_i + cc_i x_{i+1} = d_i
    // (row 0 keeps its coupling aa_0 to the previous partition's last unknown)
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const int k = k0 + i;
        double a = 0.0, bb = 1.0, c = 0.0;
        if (active && k < z.nz) {
            a = z.za[k];
            bb = z.zb[k] + lam;
            c = z.zc[k];
        }
        if (i < 2) {
            const double r = 1.0 / bb;
            aa[i] = (T)(a * r);
            cc[i] = (T)(c * r);
            d[i] = C{(T)(d[i].x * r), (T)(d[i].y * r)};
        } else {
            const double r = 1.0 / (bb - a * (double)cc[i - 1]);
            aa[i] = (T)(-a * (double)aa[i - 1] * r);
            cc[i] = (T)(c * r);
            d[i] = C{(T)((d[i].x - a * d[i - 1].x) * r), (T)((d[i].y - a * d[i - 1].y) * r)};
        }
    }
    // backward: rows 1..L-2 end as aa_i x_first + x_i + cc_i x_last = d_i
#pragma unroll
    for (int i = L - 3; i >= 1; --i) {
        d[i] = C{d[i].x - cc[i] * d[i + 1].x, d[i].y - cc[i] * d[i + 1].y};
        aa[i] = aa[i] - cc[i] * aa[i + 1];
        cc[i] = -cc[i] * cc[i + 1];
    }
    if (L >= 3) {
        const T r = (T)1 / ((T)1 - cc[0] * aa[1]);
        d[0] = C{(d[0].x - cc[0] * d[1].x) * r, (d[0].y - cc[0] * d[1].y) * r};
        aa[0] = aa[0] * r;
        cc[0] = -cc[0] * cc[1] * r;
    }
    // interface system of 2P rows, ordered (first_0, last_0, first_1, ...):
    //   A_i x_{i-1} + B_i x_i + C_i x_{i+1} = D_i, solved by cyclic reduction.
    T A[2] = {aa[0], aa[L - 1]};
    T B[2] = {(T)1, (T)1};
    T Cc[2] = {cc[0], cc[L - 1]};
    C D[2] = {d[0], d[L - 1]};
    const int nrow = 2 * P;
    for (int st = 1; st < nrow; st <<= 1) {
        T nA[2], nB[2], nC[2];
        C nD[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int i = 2 * p + e;
            const int jl = i - st, jr = i + st;
            const int sl = jl & 1, sr = jr & 1;  // uniform over the wave
            const int ll = (gbase + (jl >> 1)) & 63, lr = (gbase + (jr >> 1)) & 63;
            // values of rows jl and jr (identity rows outside 0..2P-1)
            const T la = shfl_v(sl ? A[1] : A[0], ll), lb = shfl_v(sl ? B[1] : B[0], ll);
            const T lc = shfl_v(sl ? Cc[1] : Cc[0], ll);
            const T ldx = shfl_v(sl ? D[1].x : D[0].x, ll), ldy = shfl_v(sl ? D[1].y : D[0].y, ll);
            const T ra = shfl_v(sr ? A[1] : A[0], lr), rb = shfl_v(sr ? B[1] : B[0], lr);
            const T rc = shfl_v(sr ? Cc[1] : Cc[0], lr);
            const T rdx = shfl_v(sr ? D[1].x : D[0].x, lr), rdy = shfl_v(sr ? D[1].y : D[0].y, lr);
            const bool hl = jl >= 0, hr = jr < nrow;
            const T al = hl ? -A[e] / lb : (T)0;
            const T ar = hr ? -Cc[e] / rb : (T)0;
            nA[e] = hl ? al * la : (T)0;
            nC[e] = hr ? ar * rc : (T)0;
            nB[e] = B[e] + (hl ? al * lc : (T)0) + (hr ? ar * ra : (T)0);
            nD[e] = C{D[e].x + (hl ? al * ldx : (T)0) + (hr ? ar * rdx : (T)0),
                      D[e].y + (hl ? al * ldy : (T)0) + (hr ? ar * rdy : (T)0)};
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            A[e] = nA[e];
            B[e] = nB[e];
            Cc[e] = nC[e];
            D[e] = nD[e];
        }
    }
    const C xf = C{D[0].x / B[0], D[0].y / B[0]};
    const C xl = C{D[1].x / B[1], D[1].y / B[1]};
#pragma unroll
    for (int i = 1; i < L - 1; ++i)
        d[i] = C{d[i].x - aa[i] * xf.x - cc[i] * xl.x, d[i].y - aa[i] * xf.y - cc[i] * xl.y};
    d[0] = xf;
    d[L - 1] = xl;
    if constexpr (STAGE) {
        // each lane rewrites only the slots it read; then the block stores the
        // tile coalesced, leaving the (0,0) column to the zero-mode wave
        if (active) {
#pragma unroll
            for (int i = 0; i < L; ++i)
                if (k0 + i < z.nz) lds[sl * sstride + p * (L + 1) + i] = d[i];
        }
        __syncthreads();
        C* dst = spec + (size_t)s0 * z.nz;
        for (int e = threadIdx.x; e < cnt; e += 256) {
            int q = (int)((float)e * z.rcp_nz);
            int r = e - q * z.nz;
            if (r < 0) { --q; r += z.nz; } else if (r >= z.nz) { ++q; r -= z.nz; }
            if (s0 + q != 0) dst[e] = lds[q * sstride + (r / L) * (L + 1) + (r % L)];
        }
    } else if (active) {
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const int k = k0 + i;
            if (k < z.nz) colp[k] = d[i];
        }
    }
}

// Rows per lane L and lanes per system P for a column of nz rows, starting
// from the preferred L (8 unless tuned): short chains keep the serial
// elimination short and give many waves; L grows only when 64 lanes per
// system would not cover the column.
inline void tri_shape(int nz, int& L, int& P, int prefer = 8) {
    if (nz <= 8 && prefer >= 8) {
        P = 1;
        L = 2;
        while (L < nz) L *= 2;
        return;
    }
    for (L = prefer; L <= 32; L *= 2) {
        P = 1;
        while (P * L < nz) P *= 2;
        if (P <= 64) return;
    }
    L = 32;
    P = 64;
}

inline void tri_shape(const Plan& p, int& L, int& P) { tri_shape(p.nz, L, P, p.lp.tri_L); }

inline ZArgs make_zargs(const Plan& p, double* mean_out) {
    ZArgs z;
    z.nz = p.nz;
    z.mx = p.mx;
    z.ny = p.ny;
    int L = 8, P = 1;
    tri_shape(p, L, P);
    z.P = P;
    z.rcp_nz = 1.0f / (float)p.nz;
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
    return z;
}

inline int tri_tiles(const Plan& p) {
    int L = 8, P = 1;
    tri_shape(p, L, P);
    const int spb = 256 / P;
    return (p.mx * p.ny + spb - 1) / spb;
}

inline int fft_y_tiles(const Plan& p) { return p.mx * ((p.nz + p.lp.lby - 1) / p.lp.lby); }

}  // namespace psv
