// y and z passes of the eigenexpansion solve (Sec. 3.3.1):
//  * complex FFT along y over the contiguous lines spec[k][m][:];
//  * one tridiagonal solve along z per wavenumber pair (m, n) != (0, 0):
//      a_k x_{k-1} + (b_k + lx[m] + ly[n]) x_k + c_k x_{k+1} = R_k;
//  * the singular (0, 0) pair in FP64: projection of the right-hand side
//    (removal of its volume-weighted mean), flux integration from the bottom
//    wall, gauge sum_k h_k x_k = 0.
#include "internal.hpp"

namespace psv {
namespace {

template <typename TS, typename TC, int DIR>
__global__ void __launch_bounds__(256) k_fft_y(int ny, int nlines, int lb, Radices rad,
                                                c2<TS>* __restrict__ spec,
                                                const c2<TC>* __restrict__ tw, const int* done) {
    using C = c2<TC>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (done && *done) return;
    C* buf0 = reinterpret_cast<C*>(smem_raw);
    C* buf1 = buf0 + lb * ny;
    const int l0 = blockIdx.x * lb;
    const int nl = min(lb, nlines - l0);
    c2<TS>* base = spec + (size_t)l0 * ny;
    const int n = nl * ny;
    for (int t = threadIdx.x; t < n; t += blockDim.x) buf0[t] = cconv<C>(base[t]);
    __syncthreads();
    C* r = lds_fft<DIR>(buf0, buf1, ny, nl, ny, rad, tw, ny);
    for (int t = threadIdx.x; t < n; t += blockDim.x) base[t] = cconv<c2<TS>>(r[t]);
}

struct ZArgs {
    int nz, mx, ny;
    double nxny_lz;  // nx * ny * lz
    double lz;
    const double* za;
    const double* zb;
    const double* zc;
    const double* lamx;
    const double* lamy;
    const double* h;
    const double* inv_g;
    double* rhs_mean;
};

// (0,0) column, FP64, by one block: project, integrate twice, gauge.
template <typename TS>
__device__ void zero_mode(const ZArgs& z, c2<TS>* spec, double* col) {
    const size_t P = (size_t)z.mx * z.ny;
    for (int k = threadIdx.x; k < z.nz; k += blockDim.x) col[k] = (double)spec[(size_t)k * P].x;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < z.nz; ++k) s += z.h[k] * col[k];
        const double mean = s / z.lz;
        *z.rhs_mean = s / z.nxny_lz;
        // flux through face k+1: phi_k = sum_{j<=k} h_j (r_j - mean)
        // x_{k+1} = x_k + g_{k+1} phi_k, x_0 = 0
        double phi = 0.0, x = 0.0, hx = 0.0;
        double prev = 0.0;
        for (int k = 0; k < z.nz; ++k) {
            const double rk = col[k] - mean;
            if (k > 0) x = x + prev;
            col[k] = x;
            hx += z.h[k] * x;
            phi += z.h[k] * rk;
            prev = (k + 1 < z.nz) ? phi * (1.0 / z.inv_g[k + 1]) : 0.0;
        }
        col[z.nz] = hx / z.lz;
    }
    __syncthreads();
    const double shift = col[z.nz];
    for (int k = threadIdx.x; k < z.nz; k += blockDim.x) {
        using T = decltype(c2<TS>::x);
        spec[(size_t)k * P] = c2<TS>{(T)(col[k] - shift), (T)0};
    }
}

// Thread per wavenumber pair; the forward sweep stores the modified
// right-hand side in place and the pivots c'_k in `cp`.
template <typename T>
__global__ void __launch_bounds__(256) k_thomas(ZArgs z, c2<T>* __restrict__ spec,
                                                 T* __restrict__ cp, const int* done) {
    using C = c2<T>;
    __shared__ double col[2049];
    if (done && *done) return;
    const int S = z.mx * z.ny;
    const size_t P = (size_t)S;
    if (blockIdx.x == 0) zero_mode<T>(z, spec, col);
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0 || s >= S) return;
    const int m = s / z.ny;
    const int n = s - m * z.ny;
    const double lam = z.lamx[m] + z.lamy[n];
    double cpk = 0.0;
    C d{0, 0};
    for (int k = 0; k < z.nz; ++k) {
        const double ak = z.za[k];
        const double piv = z.zb[k] + lam - ak * cpk;
        const double inv = 1.0 / piv;
        cpk = z.zc[k] * inv;
        const C y = spec[(size_t)k * P + s];
        d = C{(T)(((double)y.x - ak * (double)d.x) * inv), (T)(((double)y.y - ak * (double)d.y) * inv)};
        cp[(size_t)k * P + s] = (T)cpk;
        spec[(size_t)k * P + s] = d;
    }
    C x = d;
    for (int k = z.nz - 2; k >= 0; --k) {
        const C dk = spec[(size_t)k * P + s];
        const T c = cp[(size_t)k * P + s];
        x = C{dk.x - c * x.x, dk.y - c * x.y};
        spec[(size_t)k * P + s] = x;
    }
}

}  // namespace

void launch_fft_y(const Plan& p, bool fp32, bool inverse, const int* done, hipStream_t s) {
    const int nlines = p.mx * p.nz;
    const int lb = p.lp.lby;
    const int nblk = (nlines + lb - 1) / lb;
    static const char* names[2][2] = {{"fft_y_fwd_fp64", "fft_y_inv_fp64"},
                                      {"fft_y_fwd_fp32", "fft_y_inv_fp32"}};
    TraceScope ts(p, names[fp32][inverse], s);
    if (fp32) {
        const size_t lds = (size_t)2 * lb * p.ny * sizeof(float2);
        if (inverse)
            hipLaunchKernelGGL((k_fft_y<float, float, +1>), dim3(nblk), dim3(p.lp.thr_y), lds, s,
                               p.ny, nlines, lb, p.rad_y, (float2*)p.spec, p.t.twy32, done);
        else
            hipLaunchKernelGGL((k_fft_y<float, float, -1>), dim3(nblk), dim3(p.lp.thr_y), lds, s,
                               p.ny, nlines, lb, p.rad_y, (float2*)p.spec, p.t.twy32, done);
    } else {
        const size_t lds = (size_t)2 * lb * p.ny * sizeof(double2);
        if (inverse)
            hipLaunchKernelGGL((k_fft_y<double, double, +1>), dim3(nblk), dim3(p.lp.thr_y), lds, s,
                               p.ny, nlines, lb, p.rad_y, (double2*)p.spec, p.t.twy64, done);
        else
            hipLaunchKernelGGL((k_fft_y<double, double, -1>), dim3(nblk), dim3(p.lp.thr_y), lds, s,
                               p.ny, nlines, lb, p.rad_y, (double2*)p.spec, p.t.twy64, done);
    }
    PSV_HIP(hipGetLastError());
}

void launch_thomas(const Plan& p, bool fp32, double* mean_out, const int* done, hipStream_t s) {
    ZArgs z;
    z.nz = p.nz;
    z.mx = p.mx;
    z.ny = p.ny;
    z.lz = p.grid.lz;
    z.nxny_lz = (double)p.nx * p.ny * p.grid.lz;
    z.za = p.t.za;
    z.zb = p.t.zb;
    z.zc = p.t.zc;
    z.lamx = p.t.lamx;
    z.lamy = p.t.lamy;
    z.h = p.t.h;
    z.inv_g = p.t.inv_g;
    z.rhs_mean = mean_out;
    const int S = p.mx * p.ny;
    const int thr = p.lp.thr_z;
    const int nblk = (S + thr - 1) / thr;
    TraceScope ts(p, fp32 ? "thomas_z_fp32" : "thomas_z_fp64", s);
    if (fp32)
        hipLaunchKernelGGL((k_thomas<float>), dim3(nblk), dim3(thr), 0, s, z, (float2*)p.spec,
                           (float*)p.cp, done);
    else
        hipLaunchKernelGGL((k_thomas<double>), dim3(nblk), dim3(thr), 0, s, z, (double2*)p.spec,
                           (double*)p.cp, done);
    PSV_HIP(hipGetLastError());
}

}  // namespace psv
