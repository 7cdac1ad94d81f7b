// Per-pass kernels of the y and z directions (tile bodies in pass_yz.hpp).
#include "pass_yz.hpp"

namespace psv {
namespace {

template <typename TS, typename TC, int DIR, int N>
__global__ void __launch_bounds__(256) k_fft_y_t(int ny_rt, int nz, int mx, int kb, Radices rad,
                                                  const c2<TS>* __restrict__ in,
                                                  c2<TS>* __restrict__ out,
                                                  const c2<TC>* __restrict__ tw_g, const int* done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (done && *done) return;
    fft_y_tile<TS, TC, DIR, N>(ny_rt, nz, mx, kb, rad, in, out, tw_g, blockIdx.x, smem_raw);
}

template <typename T, int L>
__global__ void __launch_bounds__(256) k_tri_wave(ZArgs z, c2<T>* __restrict__ spec, const int* done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (done && *done) return;
    tri_tile<T, L>(z, spec, blockIdx.x, smem_raw);
}

// y-line lengths with a compile-time FFT; others use the runtime one
#define PSV_Y_SIZES(X) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(512)

template <typename T, int DIR>
void fft_y_dispatch(const Plan& p, int nblk, int kb, const c2<T>* in, c2<T>* out, const c2<T>* tw,
                    const int* done, hipStream_t s) {
    const size_t lds = fft_y_lds(p.ny, kb, sizeof(c2<T>));
    switch (p.ny) {
#define PSV_CASE(n)                                                                               \
    case n:                                                                                       \
        hipLaunchKernelGGL((k_fft_y_t<T, T, DIR, n>), dim3(nblk), dim3(256), lds, s, p.ny, p.nz, \
                           p.mx, kb, p.rad_y, in, out, tw, done);                                 \
        break;
        PSV_Y_SIZES(PSV_CASE)
#undef PSV_CASE
        default:
            hipLaunchKernelGGL((k_fft_y_t<T, T, DIR, 0>), dim3(nblk), dim3(256), lds, s, p.ny, p.nz,
                               p.mx, kb, p.rad_y, in, out, tw, done);
            break;
    }
}

template <typename T>
void tri_launch(const ZArgs& z, int L, int nblk, void* spec, const int* done, hipStream_t s) {
    c2<T>* sp = reinterpret_cast<c2<T>*>(spec);
    const size_t lds = tri_lds<T>(L);
    switch (L) {
        case 2: hipLaunchKernelGGL((k_tri_wave<T, 2>), dim3(nblk), dim3(256), lds, s, z, sp, done); break;
        case 4: hipLaunchKernelGGL((k_tri_wave<T, 4>), dim3(nblk), dim3(256), lds, s, z, sp, done); break;
        case 8: hipLaunchKernelGGL((k_tri_wave<T, 8>), dim3(nblk), dim3(256), lds, s, z, sp, done); break;
        case 16: hipLaunchKernelGGL((k_tri_wave<T, 16>), dim3(nblk), dim3(256), lds, s, z, sp, done); break;
        default: hipLaunchKernelGGL((k_tri_wave<T, 32>), dim3(nblk), dim3(256), lds, s, z, sp, done); break;
    }
}

}  // namespace

void launch_fft_y(const Plan& p, bool fp32, bool inverse, const int* done, hipStream_t s) {
    const int kb = p.lp.lby;
    const int nblk = fft_y_tiles(p);
    static const char* names[2][2] = {{"fft_y_fwd_fp64", "fft_y_inv_fp64"},
                                      {"fft_y_fwd_fp32", "fft_y_inv_fp32"}};
    TraceScope ts(p, names[fp32][inverse], s);
    if (fp32) {
        if (inverse)
            fft_y_dispatch<float, +1>(p, nblk, kb, (const float2*)p.spec_t, (float2*)p.spec, p.t.twy32, done, s);
        else
            fft_y_dispatch<float, -1>(p, nblk, kb, (const float2*)p.spec, (float2*)p.spec_t, p.t.twy32, done, s);
    } else {
        if (inverse)
            fft_y_dispatch<double, +1>(p, nblk, kb, (const double2*)p.spec_t, (double2*)p.spec, p.t.twy64, done, s);
        else
            fft_y_dispatch<double, -1>(p, nblk, kb, (const double2*)p.spec, (double2*)p.spec_t, p.t.twy64, done, s);
    }
    PSV_HIP(hipGetLastError());
}

void launch_thomas(const Plan& p, bool fp32, double* mean_out, const int* done, hipStream_t s) {
    const ZArgs z = make_zargs(p, mean_out);
    int L = 8, P = 1;
    tri_shape(p, L, P);
    const int nblk = tri_tiles(p);
    TraceScope ts(p, fp32 ? "thomas_z_fp32" : "thomas_z_fp64", s);
    if (fp32)
        tri_launch<float>(z, L, nblk, p.spec_t, done, s);
    else
        tri_launch<double>(z, L, nblk, p.spec_t, done, s);
    PSV_HIP(hipGetLastError());
}

}  // namespace psv
