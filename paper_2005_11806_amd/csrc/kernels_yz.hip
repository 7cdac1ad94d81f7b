// Per-pass kernels of the y and z directions (tile bodies in pass_yz.hpp) and
// the plan-time interface factor table.
#include "pass_yz.hpp"

namespace psv {
namespace {

template <typename T, int N, int KC, bool INV>
__global__ void __launch_bounds__(256) k_yz(ZArgs z, Radices rad, c2<T>* __restrict__ spec,
                                            const c2<T>* __restrict__ tw_g, const int* done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (done && *done) return;
    if constexpr (INV)
        yz_inv_tile<T, N, KC>(z, rad, spec, tw_g, blockIdx.x, smem_raw);
    else
        yz_fwd_tile<T, N, KC>(z, rad, spec, tw_g, blockIdx.x, smem_raw);
}

// Two-dimensional problems (ny = 1): the y transform is the identity and a y
// tile would hold a single system, so here one thread takes the chunk of one
// wavenumber m (consecutive threads, consecutive m: the rows of a plane are
// read and written whole). Same arithmetic as the tiles: the forward chunk is
// eliminated in registers (rows past nz read as 0), the inverse one
// back-substituted in place.
template <typename T, int KC, bool INV>
__global__ void __launch_bounds__(256) k_z2d(ZArgs z, c2<T>* __restrict__ spec, const int* done) {
    if (done && *done) return;
    const int m = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (m == 0 || m >= z.mx) return;  // the (0,0) pair is solved apart
    const int k0 = (int)blockIdx.y * KC;
    const int nl = min(KC, z.nz - k0);
    const int SP = z.mx;  // elements per plane when ny = 1
    c2<T>* col = spec + (size_t)k0 * SP + m;
    const double lam = z.lamx[m] + z.lamy[0];
    if constexpr (INV) {
        chunk_substitute<T, KC>(z, k0, nl, lam, col, SP);
    } else {
        c2<T> v[KC];
#pragma unroll
        for (int i = 0; i < KC; ++i) v[i] = i < nl ? col[(size_t)i * SP] : c2<T>{(T)0, (T)0};
        chunk_eliminate<T, KC>(z, k0, lam, v, 1);
#pragma unroll
        for (int i = 0; i < KC; ++i)
            if (i < nl) col[(size_t)i * SP] = v[i];
    }
}

template <typename T, bool INV>
void z2d_launch(const Plan& p, const ZArgs& z, c2<T>* spec, const int* done, hipStream_t s) {
    const dim3 grid((p.mx + 255) / 256, (p.nz + p.lp.kc - 1) / p.lp.kc);
    switch (p.lp.kc) {
        case 4: hipLaunchKernelGGL((k_z2d<T, 4, INV>), grid, dim3(256), 0, s, z, spec, done); break;
        case 8: hipLaunchKernelGGL((k_z2d<T, 8, INV>), grid, dim3(256), 0, s, z, spec, done); break;
        default: hipLaunchKernelGGL((k_z2d<T, 16, INV>), grid, dim3(256), 0, s, z, spec, done); break;
    }
}

template <typename T, int QM>
__global__ void __launch_bounds__(IFC_THREADS) k_ifc(ZArgs z, c2<T>* __restrict__ spec, const int* done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (done && *done) return;
    ifc_tile<T, QM>(z, spec, blockIdx.x, smem_raw);
}

template <typename T, int QM>
void ifc_launch(const Plan& p, const ZArgs& z, const int* done, hipStream_t s) {
    const size_t lds = ifc_lds(p);
    allow_lds(k_ifc<T, QM>, lds);
    hipLaunchKernelGGL((k_ifc<T, QM>), dim3(ifc_tiles(p)), dim3(IFC_THREADS), lds, s, z,
                       reinterpret_cast<c2<T>*>(p.spec), done);
}

template <typename T>
void ifc_dispatch(const Plan& p, const ZArgs& z, const int* done, hipStream_t s) {
    switch (ifc_qmax(2 * z.nc)) {
        case 2: ifc_launch<T, 2>(p, z, done, s); break;
        case 4: ifc_launch<T, 4>(p, z, done, s); break;
        case 8: ifc_launch<T, 8>(p, z, done, s); break;
        default: ifc_launch<T, 16>(p, z, done, s); break;
    }
}

constexpr int TAB_THREADS = 64;

template <typename T>
__global__ void __launch_bounds__(TAB_THREADS) k_ifc_table(ZArgs z, T* __restrict__ tab) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int s = blockIdx.x * TAB_THREADS + (int)threadIdx.x;
    if (s >= z.mx * z.ny) return;
    c2<double>* scratch = reinterpret_cast<c2<double>*>(smem_raw) + threadIdx.x;
    ifc_table_pair<T>(z, s, tab, scratch, TAB_THREADS);
}

template <typename T, int N, int KC, bool INV>
void yz_launch(const Plan& p, const ZArgs& z, c2<T>* spec, const c2<T>* tw, const int* done,
               hipStream_t s) {
    const size_t lds = yz_lds(p.ny, KC, sizeof(c2<T>));
    allow_lds(k_yz<T, N, KC, INV>, lds);
    hipLaunchKernelGGL((k_yz<T, N, KC, INV>), dim3(yz_tiles(p)), dim3(256), lds, s, z, p.rad_y,
                       spec, tw, done);
}

template <typename T, int N, bool INV>
void yz_dispatch_kc(const Plan& p, const ZArgs& z, c2<T>* spec, const c2<T>* tw, const int* done,
                    hipStream_t s) {
    switch (p.lp.kc) {
        case 4: yz_launch<T, N, 4, INV>(p, z, spec, tw, done, s); break;
        case 8: yz_launch<T, N, 8, INV>(p, z, spec, tw, done, s); break;
        default: yz_launch<T, N, 16, INV>(p, z, spec, tw, done, s); break;
    }
}

template <typename T, bool INV>
void yz_dispatch(const Plan& p, const ZArgs& z, c2<T>* spec, const c2<T>* tw, const int* done,
                 hipStream_t s) {
    if (p.ny == 1) {
        z2d_launch<T, INV>(p, z, spec, done, s);
        return;
    }
    switch (p.ny) {
#define PSV_CASE(n) case n: yz_dispatch_kc<T, n, INV>(p, z, spec, tw, done, s); break;
        PSV_YZ_SIZES(PSV_CASE)
#undef PSV_CASE
        default: yz_dispatch_kc<T, 0, INV>(p, z, spec, tw, done, s); break;
    }
}

void check_precision(const Plan& p, bool fp32) {
    if (fp32 != (p.opts.precision == PSV_MIXED))
        fail(PSV_ERR_INVALID_ARG, "z pass precision differs from the plan's");
}

}  // namespace

void launch_yz(const Plan& p, bool fp32, bool inverse, const int* done, hipStream_t s) {
    check_precision(p, fp32);
    static const char* names[2][2] = {{"yz_fwd_fp64", "yz_inv_fp64"}, {"yz_fwd_fp32", "yz_inv_fp32"}};
    TraceScope ts(p, names[fp32][inverse], s);
    const ZArgs z = make_zargs(p, nullptr);
    if (fp32) {
        if (inverse)
            yz_dispatch<float, true>(p, z, (float2*)p.spec, p.t.twy32, done, s);
        else
            yz_dispatch<float, false>(p, z, (float2*)p.spec, p.t.twy32, done, s);
    } else {
        if (inverse)
            yz_dispatch<double, true>(p, z, (double2*)p.spec, p.t.twy64, done, s);
        else
            yz_dispatch<double, false>(p, z, (double2*)p.spec, p.t.twy64, done, s);
    }
    PSV_HIP(hipGetLastError());
}

void launch_interface(const Plan& p, bool fp32, double* mean_out, const int* done, hipStream_t s) {
    check_precision(p, fp32);
    const ZArgs z = make_zargs(p, mean_out);
    TraceScope ts(p, fp32 ? "z_interface_fp32" : "z_interface_fp64", s);
    if (fp32)
        ifc_dispatch<float>(p, z, done, s);
    else
        ifc_dispatch<double>(p, z, done, s);
    PSV_HIP(hipGetLastError());
}

void launch_z_solve(const Plan& p, bool fp32, double* mean_out, const int* done, hipStream_t s) {
    launch_yz(p, fp32, false, done, s);
    launch_interface(p, fp32, mean_out, done, s);
    launch_yz(p, fp32, true, done, s);
}

bool kc_fits(const Plan& p, int kc) {
    if (kc != 4 && kc != 8 && kc != 16) return false;
    const size_t csz = p.opts.precision == PSV_MIXED ? sizeof(float2) : sizeof(double2);
    return yz_lds(p.ny, kc, csz) <= (size_t)LDS_MAX_BLOCK;
}

size_t ifc_table_bytes(const Plan& p, int kc) {
    const size_t esz = p.opts.precision == PSV_MIXED ? sizeof(float) : sizeof(double);
    const int nc = (p.nz + kc - 1) / kc;
    return ifc_tab_entries(ifc_shape(nc, p.mx * p.ny)) * esz;
}

void launch_ifc_table(const Plan& p, hipStream_t s) {
    const bool fp32 = p.opts.precision == PSV_MIXED;
    const ZArgs z = make_zargs(p, nullptr);
    const int nblk = (p.mx * p.ny + TAB_THREADS - 1) / TAB_THREADS;
    const size_t lds = (size_t)p.lp.kc * TAB_THREADS * sizeof(double2);
    if (fp32) {
        allow_lds(k_ifc_table<float>, lds);
        hipLaunchKernelGGL(k_ifc_table<float>, dim3(nblk), dim3(TAB_THREADS), lds, s, z,
                           (float*)p.ifc_tab);
    } else {
        allow_lds(k_ifc_table<double>, lds);
        hipLaunchKernelGGL(k_ifc_table<double>, dim3(nblk), dim3(TAB_THREADS), lds, s, z,
                           (double*)p.ifc_tab);
    }
    PSV_HIP(hipGetLastError());
}

void plan_set_kc(Plan& p, int kc) {
    if (!kc_fits(p, kc)) fail(PSV_ERR_UNSUPPORTED_SIZE, "chunk rows do not fit the LDS of a block");
    const size_t bytes = ifc_table_bytes(p, kc);
    if (bytes > p.ifc_tab_bytes) {
        if (p.ifc_tab) PSV_HIP(hipFree(p.ifc_tab));
        p.ifc_tab = nullptr;
        p.ifc_tab_bytes = 0;
        PSV_HIP(hipMalloc(&p.ifc_tab, bytes));
        p.ifc_tab_bytes = bytes;
    }
    p.lp.kc = kc;
    launch_ifc_table(p, nullptr);
    PSV_HIP(hipDeviceSynchronize());
}

}  // namespace psv
