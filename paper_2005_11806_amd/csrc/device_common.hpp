// Device-side building blocks shared by the kernels of libpsv: complex
// arithmetic on HIP vector types, butterflies and a Stockham autosort FFT
// over batches of lines held in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psv {

template <typename T> struct V2;
template <> struct V2<double> { using t = double2; };
template <> struct V2<float> { using t = float2; };
template <typename T> using c2 = typename V2<T>::t;

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) { return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <typename C>
__device__ __forceinline__ C cconj(C a) { return C{a.x, -a.y}; }
template <typename C, typename T>
__device__ __forceinline__ C cscale(C a, T s) { return C{a.x * s, a.y * s}; }
// multiply by (sign * i): sign = -1 gives -i, +1 gives +i
template <int SIGN, typename C>
__device__ __forceinline__ C cmul_i(C a) {
    return SIGN > 0 ? C{-a.y, a.x} : C{a.y, -a.x};
}

template <typename D, typename S>
__device__ __forceinline__ D cconv(S a) { return D{(decltype(D::x))a.x, (decltype(D::x))a.y}; }

// Radix sequence of one FFT length (product of r[0..count-1] = n).
struct Radices {
    int n;
    int count;
    int r[12];
};

// ---------------------------------------------------------------------------
// DFT of R points in registers: V[q] = sum_r v[r] exp(DIR 2 pi i r q / R).
template <int DIR, typename C>
__device__ __forceinline__ void bfly2(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <int DIR, typename C>
__device__ __forceinline__ void bfly4(C* v) {
    C t0 = cadd(v[0], v[2]);
    C t1 = csub(v[0], v[2]);
    C t2 = cadd(v[1], v[3]);
    C t3 = cmul_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

template <int DIR, typename C>
__device__ __forceinline__ void bfly3(C* v) {
    using T = decltype(C::x);
    const T half_sqrt3 = (T)0.86602540378443864676372317075294;
    C s = cadd(v[1], v[2]);
    C d = csub(v[1], v[2]);
    C m = C{v[0].x - (T)0.5 * s.x, v[0].y - (T)0.5 * s.y};
    C rot = cmul_i<DIR>(cscale(d, half_sqrt3));
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, rot);
    v[2] = csub(m, rot);
}

template <int DIR, typename C>
__device__ __forceinline__ void bfly8(C* v) {
    using T = decltype(C::x);
    const T rs2 = (T)0.70710678118654752440084436210485;
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    bfly4<DIR>(e);
    bfly4<DIR>(o);
    // w8^q = exp(DIR 2 pi i q / 8)
    C o1 = C{(o[1].x - (T)DIR * o[1].y) * rs2, ((T)DIR * o[1].x + o[1].y) * rs2};   // * (1 + DIR i)/sqrt2
    C o2 = cmul_i<DIR>(o[2]);                                                         // * DIR i
    C o3 = C{(-o[3].x - (T)DIR * o[3].y) * rs2, ((T)DIR * o[3].x - o[3].y) * rs2};  // * (-1 + DIR i)/sqrt2
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

// One Stockham stage for butterfly j of a line: reads R points at stride L/R,
// twiddles by W^(r k) with W = exp(DIR 2 pi i / (Ns R)), k = j mod Ns, and
// writes them to (j / Ns) Ns R + k + r Ns. `tw` holds exp(-2 pi i t / twn).
template <int R, int DIR, typename C>
__device__ __forceinline__ void stockham_bfly(const C* __restrict__ in, C* __restrict__ out, int j,
                                              int nb, int Ns, const C* __restrict__ tw, int tstep) {
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[j + r * nb];
    const int k = j % Ns;
    if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
            C w = tw[r * k * tstep];
            if (DIR > 0) w.y = -w.y;
            v[r] = cmul(v[r], w);
        }
    }
    if (R == 2) bfly2<DIR>(v);
    if (R == 3) bfly3<DIR>(v);
    if (R == 4) bfly4<DIR>(v);
    if (R == 8) bfly8<DIR>(v);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[base + r * Ns] = v[r];
}

// Unnormalised FFT of `nlines` lines of length L stored in LDS at buf0 +
// line * lstride, ping-ponging with buf1. All threads of the block take part;
// returns the buffer that holds the result. Twiddles come from a table of
// exp(-2 pi i t / twn) with twn a multiple of L.
template <int DIR, typename C>
__device__ C* lds_fft(C* buf0, C* buf1, int L, int nlines, int lstride, const Radices& rp,
                      const C* __restrict__ tw, int twn) {
    C* src = buf0;
    C* dst = buf1;
    int Ns = 1;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    for (int s = 0; s < rp.count; ++s) {
        const int R = rp.r[s];
        const int nb = L / R;
        const int total = nlines * nb;
        const int tstep = twn / (Ns * R);
        for (int t = tid; t < total; t += nthr) {
            const int line = t / nb;
            const int j = t - line * nb;
            const C* in = src + line * lstride;
            C* out = dst + line * lstride;
            switch (R) {
                case 2: stockham_bfly<2, DIR>(in, out, j, nb, Ns, tw, tstep); break;
                case 3: stockham_bfly<3, DIR>(in, out, j, nb, Ns, tw, tstep); break;
                case 4: stockham_bfly<4, DIR>(in, out, j, nb, Ns, tw, tstep); break;
                default: stockham_bfly<8, DIR>(in, out, j, nb, Ns, tw, tstep); break;
            }
        }
        __syncthreads();
        C* t = src;
        src = dst;
        dst = t;
        Ns *= R;
    }
    return src;
}

// ---------------------------------------------------------------------------
// Compile-time variant: the line length N (2^a 3^b) and hence every radix,
// stride and twiddle step are constants. Blocks have 256 threads. Twiddles
// come from `tw` (usually an LDS copy) holding exp(-2 pi i t / (N * TWM)).
struct RadixList {
    int count;
    int r[12];
};

__host__ __device__ constexpr RadixList radix_list(int n) {
    RadixList L{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
    int a = 0, b = 0, m = n;
    while (m % 2 == 0) { m /= 2; ++a; }
    while (m % 3 == 0) { m /= 3; ++b; }
    while (a >= 3) { L.r[L.count++] = 8; a -= 3; }
    if (a == 2) L.r[L.count++] = 4;
    if (a == 1) L.r[L.count++] = 2;
    while (b-- > 0) L.r[L.count++] = 3;
    return L;
}

__host__ __device__ constexpr int radix_prefix(RadixList L, int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= L.r[i];
    return p;
}

// LDS layouts of FFT lines: contiguous, or with one pad element after every 8
// (the radix-R scatter of a Stockham stage then spreads over the banks
// instead of hitting the same ones); element i lives at at(i).
struct NoPad {
    __host__ __device__ static constexpr int at(int i) { return i; }
    __host__ __device__ static constexpr bool linear(int) { return true; }
    __host__ __device__ static constexpr int step(int s) { return s; }
};
struct Pad8 {
    __host__ __device__ static constexpr int at(int i) { return i + (i >> 3); }
    // at(i + k s) = at(i) + k step(s) whenever s is a multiple of 8, so the
    // addresses of a butterfly are one base plus constant offsets
    __host__ __device__ static constexpr bool linear(int s) { return s % 8 == 0; }
    __host__ __device__ static constexpr int step(int s) { return s + s / 8; }
};

// Butterfly j of a radix-R Stockham stage (NS = product of the earlier
// radices, NB = N / R) of the line starting at element off: load with
// twiddles and transform into v, then store.
template <int R, int DIR, int NS, int NB, int TSTEP, typename P = NoPad, typename C>
__device__ __forceinline__ void stockham_load_ct(const C* __restrict__ in, int j,
                                                 const C* __restrict__ tw, C* v, int off = 0) {
    if constexpr (P::linear(NB)) {
        const int b = P::at(off + j);
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = in[b + r * P::step(NB)];
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = in[P::at(off + j + r * NB)];
    }
    const int k = j % NS;
    if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
            C w = tw[r * k * TSTEP];
            if (DIR > 0) w.y = -w.y;
            v[r] = cmul(v[r], w);
        }
    }
    if (R == 2) bfly2<DIR>(v);
    if (R == 3) bfly3<DIR>(v);
    if (R == 4) bfly4<DIR>(v);
    if (R == 8) bfly8<DIR>(v);
}

// A8: off is a multiple of 8 (lines of a length divisible by 8), so in a
// first stage (NS = 1) with R dividing 8 the R outputs of a butterfly stay in
// one group of 8 elements.
template <int R, int NS, typename P = NoPad, bool A8 = false, typename C>
__device__ __forceinline__ void stockham_store_ct(C* __restrict__ out, int j, const C* v,
                                                  int off = 0) {
    const int base = off + (j / NS) * NS * R + j % NS;
    if constexpr (P::linear(NS)) {
        const int b = P::at(base);
#pragma unroll
        for (int r = 0; r < R; ++r) out[b + r * P::step(NS)] = v[r];
    } else if constexpr (A8 && NS == 1 && 8 % R == 0) {
        const int b = P::at(base);
#pragma unroll
        for (int r = 0; r < R; ++r) out[b + r] = v[r];
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) out[P::at(base + r * NS)] = v[r];
    }
}

// Two-buffer variant: stage S reads src and writes dst (both in layout P,
// line l starting at element l * lstride, lstride a multiple of 8 when N is),
// then the buffers swap. Returns the buffer holding the result; ends with the
// block synchronised.
template <int N, int S, int DIR, int TWM, typename P = NoPad, typename C>
__device__ __forceinline__ C* fft_stages(C* src, C* dst, int nlines, int lstride,
                                         const C* __restrict__ tw) {
    constexpr RadixList RL = radix_list(N);
    if constexpr (S == RL.count) {
        return src;
    } else {
        constexpr int R = RL.r[S];
        constexpr int NS = radix_prefix(RL, S);
        constexpr int NB = N / R;
        constexpr int TSTEP = (N / (NS * R)) * TWM;
        const int total = nlines * NB;
        for (int t = threadIdx.x; t < total; t += 256) {
            const int line = t / NB;
            const int j = t - line * NB;
            C v[R];
            stockham_load_ct<R, DIR, NS, NB, TSTEP, P>(src, j, tw, v, line * lstride);
            stockham_store_ct<R, NS, P, N % 8 == 0>(dst, j, v, line * lstride);
        }
        __syncthreads();
        return fft_stages<N, S + 1, DIR, TWM, P>(dst, src, nlines, lstride, tw);
    }
}

// In-place variant for NL lines of length N stored one after the other in
// one LDS buffer in layout P: every stage reads all of its butterflies into
// registers (a thread takes butterflies t, t + 256, ...), waits for the block,
// then writes. Ends with the block synchronised.
template <int N, int S, int DIR, int TWM, int NL, typename P = NoPad, typename C>
__device__ __forceinline__ void fft_inplace(C* buf, const C* __restrict__ tw) {
    constexpr RadixList RL = radix_list(N);
    if constexpr (S < RL.count) {
        constexpr int R = RL.r[S];
        constexpr int NS = radix_prefix(RL, S);
        constexpr int NB = N / R;
        constexpr int TSTEP = (N / (NS * R)) * TWM;
        constexpr int TOTAL = NL * NB;
        constexpr int IT = (TOTAL + 255) / 256;
        C v[IT][R];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int t = (int)threadIdx.x + it * 256;
            if (TOTAL % 256 == 0 || t < TOTAL) {
                const int line = t / NB;
                stockham_load_ct<R, DIR, NS, NB, TSTEP, P>(buf, t - line * NB, tw, v[it], line * N);
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int t = (int)threadIdx.x + it * 256;
            if (TOTAL % 256 == 0 || t < TOTAL) {
                const int line = t / NB;
                stockham_store_ct<R, NS, P, N % 8 == 0>(buf, t - line * NB, v[it], line * N);
            }
        }
        __syncthreads();
        fft_inplace<N, S + 1, DIR, TWM, NL, P>(buf, tw);
    }
}

// 1/s: hardware reciprocal refined by two Newton steps (correctly rounded on
// every input measured)
__device__ __forceinline__ double rcp_nr(double s) {
    double r = __builtin_amdgcn_rcp(s);
    r = fma(r, fma(-s, r, 1.0), r);
    return fma(r, fma(-s, r, 1.0), r);
}

// 1/s: hardware reciprocal refined by one Newton step (within about 11 ulp),
// for the face coefficients of the stencils, where the error is far below the
// solve's own rounding
__device__ __forceinline__ double rcp_nr1(double s) {
    const double r = __builtin_amdgcn_rcp(s);
    return fma(r, fma(-s, r, 1.0), r);
}

// N = 0 selects the runtime-length routine above (layout P applies to N > 0
// only; the runtime routine reads and writes unpadded lines).
template <int N, int DIR, int TWM, typename P = NoPad, typename C>
__device__ __forceinline__ C* lds_fft_n(C* buf0, C* buf1, int L, int nlines, int lstride,
                                        const Radices& rp, const C* __restrict__ tw) {
    if constexpr (N > 0) {
        return fft_stages<N, 0, DIR, TWM, P>(buf0, buf1, nlines, lstride, tw);
    } else {
        return lds_fft<DIR>(buf0, buf1, L, nlines, lstride, rp, tw, L * TWM);
    }
}

// Block copy of n elements (256 threads), G per thread in flight: get(t) is
// evaluated for G indices before put(t, v) runs for any of them, so their
// global loads overlap (a plain strided loop waits for each load before the
// LDS write that follows it). get must accept any t < n; slots past n call
// it again with the first index of the round and are not put. The first
// round is straight-line code: at a loop header the compiler's wait
// insertion would also wait for loads the caller issued before the copy.
template <int G, typename V, typename Get, typename Put>
__device__ __forceinline__ void block_copy(int n, Get&& get, Put&& put) {
    auto round = [&](int t0) {
        V v[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int t = t0 + j * 256;
            v[j] = get(t < n ? t : t0);
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int t = t0 + j * 256;
            if (t < n) put(t, v[j]);
        }
    };
    if ((int)threadIdx.x < n) round((int)threadIdx.x);
    for (int t0 = (int)threadIdx.x + G * 256; t0 < n; t0 += G * 256) round(t0);
}

// Direct global-to-LDS load of one 16-byte element per active lane (gfx950
// global_load_lds_dwordx4): lane i of the wave writes lds_base + 16 i bytes,
// lds_base being the same on every lane. Nothing passes through registers;
// the data is in LDS after lds_dma_wait() and a block barrier.
__device__ __forceinline__ void lds_dma16(const void* src, void* lds_base) {
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds_base, 16, 0, 0);
}
// This thread's share of sum_b p[stride b + off] over b < nb (b = thread +
// 256 i, in a block of 256 threads), with U loads in flight per round: a
// plain loop waits for each load in turn, which took a single block 50 us
// over the 32768 partials of a 256x256x512 forward pass. The order of the
// additions is fixed.
__device__ __forceinline__ double thread_share(const double* p, int nb, int stride, int off) {
    constexpr int U = 16;
    double acc[U] = {};
    int b = threadIdx.x;
    for (; b + (U - 1) * 256 < nb; b += U * 256) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = p[(size_t)stride * (b + u * 256) + off];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] += v[u];
    }
    for (; b < nb; b += 256) acc[0] += p[(size_t)stride * b + off];
#pragma unroll
    for (int h = U / 2; h > 0; h /= 2)
#pragma unroll
        for (int u = 0; u < h; ++u) acc[u] += acc[u + h];
    return acc[0];
}
// The same for two interleaved sums (p[2 b], p[2 b + 1]) in one pass.
__device__ __forceinline__ double2 thread_share2(const double* p, int nb) {
    constexpr int U = 16;
    const double2* p2 = reinterpret_cast<const double2*>(p);
    double2 acc[U] = {};
    int b = threadIdx.x;
    for (; b + (U - 1) * 256 < nb; b += U * 256) {
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = p2[b + u * 256];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = double2{acc[u].x + v[u].x, acc[u].y + v[u].y};
    }
    for (; b < nb; b += 256) acc[0] = double2{acc[0].x + p2[b].x, acc[0].y + p2[b].y};
#pragma unroll
    for (int h = U / 2; h > 0; h /= 2)
#pragma unroll
        for (int u = 0; u < h; ++u) acc[u] = double2{acc[u].x + acc[u + h].x, acc[u].y + acc[u + h].y};
    return acc[0];
}

// Non-temporal (streaming) accesses, for data that no later pass of the
// solve reads from the caches: the solution p (written last), the density
// as the min reduction reads it, and the interface factor table. On the
// 256x256x512 solve they took the inverse x pass from 119 to 101 us, the min
// pass from 80 to 47 us and the interface pass from 58 to 52 us; on the
// spectrum, which the next pass reads, they lose.
__device__ __forceinline__ void st_stream(double2* p, double2 v) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(d2v{v.x, v.y}, reinterpret_cast<d2v*>(p));
}
__device__ __forceinline__ double2 ld_stream(const double2* p) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
    return double2{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
    return __builtin_nontemporal_load(p);
}

// Waits for this wave's vector memory loads, the direct-to-LDS ones included
// (vmcnt(0); expcnt and lgkmcnt left at their maxima).
__device__ __forceinline__ void lds_dma_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Block-wide sum of one double per thread (blockDim.x <= 1024, multiple of 64).
__device__ inline double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) s += sh[w];
    }
    return s;  // valid on thread 0
}

// Blocks are dispatched round-robin over the 8 XCDs; remap so that each XCD
// walks a contiguous range of block indices (of planes and lines), and the
// neighbouring lines and planes a stencil reads stay in its L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, i = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// Forward x tiles in line windows: XCD x takes tiles x w .. x w + w - 1 of
// every plane (w = tiles per plane / 8), plane after plane. The z
// neighbours a tile reads are then the rows of the tiles just before and
// after it in the same XCD's sweep, fetched at about the same time, and the
// y neighbours come from another XCD only at the window's two edges. (With
// contiguous plane ranges an XCD works on about two planes at once and the
// neighbouring planes of p and rho leave its L2 between their uses.)
__device__ __forceinline__ int xcd_windows(int b, int w, int tiles) {
    const int x = b & 7, i = b >> 3;
    const int k = i / w;
    return k * tiles + x * w + (i - k * w);
}

}  // namespace psv
