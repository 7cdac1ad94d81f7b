// Pointwise and reduction kernels around the solve: min(rho) with its first
// index (rho0 of Method I, Sec. 3.3.1), residual norms, the mixture density
// (Sec. 2.2, Eq. eq_22), the discrete divergence, input scans and the
// face terms of the adjoint of one Method-I step.
// Reductions are two-stage (per-block partials, then one block) so that
// their results do not depend on scheduling.
#include <algorithm>
#include <cstdint>

#include "internal.hpp"

namespace psv {
namespace {

constexpr int RB = 256;      // threads per reduction block
constexpr int RMAXB = 2048;  // partial blocks of a reduction

// (value, index) pair that comes first: smaller value, then smaller index
__device__ __forceinline__ void argmin_merge(double& v, int& i, double v2, int i2) {
    if (v2 < v || (v2 == v && i2 < i)) {
        v = v2;
        i = i2;
    }
}

// Block-wide argmin_merge of one pair per thread; the result is on thread 0.
__device__ __forceinline__ void block_argmin(double& v, int& i, double* sv, int* si) {
    for (int o = 32; o > 0; o >>= 1) argmin_merge(v, i, __shfl_down(v, o, 64), __shfl_down(i, o, 64));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sv[w] = v;
        si[w] = i;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k < RB / 64; ++k) argmin_merge(v, i, sv[k], si[k]);
}

// Per-block minimum of a contiguous share of x[0, n) and the first index
// where it occurs: pairs (16-byte loads), eight per thread in flight, each
// thread visiting its pairs in increasing index order so that a strict '<'
// keeps its first minimum. A second launch merges the blocks' pairs (a
// device-scope fence per block, to merge in the last block instead, writes
// back its L2 and costs more than the launch).
__global__ void __launch_bounds__(RB) k_min_partial(const double* __restrict__ x, size_t n,
                                                    double* pv, int* pi) {
    __shared__ double sv[RB / 64];
    __shared__ int si[RB / 64];
    double best = __builtin_inf();
    int bi = 0x7fffffff;
    constexpr int U = 8;
    const double2* x2 = reinterpret_cast<const double2*>(x);
    const size_t n2 = n / 2;
    const size_t chunk = (n2 + gridDim.x - 1) / gridDim.x;
    const size_t c0 = (size_t)blockIdx.x * chunk;
    const size_t c1 = c0 + chunk < n2 ? c0 + chunk : n2;
    size_t c = c0 + threadIdx.x;
    for (; c + (U - 1) * RB < c1; c += U * RB) {
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld_stream(x2 + c + u * RB);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (v[u].x < best) { best = v[u].x; bi = (int)(2 * (c + u * RB)); }
            if (v[u].y < best) { best = v[u].y; bi = (int)(2 * (c + u * RB) + 1); }
        }
    }
    for (; c < c1; c += RB) {
        const double2 v = ld_stream(x2 + c);
        if (v.x < best) { best = v.x; bi = (int)(2 * c); }
        if (v.y < best) { best = v.y; bi = (int)(2 * c + 1); }
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0 && x[n - 1] < best) {
        best = x[n - 1];
        bi = (int)(n - 1);
    }
    block_argmin(best, bi, sv, si);
    if (threadIdx.x == 0) {
        pv[blockIdx.x] = best;
        pi[blockIdx.x] = bi;
    }
}

__global__ void __launch_bounds__(RB) k_min_final(const double* pv, const int* pi, int nb,
                                                  double* out, int* argmin) {
    __shared__ double sv[RB / 64];
    __shared__ int si[RB / 64];
    double best = __builtin_inf();
    int bi = 0x7fffffff;
    for (int b = threadIdx.x; b < nb; b += RB) argmin_merge(best, bi, pv[b], pi[b]);
    block_argmin(best, bi, sv, si);
    if (threadIdx.x == 0) {
        *out = best;
        if (argmin) *argmin = bi;
    }
}

// Largest value (no index), pairs of doubles, eight in flight per thread.
__global__ void __launch_bounds__(RB) k_max_partial(const double* __restrict__ x, size_t n,
                                                    double* pv) {
    __shared__ double sv[RB];
    double best = -__builtin_inf();
    constexpr int U = 8;
    const double2* x2 = reinterpret_cast<const double2*>(x);
    const size_t n2 = n / 2, stride = (size_t)gridDim.x * RB;
    size_t c = (size_t)blockIdx.x * RB + threadIdx.x;
    for (; c + (U - 1) * stride < n2; c += U * stride) {
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = x2[c + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) best = fmax(best, fmax(v[u].x, v[u].y));
    }
    for (; c < n2; c += stride) best = fmax(best, fmax(x2[c].x, x2[c].y));
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) best = fmax(best, x[n - 1]);
    sv[threadIdx.x] = best;
    __syncthreads();
    for (int o = RB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sv[threadIdx.x] = fmax(sv[threadIdx.x], sv[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) pv[blockIdx.x] = sv[0];
}

// scal[S_RHOMAX] = max of the partials; scal[S_OMEGA] = 2 a b / (a + b) with
// a = scal[S_RHO0] (min rho), b = max rho.
__global__ void __launch_bounds__(RB) k_harmonic_final(const double* pv, int nb, double* scal) {
    __shared__ double sv[RB];
    double best = -__builtin_inf();
    for (int b = threadIdx.x; b < nb; b += RB) best = fmax(best, pv[b]);
    sv[threadIdx.x] = best;
    __syncthreads();
    for (int o = RB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sv[threadIdx.x] = fmax(sv[threadIdx.x], sv[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double a = scal[S_RHO0], b = sv[0];
        scal[S_RHOMAX] = b;
        scal[S_OMEGA] = 2.0 * a * b / (a + b);
    }
}

// First stage of a sum over a long partial array: block i of the grid sums
// its contiguous share of the nb entries of each of the `per` interleaved
// sums (per <= 2) into out[per i + q]. One block reading all 32768 partials
// of a 256x256x512 forward pass waits on memory round after round (25-50
// us); split over STAGE1_BLOCKS blocks it does not. Skipped when *done.
constexpr int STAGE1_BLOCKS = 32;
__global__ void __launch_bounds__(RB) k_partials_stage1(const double* partials, int nb, int per,
                                                        double* out, const int* done) {
    __shared__ double sh[16];
    if (done && *done) return;
    const int b0 = (int)((long long)nb * blockIdx.x / gridDim.x);
    const int b1 = (int)((long long)nb * (blockIdx.x + 1) / gridDim.x);
    auto at = [&](int b, int q) { return partials[(size_t)per * b + q]; };
    for (int q = 0; q < per; ++q) {
        double v = 0.0;
        int b = b0 + (int)threadIdx.x;
        for (; b + 3 * RB < b1; b += 4 * RB) {  // four loads in flight
            const double t0 = at(b, q), t1 = at(b + RB, q), t2 = at(b + 2 * RB, q), t3 = at(b + 3 * RB, q);
            v += (t0 + t1) + (t2 + t3);
        }
        for (; b < b1; b += RB) v += at(b, q);
        const double t = block_sum(v, sh);
        if (threadIdx.x == 0) out[per * blockIdx.x + q] = t;
    }
}

// Sum of `per` interleaved partial sums over nb blocks.
__global__ void __launch_bounds__(RB) k_sum_partials(const double* partials, int nb, int per,
                                                     double* out) {
    __shared__ double sh[16];
    if (per == 2) {  // both sums in one pass over the pairs
        const double2 ab = thread_share2(partials, nb);
        const double a = block_sum(ab.x, sh);
        if (threadIdx.x == 0) out[0] = a;
        __syncthreads();
        const double b = block_sum(ab.y, sh);
        if (threadIdx.x == 0) out[1] = b;
        return;
    }
    for (int q = 0; q < per; ++q) {
        const double s = block_sum(thread_share(partials, nb, per, q), sh);
        if (threadIdx.x == 0) out[q] = s;
        __syncthreads();
    }
}

// relres = sqrt(sum res^2 / sum r^2); sets flags[F_DONE] when <= tol.
__global__ void k_relres_final(double* scal, int* flags, double tol) {
    if (threadIdx.x == 0) {
        const double r2 = scal[S_R2];
        const double rr = r2 > 0.0 ? sqrt(scal[S_RES2] / r2) : 0.0;
        scal[S_RELRES] = rr;
        if (tol > 0.0 && rr <= tol) flags[F_DONE] = 1;
    }
}

__global__ void k_refine_reset(double* scal, int* flags) {
    if (threadIdx.x < S_NHIST) scal[S_HIST + threadIdx.x] = __builtin_nan("");
    if (threadIdx.x == 0) {
        flags[F_DONE] = 0;
        flags[F_STEPS] = 0;
        flags[F_CONV] = 0;
    }
}

__global__ void __launch_bounds__(RB) k_refine_check(const double* partials, int nb, int sweep,
                                                     int max_refine, double tol, double* scal,
                                                     int* flags) {
    __shared__ double sh[16];
    if (flags[F_DONE]) return;  // uniform over the block
    const double2 ab = thread_share2(partials, nb);
    const double a = block_sum(ab.x, sh);
    __syncthreads();
    const double b = block_sum(ab.y, sh);
    if (threadIdx.x == 0) {
        const double rr = b > 0.0 ? sqrt(a / b) : 0.0;
        scal[S_RELRES] = rr;
        if (sweep < S_NHIST) scal[S_HIST + sweep] = rr;
        if (rr <= tol) {
            flags[F_DONE] = 1;
            flags[F_CONV] = 1;
        } else if (sweep >= max_refine || !isfinite(rr)) {
            flags[F_DONE] = 1;
        } else {
            flags[F_STEPS] += 1;
        }
    }
}

__global__ void k_m3_reset(int* flags) {
    if (threadIdx.x == 0) {
        flags[F_DONE] = 0;
        flags[F_STEPS] = 0;
        flags[F_CONV] = 0;
    }
}

__global__ void __launch_bounds__(RB) k_m3_check(const double* partials, int nb, double dt,
                                                 double eps_t, int has_p, int max_iter,
                                                 double* scal, int* flags) {
    __shared__ double sh[16];
    if (flags[F_DONE]) return;  // uniform over the block
    const double eps = dt * block_sum(thread_share(partials, nb, 1, 0), sh);
    if (threadIdx.x != 0) return;
    if (!has_p) {
        scal[S_EPS0] = eps;
    } else {
        scal[S_EPS] = eps;
        if (eps <= eps_t) {
            flags[F_CONV] = 1;
            flags[F_DONE] = 1;
            return;
        }
        if (flags[F_STEPS] >= max_iter) {
            flags[F_DONE] = 1;
            return;
        }
    }
    flags[F_STEPS] += 1;
}

__global__ void k_set_scalar(double* dst, double v) {
    if (threadIdx.x == 0) *dst = v;
}

struct Geo {
    int nx, ny, nz;
    double inv_dx, inv_dy;
    const double* inv_h;
    const double* inv_g;
    const double* vol;
};

// res = r - mean - L p ; partial sums of res^2 and (r - mean)^2. One thread
// per pair of cells (2q, 2q+1) of an x-line (nx is even), 16-byte loads,
// 32-bit index arithmetic (every index is below nx ny nz < 2^31).
__global__ void __launch_bounds__(RB) k_residual(Geo g, const double* __restrict__ r,
                                                 const double* __restrict__ p,
                                                 const double* mean_p, double* partials) {
    __shared__ double sh[16];
    const unsigned M = (unsigned)g.nx / 2u;  // pairs per line
    const unsigned npair = M * (unsigned)g.ny * (unsigned)g.nz;
    const unsigned pl2 = M * (unsigned)g.ny;  // pairs per plane
    const double2* p2 = reinterpret_cast<const double2*>(p);
    const double2* r2 = reinterpret_cast<const double2*>(r);
    const double mean = *mean_p;
    const double idx2 = g.inv_dx * g.inv_dx, idy2 = g.inv_dy * g.inv_dy;
    double s1 = 0.0, s2 = 0.0;
    for (unsigned q = blockIdx.x * RB + threadIdx.x; q < npair; q += gridDim.x * RB) {
        const unsigned line = q / M, n = q - line * M;
        const unsigned k = line / (unsigned)g.ny, j = line - k * (unsigned)g.ny;
        const unsigned row = q - n;  // first pair of the line
        const double2 pc = p2[q];
        const double pw = p2[row + (n == 0 ? M - 1 : n - 1)].y;
        const double pe = p2[row + (n + 1 == M ? 0 : n + 1)].x;
        const double2 pn = p2[j + 1 == (unsigned)g.ny ? q - j * M : q + M];
        const double2 ps = p2[j == 0 ? q + ((unsigned)g.ny - 1) * M : q - M];
        double l0 = ((pc.y - pc.x) - (pc.x - pw)) * idx2 + ((pn.x - pc.x) - (pc.x - ps.x)) * idy2;
        double l1 = ((pe - pc.y) - (pc.y - pc.x)) * idx2 + ((pn.y - pc.y) - (pc.y - ps.y)) * idy2;
        double ft0 = 0.0, ft1 = 0.0, fb0 = 0.0, fb1 = 0.0;  // wall fluxes are zero
        if (k + 1 < (unsigned)g.nz) {
            const double2 pt = p2[q + pl2];
            ft0 = (pt.x - pc.x) * g.inv_g[k + 1];
            ft1 = (pt.y - pc.y) * g.inv_g[k + 1];
        }
        if (k > 0) {
            const double2 pb = p2[q - pl2];
            fb0 = (pc.x - pb.x) * g.inv_g[k];
            fb1 = (pc.y - pb.y) * g.inv_g[k];
        }
        l0 += (ft0 - fb0) * g.inv_h[k];
        l1 += (ft1 - fb1) * g.inv_h[k];
        const double2 rv = r2[q];
        const double rp0 = rv.x - mean, rp1 = rv.y - mean;
        const double e0 = rp0 - l0, e1 = rp1 - l1;
        s1 += e0 * e0 + e1 * e1;
        s2 += rp0 * rp0 + rp1 * rp1;
    }
    const double a = block_sum(s1, sh);
    __syncthreads();
    const double b = block_sum(s2, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = a;
        partials[2 * blockIdx.x + 1] = b;
    }
}

__global__ void k_density(size_t n, const double* __restrict__ phi, const double* __restrict__ rg,
                          double rl, double* __restrict__ out) {
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (size_t)gridDim.x * blockDim.x) {
        const double f = phi[c];
        out[c] = rg[c] * f + rl * (1.0 - f);
    }
}

// (i, j, k) of cell c with 32-bit arithmetic (every index is below 2^31)
__device__ __forceinline__ void cell_ijk(unsigned c, const Geo& g, unsigned& i, unsigned& j,
                                         unsigned& k) {
    const unsigned line = c / (unsigned)g.nx;
    i = c - line * (unsigned)g.nx;
    k = line / (unsigned)g.ny;
    j = line - k * (unsigned)g.ny;
}

// out = scale (D u - target), target may be null. u is the MAC face field:
// ux on the face between cells i and i+1, uy likewise, uz [nz+1][ny][nx] with
// the bottom face of cell c at index c and the top at c + nx ny.
__global__ void k_divergence(Geo g, const double* __restrict__ ux, const double* __restrict__ uy,
                             const double* __restrict__ uz, const double* __restrict__ target,
                             double scale, double* __restrict__ out) {
    const unsigned nx = (unsigned)g.nx, plane = nx * (unsigned)g.ny;
    const unsigned n = plane * (unsigned)g.nz;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        unsigned i, j, k;
        cell_ijk(c, g, i, j, k);
        const double dx = ux[c] - ux[i == 0 ? c + nx - 1 : c - 1];
        const double dy = uy[c] - uy[j == 0 ? c + plane - nx : c - nx];
        const double dz = uz[c + plane] - uz[c];
        double d = dx * g.inv_dx + dy * g.inv_dy + dz * g.inv_h[k];
        if (target) d -= target[c];
        out[c] = d * scale;
    }
}

// Correction step of Method III (Eq. corr): u = u* - dt rho_f^-1 G p on every
// interior face, rho_f = (rho_L + rho_R)/2; the two wall planes of uz are
// copied (zero normal velocity).
__global__ void k_correct_velocity(Geo g, const double* __restrict__ ux, const double* __restrict__ uy,
                                   const double* __restrict__ uz, const double* __restrict__ p,
                                   const double* __restrict__ rho, double dt,
                                   double* __restrict__ ox, double* __restrict__ oy,
                                   double* __restrict__ oz) {
    const unsigned nx = (unsigned)g.nx, plane = nx * (unsigned)g.ny;
    const unsigned n = plane * (unsigned)g.nz;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        unsigned i, j, k;
        cell_ijk(c, g, i, j, k);
        const double pc = p[c], rc = rho[c];
        const unsigned ce = i + 1 == nx ? c + 1 - nx : c + 1;
        const unsigned cn = j + 1 == (unsigned)g.ny ? c + nx - plane : c + nx;
        ox[c] = ux[c] - dt * 2.0 * (p[ce] - pc) * g.inv_dx / (rc + rho[ce]);
        oy[c] = uy[c] - dt * 2.0 * (p[cn] - pc) * g.inv_dy / (rc + rho[cn]);
        if (k == 0)
            oz[c] = uz[c];
        else
            oz[c] = uz[c] - dt * 2.0 * (pc - p[c - plane]) * g.inv_g[k] / (rho[c - plane] + rc);
        if (k + 1 == (unsigned)g.nz) oz[c + plane] = uz[c + plane];
    }
}

// Adjoint face terms of one Method-I step for loss = sum(w p). The solve S is
// self-adjoint in the volume-weighted inner product, so S^T w = V S(V^-1 w);
// the kernel receives x = S(V^-1 w) and forms lam = V x. With beta_f =
// 1 - rho0/rho_f and rho_f = (rho_L + rho_R)/2:
//   (D^T lam)_f = lam_L/h_L - lam_R/h_R, gface = (D^T lam)_f (G p_prev)_f,
//   grad_f[c]    = rho0 lam_c,
//   grad_rho[c]  = sum over the 6 faces of c of gface rho0 / (2 rho_f^2),
//   grad_p[c]    = (G^T (beta D^T lam))_c,
//   partials     = sum lam f - sum over faces (each once) of gface / rho_f.
struct AdjArgs {
    const double* x;  // S(V^-1 w)
    const double* f;
    const double* rho;
    const double* pp;
    const double* rho0p;
    double* grad_f;
    double* grad_rho;
    double* grad_p;
    double* partials;
};

// One face between cells L and R of the adjoint's face products:
// t = (D^T mu)_F = mu_L ih_L - mu_R ih_R (ih the widths normal to F), g = (G p)_F,
// 1/rho_f = 2 / (rho_L + rho_R). Adds t g rho0 / (2 rho_f^2) to the grad_rho of
// both cells (gr_l, gr_r), the face's share of G^T((1 - rho0/rho_f) t) to their
// grad_p (gp_l, gp_r), and returns -t g / rho_f (the face's part of d/drho0).
struct FaceOut {
    double gr, gp_l, gp_r, r0;
};
__device__ __forceinline__ FaceOut adj_face(double mul, double ihl, double mur, double ihr,
                                            double rl, double rr, double pl, double pr,
                                            double inv_d, double rho0) {
    const double t = mul * ihl - mur * ihr;
    const double irf = 2.0 * rcp_nr(rl + rr);
    const double gf = t * ((pr - pl) * inv_d);
    const double bdt = (1.0 - rho0 * irf) * t * inv_d;
    return FaceOut{0.5 * gf * rho0 * irf * irf, -bdt, bdt, -gf * irf};
}

// Face products of the adjoint, one thread per pair of cells (2n, 2n+1) of an
// x line: 16-byte loads of x, rho and p on the pair and on its y and z
// neighbour pairs; the two x neighbours outside the pair come from the
// adjacent lanes where a wave holds them, else by single loads.
// The pair's three x faces (west, middle, east), four y faces and up to four z
// faces are evaluated once each; each cell sums the faces it touches. The
// d/drho0 partial counts each face once, at the cell on its lower (west,
// south or bottom) side. nx is even, so pairs never straddle lines.
__global__ void __launch_bounds__(RB) k_adjoint_faces(Geo g, AdjArgs a) {
    __shared__ double sh[16];
    const unsigned nx = (unsigned)g.nx, ny = (unsigned)g.ny, nz = (unsigned)g.nz;
    const unsigned M = nx / 2;
    const unsigned plane2 = M * ny, npair = plane2 * nz;  // every index is below 2^31
    const double rho0 = *a.rho0p;
    const double2* X = reinterpret_cast<const double2*>(a.x);
    const double2* RH = reinterpret_cast<const double2*>(a.rho);
    const double2* P = reinterpret_cast<const double2*>(a.pp);
    double acc = 0.0;
    // one block per RB consecutive pairs. Where a plane is a whole number of
    // blocks, a multiple of 8, and every pair has its own block, each XCD
    // takes a window of 1/8 of every plane's blocks, plane after plane (the
    // z neighbours of a block's pairs are then the pairs of the blocks just
    // before and after it in the same XCD's sweep); else each XCD takes a
    // contiguous range
    const unsigned tpp = plane2 / RB;  // blocks per plane
    const bool win = plane2 % RB == 0 && tpp % 8 == 0 && gridDim.x * RB == npair;
    const unsigned bx = win ? (unsigned)xcd_windows((int)blockIdx.x, (int)(tpp / 8), (int)tpp)
                            : (unsigned)xcd_remap((int)blockIdx.x, (int)gridDim.x);
    // x neighbours from the adjacent lanes where a wave holds whole lines (M
    // divides 64) or 64 pairs of one line (64 divides M; the wave's first and
    // last lanes load theirs); whole lane groups are active together
    const bool xl = (M % 64u) == 0 || (64u % M) == 0;
    const unsigned XG = M < 64u ? M : 64u;
    const unsigned lane = threadIdx.x & 63u;
    const int src_w = (int)((lane & ~(XG - 1)) + ((lane + XG - 1) & (XG - 1)));
    const int src_e = (int)((lane & ~(XG - 1)) + ((lane + 1) & (XG - 1)));
    for (unsigned q = bx * RB + threadIdx.x; q < npair; q += gridDim.x * RB) {
        const unsigned line = q / M;
        const unsigned n = q - line * M;
        const unsigned k = line / ny, j = line - k * ny;
        const double vk = g.vol[k], ihk = g.inv_h[k];
        const double idx = g.inv_dx, idy = g.inv_dy;
        const double2 xc = X[q], rc = RH[q], pc = P[q];
        const double m0 = vk * xc.x, m1 = vk * xc.y;
        // x neighbours outside the pair (periodic within the line)
        const unsigned cw = line * nx + (n == 0 ? nx - 1 : 2 * n - 1);
        const unsigned ce = line * nx + (n + 1 == M ? 0 : 2 * n + 2);
        double xw, rw, pw, xe, re, pe;
        if (xl) {
            xw = __shfl(xc.y, src_w, 64);
            rw = __shfl(rc.y, src_w, 64);
            pw = __shfl(pc.y, src_w, 64);
            xe = __shfl(xc.x, src_e, 64);
            re = __shfl(rc.x, src_e, 64);
            pe = __shfl(pc.x, src_e, 64);
            if (M > 64u && lane == 0) {
                xw = a.x[cw];
                rw = a.rho[cw];
                pw = a.pp[cw];
            }
            if (M > 64u && lane == 63) {
                xe = a.x[ce];
                re = a.rho[ce];
                pe = a.pp[ce];
            }
        } else {
            xw = a.x[cw];
            rw = a.rho[cw];
            pw = a.pp[cw];
            xe = a.x[ce];
            re = a.rho[ce];
            pe = a.pp[ce];
        }
        const double mw = vk * xw, me = vk * xe;
        double gr0 = 0.0, gr1 = 0.0, gp0 = 0.0, gp1 = 0.0;
        // x faces: west of 2n (lower cell outside), middle, east of 2n+1
        FaceOut f = adj_face(mw, idx, m0, idx, rw, rc.x, pw, pc.x, idx, rho0);
        gr0 += f.gr;
        gp0 += f.gp_r;
        f = adj_face(m0, idx, m1, idx, rc.x, rc.y, pc.x, pc.y, idx, rho0);
        gr0 += f.gr;
        gr1 += f.gr;
        gp0 += f.gp_l;
        gp1 += f.gp_r;
        acc += f.r0;
        f = adj_face(m1, idx, me, idx, rc.y, re, pc.y, pe, idx, rho0);
        gr1 += f.gr;
        gp1 += f.gp_l;
        acc += f.r0;
        // y faces: north (this pair lower) and south (periodic)
        {
            const unsigned qn = (j + 1 == ny) ? q + M - plane2 : q + M;
            const unsigned qs = (j == 0) ? q + plane2 - M : q - M;
            const double2 xn = X[qn], rn = RH[qn], pn = P[qn];
            const double2 xs = X[qs], rs = RH[qs], ps = P[qs];
            f = adj_face(m0, idy, vk * xn.x, idy, rc.x, rn.x, pc.x, pn.x, idy, rho0);
            gr0 += f.gr;
            gp0 += f.gp_l;
            acc += f.r0;
            f = adj_face(m1, idy, vk * xn.y, idy, rc.y, rn.y, pc.y, pn.y, idy, rho0);
            gr1 += f.gr;
            gp1 += f.gp_l;
            acc += f.r0;
            f = adj_face(vk * xs.x, idy, m0, idy, rs.x, rc.x, ps.x, pc.x, idy, rho0);
            gr0 += f.gr;
            gp0 += f.gp_r;
            f = adj_face(vk * xs.y, idy, m1, idy, rs.y, rc.y, ps.y, pc.y, idy, rho0);
            gr1 += f.gr;
            gp1 += f.gp_r;
        }
        // z faces: top (this pair lower) and bottom; none at the walls
        if (k + 1 < nz) {
            const unsigned qt = q + plane2;
            const double2 xt = X[qt], rt = RH[qt], pt = P[qt];
            const double vt = g.vol[k + 1], iht = g.inv_h[k + 1], igt = g.inv_g[k + 1];
            f = adj_face(m0, ihk, vt * xt.x, iht, rc.x, rt.x, pc.x, pt.x, igt, rho0);
            gr0 += f.gr;
            gp0 += f.gp_l;
            acc += f.r0;
            f = adj_face(m1, ihk, vt * xt.y, iht, rc.y, rt.y, pc.y, pt.y, igt, rho0);
            gr1 += f.gr;
            gp1 += f.gp_l;
            acc += f.r0;
        }
        if (k > 0) {
            const unsigned qb = q - plane2;
            const double2 xb = X[qb], rb = RH[qb], pb = P[qb];
            const double vb = g.vol[k - 1], ihb = g.inv_h[k - 1], igb = g.inv_g[k];
            f = adj_face(vb * xb.x, ihb, m0, ihk, rb.x, rc.x, pb.x, pc.x, igb, rho0);
            gr0 += f.gr;
            gp0 += f.gp_r;
            f = adj_face(vb * xb.y, ihb, m1, ihk, rb.y, rc.y, pb.y, pc.y, igb, rho0);
            gr1 += f.gr;
            gp1 += f.gp_r;
        }
        if (a.f) {
            const double2 fc = reinterpret_cast<const double2*>(a.f)[q];
            acc += m0 * fc.x + m1 * fc.y;
        }
        // the gradients are outputs no later pass reads: streaming stores
        if (a.grad_f) st_stream(reinterpret_cast<double2*>(a.grad_f) + q, double2{rho0 * m0, rho0 * m1});
        if (a.grad_rho) st_stream(reinterpret_cast<double2*>(a.grad_rho) + q, double2{gr0, gr1});
        if (a.grad_p) st_stream(reinterpret_cast<double2*>(a.grad_p) + q, double2{gp0, gp1});
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = s;
}

__global__ void k_scale_vol(Geo g, const double* __restrict__ x, double* __restrict__ out) {
    const unsigned plane = (unsigned)g.nx * (unsigned)g.ny, n = plane * (unsigned)g.nz;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
        out[c] = g.vol[c / plane] * x[c];
}

// partial sums of vol[k] r[c] (volume-weighted integral)
__global__ void __launch_bounds__(RB) k_vsum(Geo g, const double* __restrict__ r,
                                             const double* __restrict__ sc, double* partials) {
    __shared__ double sh[16];
    const unsigned plane = (unsigned)g.nx * (unsigned)g.ny, n = plane * (unsigned)g.nz;
    double acc = 0.0;
    for (unsigned c = blockIdx.x * RB + threadIdx.x; c < n; c += gridDim.x * RB) {
        const unsigned k = c / plane;
        acc += (sc ? g.vol[k] * sc[k] : g.vol[k]) * r[c];
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void k_div_scalar(double* x, double d) {
    if (threadIdx.x == 0) *x = *x / d;
}

__global__ void k_fill(size_t n, double* __restrict__ x, double v) {
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (size_t)gridDim.x * blockDim.x)
        x[c] = v;
}

__global__ void k_adjoint_argmin(double* grad_rho, const double* scal, const int* flags) {
    if (threadIdx.x == 0) grad_rho[flags[F_ARGMIN]] += scal[S_GRAD_RHO0];
}

__global__ void k_scan(size_t n, const double* __restrict__ x, int positive, int* bad) {
    int b = 0;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (size_t)gridDim.x * blockDim.x) {
        const double v = x[c];
        if (!isfinite(v)) b |= 1;
        else if (positive && !(v > 0.0)) b |= 2;
    }
    if (b) atomicOr(bad, b);
}

Geo make_geo(const Plan& p) {
    Geo g;
    g.nx = p.nx;
    g.ny = p.ny;
    g.nz = p.nz;
    g.inv_dx = 1.0 / p.dx;
    g.inv_dy = 1.0 / p.dy;
    g.inv_h = p.t.inv_h;
    g.inv_g = p.t.inv_g;
    g.vol = p.t.vol;
    return g;
}

int grid_blocks(size_t n, int thr) {
    size_t b = (n + thr - 1) / thr;
    if (b > (size_t)RMAXB) b = RMAXB;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

// One block per RB pairs of cells, bounded by the partial-sum buffer (one
// slot per block; past it the blocks stride over the pairs).
int adjoint_blocks(const Plan& p) {
    return (int)std::min<size_t>((size_t)p.n_partials, (p.ncell() / 2 + RB - 1) / RB);
}

void launch_min_reduce(const Plan& p, const double* x, double* out_scalar, int* argmin_out,
                       hipStream_t s) {
    const int nb = grid_blocks(p.ncell(), RB);
    double* pv = p.partials;
    int* pi = reinterpret_cast<int*>(p.partials + RMAXB);
    TraceScope ts(p, "min_rho", s);
    hipLaunchKernelGGL(k_min_partial, dim3(nb), dim3(RB), 0, s, x, p.ncell(), pv, pi);
    hipLaunchKernelGGL(k_min_final, dim3(1), dim3(RB), 0, s, pv, pi, nb, out_scalar, argmin_out);
    PSV_HIP(hipGetLastError());
}

void launch_harmonic_weight(const Plan& p, const double* rho, hipStream_t s) {
    launch_min_reduce(p, rho, p.scal + S_RHO0, p.flags + F_ARGMIN, s);
    const int nb = grid_blocks(p.ncell(), RB);
    hipLaunchKernelGGL(k_max_partial, dim3(nb), dim3(RB), 0, s, rho, p.ncell(), p.partials);
    hipLaunchKernelGGL(k_harmonic_final, dim3(1), dim3(RB), 0, s, p.partials, nb, p.scal);
    PSV_HIP(hipGetLastError());
}

// Long partial arrays (more than 2048 entries per sum) first go through
// k_partials_stage1 into the last 2 STAGE1_BLOCKS entries of the plan's
// partials buffer. The x passes' arrays (one or two entries per tile) never
// reach them, as the buffer holds at least 2 ny nz + 64 entries; a source
// that spans them is read by the single block directly. Returns the array
// the final single-block pass reads; nb becomes its length.
static const double* stage_partials(const Plan& p, const double* partials, int& nb, int per,
                                    const int* done, hipStream_t s) {
    double* out = p.partials + (p.n_partials - 2 * STAGE1_BLOCKS);
    const uintptr_t a0 = (uintptr_t)partials, a1 = (uintptr_t)(partials + (size_t)per * nb);
    const uintptr_t o0 = (uintptr_t)out, o1 = (uintptr_t)(out + 2 * STAGE1_BLOCKS);
    if (nb <= 2048 || per > 2 || (a0 < o1 && o0 < a1)) return partials;
    hipLaunchKernelGGL(k_partials_stage1, dim3(STAGE1_BLOCKS), dim3(RB), 0, s, partials, nb, per,
                       out, done);
    nb = STAGE1_BLOCKS;
    return out;
}

void launch_norm_finalize(const Plan& p, int nblocks, double tol, hipStream_t s) {
    const double* src = stage_partials(p, p.partials, nblocks, 2, nullptr, s);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(RB), 0, s, src, nblocks, 2,
                       p.scal + S_RES2);
    hipLaunchKernelGGL(k_relres_final, dim3(1), dim3(64), 0, s, p.scal, p.flags, tol);
    PSV_HIP(hipGetLastError());
}

void launch_refine_reset(const Plan& p, hipStream_t s) {
    hipLaunchKernelGGL(k_refine_reset, dim3(1), dim3(64), 0, s, p.scal, p.flags);
    PSV_HIP(hipGetLastError());
}

void launch_refine_check(const Plan& p, int nblocks, int sweep, int max_refine, double tol,
                         hipStream_t s) {
    const double* src = stage_partials(p, p.partials, nblocks, 2, p.flags + F_DONE, s);
    hipLaunchKernelGGL(k_refine_check, dim3(1), dim3(RB), 0, s, src, nblocks, sweep,
                       max_refine, tol, p.scal, p.flags);
    PSV_HIP(hipGetLastError());
}

void launch_residual(const Plan& p, const double* r, const double* p_sol, const double* mean,
                     hipStream_t s) {
    const int nb = grid_blocks(p.ncell(), RB);
    {
        TraceScope ts(p, "residual_fp64", s);
        hipLaunchKernelGGL(k_residual, dim3(nb), dim3(RB), 0, s, make_geo(p), r, p_sol, mean,
                           p.partials);
    }
    launch_norm_finalize(p, nb, 0.0, s);
}

void launch_set_scalar(double* dst, double v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, s, dst, v);
    PSV_HIP(hipGetLastError());
}

void launch_density(const Plan& p, const double* phi, const double* rg, double rl, double* out,
                    hipStream_t s) {
    const int nb = grid_blocks(p.ncell(), RB) * 4;
    hipLaunchKernelGGL(k_density, dim3(nb), dim3(RB), 0, s, p.ncell(), phi, rg, rl, out);
    PSV_HIP(hipGetLastError());
}

void launch_divergence(const Plan& p, const double* ux, const double* uy, const double* uz,
                       double* out, hipStream_t s) {
    launch_divergence_rhs(p, ux, uy, uz, nullptr, 1.0, out, s);
}

void launch_divergence_rhs(const Plan& p, const double* ux, const double* uy, const double* uz,
                           const double* target, double scale, double* out, hipStream_t s) {
    const int nb = grid_blocks(p.ncell(), RB) * 4;
    hipLaunchKernelGGL(k_divergence, dim3(nb), dim3(RB), 0, s, make_geo(p), ux, uy, uz, target,
                       scale, out);
    PSV_HIP(hipGetLastError());
}

void launch_correct_velocity(const Plan& p, const double* ux, const double* uy, const double* uz,
                             const double* pr, const double* rho, double dt, double* ox,
                             double* oy, double* oz, hipStream_t s) {
    const int nb = grid_blocks(p.ncell(), RB) * 4;
    TraceScope ts(p, "correct_velocity", s);
    hipLaunchKernelGGL(k_correct_velocity, dim3(nb), dim3(RB), 0, s, make_geo(p), ux, uy, uz, pr,
                       rho, dt, ox, oy, oz);
    PSV_HIP(hipGetLastError());
}

void launch_m3_reset(const Plan& p, hipStream_t s) {
    hipLaunchKernelGGL(k_m3_reset, dim3(1), dim3(64), 0, s, p.flags);
    PSV_HIP(hipGetLastError());
}

void launch_m3_check(const Plan& p, const double* partials, int nblocks, double dt, double eps_t,
                     bool has_p, int max_iter, hipStream_t s) {
    const double* src = stage_partials(p, partials, nblocks, 1, p.flags + F_DONE, s);
    hipLaunchKernelGGL(k_m3_check, dim3(1), dim3(RB), 0, s, src, nblocks, dt, eps_t,
                       has_p ? 1 : 0, max_iter, p.scal, p.flags);
    PSV_HIP(hipGetLastError());
}

void launch_sum_partials(const Plan& p, const double* partials, int nblocks, double* out,
                         hipStream_t s) {
    const double* src = stage_partials(p, partials, nblocks, 1, nullptr, s);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(RB), 0, s, src, nblocks, 1, out);
    PSV_HIP(hipGetLastError());
}

void launch_adjoint_faces(const Plan& p, const double* x, const double* f, const double* rho,
                          const double* pprev, const double* rho0, double* grad_f,
                          double* grad_rho, double* grad_p, double* partials, hipStream_t s) {
    AdjArgs a{x, f, rho, pprev, rho0, grad_f, grad_rho, grad_p, partials};
    TraceScope ts(p, "adjoint_faces", s);
    hipLaunchKernelGGL(k_adjoint_faces, dim3(adjoint_blocks(p)), dim3(RB), 0, s, make_geo(p), a);
    PSV_HIP(hipGetLastError());
}

void launch_adjoint_finalize(const Plan& p, int nblocks, double* grad_rho, int add_argmin,
                             hipStream_t s) {
    const double* src = stage_partials(p, p.partials, nblocks, 1, nullptr, s);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(RB), 0, s, src, nblocks, 1,
                       p.scal + S_GRAD_RHO0);
    if (add_argmin && grad_rho)
        hipLaunchKernelGGL(k_adjoint_argmin, dim3(1), dim3(64), 0, s, grad_rho, p.scal, p.flags);
    PSV_HIP(hipGetLastError());
}

void launch_scale_vol(const Plan& p, const double* x, double* out, hipStream_t s) {
    const int nb = grid_blocks(p.ncell(), RB) * 4;
    hipLaunchKernelGGL(k_scale_vol, dim3(nb), dim3(RB), 0, s, make_geo(p), x, out);
    PSV_HIP(hipGetLastError());
}

void launch_vmean(const Plan& p, const double* r, double* out_scalar, hipStream_t s,
                  const double* scale) {
    const int nb = grid_blocks(p.ncell(), RB);
    hipLaunchKernelGGL(k_vsum, dim3(nb), dim3(RB), 0, s, make_geo(p), r, scale, p.partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(RB), 0, s, p.partials, nb, 1, out_scalar);
    double total = 0.0;
    for (double h : p.h) total += h;
    hipLaunchKernelGGL(k_div_scalar, dim3(1), dim3(64), 0, s, out_scalar, p.dx * p.dy * total * p.nx * p.ny);
    PSV_HIP(hipGetLastError());
}

void launch_mean_finalize(const Plan& p, int nblocks, double* out_scalar, hipStream_t s) {
    const double* src = stage_partials(p, p.partials, nblocks, 1, nullptr, s);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(RB), 0, s, src, nblocks, 1, out_scalar);
    double total = 0.0;
    for (double h : p.h) total += h;
    hipLaunchKernelGGL(k_div_scalar, dim3(1), dim3(64), 0, s, out_scalar, p.dx * p.dy * total * p.nx * p.ny);
    PSV_HIP(hipGetLastError());
}

void launch_fill(double* x, size_t n, double v, hipStream_t s) {
    size_t b = (n + RB - 1) / RB;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_fill, dim3((int)(b < 1 ? 1 : b)), dim3(RB), 0, s, n, x, v);
    PSV_HIP(hipGetLastError());
}

void launch_scan_inputs(const Plan& p, const double* x, int positive, int* bad, hipStream_t s) {
    const int nb = grid_blocks(p.ncell(), RB);
    hipLaunchKernelGGL(k_scan, dim3(nb), dim3(RB), 0, s, p.ncell(), x, positive, bad);
    PSV_HIP(hipGetLastError());
}

}  // namespace psv
