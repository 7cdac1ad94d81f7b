// Batched uneven solves: one plan per problem, every pass of every problem
// expressed as tiles of the same block-level tile functions as the single
// solve (pass_x.hpp, pass_yz.hpp). Two executors share the task code:
//  * per-pass batched kernels: one launch per pass covers the tiles of all
//    problems (a block finds its problem by a prefix table); the sequence of
//    launches, refinement rounds included, is captured once in a HIP graph and
//    replayed;
//  * a persistent kernel: blocks take tickets from a global task queue (passes
//    in dependency order, problems largest first), wait on per-(problem, pass)
//    completion counters with a bounded spin, run the tile and release the
//    counter.
// Mixed precision runs the refinement rounds with device-side convergence
// flags: once a problem converges its remaining tiles return immediately.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "pass_x.hpp"
#include "pass_yz.hpp"

struct psv_batch;

namespace psv {

enum BKind : int {
    K_MINP = 0,  // partial min(rho) with first index
    K_MINF,      // rho0: given value or the reduced minimum
    K_FWD,       // assembly + forward x (CONST or METHOD1)
    K_MEAN,      // FP64 volume-weighted mean of the RHS from the forward partials (mixed)
    K_Y,         // forward y + chunk elimination of the z solve
    K_Z,         // z interface systems + zero mode (mean to S_RHS_MEAN)
    K_Z2,        // same, mean discarded (refinement corrections)
    K_YI,        // z back substitution + inverse y
    K_INV,       // inverse x, store
    K_INVADD,    // inverse x, accumulate
    K_RES,       // fused residual + forward x (refinement)
    K_NRM,       // relres from the residual partials; set done when <= tol
    K_CHK,       // standalone residual (final check)
    K_CHKF,      // relres of the final check
    K_NKIND
};

constexpr int MIN_TILE = 65536;  // cells per min tile
constexpr int RES_TILE = 2048;   // cells per residual tile
constexpr int MAX_MIN_TILES = 256;

struct ProblemDesc {
    XGeom xg;   // forward x tiles (the plan's lines per block and stencil variant)
    XGeom xgi;  // inverse x tiles (the plan's own lines per block)
    Stencil st;
    ZArgs z;  // rhs_mean set per kind at run time
    int method, fp32;
    Radices rad_y;
    const void* twx;
    const void* twy;
    void* spec;
    double* r_ws;
    double* partials;
    double* scal;
    int* flags;
    double tol;
    double vtotal;  // total volume
    size_t ncell;
    int ntiles[K_NKIND];
};

struct ProblemIO {
    const double* f;
    const double* rho;
    const double* pprev;
    double* pout;
    double rho0;  // <= 0: min(rho)
    int want_r;   // store the FP64 RHS (refinement or final check)
};

inline int kind_tiles(const Plan& p, int kind) {
    switch (kind) {
        case K_MINP: return std::min<int>(MAX_MIN_TILES, (int)((p.ncell() + MIN_TILE - 1) / MIN_TILE));
        case K_FWD: case K_RES: return fwd_x_blocks(p);
        case K_INV: case K_INVADD: return (p.ny / p.lp.lbx_inv) * p.nz;
        case K_Y: case K_YI: return yz_tiles(p);
        case K_Z: case K_Z2: return ifc_tiles(p);
        case K_CHK: return (int)((p.ncell() + RES_TILE - 1) / RES_TILE);
        default: return 1;
    }
}

// ---------------------------------------------------------------------------
// device: small tiles
__device__ void minp_tile(const ProblemDesc& D, const ProblemIO& io, int b) {
    __shared__ double sv[256];
    __shared__ int si[256];
    const int nt = D.ntiles[K_MINP];
    const size_t chunk = (D.ncell + nt - 1) / nt;
    const size_t c0 = (size_t)b * chunk, c1 = min(D.ncell, c0 + chunk);
    double best = __builtin_inf();
    int bi = 0x7fffffff;
    for (size_t c = c0 + threadIdx.x; c < c1; c += 256) {
        const double v = ld_stream(io.rho + c);  // read once per solve: streaming
        if (v < best) { best = v; bi = (int)c; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double v = sv[threadIdx.x + o];
            const int i = si[threadIdx.x + o];
            if (v < sv[threadIdx.x] || (v == sv[threadIdx.x] && i < si[threadIdx.x])) {
                sv[threadIdx.x] = v;
                si[threadIdx.x] = i;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        D.partials[b] = sv[0];
        D.partials[MAX_MIN_TILES + b] = (double)si[0];
    }
}

__device__ void minf_tile(const ProblemDesc& D, const ProblemIO& io) {
    if (threadIdx.x != 0) return;
    if (io.rho0 > 0.0) {
        D.scal[S_RHO0] = io.rho0;
        return;
    }
    const int nt = D.ntiles[K_MINP];
    double best = __builtin_inf();
    double bi = 0.0;
    for (int b = 0; b < nt; ++b) {
        const double v = D.partials[b], i = D.partials[MAX_MIN_TILES + b];
        if (v < best || (v == best && i < bi)) { best = v; bi = i; }
    }
    D.scal[S_RHO0] = best;
    D.flags[F_ARGMIN] = (int)bi;
}

// sum of `per` interleaved partials over nb tiles, on thread 0
__device__ double sum_partials(const double* p, int nb, int per, int q, double* red) {
    return block_sum(thread_share(p, nb, per, q), red);
}

__device__ void mean_tile(const ProblemDesc& D, double* red) {
    const double s = sum_partials(D.partials, D.ntiles[K_FWD], 1, 0, red);
    if (threadIdx.x == 0) D.scal[S_RHS_MEAN] = s / D.vtotal;
}

__device__ void nrm_tile(const ProblemDesc& D, int ntiles, double* red, bool set_done) {
    const double2 ab = thread_share2(D.partials, ntiles);
    const double a = block_sum(ab.x, red);
    __syncthreads();
    const double b = block_sum(ab.y, red);
    if (threadIdx.x == 0) {
        const double rr = b > 0.0 ? sqrt(a / b) : 0.0;
        D.scal[S_RELRES] = rr;
        if (set_done && rr <= D.tol) D.flags[F_DONE] = 1;
        if (set_done) D.flags[F_STEPS] += (rr <= D.tol) ? 0 : 1;
    }
}

__device__ void chk_tile(const ProblemDesc& D, const ProblemIO& io, int b, double* red) {
    const XGeom& g = D.xg;
    const double mean = D.scal[S_RHS_MEAN];
    const size_t c0 = (size_t)b * RES_TILE;
    double s1 = 0.0, s2 = 0.0;
    for (int t = threadIdx.x; t < RES_TILE; t += 256) {
        const size_t c = c0 + t;
        if (c >= D.ncell) break;
        const int i = (int)(c % g.nx);
        const size_t q = c / g.nx;
        const int j = (int)(q % g.ny);
        const int k = (int)(q / g.ny);
        const double rp = D.r_ws[c] - mean;
        const double res = rp - lap_cell(io.pout, i, j, k, g, D.st);
        s1 += res * res;
        s2 += rp * rp;
    }
    const double a = block_sum(s1, red);
    __syncthreads();
    const double bb = block_sum(s2, red);
    if (threadIdx.x == 0) {
        D.partials[2 * b] = a;
        D.partials[2 * b + 1] = bb;
    }
}

// ---------------------------------------------------------------------------
// device: one tile of one pass of one problem
#define PSV_BX_SIZES(X) X(16) X(24) X(32) X(48) X(64) X(96) X(128)

template <typename T, int MODE, bool STAGE>
__device__ __forceinline__ void run_fwd_s(const ProblemDesc& D, const FwdArgs& a, int b,
                                          unsigned char* smem, double* red) {
    const c2<T>* tw = reinterpret_cast<const c2<T>*>(D.twx);
    c2<T>* sp = reinterpret_cast<c2<T>*>(D.spec);
    switch (D.xg.M) {
#define PSV_CASE(n) case n: fwd_x_tile<T, T, MODE, n, STAGE>(D.xg, D.st, a, tw, sp, b, smem, red); return;
        PSV_BX_SIZES(PSV_CASE)
#undef PSV_CASE
        default: fwd_x_tile<T, T, MODE, 0, STAGE>(D.xg, D.st, a, tw, sp, b, smem, red); return;
    }
}

// Forward x tile in the problem's stencil variant: SEL = 1 staged rows, 0
// direct loads (per-pass kernels, one launch per variant), -1 chosen from the
// problem's geometry at run time (persistent kernel). The constant-
// coefficient copy has no stencil and always takes the staged variant.
template <typename T, int MODE, int SEL>
__device__ __forceinline__ void run_fwd(const ProblemDesc& D, const FwdArgs& a, int b,
                                        unsigned char* smem, double* red) {
    if constexpr (MODE == FWD_CONST || SEL == 1) {
        run_fwd_s<T, MODE, true>(D, a, b, smem, red);
    } else if constexpr (SEL == 0) {
        run_fwd_s<T, MODE, false>(D, a, b, smem, red);
    } else {
        if (D.xg.stage)
            run_fwd_s<T, MODE, true>(D, a, b, smem, red);
        else
            run_fwd_s<T, MODE, false>(D, a, b, smem, red);
    }
}

template <typename T, int MODE>
__device__ __forceinline__ void run_inv(const ProblemDesc& D, double* out, int b, unsigned char* smem) {
    const c2<T>* tw = reinterpret_cast<const c2<T>*>(D.twx);
    const c2<T>* sp = reinterpret_cast<const c2<T>*>(D.spec);
    const double sc = 2.0 / ((double)D.xg.nx * D.xg.ny);
    switch (D.xgi.M) {
#define PSV_CASE(n) case n: inv_x_tile<T, T, MODE, n>(D.xgi, tw, sp, out, D.st.vol, sc, b, smem); return;
        PSV_BX_SIZES(PSV_CASE)
#undef PSV_CASE
        default: inv_x_tile<T, T, MODE, 0>(D.xgi, tw, sp, out, D.st.vol, sc, b, smem); return;
    }
}

template <typename T, bool INV, int N>
__device__ __forceinline__ void yz_tile(const ProblemDesc& D, c2<T>* sp, const c2<T>* tw, int b,
                                        unsigned char* smem) {
    with_kc(D.z.kc, [&](auto kc) {
        constexpr int KC = decltype(kc)::value;
        if constexpr (INV)
            yz_inv_tile<T, N, KC>(D.z, D.rad_y, sp, tw, b, smem);
        else
            yz_fwd_tile<T, N, KC>(D.z, D.rad_y, sp, tw, b, smem);
    });
}

template <typename T, bool INV>
__device__ __forceinline__ void run_yz(const ProblemDesc& D, int b, unsigned char* smem) {
    const c2<T>* tw = reinterpret_cast<const c2<T>*>(D.twy);
    c2<T>* sp = reinterpret_cast<c2<T>*>(D.spec);
    switch (D.xg.ny) {
#define PSV_CASE(n) case n: yz_tile<T, INV, n>(D, sp, tw, b, smem); return;
        PSV_YZ_SIZES(PSV_CASE)
#undef PSV_CASE
        default: yz_tile<T, INV, 0>(D, sp, tw, b, smem); return;
    }
}

template <typename T>
__device__ __forceinline__ void run_ifc(const ProblemDesc& D, double* mean_out, int b,
                                        unsigned char* smem) {
    ZArgs z = D.z;
    z.rhs_mean = mean_out;
    ifc_tile<T>(z, reinterpret_cast<c2<T>*>(D.spec), b, smem);
}

template <typename T, int KIND, int SEL = -1>
__device__ __forceinline__ void run_task(const ProblemDesc& D, const ProblemIO& io, int b,
                                         unsigned char* smem, double* red) {
    // The done flag is cleared before the first pass and set only by the norm
    // tile of a refinement round, so every tile of a converged problem may
    // return at once.
    if (D.fp32 && D.flags[F_DONE]) return;
    if constexpr (KIND == K_MINP) {
        minp_tile(D, io, b);
    } else if constexpr (KIND == K_MINF) {
        minf_tile(D, io);
    } else if constexpr (KIND == K_FWD) {
        FwdArgs a{};
        a.f = io.f;
        a.rho = io.rho;
        a.pprev = io.pprev;
        a.rho0 = D.scal + S_RHO0;
        a.r_out = io.want_r ? D.r_ws : nullptr;
        a.partials = D.fp32 ? D.partials : nullptr;
        if (D.method == PSV_SPLIT_RHO0) {
            a.mode = FWD_METHOD1;
            run_fwd<T, FWD_METHOD1, SEL>(D, a, b, smem, red);
        } else {
            a.mode = FWD_CONST;
            run_fwd<T, FWD_CONST, SEL>(D, a, b, smem, red);
        }
    } else if constexpr (KIND == K_MEAN) {
        mean_tile(D, red);
    } else if constexpr (KIND == K_Y) {
        run_yz<T, false>(D, b, smem);
    } else if constexpr (KIND == K_YI) {
        run_yz<T, true>(D, b, smem);
    } else if constexpr (KIND == K_Z) {
        run_ifc<T>(D, D.scal + (D.fp32 ? S_MEAN2 : S_RHS_MEAN), b, smem);
    } else if constexpr (KIND == K_Z2) {
        run_ifc<T>(D, D.scal + S_MEAN2, b, smem);
    } else if constexpr (KIND == K_INV) {
        run_inv<T, INV_STORE>(D, io.pout, b, smem);
    } else if constexpr (KIND == K_INVADD) {
        run_inv<T, INV_ADD>(D, io.pout, b, smem);
    } else if constexpr (KIND == K_RES) {
        FwdArgs a{};
        a.mode = FWD_RESID;
        a.r_in = D.r_ws;
        a.pprev = io.pout;
        a.mean = D.scal + S_RHS_MEAN;
        a.partials = D.partials;
        run_fwd<T, FWD_RESID, SEL>(D, a, b, smem, red);
    } else if constexpr (KIND == K_NRM) {
        nrm_tile(D, D.ntiles[K_RES], red, true);
    } else if constexpr (KIND == K_CHK) {
        chk_tile(D, io, b, red);
    } else if constexpr (KIND == K_CHKF) {
        nrm_tile(D, D.ntiles[K_CHK], red, false);
    }
}

// Per-pass batched kernel: block -> (problem, tile) through start[] (prefix of
// tile counts, nprob + 1 entries). SEL: stencil variant of the forward x
// kinds (problems of the other variant have no tiles in this launch).
template <typename T, int KIND, int SEL>
__global__ void __launch_bounds__(256) k_batch_pass(const ProblemDesc* __restrict__ desc,
                                                     const ProblemIO* __restrict__ io,
                                                     const int* __restrict__ start, int nprob) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[16];
    const int blk = blockIdx.x;
    int lo = 0, hi = nprob;  // largest p with start[p] <= blk
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= blk) lo = mid; else hi = mid;
    }
    run_task<T, KIND, SEL>(desc[lo], io[lo], blk - start[lo], smem_raw, red);
}

// Persistent executor. Tasks are int4 {problem, level, tile, tiles of the
// previous level of that problem}; the queue holds every level of every
// problem, level by level, problems largest first, so whatever a task waits
// for was dequeued earlier by a running block and the wait always ends.
// A wait that exceeds the spin budget sets *error and the block carries on
// (the kernel always drains); the host then reports the failure.
struct PersistArgs {
    const ProblemDesc* desc;
    const ProblemIO* io;
    const int4* tasks;
    const int* kinds;  // kind of each level
    int* counters;     // [nprob][nlevels] completed tiles
    int* ticket;
    int* error;
    int ntasks;
    int nlevels;
    int chunk;  // tasks per ticket
};

constexpr long long SPIN_LIMIT = 1ll << 22;  // x s_sleep(2): well above any legitimate wait

template <typename T>
__device__ __forceinline__ void run_kind(int kind, const ProblemDesc& D, const ProblemIO& io, int b,
                                         unsigned char* smem, double* red) {
    switch (kind) {
#define PSV_K(k) case k: run_task<T, k>(D, io, b, smem, red); break;
        PSV_K(K_MINP) PSV_K(K_MINF) PSV_K(K_FWD) PSV_K(K_MEAN) PSV_K(K_Y) PSV_K(K_Z) PSV_K(K_Z2)
        PSV_K(K_YI) PSV_K(K_INV) PSV_K(K_INVADD) PSV_K(K_RES) PSV_K(K_NRM) PSV_K(K_CHK)
        PSV_K(K_CHKF)
#undef PSV_K
        default: break;
    }
}

// Tickets hand out TICKET_TASKS consecutive tasks at a time. The queue is
// ordered by pass, so a run of tasks usually shares its (problem, pass): the
// block waits on that group's dependency once and releases its completions
// with one counter update. The smallest unfinished task always has its
// dependencies (earlier in the queue) done and is the current task of its
// block, so the executor cannot deadlock.
// Synchronisation is costly on a multi-XCD GPU: each XCD has its own L2, so
// a release at device scope writes the L2's dirty lines back and an acquire
// invalidates the caches. Only thread 0 of a block releases (one atomic per
// run of completions, no separate fence) and acquires (the wait's atomic
// load, then a block barrier). Longer tickets mean fewer of both but leave
// fewer blocks working on each pass while the others wait on it: on a batch
// of 64 problems of 0.26-3.1 million cells, 8 tasks per ticket took 25.6 ms,
// 4 took 29.2, 32 took 30.6 and 128 took 57.5.
constexpr int TICKET_TASKS = 8;

template <typename T>
__global__ void __launch_bounds__(256) k_batch_persistent(PersistArgs A) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[16];
    __shared__ int s_task;
    for (;;) {
        __syncthreads();  // the previous task is done with LDS and s_task
        if (threadIdx.x == 0) s_task = atomicAdd(A.ticket, A.chunk);
        __syncthreads();
        const int t0 = s_task;
        if (t0 >= A.ntasks) break;
        const int t1 = min(t0 + A.chunk, A.ntasks);
        int* cnt_done = nullptr;  // counter of the group whose completions are pending
        int pending = 0;
        for (int t = t0; t < t1; ++t) {
            const int4 tk = A.tasks[t];
            int* cnt = A.counters + (size_t)tk.x * A.nlevels;
            if (cnt + tk.y != cnt_done) {
                if (pending && threadIdx.x == 0)
                    __hip_atomic_fetch_add(cnt_done, pending, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                pending = 0;
                cnt_done = cnt + tk.y;
                if (threadIdx.x == 0 && tk.y > 0) {
                    long long spins = 0;
                    while (__hip_atomic_load(cnt + tk.y - 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < tk.w) {
                        __builtin_amdgcn_s_sleep(2);
                        if (++spins > SPIN_LIMIT) {
                            atomicOr(A.error, 1);
                            break;
                        }
                        // once any wait has failed, no block waits again: the drain is bounded
                        if ((spins & 255) == 0 &&
                            __hip_atomic_load(A.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                            break;
                    }
                }
                __syncthreads();  // thread 0's acquire covers the block (one L1 per CU)
            }
            run_kind<T>(A.kinds[tk.y], A.desc[tk.x], A.io[tk.x], tk.z, smem_raw, red);
            __syncthreads();  // the tile is complete and its LDS free
            ++pending;
        }
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(cnt_done, pending, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_persist_reset(ProblemDesc* desc, int n, int* counters, int ncount, int* ticket,
                                int* error) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        desc[i].flags[F_DONE] = 0;
        desc[i].flags[F_STEPS] = 0;
    }
    if (i < ncount) counters[i] = 0;
    if (i == 0) {
        *ticket = 0;
        *error = 0;
    }
}

// ---------------------------------------------------------------------------
// host
struct PassLaunch {
    int kind;
    int sel;     // forward x kinds: stencil variant of this launch (1 staged, 0 direct)
    int refine;  // refinement tile: skipped when the problem converged
    int nblk;
    size_t lds;
    int* d_start;
};

}  // namespace psv

struct psv_batch {
    std::vector<psv::Plan*> plans;
    psv_opts opts{};
    int n = 0;
    bool fp32 = false;
    psv::ProblemDesc* d_desc = nullptr;
    psv::ProblemIO* d_io = nullptr;
    psv::ProblemIO* h_io = nullptr;  // pinned
    // the copy of h_io to d_io reads h_io when the stream reaches it: the next
    // call waits for this event before it rewrites the table
    hipEvent_t io_copied = nullptr;
    bool io_pending = false;
    std::vector<psv::PassLaunch> seq[2];  // per graph: without / with the final check
    std::vector<int*> starts[2];
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int device = 0;
    // persistent executor (per graph)
    int persistent = 0;
    int4* d_tasks[2] = {nullptr, nullptr};
    int* d_kinds[2] = {nullptr, nullptr};
    int ntasks[2] = {0, 0};
    int nlevels[2] = {0, 0};
    size_t plds[2] = {0, 0};
    int* d_counters = nullptr;  // sized for the longer sequence
    int ncounters = 0;
    int* d_ticket = nullptr;    // [0] ticket, [1] error
    int* h_err = nullptr;       // pinned
};

namespace psv {

void plan_init(Plan& p, const psv_grid& g, const psv_opts& o, bool alloc_ws);
void plan_free(Plan& p);

static size_t kind_lds(const Plan& p, int kind, bool fp32) {
    const size_t cs = fp32 ? sizeof(float2) : sizeof(double2);
    switch (kind) {
        case K_FWD: case K_RES: return fwd_x_lds(make_xgeom(p), cs);
        case K_INV: case K_INVADD: return inv_x_lds(make_xgeom(p, true), cs);
        case K_Y: case K_YI: return yz_lds(p.ny, p.lp.kc, cs);
        case K_Z: case K_Z2: return ifc_lds(p);
        default: return 0;
    }
}

template <typename T, int KIND, int SEL>
static void launch_pass_k(const psv_batch& B, const PassLaunch& L, hipStream_t s) {
    allow_lds(k_batch_pass<T, KIND, SEL>, L.lds);
    hipLaunchKernelGGL((k_batch_pass<T, KIND, SEL>), dim3(L.nblk), dim3(256), L.lds, s, B.d_desc,
                       B.d_io, L.d_start, B.n);
}

template <typename T>
static void launch_pass(const psv_batch& B, const PassLaunch& L, hipStream_t s) {
    switch (L.kind) {
#define PSV_K(k) case k: launch_pass_k<T, k, 1>(B, L, s); break;
        PSV_K(K_MINP) PSV_K(K_MINF) PSV_K(K_MEAN) PSV_K(K_Y) PSV_K(K_Z) PSV_K(K_Z2)
        PSV_K(K_YI) PSV_K(K_INV) PSV_K(K_INVADD) PSV_K(K_NRM) PSV_K(K_CHK) PSV_K(K_CHKF)
#undef PSV_K
        case K_FWD:
            if (L.sel) launch_pass_k<T, K_FWD, 1>(B, L, s); else launch_pass_k<T, K_FWD, 0>(B, L, s);
            break;
        case K_RES:
            if (L.sel) launch_pass_k<T, K_RES, 1>(B, L, s); else launch_pass_k<T, K_RES, 0>(B, L, s);
            break;
    }
    PSV_HIP(hipGetLastError());
}

__global__ void k_batch_reset(ProblemDesc* desc, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) {
        desc[p].flags[F_DONE] = 0;
        desc[p].flags[F_STEPS] = 0;
    }
}

std::vector<int> batch_sequence(bool fp32, int method, int rounds, bool check) {
    std::vector<int> k;
    if (method == PSV_SPLIT_RHO0) {
        k.push_back(K_MINP);
        k.push_back(K_MINF);
    }
    k.push_back(K_FWD);
    if (fp32) k.push_back(K_MEAN);
    k.insert(k.end(), {K_Y, K_Z, K_YI, K_INV});
    if (fp32) {
        for (int r = 0; r < rounds; ++r) k.insert(k.end(), {K_RES, K_NRM, K_Y, K_Z2, K_YI, K_INVADD});
    }
    if (check || fp32) k.insert(k.end(), {K_CHK, K_CHKF});
    return k;
}

void batch_build(psv_batch& B, bool check) {
    const int gi = check ? 1 : 0;
    const int rounds = B.fp32 ? std::max(1, std::min(B.opts.max_refine, 3)) : 0;
    const std::vector<int> kinds = batch_sequence(B.fp32, B.opts.method, rounds, check);
    B.seq[gi].clear();
    for (int kind : kinds) {
        // the forward x kinds of a Method-I batch run as one launch per
        // stencil variant, each over the problems whose plan takes it
        const bool split = (kind == K_FWD && B.opts.method == PSV_SPLIT_RHO0) || kind == K_RES;
        for (int sel : {1, 0}) {
            if (!split && sel == 0) continue;
            PassLaunch L{};
            L.kind = kind;
            L.sel = sel;
            std::vector<int> st(B.n + 1, 0);
            size_t lds = 0;
            for (int p = 0; p < B.n; ++p) {
                const bool mine = !split || B.plans[p]->lp.xstage == sel;
                st[p + 1] = st[p] + (mine ? kind_tiles(*B.plans[p], kind) : 0);
                if (mine) lds = std::max(lds, kind_lds(*B.plans[p], kind, B.fp32));
            }
            if (st[B.n] == 0) continue;
            L.nblk = st[B.n];
            L.lds = lds;
            int* d = nullptr;
            PSV_HIP(hipMalloc(&d, st.size() * sizeof(int)));
            PSV_HIP(hipMemcpy(d, st.data(), st.size() * sizeof(int), hipMemcpyHostToDevice));
            B.starts[gi].push_back(d);
            L.d_start = d;
            B.seq[gi].push_back(L);
        }
    }
    // persistent queue: level by level, problems largest first (LPT)
    std::vector<int> order(B.n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return B.plans[a]->ncell() > B.plans[b]->ncell();
    });
    std::vector<int4> tasks;
    const int nlev = (int)kinds.size();
    size_t plds = 0;
    for (int lev = 0; lev < nlev; ++lev) {
        for (int p : order) {
            const int nt = kind_tiles(*B.plans[p], kinds[lev]);
            const int dep = lev > 0 ? kind_tiles(*B.plans[p], kinds[lev - 1]) : 0;
            for (int t = 0; t < nt; ++t) tasks.push_back(int4{p, lev, t, dep});
            plds = std::max(plds, kind_lds(*B.plans[p], kinds[lev], B.fp32));
        }
    }
    B.ntasks[gi] = (int)tasks.size();
    B.nlevels[gi] = nlev;
    B.plds[gi] = plds;
    PSV_HIP(hipMalloc(&B.d_tasks[gi], tasks.size() * sizeof(int4)));
    PSV_HIP(hipMemcpy(B.d_tasks[gi], tasks.data(), tasks.size() * sizeof(int4), hipMemcpyHostToDevice));
    PSV_HIP(hipMalloc(&B.d_kinds[gi], kinds.size() * sizeof(int)));
    PSV_HIP(hipMemcpy(B.d_kinds[gi], kinds.data(), kinds.size() * sizeof(int), hipMemcpyHostToDevice));
    if (B.n * nlev > B.ncounters) {
        if (B.d_counters) PSV_HIP(hipFree(B.d_counters));
        B.ncounters = B.n * nlev;
        PSV_HIP(hipMalloc(&B.d_counters, B.ncounters * sizeof(int)));
    }
}

template <typename T>
static void launch_persistent(const psv_batch& B, int gi, hipStream_t s) {
    const int ncount = B.n * B.nlevels[gi];
    const int rn = std::max(B.n, ncount);
    hipLaunchKernelGGL(k_persist_reset, dim3((rn + 255) / 256), dim3(256), 0, s, B.d_desc, B.n,
                       B.d_counters, ncount, B.d_ticket, B.d_ticket + 1);
    int per_cu = 0, ncu = 0;
    allow_lds(k_batch_persistent<T>, B.plds[gi]);
    PSV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent<T>, 256,
                                                         B.plds[gi]));
    PSV_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, B.device));
    const int grid = std::max(1, std::min(per_cu, 8) * ncu);
    PersistArgs A{B.d_desc, B.d_io, B.d_tasks[gi], B.d_kinds[gi], B.d_counters,
                  B.d_ticket, B.d_ticket + 1, B.ntasks[gi], B.nlevels[gi], TICKET_TASKS};
    hipLaunchKernelGGL(k_batch_persistent<T>, dim3(grid), dim3(256), B.plds[gi], s, A);
    PSV_HIP(hipGetLastError());
}

void batch_enqueue(const psv_batch& B, int gi, hipStream_t s) {
    if (B.persistent) {
        if (B.fp32)
            launch_persistent<float>(B, gi, s);
        else
            launch_persistent<double>(B, gi, s);
        return;
    }
    hipLaunchKernelGGL(k_batch_reset, dim3((B.n + 255) / 256), dim3(256), 0, s, B.d_desc, B.n);
    for (const PassLaunch& L : B.seq[gi]) {
        if (B.fp32)
            launch_pass<float>(B, L, s);
        else
            launch_pass<double>(B, L, s);
    }
}

void batch_create(psv_batch& B, int n, const psv_grid* grids, const psv_opts& o) {
    B.n = n;
    B.opts = o;
    B.fp32 = o.precision == PSV_MIXED;
    PSV_HIP(hipGetDevice(&B.device));
    std::vector<ProblemDesc> desc(n);
    for (int p = 0; p < n; ++p) {
        Plan* pl = new Plan();
        B.plans.push_back(pl);
        plan_init(*pl, grids[p], o, true);
        const int need = 2 * kind_tiles(*pl, K_CHK) + 64;
        if (need > pl->n_partials) {
            PSV_HIP(hipFree(pl->partials));
            pl->n_partials = need;
            PSV_HIP(hipMalloc(&pl->partials, need * sizeof(double)));
        }
        ProblemDesc& D = desc[p];
        std::memset(&D, 0, sizeof(D));
        D.xg = make_xgeom(*pl);
        D.xgi = make_xgeom(*pl, true);
        D.st = Stencil{pl->t.inv_h, pl->t.inv_g, pl->t.vol};
        D.z = make_zargs(*pl, pl->scal + S_RHS_MEAN);
        D.method = o.method;
        D.fp32 = B.fp32 ? 1 : 0;
        D.rad_y = pl->rad_y;
        D.twx = B.fp32 ? (const void*)pl->t.twx32 : (const void*)pl->t.twx64;
        D.twy = B.fp32 ? (const void*)pl->t.twy32 : (const void*)pl->t.twy64;
        D.spec = pl->spec;
        D.r_ws = pl->r_ws;
        D.partials = pl->partials;
        D.scal = pl->scal;
        D.flags = pl->flags;
        D.tol = pl->opts.tol;
        double hsum = 0.0;
        for (double h : pl->h) hsum += h;
        D.vtotal = pl->dx * pl->dy * hsum * pl->nx * pl->ny;
        D.ncell = pl->ncell();
        for (int k = 0; k < K_NKIND; ++k) D.ntiles[k] = kind_tiles(*pl, k);
    }
    PSV_HIP(hipMalloc(&B.d_desc, n * sizeof(ProblemDesc)));
    PSV_HIP(hipMemcpy(B.d_desc, desc.data(), n * sizeof(ProblemDesc), hipMemcpyHostToDevice));
    PSV_HIP(hipMalloc(&B.d_io, n * sizeof(ProblemIO)));
    PSV_HIP(hipHostMalloc(&B.h_io, n * sizeof(ProblemIO)));
    std::memset(B.h_io, 0, n * sizeof(ProblemIO));
    PSV_HIP(hipEventCreateWithFlags(&B.io_copied, hipEventDisableTiming));
    PSV_HIP(hipMalloc(&B.d_ticket, 2 * sizeof(int)));
    PSV_HIP(hipHostMalloc(&B.h_err, sizeof(int)));
    *B.h_err = 0;
    B.persistent = (o.batch_executor == 2) ? 1 : 0;
}

void batch_free(psv_batch& B) {
    for (int i = 0; i < 2; ++i) {
        if (B.exec[i]) (void)hipGraphExecDestroy(B.exec[i]);
        if (B.graph[i]) (void)hipGraphDestroy(B.graph[i]);
    }
    for (int i = 0; i < 2; ++i) {
        for (int* d : B.starts[i]) (void)hipFree(d);
        if (B.d_tasks[i]) (void)hipFree(B.d_tasks[i]);
        if (B.d_kinds[i]) (void)hipFree(B.d_kinds[i]);
    }
    if (B.d_counters) (void)hipFree(B.d_counters);
    if (B.d_ticket) (void)hipFree(B.d_ticket);
    if (B.h_err) (void)hipHostFree(B.h_err);
    for (Plan* p : B.plans) {
        plan_free(*p);
        delete p;
    }
    if (B.d_desc) (void)hipFree(B.d_desc);
    if (B.d_io) (void)hipFree(B.d_io);
    if (B.h_io) (void)hipHostFree(B.h_io);
    if (B.io_copied) (void)hipEventDestroy(B.io_copied);
}

// One batched solve: upload the per-call pointer table, then replay the
// captured graph (captured on first use for this `check` setting).
void batch_solve(psv_batch& B, hipStream_t s, bool check) {
    PSV_HIP(hipMemcpyAsync(B.d_io, B.h_io, B.n * sizeof(ProblemIO), hipMemcpyHostToDevice, s));
    PSV_HIP(hipEventRecord(B.io_copied, s));
    B.io_pending = true;
    const int gi = check ? 1 : 0;
    if (!B.exec[gi]) {
        batch_build(B, check);
        hipStream_t cs;
        PSV_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        PSV_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        batch_enqueue(B, gi, cs);
        PSV_HIP(hipStreamEndCapture(cs, &B.graph[gi]));
        PSV_HIP(hipGraphInstantiate(&B.exec[gi], B.graph[gi], nullptr, nullptr, 0));
        PSV_HIP(hipStreamDestroy(cs));
    }
    PSV_HIP(hipGraphLaunch(B.exec[gi], s));
}

psv_batch* batch_new() { return new psv_batch(); }

void batch_delete(psv_batch* b) {
    batch_free(*b);
    delete b;
}

int batch_size(const psv_batch& B) { return B.n; }
int batch_method(const psv_batch& B) { return B.opts.method; }
bool batch_fp32(const psv_batch& B) { return B.fp32; }

void batch_set_io(psv_batch& B, int p, const double* f, const double* rho, const double* pprev,
                  double* pout, double rho0, bool want_r) {
    // the previous call's copy of the table may still be queued behind work
    // on its stream
    if (B.io_pending) {
        PSV_HIP(hipEventSynchronize(B.io_copied));
        B.io_pending = false;
    }
    ProblemIO& io = B.h_io[p];
    io.f = f;
    io.rho = rho;
    io.pprev = pprev;
    io.pout = pout;
    io.rho0 = rho0;
    io.want_r = want_r ? 1 : 0;
}

// Synchronises and fills one psv_info per problem; false if a mixed-precision
// problem missed its tolerance.
bool batch_infos(psv_batch& B, hipStream_t s, psv_info* infos) {
    PSV_HIP(hipStreamSynchronize(s));
    if (B.persistent) {
        PSV_HIP(hipMemcpy(B.h_err, B.d_ticket + 1, sizeof(int), hipMemcpyDeviceToHost));
        if (*B.h_err) fail(PSV_ERR_HIP, "persistent batch: a dependency wait exceeded its spin budget");
    }
    bool ok = true;
    for (int p = 0; p < B.n; ++p) {
        Plan& P = *B.plans[p];
        PSV_HIP(hipMemcpy(P.host_scal, P.scal, S_NSCAL * sizeof(double), hipMemcpyDeviceToHost));
        PSV_HIP(hipMemcpy(P.host_flags, P.flags, F_NFLAG * sizeof(int), hipMemcpyDeviceToHost));
        infos[p].refine_steps = P.host_flags[F_STEPS];
        infos[p].relres = P.host_scal[S_RELRES];
        infos[p].rhs_mean_removed = P.host_scal[S_RHS_MEAN];
        infos[p].rho0_used = P.host_scal[S_RHO0];
        for (int i = 0; i < PSV_RELRES_HISTORY; ++i) infos[p].relres_sweep[i] = NAN;
        if (B.fp32 && !(infos[p].relres <= P.opts.tol)) ok = false;
    }
    return ok;
}

}  // namespace psv
