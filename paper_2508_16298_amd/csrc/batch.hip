// Many independent chains of uneven lattice sizes advanced together
// (configuration with one chain per lattice, all on one device).
//
// Each chain keeps its own handle (bond tables, e^{i theta} caches, solver
// workspace).  The chains' angles, momenta and forces live in concatenated
// arrays, so the leapfrog kick and drift are one launch for all chains and
// the e^{i theta} caches are rebuilt by one launch per precision.  The
// solves -- where the time goes -- run batched: one launch of k_b_cg_iter
// performs one CG iteration of every chain, a workgroup per (chain, time
// slice) taken from a work list; every chain has its own scalar slots, its
// own reliable updates and its own stop state, decided on the device.  A
// chunk of kChunk iteration launches followed by the batched reliable-update
// step (FP64 O x, residual replacement, check) is captured once into a
// hipGraph and replayed; the host only polls a per-chain result record
// between replays, one replay ahead.  Finished chains are frozen in the
// device table and their workgroups exit at once.
//
// Tile shape (cells per thread, exchange buffers) is chosen per working
// precision when the batch is created, by timing every candidate on the
// batch's own lattices (the autotuner).
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cg_body.h"

namespace qh {

static constexpr int kChunk = kCap + 1;  // iteration launches per replay
static constexpr int kBS = 256;          // launch bound of the batched slice kernels
static constexpr int kNRes = 8;          // doubles per chain in the result record

// per-chain record of a finished solve
enum { RS_ITERS = 0, RS_TRUE = 1, RS_B2 = 2, RS_NREL = 3, RS_DONE = 4 };

template <typename R>
struct ChainDev {
    Lat lt;
    CgBufs<R> B;
    const cplx<R>* gauge;
    const cplx<double>* gauge64;
    double* scal;  // this chain's two slots of S_NSLOT doubles
    Coef<R> co;
    Coef<double> co64;
    int maxit;   // host: iteration budget of the solve
    int mixed;   // host: 1 for the mixed-precision recursion
    int it0;     // device: iterations done at the start of the current chunk
    int rel0;    // device: parity of the iterations since the last update at the start of the chunk
    int frozen;  // device: 1 once the solve of this chain is final
};

// A workgroup of kBS threads runs kBS / G consecutive slices tau0, tau0 + 1,
// ... of one chain, a group of G threads per slice (G: the smallest power of
// two from 16 up with G x cells per thread >= the slice's cells).  Groups past
// the chain's last slice are padding: they take part in the barriers, own no
// cell and write nothing.
struct Blk {
    int chain, tau0, G;  // chain < 0: padding block
};

// This thread's group: its slice (an in-range stand-in for padding groups),
// its exchange buffers (gbytes each, in group order) and the workgroup's
// reduction scratch after the last group's buffers.
__device__ __forceinline__ Tile blk_tile(const Blk& b, int Nt, unsigned char* smem, size_t gbytes, int& tau) {
    const int g = (int)threadIdx.x / b.G;
    tau = b.tau0 + g;
    const bool valid = tau < Nt;
    if (!valid) tau = b.tau0;
    return Tile{(int)threadIdx.x - g * b.G, b.G, valid, smem + g * gbytes,
                reinterpret_cast<double*>(smem + (size_t)(kBS / b.G) * gbytes)};
}

template <typename R, int NB>
__device__ __forceinline__ size_t group_lds(const Lat& lt) {
    return (size_t)NB * 2 * lt.Vs * sizeof(cplx<R>);
}


// ---------------------------------------------------------------------------
// Batched slice kernels: block -> (chain, tau) from the work list
// ---------------------------------------------------------------------------
template <typename R, int MC, int NB>
__global__ __launch_bounds__(kBS) void k_b_cg_start(const ChainDev<R>* __restrict__ tab, const Blk* __restrict__ blk,
                                                    double* __restrict__ res) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Blk b = blk[blockIdx.x];
    if (b.chain < 0) return;
    const ChainDev<R>& d = tab[b.chain];
    int tau;
    const Tile tl = blk_tile(b, d.lt.Nt, smem, group_lds<R, NB>(d.lt), tau);
    cg_start_body<R, MC, NB>(d.lt, d.B, d.gauge, d.co, d.scal, tau, tl.valid && tau == 0, tl);
    if (b.tau0 == 0 && threadIdx.x < kNRes) res[kNRes * b.chain + threadIdx.x] = 0.0;
}

template <typename R, int MC, int NB>
__global__ __launch_bounds__(kBS) void k_b_cg_iter(const ChainDev<R>* __restrict__ tab, const Blk* __restrict__ blk,
                                                   int kpar, int k, double tol2) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Blk b = blk[blockIdx.x];
    if (b.chain < 0) return;
    const ChainDev<R>& d = tab[b.chain];
    if (d.frozen) return;
    const int it = d.it0 + k;  // the iteration count if the chain ran every launch of this chunk
    if (it >= d.maxit) {
        // budget used: carry the state over, mark it for the final true residual
        if (b.tau0 == 0 && threadIdx.x < S_NSLOT) {
            double v = d.scal[S_NSLOT * kpar + threadIdx.x];
            if (threadIdx.x == S_DONE && v == 0.0) v = 6.0;
            d.scal[S_NSLOT * (kpar ^ 1) + threadIdx.x] = v;
        }
        return;
    }
    int tau;
    const Tile tl = blk_tile(b, d.lt.Nt, smem, group_lds<R, NB>(d.lt), tau);
    cg_iter_body<R, MC, NB>(d.lt, d.B, d.gauge, d.co, d.scal, kpar, (d.rel0 + k) & 1, tol2, d.mixed, d.maxit, tau,
                            tl.valid && tau == 0, tl);
}

// FP64 O x of the chains that stopped or paused
template <typename R, int MC, int NB>
__global__ __launch_bounds__(kBS) void k_b_ox(const ChainDev<R>* __restrict__ tab, const Blk* __restrict__ blk,
                                              int kpar) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Blk b = blk[blockIdx.x];
    if (b.chain < 0) return;
    const ChainDev<R>& d = tab[b.chain];
    if (d.frozen || !gate_open(d.scal[S_NSLOT * kpar + S_DONE])) return;
    int tau;
    const Tile tl = blk_tile(b, d.lt.Nt, smem, group_lds<double, NB>(d.lt), tau);
    SliceCtx<MC> c;
    slice_ctx<MC>(d.lt, c, tau, tl);
    const size_t Vs = d.lt.Vs;
    cplx<double> hm[MC][12], ht[MC][12];
    hops_of<double, MC>(d.gauge64, d.lt, c.tm, c.idx, d.co64, hm);
    hops_of<double, MC>(d.gauge64, d.lt, c.tau, c.idx, d.co64, ht);
    Cells<double, MC> vm, vt, vn, o;
    load_cells<double, MC>(vm, d.B.x + c.tm * Vs, c.g, c.own);
    load_cells<double, MC>(vt, d.B.x + c.tau * Vs, c.g, c.own);
    load_cells<double, MC>(vn, d.B.x + c.tp * Vs, c.g, c.own);
    mdagm_cells<double, MC, NB>(vm, vt, vn, hm, ht, c.g, c.own, d.co64, c.tau == 0 ? -1.0 : 1.0,
                                c.tau == d.lt.Nt - 1 ? -1.0 : 1.0, reinterpret_cast<cplx<double>*>(tl.buf), d.lt.Vs, o);
    store_cells<double, MC>(o, const_cast<cplx<double>*>(d.B.Ox) + c.tau * Vs, c.g, c.own);
}

template <typename R, int MC, int NB>
__global__ __launch_bounds__(kBS) void k_b_cg_replace(const ChainDev<R>* __restrict__ tab,
                                                      const Blk* __restrict__ blk, int kpar) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Blk b = blk[blockIdx.x];
    if (b.chain < 0) return;
    const ChainDev<R>& d = tab[b.chain];
    if (d.frozen || !gate_open(d.scal[S_NSLOT * kpar + S_DONE])) return;
    int tau;
    const Tile tl = blk_tile(b, d.lt.Nt, smem, group_lds<R, NB>(d.lt), tau);
    cg_replace_body<R, MC, NB>(d.lt, d.B, d.gauge, d.co, d.scal, kpar, tau, tl);
}

// One block per chain: the FP64 true residual decides -- converged (5),
// failed (4: budget used, no progress across three updates, non-finite) or
// resume (0, with a restart beta = 0 on the FP64 path and after a
// non-positive denominator).  Writes the chain's result record when final.
template <typename R>
__global__ void k_b_cg_check(ChainDev<R>* __restrict__ tab, int kpar, double* __restrict__ res) {
    __shared__ double red[kNP * 16 + 16];
    ChainDev<R>* d = tab + blockIdx.x;
    if (d->frozen) return;
    double* sl = d->scal + S_NSLOT * kpar;
    const double done = sl[S_DONE];
    const int it = (int)sl[S_ITERS];
    int nd = done == 4.0 ? 4 : -1;
    if (gate_open(done)) {
        double pr[kNP];
        reduce_partials(d->B.part, d->lt.Nt, whole_block_tile(nullptr, red), pr);  // the replacement's (parity 0)
        if (threadIdx.x == 0) {
            const double tr = pr[5];
            const int stall = (it + 1 == (int)sl[S_LASTUP]) ? (int)sl[S_STALL] + 1 : 0;
            sl[S_STALL] = stall;
            sl[S_LASTUP] = it + 1;
            sl[S_NREL] += 1.0;
            sl[S_TRUE] = tr;
            if (!isfinite(tr))
                nd = 4;
            else if (tr <= sl[S_TARGET])
                nd = 5;
            else if (it >= d->maxit || stall >= 3)
                nd = 4;
            else {
                nd = 0;
                if (!d->mixed || done == 3.0) sl[S_FIRST] = 1.0;
                sl[S_ITUPD] = it;
                sl[S_RRUPD] = pr[0];
            }
            sl[S_DONE] = nd;
        }
    }
    if (threadIdx.x == 0) {
        d->it0 = it;
        d->rel0 = (it - (int)sl[S_ITUPD]) & 1;
        if (nd == 4 || nd == 5) {
            d->frozen = 1;
            double* r = res + kNRes * blockIdx.x;
            r[RS_ITERS] = it;
            r[RS_TRUE] = sl[S_TRUE];
            r[RS_B2] = sl[S_B2];
            r[RS_NREL] = sl[S_NREL];
            r[RS_DONE] = nd;
        }
    }
}

// e^{i theta} caches of every chain (same arithmetic as the single-lattice
// cache: FP64 sincos rounded once)
template <typename R>
__global__ void k_b_gauge(const ChainDev<R>* __restrict__ tab, const double* __restrict__ theta,
                          const int64_t* __restrict__ toff) {
    const int c = blockIdx.y;
    const int64_t o = toff[c], n = toff[c + 1] - o;
    cplx<R>* g = const_cast<cplx<R>*>(tab[c].gauge);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s, co;
        sincos(theta[o + i], &s, &co);
        g[i] = mk<R>((R)co, (R)s);
    }
}

}  // namespace qh

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct qedhmc_batch {
    int n = 0;
    hipStream_t user = nullptr;    // the caller's stream
    hipStream_t stream = nullptr;  // the batch's own stream (graph capture needs a non-null stream)
    hipEvent_t ev_in = nullptr;    // orders the batch's work after the caller's
    size_t max_lds = 0;
    std::vector<qedhmc_params> params;
    std::vector<qedhmc_ctx*> ctx;
    std::vector<int64_t> toff;  // theta / momentum / force offsets in doubles (2N per chain), n + 1
    std::vector<int64_t> voff;  // vector offsets in complex elements (N per chain), n + 1
    int maxL = 0, maxVs = 0, maxcell = 0;
    int nblocks[4] = {0, 0, 0, 0};                  // work-list length per tile shape
    qh::Blk* d_blk[4] = {nullptr, nullptr, nullptr, nullptr};  // work list per tile shape
    int64_t* d_toff = nullptr;
    double* d_scal = nullptr;  // n x 2 x S_NSLOT
    double* d_res = nullptr;   // n x kNRes
    void* d_tab[2] = {nullptr, nullptr};  // ChainDev<float>[n], ChainDev<double>[n]
    void* h_tab[2] = {nullptr, nullptr};
    double* h_res[2] = {nullptr, nullptr};  // pinned, one per replay in flight
    hipEvent_t ev[2] = {nullptr, nullptr};
    double *mom = nullptr, *force = nullptr, *force_b = nullptr, *theta0 = nullptr;  // concatenated, 2N per chain
    int shape[2] = {0, 0};          // chosen tile shape per working precision (FP32, FP64)
    float tune_us[2][4] = {};       // per-iteration time of each candidate (0: not a candidate)
    hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [R is double][start parity]
    double graph_tol2[2][2] = {{-1, -1}, {-1, -1}};
    // every chain reads chain 0's phase caches: one gauge field, many right-hand
    // sides (the multi-RHS solve of the stochastic estimation)
    bool shared = false;
};

namespace qh {

// tile shapes: (cells per thread, exchange buffers)
static constexpr int kShapeMC[4] = {1, 2, 1, 2};
static constexpr int kShapeNB[4] = {2, 2, 1, 1};

template <typename F>
static qedhmc_status with_bshape(int shape, F&& f) {
    switch (shape) {
        case 0: return f.template operator()<1, 2>();
        case 1: return f.template operator()<2, 2>();
        case 2: return f.template operator()<1, 1>();
        default: return f.template operator()<2, 1>();
    }
}

// threads per slice of a chain under a tile shape (0: the slice does not fit)
static int group_threads(const Lat& lt, int shape) {
    const int need = (lt.ncell + kShapeMC[shape] - 1) / kShapeMC[shape];
    int G = 16;
    while (G < need) G *= 2;
    return G <= kBS ? G : 0;
}

// dynamic LDS of a workgroup: the exchange buffers of its kBS / G groups (the
// largest over the chains) and the reduction scratch
static size_t shape_lds(const qedhmc_batch* b, int shape, size_t csz) {
    size_t most = 0;
    for (const qedhmc_ctx* h : b->ctx) {
        const int G = group_threads(h->lat, shape);
        if (G > 0) most = std::max(most, (size_t)(kBS / G) * kShapeNB[shape] * 2 * h->lat.Vs * csz);
    }
    return most + (kNP * 16 + 16) * sizeof(double);
}

static bool shape_ok(const qedhmc_batch* b, int shape) {
    for (const qedhmc_ctx* h : b->ctx)
        if (group_threads(h->lat, shape) == 0) return false;
    return shape_lds(b, shape, sizeof(cplx<double>)) <= b->max_lds;
}

// Work list of a tile shape: one entry per run of kBS / G consecutive slices
// of a chain.  Workgroup i runs on XCD i mod 8, so the list is dealt out in 8
// contiguous ranges and each XCD's L2 sees whole runs of neighbouring slices
// (the tau - 1 / tau + 1 halos stay local).
static std::vector<Blk> work_list(const qedhmc_batch* b, int shape) {
    std::vector<Blk> work;
    for (int c = 0; c < b->n; c++) {
        const Lat& lt = b->ctx[c]->lat;
        const int G = group_threads(lt, shape), T = kBS / G;
        for (int tau0 = 0; tau0 < lt.Nt; tau0 += T) work.push_back({c, tau0, G});
    }
    const size_t per = (work.size() + 7) / 8;
    std::vector<Blk> blk(per * 8, Blk{-1, 0, kBS});
    for (size_t i = 0; i < blk.size(); i++) {
        const size_t w = (i % 8) * per + i / 8;
        if (w < work.size()) blk[i] = work[w];
    }
    return blk;
}

template <typename K>
static qedhmc_status set_lds(K kern, size_t bytes) {
    if (bytes > 65536)
        QH_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return QEDHMC_OK;
}

template <typename R>
static qedhmc_status set_attrs(qedhmc_batch* b, int shape) {
    return with_bshape(shape, [&]<int MC, int NB>() -> qedhmc_status {
        const size_t l = shape_lds(b, shape, sizeof(cplx<R>)), l64 = shape_lds(b, shape, sizeof(cplx<double>));
        QH_TRY(set_lds(k_b_cg_start<R, MC, NB>, l));
        QH_TRY(set_lds(k_b_cg_iter<R, MC, NB>, l));
        QH_TRY(set_lds(k_b_cg_replace<R, MC, NB>, l));
        QH_TRY(set_lds(k_b_ox<R, MC, NB>, l64));
        return QEDHMC_OK;
    });
}

template <typename R>
static constexpr int pidx() {
    return sizeof(R) == 8 ? 1 : 0;
}

template <typename R>
static ChainDev<R>* host_tab(qedhmc_batch* b) {
    return reinterpret_cast<ChainDev<R>*>(b->h_tab[pidx<R>()]);
}

template <typename R>
static const ChainDev<R>* dev_tab(qedhmc_batch* b) {
    return reinterpret_cast<const ChainDev<R>*>(b->d_tab[pidx<R>()]);
}

// static part of a chain's table row; the solve fills rhs, x, maxit, mixed
template <typename R>
static void init_tab(qedhmc_batch* b) {
    ChainDev<R>* tab = host_tab<R>(b);
    for (int c = 0; c < b->n; c++) {
        qedhmc_ctx* h = b->ctx[c];
        ChainDev<R>& d = tab[c];
        d = ChainDev<R>{};
        d.lt = h->lat;
        const size_t N = (size_t)h->lat.Nt * h->lat.Vs;
        cplx<R>* base = reinterpret_cast<cplx<R>*>(h->cg_arena);
        d.B.r[0] = base;
        d.B.r[1] = base + N;
        d.B.s[0] = base + 2 * N;
        d.B.s[1] = base + 3 * N;
        d.B.w[0] = base + 4 * N;
        d.B.w[1] = base + 5 * N;
        d.B.p = base + 6 * N;
        d.B.Ox = reinterpret_cast<const cplx<double>*>(h->ws[3]);
        d.B.part = h->partial;
        qedhmc_ctx* hg = b->shared ? b->ctx[0] : h;
        d.gauge = gauge_for<R>(hg);
        d.gauge64 = hg->gauge64;
        d.scal = b->d_scal + (size_t)c * 2 * S_NSLOT;
        d.co = coef_of<R>(h->p);
        d.co64 = coef_of<double>(h->p);
    }
}

template <typename R>
static qedhmc_status push_tab(qedhmc_batch* b, const std::vector<const double*>& rhs, const std::vector<double*>& x,
                              int maxit, bool mixed) {
    ChainDev<R>* tab = host_tab<R>(b);
    for (int c = 0; c < b->n; c++) {
        tab[c].B.rhs = reinterpret_cast<const cplx<double>*>(rhs[c]);
        tab[c].B.x = reinterpret_cast<cplx<double>*>(x[c]);
        tab[c].maxit = maxit;
        tab[c].mixed = mixed ? 1 : 0;
        tab[c].it0 = 0;
        tab[c].rel0 = 0;
        tab[c].frozen = 0;
    }
    QH_HIP(hipMemcpyAsync(b->d_tab[pidx<R>()], tab, b->n * sizeof(ChainDev<R>), hipMemcpyHostToDevice, b->stream));
    return QEDHMC_OK;
}

template <typename R>
static qedhmc_status launch_start(qedhmc_batch* b, int shape) {
    return with_bshape(shape, [&]<int MC, int NB>() -> qedhmc_status {
        hipLaunchKernelGGL((k_b_cg_start<R, MC, NB>), dim3(b->nblocks[shape]), dim3(kBS),
                           shape_lds(b, shape, sizeof(cplx<R>)), b->stream, dev_tab<R>(b), b->d_blk[shape], b->d_res);
        QH_HIP(hipGetLastError());
        return QEDHMC_OK;
    });
}

template <typename R>
static qedhmc_status launch_iters(qedhmc_batch* b, int shape, int kpar, int count, double tol2) {
    return with_bshape(shape, [&]<int MC, int NB>() -> qedhmc_status {
        const size_t lds = shape_lds(b, shape, sizeof(cplx<R>));
        for (int k = 0; k < count; k++)
            hipLaunchKernelGGL((k_b_cg_iter<R, MC, NB>), dim3(b->nblocks[shape]), dim3(kBS), lds, b->stream,
                               dev_tab<R>(b), b->d_blk[shape], kpar ^ (k & 1), k, tol2);
        QH_HIP(hipGetLastError());
        return QEDHMC_OK;
    });
}

template <typename R>
static qedhmc_status launch_update(qedhmc_batch* b, int shape, int kpar) {
    QH_TRY(with_bshape(shape, [&]<int MC, int NB>() -> qedhmc_status {
        hipLaunchKernelGGL((k_b_ox<R, MC, NB>), dim3(b->nblocks[shape]), dim3(kBS),
                           shape_lds(b, shape, sizeof(cplx<double>)), b->stream, dev_tab<R>(b), b->d_blk[shape], kpar);
        hipLaunchKernelGGL((k_b_cg_replace<R, MC, NB>), dim3(b->nblocks[shape]), dim3(kBS),
                           shape_lds(b, shape, sizeof(cplx<R>)), b->stream, dev_tab<R>(b), b->d_blk[shape], kpar);
        return QEDHMC_OK;
    }));
    hipLaunchKernelGGL(k_b_cg_check<R>, dim3(b->n), dim3(64), 0, b->stream,
                       reinterpret_cast<ChainDev<R>*>(b->d_tab[pidx<R>()]), kpar, b->d_res);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// One replay: kChunk iterations from launch parity kpar0, then the batched
// reliable-update step at parity kpar0 ^ 1.
template <typename R>
static qedhmc_status replay(qedhmc_batch* b, int kpar0, double tol2) {
    hipGraphExec_t& ex = b->graph[pidx<R>()][kpar0];
    if (ex && b->graph_tol2[pidx<R>()][kpar0] != tol2) {
        QH_HIP(hipGraphExecDestroy(ex));
        ex = nullptr;
    }
    if (!ex) {
        hipGraph_t g = nullptr;
        QH_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        qedhmc_status st = launch_iters<R>(b, b->shape[pidx<R>()], kpar0, kChunk, tol2);
        if (st == QEDHMC_OK) st = launch_update<R>(b, b->shape[pidx<R>()], kpar0 ^ (kChunk & 1));
        const hipError_t e = hipStreamEndCapture(b->stream, &g);
        if (st != QEDHMC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        QH_HIP(e);
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        QH_HIP(ei);
        b->graph_tol2[pidx<R>()][kpar0] = tol2;
    }
    QH_HIP(hipGraphLaunch(ex, b->stream));
    return QEDHMC_OK;
}

struct SolveOut {
    std::vector<int> iters, nrel, status;
    std::vector<double> rel;
};

// Solve M^dag M x_c = rhs_c for every chain (gauge caches of the working
// precision and FP64 already built).
template <typename R>
static qedhmc_status batch_cg(qedhmc_batch* b, const std::vector<const double*>& rhs, const std::vector<double*>& x,
                              double tol, int maxit, bool mixed, SolveOut& out) {
    const int n = b->n;
    QH_TRY(push_tab<R>(b, rhs, x, maxit, mixed));
    QH_TRY(launch_start<R>(b, b->shape[pidx<R>()]));
    const double tol2 = tol * tol;
    const long max_replays = 3L * ((long)maxit / kChunk + 2) + 8;
    auto all_final = [&](const double* r) {
        for (int c = 0; c < n; c++)
            if (r[kNRes * c + RS_DONE] != 4.0 && r[kNRes * c + RS_DONE] != 5.0) return false;
        return true;
    };
    auto enqueue = [&](int kpar, int slot) -> qedhmc_status {
        QH_TRY(replay<R>(b, kpar, tol2));
        QH_HIP(hipMemcpyAsync(b->h_res[slot], b->d_res, (size_t)n * kNRes * sizeof(double), hipMemcpyDeviceToHost,
                              b->stream));
        QH_HIP(hipEventRecord(b->ev[slot], b->stream));
        return QEDHMC_OK;
    };
    // two replays in flight: the host looks at replay j while j + 1 runs
    int kpar = 0, cur = 0;
    long replays = 0;
    QH_TRY(enqueue(kpar, cur));
    kpar ^= (kChunk & 1);
    replays++;
    bool done = false;
    while (!done) {
        const bool more = replays < max_replays;
        if (more) {
            QH_TRY(enqueue(kpar, cur ^ 1));
            kpar ^= (kChunk & 1);
            replays++;
        }
        QH_HIP(hipEventSynchronize(b->ev[cur]));
        done = all_final(b->h_res[cur]);
        if (!done && !more) {
            QH_HIP(hipStreamSynchronize(b->stream));
            if (!all_final(b->h_res[cur ^ 1])) {
                set_error("batched CG: chains still running after the replay limit");
                return QEDHMC_ENOCONV;
            }
            cur ^= 1;
            done = true;
        }
        if (!done) cur ^= 1;
    }
    QH_HIP(hipStreamSynchronize(b->stream));
    const double* r = b->h_res[cur];
    out.iters.assign(n, 0);
    out.nrel.assign(n, 0);
    out.status.assign(n, QEDHMC_OK);
    out.rel.assign(n, 0.0);
    for (int c = 0; c < n; c++) {
        const double* rc = r + kNRes * c;
        out.iters[c] = (int)rc[RS_ITERS];
        out.nrel[c] = (int)rc[RS_NREL];
        out.rel[c] = rc[RS_B2] > 0.0 ? std::sqrt(rc[RS_TRUE] / rc[RS_B2]) : 0.0;
        out.status[c] = rc[RS_DONE] == 5.0 ? QEDHMC_OK : QEDHMC_ENOCONV;
    }
    return QEDHMC_OK;
}

template <typename R>
static qedhmc_status launch_gauge(qedhmc_batch* b, const double* theta_all) {
    int64_t most = 0;
    for (int c = 0; c < b->n; c++) most = std::max(most, b->toff[c + 1] - b->toff[c]);
    const int gx = (int)std::min<int64_t>((most + 255) / 256, 64);
    hipLaunchKernelGGL(k_b_gauge<R>, dim3(gx, b->n), dim3(256), 0, b->stream, dev_tab<R>(b), theta_all, b->d_toff);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// Time every tile shape on the batch's own lattices: angles and right-hand
// sides from the heat bath (Gaussian angles: a disordered but well-posed
// system), 4 warm-up and 24 timed iterations of the recursion in the working
// precision R, best of two.  The fastest shape is kept for R.
template <typename R>
static qedhmc_status autotune(qedhmc_batch* b, const std::vector<const double*>& rhs, const std::vector<double*>& x) {
    hipEvent_t e0, e1;
    QH_HIP(hipEventCreate(&e0));
    QH_HIP(hipEventCreate(&e1));
    float best = 0.0f;
    int best_shape = -1;
    qedhmc_status st = QEDHMC_OK;
    float* us_out = b->tune_us[pidx<R>()];
    for (int s = 0; s < 4 && st == QEDHMC_OK; s++) {
        us_out[s] = 0.0f;
        if (!shape_ok(b, s)) continue;
        float t_best = 0.0f;
        for (int rep = 0; rep < 2 && st == QEDHMC_OK; rep++) {
            st = push_tab<R>(b, rhs, x, 1 << 30, false);
            if (st == QEDHMC_OK) st = launch_start<R>(b, s);
            if (st == QEDHMC_OK) st = launch_iters<R>(b, s, 0, 4, 0.0);
            if (st != QEDHMC_OK) break;
            if (hipEventRecord(e0, b->stream) != hipSuccess) st = hip_fail(hipGetLastError(), "event");
            if (st == QEDHMC_OK) st = launch_iters<R>(b, s, 0, 24, 0.0);
            if (st == QEDHMC_OK && hipEventRecord(e1, b->stream) != hipSuccess) st = hip_fail(hipGetLastError(), "event");
            float ms = 0.0f;
            if (st == QEDHMC_OK && hipEventSynchronize(e1) != hipSuccess) st = hip_fail(hipGetLastError(), "sync");
            if (st == QEDHMC_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                st = hip_fail(hipGetLastError(), "time");
            const float us = 1000.0f * ms / 24.0f;
            if (st == QEDHMC_OK && (rep == 0 || us < t_best)) t_best = us;
        }
        if (st != QEDHMC_OK) break;
        us_out[s] = t_best;
        if (best_shape < 0 || t_best < best) {
            best = t_best;
            best_shape = s;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != QEDHMC_OK) return st;
    if (best_shape < 0) {
        set_error("batch: no tile shape fits these lattices (L up to 44 with two cells per thread)");
        return QEDHMC_EUNSUPPORTED;
    }
    b->shape[pidx<R>()] = best_shape;
    return QEDHMC_OK;
}

static qedhmc_status autotune_all(qedhmc_batch* b) {
    const int n = b->n;
    std::vector<const double*> rhs(n);
    std::vector<double*> x(n);
    for (int c = 0; c < n; c++) {
        qedhmc_ctx* h = b->ctx[c];
        QH_TRY(launch_heatbath(h, ~0ull, b->theta0 + b->toff[c], (double*)h->ws[5]));
        rhs[c] = (const double*)h->ws[5];
        x[c] = (double*)h->ws[6];
    }
    QH_TRY(launch_gauge<float>(b, b->theta0));
    QH_TRY(launch_gauge<double>(b, b->theta0));
    QH_TRY(autotune<float>(b, rhs, x));
    return autotune<double>(b, rhs, x);
}

}  // namespace qh

using namespace qh;

namespace {

// order the batch's own stream after everything the caller has enqueued
qedhmc_status enter(qedhmc_batch* b) {
    QH_HIP(hipEventRecord(b->ev_in, b->user));
    QH_HIP(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    return QEDHMC_OK;
}

qedhmc_status batch_fail(qedhmc_batch* b, qedhmc_status st) {
    qedhmc_batch_destroy(b);
    return st;
}

}  // namespace

extern "C" {

qedhmc_status qedhmc_batch_create(const qedhmc_params* params, int32_t n_chains, void* stream, qedhmc_batch_t* out) {
    if (!params || !out || n_chains < 1) {
        set_error("batch: null argument or no chains");
        return QEDHMC_EINVAL;
    }
    *out = nullptr;
    qedhmc_batch* b = new (std::nothrow) qedhmc_batch{};
    if (!b) {
        set_error("batch: out of host memory");
        return QEDHMC_ENOMEM;
    }
    b->n = n_chains;
    b->user = (hipStream_t)stream;
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        set_error("batch: stream or event creation failed");
        return batch_fail(b, QEDHMC_EHIP);
    }
    if (enter(b) != QEDHMC_OK) return batch_fail(b, QEDHMC_EHIP);
    b->params.assign(params, params + n_chains);
    b->toff.assign(n_chains + 1, 0);
    b->voff.assign(n_chains + 1, 0);
    for (int c = 0; c < n_chains; c++) {
        qedhmc_ctx* h = nullptr;
        const qedhmc_status st = qedhmc_init_lattice(&params[c], b->stream, &h);
        if (st != QEDHMC_OK) return batch_fail(b, st);
        b->ctx.push_back(h);
        const int64_t N = (int64_t)h->lat.Nt * h->lat.Vs;
        b->toff[c + 1] = b->toff[c] + 2 * N;
        b->voff[c + 1] = b->voff[c] + N;
        b->maxL = std::max(b->maxL, h->lat.L);
        b->maxVs = std::max(b->maxVs, h->lat.Vs);
        b->maxcell = std::max(b->maxcell, h->lat.ncell);
        b->max_lds = h->max_lds;
    }
    const size_t tot = (size_t)b->toff[n_chains];
    bool ok = true;
    std::vector<Blk> blk[4];
    for (int s = 0; s < 4 && ok; s++) {
        if (!shape_ok(b, s)) continue;
        blk[s] = work_list(b, s);
        b->nblocks[s] = (int)blk[s].size();
        ok = hipMalloc(&b->d_blk[s], blk[s].size() * sizeof(Blk)) == hipSuccess;
    }
    ok = ok && hipMalloc(&b->d_toff, (n_chains + 1) * sizeof(int64_t)) == hipSuccess;
    ok = ok && hipMalloc(&b->d_scal, (size_t)n_chains * 2 * S_NSLOT * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&b->d_res, (size_t)n_chains * kNRes * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&b->d_tab[0], n_chains * sizeof(ChainDev<float>)) == hipSuccess;
    ok = ok && hipMalloc(&b->d_tab[1], n_chains * sizeof(ChainDev<double>)) == hipSuccess;
    ok = ok && hipMalloc(&b->mom, tot * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&b->force, tot * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&b->force_b, tot * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&b->theta0, tot * sizeof(double)) == hipSuccess;
    for (int k = 0; k < 2 && ok; k++) {
        ok = hipHostMalloc(&b->h_tab[k], n_chains * sizeof(ChainDev<double>), hipHostMallocDefault) == hipSuccess;
        ok = ok && hipHostMalloc((void**)&b->h_res[k], (size_t)n_chains * kNRes * sizeof(double),
                                 hipHostMallocDefault) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&b->ev[k], hipEventDisableTiming) == hipSuccess;
    }
    for (int s = 0; s < 4 && ok; s++)
        if (b->d_blk[s])
            ok = hipMemcpyAsync(b->d_blk[s], blk[s].data(), blk[s].size() * sizeof(Blk), hipMemcpyHostToDevice,
                                b->stream) == hipSuccess;
    if (ok)
        ok = hipMemcpyAsync(b->d_toff, b->toff.data(), (n_chains + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                            b->stream) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        set_error("batch: device or pinned allocation failed");
        return batch_fail(b, QEDHMC_ENOMEM);
    }
    // the device tables must hold the static rows (gauge caches, workspace)
    // before any kernel reads them: the gauge kernels run before the first
    // solve pushes its per-solve fields
    init_tab<float>(b);
    init_tab<double>(b);
    {
        const std::vector<const double*> no_rhs(n_chains, nullptr);
        const std::vector<double*> no_x(n_chains, nullptr);
        qedhmc_status st = push_tab<float>(b, no_rhs, no_x, 0, false);
        if (st == QEDHMC_OK) st = push_tab<double>(b, no_rhs, no_x, 0, false);
        // the host rows are rewritten by the next push: let these copies land first
        if (st == QEDHMC_OK && hipStreamSynchronize(b->stream) != hipSuccess)
            st = hip_fail(hipGetLastError(), "batch create");
        if (st != QEDHMC_OK) return batch_fail(b, st);
    }
    for (int s = 0; s < 4; s++) {
        if (!shape_ok(b, s)) continue;
        qedhmc_status st = set_attrs<float>(b, s);
        if (st == QEDHMC_OK) st = set_attrs<double>(b, s);
        if (st != QEDHMC_OK) return batch_fail(b, st);
    }
    qedhmc_status st = autotune_all(b);
    if (st == QEDHMC_OK && hipStreamSynchronize(b->stream) != hipSuccess) st = hip_fail(hipGetLastError(), "batch create");
    if (st != QEDHMC_OK) return batch_fail(b, st);
    *out = b;
    return QEDHMC_OK;
}

qedhmc_status qedhmc_batch_destroy(qedhmc_batch_t b) {
    if (!b) return QEDHMC_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (auto* h : b->ctx) qedhmc_destroy(h);
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++)
            if (b->graph[i][j]) (void)hipGraphExecDestroy(b->graph[i][j]);
    for (int s = 0; s < 4; s++) (void)hipFree(b->d_blk[s]);
    (void)hipFree(b->d_toff);
    (void)hipFree(b->d_scal);
    (void)hipFree(b->d_res);
    (void)hipFree(b->mom);
    (void)hipFree(b->force);
    (void)hipFree(b->force_b);
    (void)hipFree(b->theta0);
    for (int k = 0; k < 2; k++) {
        (void)hipFree(b->d_tab[k]);
        if (b->h_tab[k]) (void)hipHostFree(b->h_tab[k]);
        if (b->h_res[k]) (void)hipHostFree(b->h_res[k]);
        if (b->ev[k]) (void)hipEventDestroy(b->ev[k]);
    }
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return QEDHMC_OK;
}

qedhmc_status qedhmc_batch_layout(qedhmc_batch_t b, int64_t* theta_off, int64_t* vec_off) {
    if (!b || !theta_off || !vec_off) {
        set_error("batch: null argument");
        return QEDHMC_EINVAL;
    }
    for (int c = 0; c <= b->n; c++) {
        theta_off[c] = b->toff[c];
        vec_off[c] = b->voff[c];
    }
    return QEDHMC_OK;
}

qedhmc_status qedhmc_batch_tile(qedhmc_batch_t b, qedhmc_precision prec, int32_t* cells_per_thread,
                                int32_t* threads, int32_t* exchange_buffers, float* us_per_iter) {
    if (!b || !cells_per_thread || !threads || !exchange_buffers || !us_per_iter ||
        (prec != QEDHMC_FP64 && prec != QEDHMC_FP32)) {
        set_error("batch: null argument or bad precision");
        return QEDHMC_EINVAL;
    }
    const int pi = prec == QEDHMC_FP64 ? 1 : 0;
    const int s = b->shape[pi];
    *cells_per_thread = kShapeMC[s];
    *threads = kBS;
    *exchange_buffers = kShapeNB[s];
    for (int k = 0; k < 4; k++) us_per_iter[k] = b->tune_us[pi][k];
    return QEDHMC_OK;
}

static qedhmc_status batch_args(qedhmc_batch* b, const void* a, const void* c, double tol, int maxit,
                                qedhmc_precision prec) {
    if (!b || !a || !c) {
        set_error("batch: null argument");
        return QEDHMC_EINVAL;
    }
    if (!(tol > 0.0) || maxit < 1 || (prec != QEDHMC_FP64 && prec != QEDHMC_FP32)) {
        set_error("batch: bad solver arguments");
        return QEDHMC_EINVAL;
    }
    return QEDHMC_OK;
}

static qedhmc_status batch_solve(qedhmc_batch* b, const double* theta_all, const std::vector<const double*>& rhs,
                                 const std::vector<double*>& x, double tol, int maxit, qedhmc_precision prec,
                                 SolveOut& so) {
    QH_TRY(launch_gauge<double>(b, theta_all));
    if (prec == QEDHMC_FP64) return batch_cg<double>(b, rhs, x, tol, maxit, false, so);
    QH_TRY(launch_gauge<float>(b, theta_all));
    return batch_cg<float>(b, rhs, x, tol, maxit, true, so);
}

qedhmc_status qedhmc_batch_cg_solve(qedhmc_batch_t b, const double* theta_all, const double* rhs_all, double* x_all,
                                    double tol, int32_t maxit, qedhmc_precision prec, int32_t* iters,
                                    double* true_rel) {
    QH_TRY(batch_args(b, theta_all, rhs_all, tol, maxit, prec));
    if (!x_all || !iters || !true_rel) {
        set_error("batch: null argument");
        return QEDHMC_EINVAL;
    }
    QH_TRY(enter(b));
    std::vector<const double*> rhs(b->n);
    std::vector<double*> x(b->n);
    for (int c = 0; c < b->n; c++) {
        rhs[c] = rhs_all + 2 * b->voff[c];
        x[c] = x_all + 2 * b->voff[c];
    }
    SolveOut so;
    QH_TRY(batch_solve(b, theta_all, rhs, x, tol, maxit, prec, so));
    qedhmc_status st = QEDHMC_OK;
    for (int c = 0; c < b->n; c++) {
        iters[c] = so.iters[c];
        true_rel[c] = so.rel[c];
        if (so.status[c] != QEDHMC_OK) st = QEDHMC_ENOCONV;
    }
    if (st != QEDHMC_OK) set_error("batched CG: at least one chain did not converge");
    return st;
}

}  // extern "C"

namespace qh {

qedhmc_status batch_create_shared(const qedhmc_params& params, int n, void* stream, qedhmc_batch** out) {
    *out = nullptr;
    const std::vector<qedhmc_params> ps(n, params);
    qedhmc_batch* b = nullptr;
    QH_TRY(qedhmc_batch_create(ps.data(), n, stream, &b));
    b->shared = true;
    init_tab<float>(b);
    init_tab<double>(b);
    const std::vector<const double*> no_rhs(n, nullptr);
    const std::vector<double*> no_x(n, nullptr);
    qedhmc_status st = push_tab<float>(b, no_rhs, no_x, 0, false);
    if (st == QEDHMC_OK) st = push_tab<double>(b, no_rhs, no_x, 0, false);
    if (st == QEDHMC_OK && hipStreamSynchronize(b->stream) != hipSuccess)
        st = hip_fail(hipGetLastError(), "shared batch create");
    if (st != QEDHMC_OK) return batch_fail(b, st);
    *out = b;
    return QEDHMC_OK;
}

qedhmc_ctx* batch_ctx0(qedhmc_batch* b) { return b->ctx[0]; }

qedhmc_status batch_enter(qedhmc_batch* b) { return enter(b); }

qedhmc_status batch_solve_shared(qedhmc_batch* b, const double* theta, const double* rhs_all, double* x_all,
                                 double tol, int maxit, qedhmc_precision prec, int32_t* iters, double* true_rel) {
    if (!b->shared) {
        set_error("batch_solve_shared needs a batch made by batch_create_shared");
        return QEDHMC_EINVAL;
    }
    QH_TRY(batch_args(b, theta, rhs_all, tol, maxit, prec));
    QH_TRY(enter(b));
    qedhmc_ctx* h0 = b->ctx[0];
    QH_TRY(ensure_gauge(h0, theta, QEDHMC_FP64));
    if (prec != QEDHMC_FP64) QH_TRY(ensure_gauge(h0, theta, QEDHMC_FP32));
    const int64_t N = b->voff[1];
    std::vector<const double*> rhs(b->n);
    std::vector<double*> x(b->n);
    for (int c = 0; c < b->n; c++) {
        rhs[c] = rhs_all + 2 * N * c;
        x[c] = x_all + 2 * N * c;
    }
    SolveOut so;
    if (prec == QEDHMC_FP64)
        QH_TRY(batch_cg<double>(b, rhs, x, tol, maxit, false, so));
    else
        QH_TRY(batch_cg<float>(b, rhs, x, tol, maxit, true, so));
    qedhmc_status st = QEDHMC_OK;
    for (int c = 0; c < b->n; c++) {
        iters[c] = so.iters[c];
        true_rel[c] = so.rel[c];
        if (so.status[c] != QEDHMC_OK) st = QEDHMC_ENOCONV;
    }
    if (st != QEDHMC_OK) set_error("multi-RHS CG: at least one right-hand side did not converge");
    return st;
}

}  // namespace qh

extern "C" {

qedhmc_status qedhmc_batch_trajectory(qedhmc_batch_t b, double* theta_all, uint64_t traj, int32_t n_steps,
                                      double traj_len, double tol, int32_t maxit, qedhmc_precision prec,
                                      qedhmc_traj_result* out) {
    QH_TRY(batch_args(b, theta_all, out, tol, maxit, prec));
    if (n_steps < 1 || !(traj_len > 0.0)) {
        set_error("batch: bad trajectory arguments");
        return QEDHMC_EINVAL;
    }
    QH_TRY(enter(b));
    const int n = b->n;
    const double dt = traj_len / n_steps;
    const size_t tot = (size_t)b->toff[n];
    qedhmc_ctx* h0 = b->ctx[0];
    std::vector<const double*> eta(n);
    std::vector<double*> X(n);
    for (int c = 0; c < n; c++) {
        std::memset(&out[c], 0, sizeof(out[c]));
        eta[c] = (const double*)b->ctx[c]->ws[5];
        X[c] = (double*)b->ctx[c]->ws[6];
    }
    auto th = [&](int c) { return theta_all + b->toff[c]; };
    auto sl = [&](double* base, int c) { return base + b->toff[c]; };
    SolveOut so;
    auto solve_all = [&]() -> qedhmc_status {
        QH_TRY(batch_solve(b, theta_all, eta, X, tol, maxit, prec, so));
        for (int c = 0; c < n; c++) {
            out[c].n_solves++;
            out[c].cg_iters_total += so.iters[c];
            out[c].cg_iters_max = std::max(out[c].cg_iters_max, so.iters[c]);
            out[c].max_true_resid = std::max(out[c].max_true_resid, so.rel[c]);
            out[c].reliable_updates += so.nrel[c];
            if (so.status[c] != QEDHMC_OK) out[c].status = 2;
        }
        return QEDHMC_OK;
    };
    auto forces = [&](int slot) -> qedhmc_status {
        for (int c = 0; c < n; c++) {
            qedhmc_ctx* h = b->ctx[c];
            QH_TRY(launch_force(h, prec, X[c], sl(b->force, c)));
            QH_TRY(launch_bosonic(h, th(c), sl(b->force_b, c), h->scal + 64 + slot));
        }
        return QEDHMC_OK;
    };
    // (i) heat bath, eta = M^dag R
    QH_HIP(hipMemcpyAsync(b->theta0, theta_all, tot * sizeof(double), hipMemcpyDeviceToDevice, b->stream));
    QH_TRY(launch_gauge<double>(b, theta_all));
    for (int c = 0; c < n; c++) {
        qedhmc_ctx* h = b->ctx[c];
        QH_TRY(launch_heatbath(h, traj, sl(b->mom, c), (double*)h->ws[4]));
        QH_TRY(launch_apply_M(h, QEDHMC_FP64, h->ws[4], h->ws[5], 1));
    }
    // H at the start
    QH_TRY(solve_all());
    for (int c = 0; c < n; c++) {
        qedhmc_ctx* h = b->ctx[c];
        const size_t N = (size_t)h->lat.Nt * h->lat.Vs;
        QH_TRY(launch_dot_re(h, eta[c], X[c], 2 * N, h->scal + 64 + 2));
        QH_TRY(launch_sumsq(h, sl(b->mom, c), 2 * N, h->scal + 64 + 1));
    }
    QH_TRY(forces(0));
    // (ii) leapfrog, all chains in step
    for (int step = 0; step < n_steps; step++) {
        QH_TRY(launch_kick(h0, b->mom, b->force, b->force_b, 0.5 * dt, tot));
        QH_TRY(launch_drift(h0, theta_all, b->mom, 2.0 * dt, tot));
        QH_TRY(solve_all());
        QH_TRY(forces(3));
        QH_TRY(launch_kick(h0, b->mom, b->force, b->force_b, 0.5 * dt, tot));
    }
    // H at the end, (iii) Metropolis per chain, restore on rejection
    for (int c = 0; c < n; c++) {
        qedhmc_ctx* h = b->ctx[c];
        const size_t N = (size_t)h->lat.Nt * h->lat.Vs;
        double* sc = h->scal + 64;
        QH_TRY(launch_dot_re(h, eta[c], X[c], 2 * N, sc + 5));
        QH_TRY(launch_sumsq(h, sl(b->mom, c), 2 * N, sc + 4));
        // a chain with an unconverged solve rejects its proposal
        QH_TRY(launch_metropolis(h, traj, out[c].status != 0, sc));
        QH_TRY(launch_restore(h, theta_all + b->toff[c], b->theta0 + b->toff[c], sc, 2 * N));
        QH_HIP(hipMemcpyAsync(h->h_pinned, sc, 9 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    }
    QH_HIP(hipStreamSynchronize(b->stream));
    for (int c = 0; c < n; c++) {
        const double* v = b->ctx[c]->h_pinned;
        out[c].SB0 = v[0];
        out[c].K0 = v[1];
        out[c].SF0 = v[2];
        out[c].SB1 = v[3];
        out[c].K1 = v[4];
        out[c].SF1 = v[5];
        out[c].H0 = v[0] + v[1] + v[2];
        out[c].H1 = v[3] + v[4] + v[5];
        out[c].dH = v[6];
        out[c].u = v[7];
        out[c].accepted = v[8] != 0.0 ? 1 : 0;
    }
    for (int c = 0; c < n; c++)
        if (out[c].status != 0) {
            set_error("batch: a solve of chain " + std::to_string(c) +
                      " did not converge; its proposal was rejected");
            return QEDHMC_ENOCONV;
        }
    return QEDHMC_OK;
}

}  // extern "C"
