// Conjugate gradient on O = M^dag M without preconditioner: the kernels
// (thin wrappers over the device bodies of cg_body.h, one workgroup per
// time slice) and the host driver that launches them in chunks, reads the
// stop flag once per chunk and runs the FP64 reliable updates.
#include <cstdlib>

#include "cg_body.h"

namespace qh {

template <typename R, int MC, int NB, int BS>
__global__ __launch_bounds__(BS) void k_cg_start(Lat lt, CgBufs<R> B, const cplx<R>* __restrict__ gauge, Coef<R> co,
                                                 double* __restrict__ scal) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tau = slice_of_block(blockIdx.x, lt.Nt);
    if (tau < 0) return;
    const Tile tl = whole_block_tile(smem, reinterpret_cast<double*>(smem + (size_t)NB * 2 * lt.Vs * sizeof(cplx<R>)));
    cg_start_body<R, MC, NB>(lt, B, gauge, co, scal, tau, tau == 0, tl);
}

template <typename R, int MC, int NB, int BS>
__global__ __launch_bounds__(BS) void k_cg_iter(Lat lt, CgBufs<R> B, const cplx<R>* __restrict__ gauge, Coef<R> co,
                                                double* __restrict__ scal, int kpar, int ipar, double tol2,
                                                int mixed) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tau = slice_of_block(blockIdx.x, lt.Nt);
    if (tau < 0) return;
    const Tile tl = whole_block_tile(smem, reinterpret_cast<double*>(smem + (size_t)NB * 2 * lt.Vs * sizeof(cplx<R>)));
    cg_iter_body<R, MC, NB>(lt, B, gauge, co, scal, kpar, ipar, tol2, mixed, tau, tau == 0, tl);
}

template <typename R, int MC, int NB, int BS>
__global__ __launch_bounds__(BS) void k_cg_replace(Lat lt, CgBufs<R> B, const cplx<R>* __restrict__ gauge,
                                                   Coef<R> co, const double* __restrict__ scal, int kpar) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tau = slice_of_block(blockIdx.x, lt.Nt);
    if (tau < 0) return;
    const Tile tl = whole_block_tile(smem, reinterpret_cast<double*>(smem + (size_t)NB * 2 * lt.Vs * sizeof(cplx<R>)));
    cg_replace_body<R, MC, NB>(lt, B, gauge, co, scal, kpar, tau, tl);
}

__global__ void k_cg_check(double* __restrict__ scal, int kpar, const double* __restrict__ part, int Nt,
                           int restart) {
    __shared__ double red[kNP * 16 + 16];
    cg_check_body(scal, kpar, part, Nt, restart, red);
}


// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
template <typename R>
static CgBufs<R> bufs_of(qedhmc_ctx* h, const double* rhs, double* x) {
    CgBufs<R> B;
    const size_t N = (size_t)h->lat.Nt * h->lat.Vs;
    cplx<R>* base = reinterpret_cast<cplx<R>*>(h->cg_arena);
    B.r[0] = base;
    B.r[1] = base + N;
    B.s[0] = base + 2 * N;
    B.s[1] = base + 3 * N;
    B.w[0] = base + 4 * N;
    B.w[1] = base + 5 * N;
    B.p = base + 6 * N;
    B.x = reinterpret_cast<cplx<double>*>(x);
    B.rhs = reinterpret_cast<const cplx<double>*>(rhs);
    B.Ox = reinterpret_cast<const cplx<double>*>(h->ws[3]);
    B.part = h->partial;
    return B;
}

template <typename R>
static qedhmc_status launch_start(qedhmc_ctx* h, const CgBufs<R>& B) {
    return with_shape<R>(h, [&]<int MC, int NB, int BS>(int nt, size_t lds) -> qedhmc_status {
        QH_TRY(lds_attr(h, k_cg_start<R, MC, NB, BS>, lds));
        hipLaunchKernelGGL((k_cg_start<R, MC, NB, BS>), dim3(slice_grid(h->lat.Nt)), dim3(nt), lds, h->stream, h->lat, B,
                           gauge_for<R>(h), coef_of<R>(h->p), h->scal);
        QH_HIP(hipGetLastError());
        return QEDHMC_OK;
    });
}

template <typename R>
static qedhmc_status launch_iters(qedhmc_ctx* h, const CgBufs<R>& B, int& kpar, int it0, int count, double tol2,
                                  int mixed) {
    return with_shape<R>(h, [&]<int MC, int NB, int BS>(int nt, size_t lds) -> qedhmc_status {
        QH_TRY(lds_attr(h, k_cg_iter<R, MC, NB, BS>, lds));
        const Coef<R> co = coef_of<R>(h->p);
        const cplx<R>* g = gauge_for<R>(h);
        const int cls = sizeof(R) == 4 ? QEDHMC_K_CG_FP32 : QEDHMC_K_CG_FP64;
        for (int k = 0; k < count; k++) {
            hipEvent_t e0, e1;
            const int ipar = (it0 + k) & 1;
            if (prof_sample(h, cls, e0, e1))
                hipExtLaunchKernelGGL((k_cg_iter<R, MC, NB, BS>), dim3(slice_grid(h->lat.Nt)), dim3(nt), lds, h->stream, e0, e1,
                                      0, h->lat, B, g, co, h->scal, kpar, ipar, tol2, mixed);
            else
                hipLaunchKernelGGL((k_cg_iter<R, MC, NB, BS>), dim3(slice_grid(h->lat.Nt)), dim3(nt), lds, h->stream, h->lat, B,
                                   g, co, h->scal, kpar, ipar, tol2, mixed);
            kpar ^= 1;
        }
        QH_HIP(hipGetLastError());
        return QEDHMC_OK;
    });
}

// One chunk of `count` iteration launches from launch parity kpar and buffer
// parity ipar0, replayed from a graph captured the first time this
// (buffers, tolerance, precision, chunk) combination is seen.
template <typename R>
static qedhmc_status launch_iters_graph(qedhmc_ctx* h, const CgBufs<R>& B, int kpar, int ipar0, int count,
                                        double tol2, int mixed) {
    qedhmc_ctx::CgGraph& gr = h->cg_graph[sizeof(R) == 8 ? 1 : 0][kpar][ipar0];
    if (gr.exec && (gr.x != B.x || gr.rhs != B.rhs || gr.tol2 != tol2 || gr.mixed != mixed || gr.count != count)) {
        QH_HIP(hipGraphExecDestroy(gr.exec));
        gr.exec = nullptr;
    }
    if (!gr.exec) {
        if (!h->cap_stream) QH_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        // kernel attributes before the capture
        QH_TRY(with_shape<R>(h, [&]<int MC, int NB, int BS>(int nt, size_t lds) -> qedhmc_status {
            return lds_attr(h, k_cg_iter<R, MC, NB, BS>, lds);
        }));
        hipStream_t user = h->stream;
        const int prof = h->prof_every;
        h->stream = h->cap_stream;
        h->prof_every = 0;  // no event launches inside a graph
        hipGraph_t g = nullptr;
        qedhmc_status st = QEDHMC_OK;
        hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            int kp = kpar;
            st = launch_iters<R>(h, B, kp, ipar0, count, tol2, mixed);
            e = hipStreamEndCapture(h->cap_stream, &g);
        }
        h->stream = user;
        h->prof_every = prof;
        if (st != QEDHMC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        QH_HIP(e);
        e = hipGraphInstantiate(&gr.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        QH_HIP(e);
        gr.x = B.x;
        gr.rhs = B.rhs;
        gr.tol2 = tol2;
        gr.mixed = mixed;
        gr.count = count;
    }
    // kernel timing: an event pair around the whole replay (the replay is
    // nothing but `count` back-to-back launches of the iteration kernel)
    hipEvent_t e0, e1;
    const bool timed = prof_sample_n(h, sizeof(R) == 4 ? QEDHMC_K_CG_FP32 : QEDHMC_K_CG_FP64, count, e0, e1);
    if (timed) QH_HIP(hipEventRecord(e0, h->stream));
    QH_HIP(hipGraphLaunch(gr.exec, h->stream));
    if (timed) QH_HIP(hipEventRecord(e1, h->stream));
    return QEDHMC_OK;
}

template <typename R>
static qedhmc_status launch_true(qedhmc_ctx* h, const CgBufs<R>& B, const double* x, int kpar, int restart) {
    QH_TRY(launch_mdagm(h, QEDHMC_FP64, x, h->ws[3], nullptr));
    QH_TRY(with_shape<R>(h, [&]<int MC, int NB, int BS>(int nt, size_t lds) -> qedhmc_status {
        QH_TRY(lds_attr(h, k_cg_replace<R, MC, NB, BS>, lds));
        hipLaunchKernelGGL((k_cg_replace<R, MC, NB, BS>), dim3(slice_grid(h->lat.Nt)), dim3(nt), lds, h->stream, h->lat, B,
                           gauge_for<R>(h), coef_of<R>(h->p), (const double*)h->scal, kpar);
        QH_HIP(hipGetLastError());
        return QEDHMC_OK;
    }));
    hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(256), 0, h->stream, h->scal, kpar, (const double*)h->partial,
                       h->lat.Nt, restart);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

template <typename R>
static qedhmc_status cg_t(qedhmc_ctx* h, const double* rhs, double* x, double tol, int maxit, qedhmc_precision prec,
                          int* iters, double* true_rel, int* n_reliable) {
    const bool mixed = prec != QEDHMC_FP64;
    const CgBufs<R> B = bufs_of<R>(h, rhs, x);
    // chunk of launches between host checks; the mixed path pauses itself at
    // most every kCap + 1 launches
    const int chunk = mixed ? kCap + 1 : 64;
    int kpar = 0, nrel = 0, it = 0, stalled = 0, last_it = -1;
    double rel = 1.0;
    bool converged = false, broken = false;
    static const bool trace = std::getenv("QEDHMC_CG_TRACE") != nullptr;
    // QEDHMC_NO_GRAPH (read per solve) launches every chunk directly
    const bool no_graph = std::getenv("QEDHMC_NO_GRAPH") != nullptr;
    QH_TRY(launch_start<R>(h, B));
    while (true) {
        const int left = maxit - it;
        // full chunks replay a captured graph
        if (left >= chunk && !no_graph) {
            QH_TRY(launch_iters_graph<R>(h, B, kpar, it & 1, chunk, tol * tol, mixed ? 1 : 0));
            if (chunk & 1) kpar ^= 1;
        } else if (left > 0) {
            QH_TRY(launch_iters<R>(h, B, kpar, it, left < chunk ? left : chunk, tol * tol, mixed ? 1 : 0));
        }
        QH_TRY(read_slot(h, kpar));
        it = (int)h->h_pinned[S_ITERS];
        const double flag = h->h_pinned[S_DONE];
        if (flag == 0.0 && it < maxit) continue;
        if (flag == 4.0) {
            broken = true;
            set_error("CG breakdown: non-finite inner products after " + std::to_string(it) + " iterations");
            break;
        }
        // every stop / pause must be followed by progress, else give up
        stalled = (it == last_it) ? stalled + 1 : 0;
        last_it = it;
        if (stalled >= 3) {
            set_error("CG made no progress across reliable updates at iteration " + std::to_string(it));
            break;
        }
        // stop, pause or maxit: FP64 true residual decides
        QH_TRY(launch_true<R>(h, B, x, kpar, (!mixed || flag == 3.0) ? 1 : 0));
        nrel++;
        QH_TRY(read_slot(h, kpar));
        const double b2 = h->h_pinned[S_B2];
        rel = b2 > 0.0 ? std::sqrt(h->h_pinned[S_TRUE] / b2) : 0.0;
        if (trace)
            std::fprintf(stderr, "cg it=%d flag=%g true_rel=%.3e gamma=%.3e\n", it, flag, rel, h->h_pinned[S_GCUR]);
        if (!std::isfinite(rel)) {
            broken = true;
            set_error("CG breakdown: non-finite true residual after " + std::to_string(it) + " iterations");
            break;
        }
        if (h->h_pinned[S_DONE] == 1.0) {
            converged = true;
            break;
        }
        if (it >= maxit) break;
    }
    if (iters) *iters = it;
    if (true_rel) *true_rel = rel;
    if (n_reliable) *n_reliable = nrel;
    if (broken) return QEDHMC_ENOCONV;
    return converged ? QEDHMC_OK : QEDHMC_ENOCONV;
}

qedhmc_status cg_solve_impl(qedhmc_ctx* h, const double* rhs, double* x, double tol, int maxit,
                            qedhmc_precision prec, int* iters, double* true_rel, int* n_reliable) {
    if (h->lat.ncell > 1024) return cg2_solve_impl(h, rhs, x, tol, maxit, prec, iters, true_rel, n_reliable);
    if (prec == QEDHMC_FP64) return cg_t<double>(h, rhs, x, tol, maxit, prec, iters, true_rel, n_reliable);
    return cg_t<float>(h, rhs, x, tol, maxit, prec, iters, true_rel, n_reliable);
}

}  // namespace qh
