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
                                                int mixed, int maxit) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tau = slice_of_block(blockIdx.x, lt.Nt);
    if (tau < 0) return;
    const Tile tl = whole_block_tile(smem, reinterpret_cast<double*>(smem + (size_t)NB * 2 * lt.Vs * sizeof(cplx<R>)));
    cg_iter_body<R, MC, NB>(lt, B, gauge, co, scal, kpar, ipar, tol2, mixed, maxit, tau, tau == 0, tl);
}

template <typename R, int MC, int NB, int BS>
__global__ __launch_bounds__(BS) void k_cg_replace(Lat lt, CgBufs<R> B, const cplx<R>* __restrict__ gauge,
                                                   Coef<R> co, const double* __restrict__ scal, int kpar,
                                                   int gated) {
    if (gated && !gate_open(scal[S_NSLOT * kpar + S_DONE])) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tau = slice_of_block(blockIdx.x, lt.Nt);
    if (tau < 0) return;
    const Tile tl = whole_block_tile(smem, reinterpret_cast<double*>(smem + (size_t)NB * 2 * lt.Vs * sizeof(cplx<R>)));
    cg_replace_body<R, MC, NB>(lt, B, gauge, co, scal, kpar, tau, tl);
}

// The reliable-update decision on the device, after the gated FP64 O x and
// replacement: converged (5) when the FP64 true residual meets the target;
// failed (4) on a non-finite residual, the iteration budget used or no
// progress across three updates, or a breakdown flagged by the recursion;
// otherwise resume (0; restart with beta = 0 after a non-positive
// denominator, and after every update with restart_all: the FP64 path's
// p = r).  A solve already final is left as it is.  The record (kept in
// device memory across rounds) is also stored to out, a slot of pinned host
// memory, so the host needs no copy.
__global__ void k_cg_check_dev(double* __restrict__ scal, int kpar, const double* __restrict__ part, int Nt,
                               int maxit, int restart_all, double* __restrict__ rec, double* __restrict__ out) {
    __shared__ double red[kNP * 16 + 16];
    double* sl = scal + S_NSLOT * kpar;
    const double done = sl[S_DONE];
    const int it = (int)sl[S_ITERS];
    int nd = -1, why = 0;
    double est = sl[S_GCUR];
    if (done == 4.0 && rec[CR_DONE] != 4.0) {
        nd = 4;
        why = WHY_BREAKDOWN;
    }
    if (gate_open(done)) {
        double pr[kNP];
        reduce_partials(part, Nt, whole_block_tile(nullptr, red), pr);  // the replacement's (parity 0)
        if (threadIdx.x == 0) {
            const double tr = pr[5];
            const int stall = (it + 1 == (int)sl[S_LASTUP]) ? (int)sl[S_STALL] + 1 : 0;
            sl[S_STALL] = stall;
            sl[S_LASTUP] = it + 1;
            sl[S_NREL] += 1.0;
            sl[S_TRUE] = tr;
            est = tr;
            if (!isfinite(tr)) {
                nd = 4;
                why = WHY_NONFINITE;
            } else if (tr <= sl[S_TARGET]) {
                nd = 5;
            } else if (it >= maxit || stall >= 3) {
                nd = 4;
                why = it >= maxit ? WHY_BUDGET : WHY_STALL;
            } else {
                nd = 0;
                if (restart_all || done == 3.0) sl[S_FIRST] = 1.0;
                sl[S_ITUPD] = it;
                sl[S_RRUPD] = pr[0];
            }
        }
    }
    if (threadIdx.x == 0) {
        rec[CR_ITERS] = it;
        rec[CR_B2] = sl[S_B2];
        rec[CR_EST] = est;
        if (nd >= 0) {
            sl[S_DONE] = nd;
            rec[CR_TRUE] = sl[S_TRUE];
            rec[CR_NREL] = sl[S_NREL];
            rec[CR_DONE] = nd;
            rec[CR_WHY] = why;
        }
#pragma unroll
        for (int k = 0; k < CR_N; k++) out[k] = rec[k];
    }
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
                                  int mixed, int maxit) {
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
                                      0, h->lat, B, g, co, h->scal, kpar, ipar, tol2, mixed, maxit);
            else
                hipLaunchKernelGGL((k_cg_iter<R, MC, NB, BS>), dim3(slice_grid(h->lat.Nt)), dim3(nt), lds, h->stream, h->lat, B,
                                   g, co, h->scal, kpar, ipar, tol2, mixed, maxit);
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
                                        double tol2, int mixed, int maxit) {
    qedhmc_ctx::CgGraph& gr = h->cg_graph[sizeof(R) == 8 ? 1 : 0][kpar][ipar0];
    if (gr.exec && (gr.x != B.x || gr.rhs != B.rhs || gr.tol2 != tol2 || gr.mixed != mixed || gr.count != count ||
                    gr.maxit != maxit)) {
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
            st = launch_iters<R>(h, B, kp, ipar0, count, tol2, mixed, maxit);
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
        gr.maxit = maxit;
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

// FP64 O x and the replacement of r, w, s and the partials; gated: both skip
// unless slot kpar asks for a reliable update
template <typename R>
static qedhmc_status launch_replace(qedhmc_ctx* h, const CgBufs<R>& B, const double* x, int kpar, bool gated) {
    QH_TRY(launch_mdagm(h, QEDHMC_FP64, x, h->ws[3], gated ? h->scal + S_NSLOT * kpar + S_DONE : nullptr));
    return with_shape<R>(h, [&]<int MC, int NB, int BS>(int nt, size_t lds) -> qedhmc_status {
        QH_TRY(lds_attr(h, k_cg_replace<R, MC, NB, BS>, lds));
        hipLaunchKernelGGL((k_cg_replace<R, MC, NB, BS>), dim3(slice_grid(h->lat.Nt)), dim3(nt), lds, h->stream, h->lat, B,
                           gauge_for<R>(h), coef_of<R>(h->p), (const double*)h->scal, kpar, gated ? 1 : 0);
        QH_HIP(hipGetLastError());
        return QEDHMC_OK;
    });
}

template <typename R>
static qedhmc_status launch_true(qedhmc_ctx* h, const CgBufs<R>& B, const double* x, int kpar, int restart) {
    QH_TRY(launch_replace<R>(h, B, x, kpar, false));
    hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(256), 0, h->stream, h->scal, kpar, (const double*)h->partial,
                       h->lat.Nt, restart);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// The solve with every decision taken on the device.  A round is a graph
// replay of a chunk of iteration launches followed by the FP64 O x, the
// replacement and the decision, all gated on the slot's stop flag.  Mixed:
// kCap + 1 launches, within which the recursion pauses itself, so every round
// ends in a reliable update and the next one starts at buffer parity 0 on the
// other launch parity (the count is odd).  FP64: 64 launches and no pauses;
// a round either stops (then updates, resuming at buffer parity 0) or runs
// all 64 iterations (an even count: parities unchanged), so every round
// starts at launch and buffer parity 0.  The host keeps the next round
// queued behind the running one and reads each round's record from pinned
// memory through an event, so the GPU does not wait for the host between
// rounds.  The round after the last is skipped when the residual estimates of
// the last two rounds, extrapolated geometrically, say the running round
// converges; a wrong guess costs one host round trip.
template <typename R>
static qedhmc_status cg_pipelined(qedhmc_ctx* h, const CgBufs<R>& B, double* x, double tol, int maxit, bool mixed,
                                  int* iters, double* true_rel, int* n_reliable) {
    const int chunk = mixed ? kCap + 1 : 64;
    static_assert((kCap + 1) & 1, "mixed rounds alternate the launch parity");
    double* rec = h->scal + kRecOff;
    for (auto& e : h->cg_ev)
        if (!e) QH_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    QH_TRY(launch_start<R>(h, B));
    QH_HIP(hipMemsetAsync(rec, 0, CR_N * sizeof(double), h->stream));
    auto round = [&](long n) -> qedhmc_status {
        const int kp = (chunk & 1) ? (int)(n & 1) : 0, ke = kp ^ (chunk & 1);
        QH_TRY(launch_iters_graph<R>(h, B, kp, 0, chunk, tol * tol, mixed ? 1 : 0, maxit));
        QH_TRY(launch_replace<R>(h, B, x, ke, true));
        hipLaunchKernelGGL(k_cg_check_dev, dim3(1), dim3(256), 0, h->stream, h->scal, ke, (const double*)h->partial,
                           h->lat.Nt, maxit, mixed ? 0 : 1, rec, h->h_pinned + 32 + 16 * (n & 1));
        QH_HIP(hipGetLastError());
        QH_HIP(hipEventRecord(h->cg_ev[n & 1], h->stream));
        return QEDHMC_OK;
    };
    // every round that does not end the solve advances the iteration count
    // or the count of updates without progress, which ends it at 3
    const long max_rounds = 4L * maxit + 16;
    long queued = 0;
    double prev = -1.0;
    const double* r = nullptr;
    QH_TRY(round(queued++));
    QH_TRY(round(queued++));
    for (long n = 0;; n++) {
        // queued: round n, and rounds n + 1 and n + 2 unless held back
        QH_HIP(hipEventSynchronize(h->cg_ev[n & 1]));
        r = h->h_pinned + 32 + 16 * (n & 1);
        if (r[CR_DONE] == 4.0 || r[CR_DONE] == 5.0) break;
        if (n + 2 >= max_rounds) {
            QH_HIP(hipStreamSynchronize(h->stream));
            set_error("CG did not end within " + std::to_string(max_rounds) + " rounds");
            return QEDHMC_ENOCONV;
        }
        if (queued < n + 2) QH_TRY(round(queued++));  // round n + 1 was held back wrongly
        const double tr = r[CR_EST], target = tol * tol * r[CR_B2];
        const bool last = prev > 0.0 && tr > 0.0 && tr * (tr / prev) <= target;
        prev = tr;
        if (!last && queued < n + 3) QH_TRY(round(queued++));
    }
    QH_HIP(hipStreamSynchronize(h->stream));  // a round queued past the end runs as no-ops
    const int it = (int)r[CR_ITERS];
    const double b2 = r[CR_B2], rel = b2 > 0.0 ? std::sqrt(r[CR_TRUE] / b2) : 0.0;
    if (iters) *iters = it;
    if (true_rel) *true_rel = rel;
    if (n_reliable) *n_reliable = (int)r[CR_NREL];
    if (r[CR_DONE] == 5.0) return QEDHMC_OK;
    switch ((int)r[CR_WHY]) {
        case WHY_BREAKDOWN:
            set_error("CG breakdown: non-finite inner products after " + std::to_string(it) + " iterations");
            break;
        case WHY_NONFINITE:
            set_error("CG breakdown: non-finite true residual after " + std::to_string(it) + " iterations");
            break;
        case WHY_STALL:
            set_error("CG made no progress across reliable updates at iteration " + std::to_string(it));
            break;
        default:
            break;
    }
    return QEDHMC_ENOCONV;
}

template <typename R>
static qedhmc_status cg_t(qedhmc_ctx* h, const double* rhs, double* x, double tol, int maxit, qedhmc_precision prec,
                          int* iters, double* true_rel, int* n_reliable) {
    const bool mixed = prec != QEDHMC_FP64;
    const CgBufs<R> B = bufs_of<R>(h, rhs, x);
    // QEDHMC_NO_GRAPH (read per solve) launches every chunk directly from a
    // host-driven loop
    const bool no_graph = std::getenv("QEDHMC_NO_GRAPH") != nullptr;
    if (!no_graph) return cg_pipelined<R>(h, B, x, tol, maxit, mixed, iters, true_rel, n_reliable);
    // chunk of launches between host checks; the mixed path pauses itself at
    // most every kCap + 1 launches
    const int chunk = mixed ? kCap + 1 : 64;
    int kpar = 0, nrel = 0, it = 0, itupd = 0, stalled = 0, last_it = -1;
    double rel = 1.0;
    bool converged = false, broken = false;
    static const bool trace = std::getenv("QEDHMC_CG_TRACE") != nullptr;
    QH_TRY(launch_start<R>(h, B));
    while (true) {
        const int left = maxit - it;
        // full chunks replay a captured graph
        // buffer parity: iterations since the last reliable update
        if (left >= chunk && !no_graph) {
            QH_TRY(launch_iters_graph<R>(h, B, kpar, (it - itupd) & 1, chunk, tol * tol, mixed ? 1 : 0, maxit));
            if (chunk & 1) kpar ^= 1;
        } else if (left > 0) {
            QH_TRY(launch_iters<R>(h, B, kpar, it - itupd, left < chunk ? left : chunk, tol * tol, mixed ? 1 : 0,
                                   maxit));
        }
        QH_TRY(read_slot(h, kpar));
        it = (int)h->h_pinned[S_ITERS];
        itupd = (int)h->h_pinned[S_ITUPD];
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
        itupd = (int)h->h_pinned[S_ITUPD];
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
