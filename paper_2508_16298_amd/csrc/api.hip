// C ABI of libqedhmc: handle lifetime, argument checks, and the host-side
// orchestration of the trajectory (Methods, HQMC steps (i)-(iv)).
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <unordered_set>

#include "net_internal.h"
#include "qedhmc_internal.h"

namespace qh {

qedhmc_status allow_lds(const void* k, size_t max_lds) {
    static std::mutex m;
    static std::unordered_set<const void*> done;
    std::lock_guard<std::mutex> g(m);
    if (done.count(k)) return QEDHMC_OK;
    // the dynamic room is what the kernel's static LDS leaves of the limit
    hipFuncAttributes fa{};
    QH_HIP(hipFuncGetAttributes(&fa, k));
    const size_t room = max_lds > fa.sharedSizeBytes ? max_lds - fa.sharedSizeBytes : 0;
    QH_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)room));
    done.insert(k);
    return QEDHMC_OK;
}

qedhmc_status blocks_per_cu(const void* k, int threads, size_t lds, int* out) {
    static std::mutex m;
    static std::map<std::tuple<const void*, int, size_t>, int> cache;
    std::lock_guard<std::mutex> g(m);
    const auto key = std::make_tuple(k, threads, lds);
    auto it = cache.find(key);
    if (it == cache.end()) {
        int n = 0;
        QH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, threads, lds));
        it = cache.emplace(key, n).first;
    }
    *out = it->second;
    return QEDHMC_OK;
}

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

qedhmc_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return QEDHMC_EHIP;
}

static qedhmc_status einval(const char* msg) {
    g_err = msg;
    return QEDHMC_EINVAL;
}

bool prof_sample_n(qedhmc_ctx* h, int cls, int n, hipEvent_t& e0, hipEvent_t& e1) {
    if (h->prof_every <= 0 || !h->prof_ready) return false;
    if ((h->prof_seen[cls]++ % h->prof_every) != 0) return false;
    if (h->prof_pending == 64 && prof_drain(h) != QEDHMC_OK) return false;
    const int k = h->prof_pending++;
    h->prof_cls[k] = cls;
    h->prof_weight[k] = n;
    e0 = h->prof_ev[k][0];
    e1 = h->prof_ev[k][1];
    return true;
}

bool prof_sample(qedhmc_ctx* h, int cls, hipEvent_t& e0, hipEvent_t& e1) { return prof_sample_n(h, cls, 1, e0, e1); }

qedhmc_status prof_drain(qedhmc_ctx* h) {
    for (int k = 0; k < h->prof_pending; k++) {
        QH_HIP(hipEventSynchronize(h->prof_ev[k][1]));
        float ms = 0.f;
        QH_HIP(hipEventElapsedTime(&ms, h->prof_ev[k][0], h->prof_ev[k][1]));
        h->prof_count[h->prof_cls[k]] += h->prof_weight[k];
        h->prof_ms[h->prof_cls[k]] += ms;
    }
    h->prof_pending = 0;
    return QEDHMC_OK;
}

}  // namespace qh

using namespace qh;

#define CHECK_H(h) \
    if (!(h)) return einval("null handle")

static size_t nsites(const qedhmc_ctx* h) { return (size_t)h->lat.Nt * h->lat.Vs; }

qedhmc_status qh::check_prec(qedhmc_precision p) {
    if (p != QEDHMC_FP64 && p != QEDHMC_FP32) return einval("bad precision");
    return QEDHMC_OK;
}

qedhmc_status qh::check_params(const qedhmc_params* params) {
    const qedhmc_params& p = *params;
    if (p.L < 2 || p.L % 2 != 0) return einval("L must be even and >= 2");
    if (p.L > 2048) return einval("L > 2048 is not supported");
    if (p.Nt < 1) return einval("Nt must be >= 1");
    if (!(p.dtau >= 0.0) || !(p.J > 0.0) || !std::isfinite(p.t) || !std::isfinite(p.K))
        return einval("bad couplings (need dtau >= 0, J > 0, finite t and K)");
    if ((size_t)p.L * p.L * p.Nt >= ((size_t)1 << 31)) return einval("lattice too large");
    if ((p.action != QEDHMC_COMPACT && p.action != QEDHMC_NONCOMPACT) || p.reserved != 0)
        return einval("bad gauge action (QEDHMC_COMPACT or QEDHMC_NONCOMPACT; reserved 0)");
    return QEDHMC_OK;
}

qedhmc_status qh::ctx_geometry(qedhmc_ctx* h, const qedhmc_params& p, void* stream) {
    h->p = p;
    h->lat.L = p.L;
    h->lat.Nt = p.Nt;
    h->lat.Vs = p.L * p.L;
    h->lat.hL = p.L / 2;
    h->lat.ncell = h->lat.hL * h->lat.hL;
    h->stream = (hipStream_t)stream;
    hipError_t e = hipGetDevice(&h->device);
    int lds = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, h->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice / attribute");
    h->max_lds = (size_t)lds;
    return QEDHMC_OK;
}

extern "C" {

const char* qedhmc_last_error(void) { return g_err.c_str(); }

qedhmc_status qedhmc_init_lattice(const qedhmc_params* params, void* stream, qedhmc_t* out) {
    if (!params || !out) return einval("null argument");
    QH_TRY(check_params(params));
    const qedhmc_params& p = *params;
    *out = nullptr;
    qedhmc_ctx* h = new (std::nothrow) qedhmc_ctx{};
    if (!h) return QEDHMC_ENOMEM;
    const qedhmc_status gst = ctx_geometry(h, p, stream);
    if (gst != QEDHMC_OK) {
        delete h;
        return gst;
    }
    hipError_t e = hipSuccess;
    const size_t N = nsites(h);
    const size_t vec = N * sizeof(cplx<double>);
    bool ok = true;
    ok = ok && hipMalloc(&h->d_tables, sizeof(int32_t) * 3 * 2 * h->lat.Vs) == hipSuccess;
    ok = ok && hipMalloc(&h->gauge64, 2 * N * sizeof(cplx<double>)) == hipSuccess;
    ok = ok && hipMalloc(&h->gauge32, 2 * N * sizeof(cplx<float>)) == hipSuccess;
    for (int k = 0; k < 12 && ok; k++) ok = hipMalloc(&h->ws[k], vec) == hipSuccess;
    ok = ok && hipMalloc(&h->cg_arena, 7 * vec) == hipSuccess;
    ok = ok && hipMalloc(&h->theta0, 2 * N * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&h->mom, 2 * N * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&h->force, 2 * N * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&h->force_b, 2 * N * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&h->partial, ((size_t)12 * p.Nt + 4096) * sizeof(double)) == hipSuccess;
    if (ok && h->lat.ncell > 1024) {
        h->tpart_tiles = std::max(mdagm_tiled_tiles(h->lat, false), mdagm_tiled_tiles(h->lat, true));
        ok = hipMalloc(&h->tpart, ((size_t)7 * p.Nt * h->tpart_tiles + p.Nt + 64) * sizeof(double)) == hipSuccess;
    }
    ok = ok && hipMalloc(&h->scal, 128 * sizeof(double)) == hipSuccess;
    ok = ok && hipHostMalloc(&h->h_pinned, 64 * sizeof(double), hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        qedhmc_destroy(h);
        g_err = "device allocation failed";
        return QEDHMC_ENOMEM;
    }
    qedhmc_status st = launch_bond_tables(h);
    if (st == QEDHMC_OK) {
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) st = hip_fail(e, "init sync");
    }
    if (st != QEDHMC_OK) {
        qedhmc_destroy(h);
        return st;
    }
    *out = h;
    return QEDHMC_OK;
}

qedhmc_status qedhmc_destroy(qedhmc_t h) {
    if (!h) return QEDHMC_OK;
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(h->d_tables);
    (void)hipFree(h->gauge64);
    (void)hipFree(h->gauge32);
    for (int k = 0; k < 12; k++) (void)hipFree(h->ws[k]);
    (void)hipFree(h->cg_arena);
    if (h->pc_dev64) (void)hipFree(h->pc_dev64);
    if (h->pc_dev32) (void)hipFree(h->pc_dev32);
    if (h->pc_roll64) (void)hipFree(h->pc_roll64);
    if (h->pc_roll32) (void)hipFree(h->pc_roll32);
    if (h->pc_spec64) (void)hipFree(h->pc_spec64);
    if (h->pc_spec32) (void)hipFree(h->pc_spec32);
    if (h->pc_tw64) (void)hipFree(h->pc_tw64);
    if (h->pc_tw32) (void)hipFree(h->pc_tw32);
    (void)hipFree(h->theta0);
    (void)hipFree(h->mom);
    (void)hipFree(h->force);
    (void)hipFree(h->force_b);
    (void)hipFree(h->partial);
    if (h->tpart) (void)hipFree(h->tpart);
    (void)hipFree(h->scal);
    if (h->h_pinned) (void)hipHostFree(h->h_pinned);
    if (h->prof_ready)
        for (int k = 0; k < 64; k++) {
            (void)hipEventDestroy(h->prof_ev[k][0]);
            (void)hipEventDestroy(h->prof_ev[k][1]);
        }
    for (auto& a : h->cg_graph)
        for (auto& b : a)
            for (auto& g : b)
                if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (auto& e : h->cg_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& a : h->pcg_graph)
        for (auto& b : a)
            for (auto& g : b)
                if (g.exec) (void)hipGraphExecDestroy(g.exec);
    for (auto& a : h->pcg_round)
        for (auto& g : a)
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
    delete h;
    return QEDHMC_OK;
}

qedhmc_status qedhmc_profile(qedhmc_t h, int32_t every) {
    CHECK_H(h);
    if (every < 0) return einval("every must be >= 0");
    if (every > 0 && !h->prof_ready) {
        for (int k = 0; k < 64; k++) {
            QH_HIP(hipEventCreate(&h->prof_ev[k][0]));
            QH_HIP(hipEventCreate(&h->prof_ev[k][1]));
        }
        h->prof_ready = true;
    }
    QH_TRY(prof_drain(h));
    h->prof_every = every;
    for (int c = 0; c < QEDHMC_K_COUNT; c++) {
        h->prof_seen[c] = 0;
        h->prof_count[c] = 0;
        h->prof_ms[c] = 0.0;
    }
    return QEDHMC_OK;
}

qedhmc_status qedhmc_profile_read(qedhmc_t h, int32_t cls, int64_t* count, double* total_ms) {
    CHECK_H(h);
    if (cls < 0 || cls >= QEDHMC_K_COUNT || !count || !total_ms) return einval("bad profile query");
    QH_HIP(hipStreamSynchronize(h->stream));
    QH_TRY(prof_drain(h));
    *count = h->prof_count[cls];
    *total_ms = h->prof_ms[cls];
    return QEDHMC_OK;
}

qedhmc_status qedhmc_set_stream(qedhmc_t h, void* stream) {
    CHECK_H(h);
    h->stream = (hipStream_t)stream;
    return QEDHMC_OK;
}

qedhmc_status qedhmc_get_bond_tables(qedhmc_t h, int32_t* host_out) {
    CHECK_H(h);
    if (!host_out) return einval("null output");
    QH_HIP(hipMemcpyAsync(host_out, h->d_tables, sizeof(int32_t) * 3 * 2 * h->lat.Vs, hipMemcpyDeviceToHost,
                          h->stream));
    QH_HIP(hipStreamSynchronize(h->stream));
    return QEDHMC_OK;
}

qedhmc_status qedhmc_apply_B(qedhmc_t h, const double* theta, int32_t tau, const void* in, void* out,
                             qedhmc_precision prec) {
    CHECK_H(h);
    if (!theta || !in || !out) return einval("null pointer");
    if (tau < 0 || tau >= h->lat.Nt) return einval("tau out of range");
    QH_TRY(check_prec(prec));
    QH_TRY(ensure_gauge(h, theta, prec));
    return launch_apply_B(h, prec, tau, in, out);
}

qedhmc_status qedhmc_apply_M(qedhmc_t h, const double* theta, const void* in, void* out, int32_t dagger,
                             qedhmc_precision prec) {
    CHECK_H(h);
    if (!theta || !in || !out) return einval("null pointer");
    if (in == out) return einval("in and out alias");
    QH_TRY(check_prec(prec));
    QH_TRY(ensure_gauge(h, theta, prec));
    return launch_apply_M(h, prec, in, out, dagger ? 1 : 0);
}

qedhmc_status qedhmc_apply_MdagM(qedhmc_t h, const double* theta, const void* in, void* out,
                                 qedhmc_precision prec) {
    CHECK_H(h);
    if (!theta || !in || !out) return einval("null pointer");
    if (in == out) return einval("in and out alias");
    QH_TRY(check_prec(prec));
    QH_TRY(ensure_gauge(h, theta, prec));
    return launch_mdagm(h, prec, in, out, nullptr);
}

// switched (nullable): with the learned preconditioner, the iteration at
// which its judge handed the solve to the fallback (-1: kept it)
static qedhmc_status solve_at(qedhmc_ctx* h, const double* theta, const double* rhs, double* x, double tol,
                              int32_t maxit, qedhmc_precision prec, qedhmc_precond pc, int32_t* iters, double* rel,
                              int* nrel, int* switched = nullptr) {
    QH_TRY(ensure_gauge(h, theta, QEDHMC_FP64));
    if (prec != QEDHMC_FP64 || pc == QEDHMC_PC_LEARNED) QH_TRY(ensure_gauge(h, theta, QEDHMC_FP32));
    int it = 0, nr = 0, sw = -1;
    double r = 0.0;
    qedhmc_status st;
    if (pc == QEDHMC_PC_LEARNED) {
        if (!h->pc_net) return einval("QEDHMC_PC_LEARNED: no network bound to the handle");
        if (prec == QEDHMC_FP64) {
            int32_t it32 = 0, sw32 = -1;
            st = qedhmc_fcg_solve(h->pc_net, theta, rhs, x, tol, maxit, h->pc_arith, h->pc_fallback, &it32, &r,
                                  &sw32);
            it = it32;
            sw = sw32;
        } else {
            st = mfcg_solve_impl(h->pc_net, rhs, x, tol, maxit, h->pc_arith, h->pc_fallback, &it, &r, &nr, &sw);
        }
    } else if (pc == QEDHMC_PC_PAPER) {
        st = pcg_solve_impl(h, rhs, x, tol, maxit, prec, &it, &r, &nr);
    } else {
        st = cg_solve_impl(h, rhs, x, tol, maxit, prec, &it, &r, &nr);
    }
    if (iters) *iters = it;
    if (rel) *rel = r;
    if (nrel) *nrel = nr;
    if (switched) *switched = sw;
    if (st == QEDHMC_ENOCONV && pc != QEDHMC_PC_LEARNED)
        set_error("CG reached maxit=" + std::to_string(maxit) + " with true residual " + std::to_string(r));
    return st;
}

static qedhmc_status check_pc(qedhmc_precond pc) {
    if (pc != QEDHMC_PC_NONE && pc != QEDHMC_PC_PAPER && pc != QEDHMC_PC_LEARNED)
        return einval("unknown preconditioner");
    return QEDHMC_OK;
}

qedhmc_status qedhmc_cg_solve(qedhmc_t h, const double* theta, const double* rhs, double* x, double tol,
                              int32_t maxit, qedhmc_precision prec, qedhmc_precond pc, int32_t* iters,
                              double* true_rel_resid) {
    CHECK_H(h);
    if (!theta || !rhs || !x) return einval("null pointer");
    if (rhs == x) return einval("rhs and x alias");
    if (!(tol > 0.0) || maxit < 1) return einval("need tol > 0 and maxit >= 1");
    QH_TRY(check_pc(pc));
    QH_TRY(check_prec(prec));
    if (pc == QEDHMC_PC_LEARNED && !h->pc_net) return einval("QEDHMC_PC_LEARNED: no network bound to the handle");
    return solve_at(h, theta, rhs, x, tol, maxit, prec, pc, iters, true_rel_resid, nullptr);
}

qedhmc_status qedhmc_set_learned_precond(qedhmc_t h, qedhmc_net_t n, qedhmc_net_arith arith,
                                         qedhmc_precond fallback) {
    CHECK_H(h);
    if (!n) {
        h->pc_net = nullptr;
        return QEDHMC_OK;
    }
    if (n->h != h) return einval("the network belongs to another lattice handle");
    if (arith != QEDHMC_NET_FP32 && arith != QEDHMC_NET_BF16) return einval("bad network arithmetic");
    if (fallback != QEDHMC_PC_NONE && fallback != QEDHMC_PC_PAPER)
        return einval("the fallback is QEDHMC_PC_NONE or QEDHMC_PC_PAPER");
    h->pc_net = n;
    h->pc_arith = arith;
    h->pc_fallback = fallback;
    return QEDHMC_OK;
}

qedhmc_status qedhmc_precond_taps(qedhmc_t h, int32_t parity, int32_t* count, double* out, int32_t capacity) {
    CHECK_H(h);
    if (!count || (parity != 0 && parity != 1) || capacity < 0 || (capacity > 0 && !out))
        return einval("bad stencil query");
    QH_TRY(ensure_paper_precond(h));
    const auto& t = h->pc_taps[parity];
    *count = (int32_t)t.size();
    for (int32_t k = 0; k < capacity && k < (int32_t)t.size(); k++) {
        out[5 * k] = t[k].dt;
        out[5 * k + 1] = t[k].dx;
        out[5 * k + 2] = t[k].dy;
        out[5 * k + 3] = t[k].gre;
        out[5 * k + 4] = t[k].gim;
    }
    return QEDHMC_OK;
}

qedhmc_status qedhmc_apply_precond(qedhmc_t h, const void* in, void* out, qedhmc_precision prec) {
    CHECK_H(h);
    if (!in || !out) return einval("null pointer");
    if (in == out) return einval("in and out alias");
    QH_TRY(check_prec(prec));
    return launch_apply_precond(h, prec, in, out);
}

qedhmc_status qedhmc_fermion_force(qedhmc_t h, const double* theta, const double* X, double* F,
                                   qedhmc_precision prec) {
    CHECK_H(h);
    if (!theta || !X || !F) return einval("null pointer");
    QH_TRY(check_prec(prec));
    QH_TRY(ensure_gauge(h, theta, prec));
    return launch_force(h, prec, X, F);
}

qedhmc_status qedhmc_bosonic_action_force(qedhmc_t h, const double* theta, double* S_B_host, double* F_B) {
    CHECK_H(h);
    if (!theta) return einval("null pointer");
    QH_TRY(launch_bosonic(h, theta, F_B, h->scal + 100));
    if (S_B_host) {
        QH_HIP(hipMemcpyAsync(h->h_pinned, h->scal + 100, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        QH_HIP(hipStreamSynchronize(h->stream));
        *S_B_host = h->h_pinned[0];
    }
    return QEDHMC_OK;
}

qedhmc_status qedhmc_heatbath(qedhmc_t h, uint64_t traj_index, double* mom, double* R) {
    CHECK_H(h);
    if (!mom || !R) return einval("null pointer");
    return launch_heatbath(h, traj_index, mom, R);
}

qedhmc_status qedhmc_hmc_trajectory(qedhmc_t h, double* theta, uint64_t traj, int32_t n_steps, double traj_len,
                                    double tol, int32_t maxit, qedhmc_precision prec, qedhmc_precond pc,
                                    qedhmc_traj_result* out) {
    CHECK_H(h);
    if (!theta || !out) return einval("null pointer");
    if (n_steps < 1 || !(traj_len > 0.0) || !(tol > 0.0) || maxit < 1) return einval("bad trajectory parameters");
    QH_TRY(check_pc(pc));
    QH_TRY(check_prec(prec));
    if (pc == QEDHMC_PC_LEARNED && !h->pc_net) return einval("QEDHMC_PC_LEARNED: no network bound to the handle");
    std::memset(out, 0, sizeof(*out));
    const size_t N = nsites(h), nb = 2 * N;
    const double dt = traj_len / n_steps;
    double* sc = h->scal + 64;  // SB0 K0 SF0 SB1 K1 SF1 dH u acc
    double* R = (double*)h->ws[4];
    double* eta = (double*)h->ws[5];
    double* X = (double*)h->ws[6];
    int it_total = 0, it_max = 0, nrel_total = 0, worst = 0;
    double max_rel = 0.0;
    // The solves after the first share eta and see theta moved by one drift:
    // each starts from the previous X (QEDHMC_WARM_START=0, read per
    // trajectory, starts every solve from zero).  It solves O e = eta - O X
    // for the correction from zero, to the tolerance that keeps the same
    // target |eta - O (X + e)| <= tol |eta|, and adds e to X; solves that
    // reach the tolerance give the same X to that tolerance, and every solver
    // (CG, PCG, flexible CG) runs unchanged.
    const char* ews = std::getenv("QEDHMC_WARM_START");
    const bool warm_ok = !(ews && *ews && std::atoi(ews) == 0);
    double* bres = (double*)h->ws[0];  // eta - O X
    double* corr = (double*)h->ws[1];  // e
    auto solve = [&](const double* th, bool warm) -> qedhmc_status {
        int32_t it = 0;
        double rel = 0.0;
        int nr = 0, sw = -1;
        qedhmc_status st = QEDHMC_OK;
        if (!(warm && warm_ok)) {
            st = solve_at(h, th, eta, X, tol, maxit, prec, pc, &it, &rel, &nr, &sw);
        } else {
            QH_TRY(ensure_gauge(h, th, QEDHMC_FP64));
            QH_TRY(launch_mdagm(h, QEDHMC_FP64, X, bres, nullptr));
            QH_TRY(launch_lincomb(h, bres, 1.0, eta, -1.0, bres, 2 * N));
            QH_TRY(launch_sumsq(h, eta, 2 * N, h->scal + 80));
            QH_TRY(launch_sumsq(h, bres, 2 * N, h->scal + 81));
            QH_HIP(hipMemcpyAsync(h->h_pinned, h->scal + 80, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
            QH_HIP(hipStreamSynchronize(h->stream));
            const double nb = std::sqrt(h->h_pinned[0]), nr0 = std::sqrt(h->h_pinned[1]);
            if (!std::isfinite(nr0)) {
                // as a solve that missed its tolerance: the proposal is rejected
                worst = 2;
                max_rel = HUGE_VAL;
                return QEDHMC_OK;
            }
            if (nr0 > tol * nb) {
                double relc = 0.0;
                st = solve_at(h, th, bres, corr, tol * nb / nr0, maxit, prec, pc, &it, &relc, &nr, &sw);
                if (st != QEDHMC_OK && st != QEDHMC_ENOCONV) return st;
                QH_TRY(launch_lincomb(h, X, 1.0, X, 1.0, corr, 2 * N));
                rel = relc * nr0 / nb;
            } else {
                rel = nb > 0.0 ? nr0 / nb : 0.0;
            }
        }
        if (st != QEDHMC_OK && st != QEDHMC_ENOCONV) return st;
        if (st == QEDHMC_ENOCONV) worst = 2;
        if (sw >= 0) out->pc_fallbacks++;
        out->n_solves++;
        it_total += it;
        if (it > it_max) it_max = it;
        if (rel > max_rel) max_rel = rel;
        nrel_total += nr;
        return QEDHMC_OK;
    };

    QH_HIP(hipMemcpyAsync(h->theta0, theta, nb * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    // (i) heat bath, eta = M^dag R
    QH_TRY(launch_heatbath(h, traj, h->mom, R));
    QH_TRY(ensure_gauge(h, theta, QEDHMC_FP64));
    QH_TRY(launch_apply_M(h, QEDHMC_FP64, R, eta, 1));
    // H at the start
    QH_TRY(solve(theta, false));
    QH_TRY(launch_dot_re(h, eta, X, 2 * N, sc + 2));
    QH_TRY(launch_sumsq(h, h->mom, nb, sc + 1));
    QH_TRY(launch_bosonic(h, theta, h->force_b, sc + 0));
    QH_TRY(ensure_gauge(h, theta, prec));
    QH_TRY(launch_force(h, prec, X, h->force));
    // (ii) leapfrog
    for (int n = 0; n < n_steps; n++) {
        QH_TRY(launch_kick(h, h->mom, h->force, h->force_b, 0.5 * dt, nb));
        QH_TRY(launch_drift(h, theta, h->mom, 2.0 * dt, nb));
        QH_TRY(solve(theta, true));
        QH_TRY(ensure_gauge(h, theta, prec));
        QH_TRY(launch_force(h, prec, X, h->force));
        QH_TRY(launch_bosonic(h, theta, h->force_b, sc + 3));
        QH_TRY(launch_kick(h, h->mom, h->force, h->force_b, 0.5 * dt, nb));
    }
    // H at the end, (iii) Metropolis, restore on rejection
    QH_TRY(launch_dot_re(h, eta, X, 2 * N, sc + 5));
    QH_TRY(launch_sumsq(h, h->mom, nb, sc + 4));
    // a solve that missed its tolerance leaves a dH that is not the leapfrog's
    // (reversibility fails), so such a trajectory is always rejected
    QH_TRY(launch_metropolis(h, traj, worst != 0, sc));
    QH_TRY(launch_restore(h, theta, h->theta0, sc, nb));
    QH_HIP(hipMemcpyAsync(h->h_pinned, sc, 9 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    QH_HIP(hipStreamSynchronize(h->stream));
    const double* v = h->h_pinned;
    out->SB0 = v[0];
    out->K0 = v[1];
    out->SF0 = v[2];
    out->SB1 = v[3];
    out->K1 = v[4];
    out->SF1 = v[5];
    out->H0 = v[0] + v[1] + v[2];
    out->H1 = v[3] + v[4] + v[5];
    out->dH = v[6];
    out->u = v[7];
    out->accepted = v[8] != 0.0 ? 1 : 0;
    out->cg_iters_total = it_total;
    out->cg_iters_max = it_max;
    out->status = worst;
    out->reliable_updates = nrel_total;
    out->max_true_resid = max_rel;
    if (worst != 0) {
        set_error("a solve of the trajectory did not converge (largest true residual " + std::to_string(max_rel) +
                  "); the proposal was rejected");
        return QEDHMC_ENOCONV;
    }
    return QEDHMC_OK;
}

}  // extern "C"
