// The paper's preconditioner (Methods, "CG method and preconditioner"; the
// banded structure of Fig. 3) and CG preconditioned with it.
//
// Construction (once per handle, on first use), following the paper's recipe
// as read for this build:
//   1. O_pi = M^dag M at pi flux (theta_x = 0, theta_y = pi x) on a build
//      lattice of kBuildL x kBuildL x kBuildNt, assembled column by column by
//      the library's own FP64 M^dag M kernel applied to unit vectors;
//   2. forward IC(0) on the host in the natural order n = tau*Vs + s,
//      O_pi ~ L L^dag on the pattern of O_pi (|O| > 1e-12 max|O|), with a
//      diagonal shift if a pivot is not positive;
//   3. the rows of G = L^{-1} at an interior site of a bulk slice, one per x
//      parity (the pi-flux unit cell), by one triangular solve each;
//   4. taps (dtau, dx, dy, g) with 0 <= dtau <= kCapTau and |g| >= kThresh
//      (the paper's matrix shows a band of 6 in tau; the reach here was
//      chosen by time to solution).
// Application: G[(tau,s),(tau-dtau, s+ds)] = g_{x(s) mod 2}(dtau, ds), with
// -1 when tau-dtau wraps (antiperiodic), and P = G^dag G as two stencil
// passes.  P is Hermitian positive definite whenever G is non-singular.
//
// PCG, one iteration = four launches (every read of a neighbouring slice
// crosses a launch boundary, so no buffer is read and written in one launch):
//   k_pcg_upd   partial sums -> beta, alpha (single reduction phase as in the
//               unpreconditioned solver, denominator <p,s> expanded);
//               p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s
//   k_pc_apply  t = G r
//   k_pc_apply  u = G^dag t
//   k_pcg_mv    w = O u and the partials <r,r>, <r,u>, <w,u>, <u,s>, <p,w>, <p,s>
// with gamma = <r, P r>; stopping and reliable updates on |r| as in cg.hip.
#include <algorithm>
#include <vector>

#include <cstdlib>
#include <cstring>
#include "cg_common.h"

namespace qh {

static constexpr int kBuildL = 8;
static constexpr int kBuildNt = 24;
static constexpr int kCapTau = QEDHMC_PC_TAU_REACH;  // tau reach of G (QEDHMC_PC_CAP overrides, up to kCapMax)
static constexpr int kCapMax = 12;
static constexpr double kThresh = 1e-3;
static constexpr int kNP7 = 7;  // PCG partials: <r,r>, <r,u>, <w,u>, <u,s>, <p,w>, <p,s>, unused

static constexpr int kPcSlots = 16;  // tau offsets per stencil pass at most (0 <= dt <= kCapMax, plus spare)

// One stencil tap of a parity's list, q = parity + c - cmin: aidx = a - amin
// (its slice in the window ring), off = b * half + (q >> 1) and plane = q & 1
// (row, column pair and column parity of the source relative to the output).
template <typename R>
struct PTap {
    int aidx;
    int off;
    int plane;
    int pad;
    cplx<R> g;
};

// ---------------------------------------------------------------------------
// Builder
// ---------------------------------------------------------------------------
__global__ void k_unit(cplx<double>* __restrict__ e, size_t n, size_t k) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        e[i] = mk<double>(i == k ? 1.0 : 0.0, 0.0);
}

// ---------------------------------------------------------------------------
// Spectral form of P.  Both passes are gathers whose taps depend only on the
// output's x parity, with space periodic and one sign flip per wrap of tau
// (the antiperiodic extension itself once N_tau exceeds a pass's tau reach).
// So each pass commutes with translations by the two-site cell (2 in x, 1 in
// y) and by one slice, and on the cell momenta kx = 2 pi nx / (L/2),
// ky = 2 pi ny / L it acts on the pair (v_even, v_odd) of a slice as a 2x2
// matrix S(k, a) per tau offset a:
//   S[p][p'](k, a) = sum over the taps (a, b, c, g) of parity p with
//                    (p + c) mod 2 = p' of g exp(i (kx (p + c - p') / 2 + ky b)).
// P = S_1 S_0 has the blocks H(k, a) = sum_{a1 + a2 = a} S_1(k, a2) S_0(k, a1)
// for a in [amin_0 + amin_1, amax_0 + amax_1], and one application is a 2D DFT
// of every slice's two parity planes, the banded tau sum
// z^(k, tau) = sum_a sign H(k, a) v^(k, tau + a) (sign -1 per wrap), and the
// inverse DFT (its 1 / (L L/2) folded into H).  Same operator, far fewer
// operations than the taps at the sizes the stencil is latency-bound at.
// ---------------------------------------------------------------------------
static constexpr int kSpecNA = 2 * kCapMax + 1;  // combined tau offsets at most
static constexpr int kSpecE = 8;                // DFT outputs per thread at most (L * L/2 <= 8192)
static constexpr int kSpecChunk = 13;           // tau offsets per load batch of the fused tau sum

static qedhmc_status build_spectral(qedhmc_ctx* h, const std::vector<HostTap> (&pass)[2][2]) {
    h->pc_spec_na = 0;
    const int L = h->lat.L, Lh = L / 2, nk = L * Lh;
    if (L % 2 || h->lat.Nt <= h->pc_cap || nk > kSpecE * 1024) return QEDHMC_OK;
    const int a0 = h->pc_pass[0].amin + h->pc_pass[1].amin, a1 = h->pc_pass[0].amax + h->pc_pass[1].amax;
    const int na = a1 - a0 + 1;
    if (na > kSpecNA) return QEDHMC_OK;
    // e^{+2 pi i j / n} by integer index, so every phase is one table entry
    auto unit = [](int n) {
        std::vector<cplx<double>> t(n);
        for (int j = 0; j < n; j++) t[j] = mk<double>(std::cos(2 * M_PI * j / n), std::sin(2 * M_PI * j / n));
        return t;
    };
    const std::vector<cplx<double>> ex = unit(Lh), ey = unit(L);
    auto pmod = [](int v, int n) { return ((v % n) + n) % n; };
    auto cmul = [](cplx<double> x, cplx<double> y) {
        return mk<double>(x.re * y.re - x.im * y.im, x.re * y.im + x.im * y.re);
    };
    std::vector<cplx<double>> H((size_t)na * 4 * nk, mk<double>(0.0, 0.0));  // [a][entry pp'][k]
    const int n0 = h->pc_pass[0].amax - h->pc_pass[0].amin + 1, n1 = h->pc_pass[1].amax - h->pc_pass[1].amin + 1;
    std::vector<cplx<double>> S0((size_t)n0 * 4), S1((size_t)n1 * 4);
    for (int ny = 0; ny < L; ny++)
        for (int nx = 0; nx < Lh; nx++) {
            const int k = ny * Lh + nx;
            for (int ps = 0; ps < 2; ps++) {
                std::vector<cplx<double>>& S = ps ? S1 : S0;
                std::fill(S.begin(), S.end(), mk<double>(0.0, 0.0));
                for (int p = 0; p < 2; p++)
                    for (const auto& t : pass[ps][p]) {
                        const int pp = pmod(p + t.dx, 2), m = (p + t.dx - pp) / 2;
                        const cplx<double> ph = cmul(ex[pmod(m * nx, Lh)], ey[pmod(t.dy * ny, L)]);
                        cplx<double>& e = S[(size_t)(t.dt - h->pc_pass[ps].amin) * 4 + 2 * p + pp];
                        const cplx<double> c = cmul(mk<double>(t.gre, t.gim), ph);
                        e.re += c.re;
                        e.im += c.im;
                    }
            }
            for (int i0 = 0; i0 < n0; i0++)
                for (int i1 = 0; i1 < n1; i1++) {
                    const int ia = h->pc_pass[0].amin + i0 + h->pc_pass[1].amin + i1 - a0;
                    for (int p = 0; p < 2; p++)
                        for (int pp = 0; pp < 2; pp++) {
                            cplx<double>& e = H[((size_t)ia * 4 + 2 * p + pp) * nk + k];
                            for (int q = 0; q < 2; q++) {
                                const cplx<double> c = cmul(S1[(size_t)i1 * 4 + 2 * p + q], S0[(size_t)i0 * 4 + 2 * q + pp]);
                                e.re += c.re;
                                e.im += c.im;
                            }
                        }
                }
        }
    const double norm = 1.0 / nk;
    for (auto& e : H) e = mk<double>(e.re * norm, e.im * norm);
    // forward twiddles e^{-2 pi i j / n}: L/2 for x, then L for y
    std::vector<cplx<double>> tw(Lh + L);
    for (int j = 0; j < Lh; j++) tw[j] = mk<double>(ex[j].re, -ex[j].im);
    for (int j = 0; j < L; j++) tw[Lh + j] = mk<double>(ey[j].re, -ey[j].im);
    std::vector<cplx<float>> H32(H.size()), tw32(tw.size());
    for (size_t i = 0; i < H.size(); i++) H32[i] = mk<float>((float)H[i].re, (float)H[i].im);
    for (size_t i = 0; i < tw.size(); i++) tw32[i] = mk<float>((float)tw[i].re, (float)tw[i].im);
    QH_HIP(hipMalloc(&h->pc_spec64, H.size() * sizeof(cplx<double>)));
    QH_HIP(hipMalloc(&h->pc_spec32, H.size() * sizeof(cplx<float>)));
    QH_HIP(hipMalloc(&h->pc_tw64, tw.size() * sizeof(cplx<double>)));
    QH_HIP(hipMalloc(&h->pc_tw32, tw.size() * sizeof(cplx<float>)));
    QH_HIP(hipMemcpyAsync(h->pc_spec64, H.data(), H.size() * sizeof(cplx<double>), hipMemcpyHostToDevice, h->stream));
    QH_HIP(hipMemcpyAsync(h->pc_spec32, H32.data(), H32.size() * sizeof(cplx<float>), hipMemcpyHostToDevice, h->stream));
    QH_HIP(hipMemcpyAsync(h->pc_tw64, tw.data(), tw.size() * sizeof(cplx<double>), hipMemcpyHostToDevice, h->stream));
    QH_HIP(hipMemcpyAsync(h->pc_tw32, tw32.data(), tw32.size() * sizeof(cplx<float>), hipMemcpyHostToDevice, h->stream));
    // the host vectors die at return: wait for the copies
    QH_HIP(hipStreamSynchronize(h->stream));
    h->pc_spec_a0 = a0;
    h->pc_spec_na = na;
    return QEDHMC_OK;
}

static qedhmc_status build_paper_precond(qedhmc_ctx* h) {
    qedhmc_params bp = h->p;
    bp.L = kBuildL;
    bp.Nt = kBuildNt;
    qedhmc_ctx* b = nullptr;
    QH_TRY(qedhmc_init_lattice(&bp, h->stream, &b));
    const int L0 = kBuildL, Vs = L0 * L0, n = Vs * kBuildNt;
    std::vector<double> th(2 * (size_t)n, 0.0);
    for (int tau = 0; tau < kBuildNt; tau++)
        for (int y = 0; y < L0; y++)
            for (int x = 0; x < L0; x++) th[(size_t)(kBuildNt + tau) * Vs + y * L0 + x] = M_PI * x;
    double *dth = nullptr, *dcols = nullptr, *de = nullptr;
    std::vector<cplx<double>> O((size_t)n * n);  // column-major: O[k * n + i] = O_ik
    qedhmc_status st = QEDHMC_OK;
    auto fail = [&](hipError_t e, const char* w) { st = hip_fail(e, w); };
    hipError_t e = hipMalloc(&dth, th.size() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&dcols, (size_t)n * n * sizeof(cplx<double>));
    if (e == hipSuccess) e = hipMalloc(&de, (size_t)n * sizeof(cplx<double>));
    if (e == hipSuccess) e = hipMemcpyAsync(dth, th.data(), th.size() * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) fail(e, "preconditioner build allocation");
    if (st == QEDHMC_OK) st = ensure_gauge(b, dth, QEDHMC_FP64);
    for (int k = 0; k < n && st == QEDHMC_OK; k++) {
        hipLaunchKernelGGL(k_unit, dim3(8), dim3(256), 0, h->stream, (cplx<double>*)de, (size_t)n, (size_t)k);
        st = launch_mdagm(b, QEDHMC_FP64, de, dcols + (size_t)2 * k * n, nullptr);
    }
    if (st == QEDHMC_OK) {
        e = hipMemcpyAsync(O.data(), dcols, O.size() * sizeof(cplx<double>), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) fail(e, "preconditioner build copy");
    }
    (void)hipFree(dth);
    (void)hipFree(dcols);
    (void)hipFree(de);
    qedhmc_destroy(b);
    if (st != QEDHMC_OK) return st;

    // IC(0), left-looking, dense storage of the lower factor (column-major)
    double omax = 0.0;
    for (const auto& z : O) omax = std::max(omax, std::hypot(z.re, z.im));
    const double cut = 1e-12 * omax;
    std::vector<cplx<double>> Lf((size_t)n * n, mk<double>(0.0, 0.0));
    double shift = 0.0;
    for (;;) {
        bool ok = true;
        std::fill(Lf.begin(), Lf.end(), mk<double>(0.0, 0.0));
        for (int k = 0; k < n && ok; k++) {
            // col[i] = A_ik - sum_{j<k} L_ij conj(L_kj), i >= k
            std::vector<cplx<double>> col(n - k);
            for (int i = k; i < n; i++) {
                cplx<double> a = O[(size_t)k * n + i];
                if (i == k) a.re += shift * O[(size_t)k * n + k].re;
                double sr = 0.0, si = 0.0;
                for (int j = 0; j < k; j++) {
                    const cplx<double> lij = Lf[(size_t)j * n + i], lkj = Lf[(size_t)j * n + k];
                    sr += lij.re * lkj.re + lij.im * lkj.im;
                    si += lij.im * lkj.re - lij.re * lkj.im;
                }
                col[i - k] = mk<double>(a.re - sr, a.im - si);
            }
            const double piv = col[0].re;
            if (!(piv > 0.0)) {
                ok = false;
                break;
            }
            const double d = std::sqrt(piv);
            Lf[(size_t)k * n + k] = mk<double>(d, 0.0);
            for (int i = k + 1; i < n; i++) {
                const cplx<double> a = O[(size_t)k * n + i];
                if (std::hypot(a.re, a.im) > cut) Lf[(size_t)k * n + i] = mk<double>(col[i - k].re / d, col[i - k].im / d);
            }
        }
        if (ok) break;
        shift = shift == 0.0 ? 1e-3 : 2 * shift;
        if (shift > 1.0) {
            set_error("preconditioner: IC(0) pivots stay non-positive");
            return QEDHMC_EUNSUPPORTED;
        }
    }
    // truncation of the taps: kThresh, or QEDHMC_PC_THRESH; tau reach:
    // kCapTau, or QEDHMC_PC_CAP (1 .. kCapMax) (both read when the
    // preconditioner is built; tuning knobs)
    double thresh = kThresh;
    if (const char* et = std::getenv("QEDHMC_PC_THRESH"); et && *et) thresh = std::atof(et);
    h->pc_cap = kCapTau;
    if (const char* ec = std::getenv("QEDHMC_PC_CAP"); ec && std::atoi(ec) > 0)
        h->pc_cap = std::min(kCapMax, std::atoi(ec));
    // rows of G = L^{-1}: x^T L = e_n0^T  <=>  L^T x = e_n0 (back substitution)
    const int tau0 = kBuildNt / 2 + 4, y0 = L0 / 2;
    for (int par = 0; par < 2; par++) {
        const int x0 = L0 / 2 + par, n0 = tau0 * Vs + y0 * L0 + x0;
        std::vector<cplx<double>> xr(n, mk<double>(0.0, 0.0));
        for (int i = n0; i >= 0; i--) {
            double re = (i == n0) ? 1.0 : 0.0, im = 0.0;
            for (int j = i + 1; j <= n0; j++) {
                const cplx<double> lji = Lf[(size_t)i * n + j], xj = xr[j];
                re -= lji.re * xj.re - lji.im * xj.im;
                im -= lji.re * xj.im + lji.im * xj.re;
            }
            const cplx<double> lii = Lf[(size_t)i * n + i];  // real positive
            xr[i] = mk<double>(re / lii.re, im / lii.re);
        }
        auto& taps = h->pc_taps[par];
        taps.clear();
        for (int m = 0; m <= n0; m++) {
            const double mag = std::hypot(xr[m].re, xr[m].im);
            if (!(mag >= thresh)) continue;
            const int tm = m / Vs, sm = m % Vs;
            const int dt = tau0 - tm;
            if (dt < 0 || dt > h->pc_cap) continue;
            const int dx = ((sm % L0 - x0 + L0 / 2) % L0 + L0) % L0 - L0 / 2;
            const int dy = ((sm / L0 - y0 + L0 / 2) % L0 + L0) % L0 - L0 / 2;
            taps.push_back({dt, dx, dy, xr[m].re, xr[m].im});
        }
        std::sort(taps.begin(), taps.end(), [](const HostTap& a, const HostTap& b) {
            if (a.dt != b.dt) return a.dt < b.dt;
            if (a.dy != b.dy) return a.dy < b.dy;
            return a.dx < b.dx;
        });
    }
    h->pc_shift = shift;
    // The two passes as gathers out(tau, y, x) = sum h in(tau + a, y + b, x + c)
    // over the tap list of the output's x parity (sign -1 where tau + a leaves
    // [0, Nt)): G takes (a, b, c, h) = (-dt, dy, dx, g) from its own parity's
    // taps; G^dag takes (dt, -dy, -dx, conj g) from every tap whose source
    // x - dx has the parity of the list it came from.
    std::vector<HostTap> pass[2][2];
    for (int par = 0; par < 2; par++) {
        for (const auto& t : h->pc_taps[par]) pass[0][par].push_back({-t.dt, t.dx, t.dy, t.gre, t.gim});
        for (int pp = 0; pp < 2; pp++)
            for (const auto& t : h->pc_taps[pp])
                if ((((par - t.dx) % 2) + 2) % 2 == pp) pass[1][par].push_back({t.dt, -t.dx, -t.dy, t.gre, -t.gim});
    }
    std::vector<PTap<double>> t64;
    std::vector<PTap<float>> t32;
    for (int ps = 0; ps < 2; ps++) {
        PcPass& g = h->pc_pass[ps];
        g.amin = g.bmin = g.cmin = 1 << 20;
        g.amax = g.bmax = g.cmax = -(1 << 20);
        for (int par = 0; par < 2; par++)
            for (const auto& t : pass[ps][par]) {
                g.amin = std::min(g.amin, t.dt);
                g.amax = std::max(g.amax, t.dt);
                g.bmin = std::min(g.bmin, t.dy);
                g.bmax = std::max(g.bmax, t.dy);
                g.cmin = std::min(g.cmin, t.dx);
                g.cmax = std::max(g.cmax, t.dx);
            }
        if (g.amin > g.amax) g.amin = g.amax = g.bmin = g.bmax = g.cmin = g.cmax = 0;
        const int half = (h->lat.L + g.cmax - g.cmin + 1) / 2;
        for (int par = 0; par < 2; par++) {
            auto& lst = pass[ps][par];
            std::stable_sort(lst.begin(), lst.end(), [](const HostTap& a, const HostTap& b) { return a.dt < b.dt; });
            g.first[par] = (int)t64.size();
            g.count[par] = (int)lst.size();
            // start of each tau-offset group (a = amin + k) within the list
            for (int k = 0; k <= kPcSlots; k++) {
                int n = 0;
                for (const auto& t : lst)
                    if (t.dt - g.amin < k) n++;
                g.gstart[par][k] = n;
            }
            for (const auto& t : lst) {
                const int aidx = t.dt - g.amin, q = par + t.dx - g.cmin;
                const int off = t.dy * half + (q >> 1), plane = q & 1;
                t64.push_back({aidx, off, plane, 0, mk<double>(t.gre, t.gim)});
                t32.push_back({aidx, off, plane, 0, mk<float>((float)t.gre, (float)t.gim)});
            }
        }
    }
    // the same passes grouped by spatial offset for the tau-rolling kernel
    // (a pass reaching exactly kRollNS tau offsets; otherwise rcount stays 0)
    std::vector<RTap<double>> r64;
    std::vector<RTap<float>> r32;
    for (int ps = 0; ps < 2; ps++) {
        PcPass& g = h->pc_pass[ps];
        const int half = (h->lat.L + g.cmax - g.cmin + 1) / 2;
        for (int par = 0; par < 2; par++) {
            g.rfirst[par] = (int)r64.size();
            g.rcount[par] = 0;
            if (g.amax - g.amin + 1 != kRollNS) continue;
            std::vector<std::pair<int, int>> offs;  // (dy, dx) in first-seen order of the sorted list
            for (const auto& t : pass[ps][par])
                if (std::find(offs.begin(), offs.end(), std::make_pair(t.dy, t.dx)) == offs.end())
                    offs.push_back({t.dy, t.dx});
            std::sort(offs.begin(), offs.end());
            for (const auto& od : offs) {
                const int q = par + od.second - g.cmin;
                RTap<double> a{od.first * half + (q >> 1), q & 1, 0, 0, {}};
                for (int k = 0; k < kRollNS; k++) a.g[k] = mk<double>(0.0, 0.0);
                for (const auto& t : pass[ps][par])
                    if (t.dy == od.first && t.dx == od.second) a.g[t.dt - g.amin] = mk<double>(t.gre, t.gim);
                RTap<float> b{a.off, a.plane, 0, 0, {}};
                for (int k = 0; k < kRollNS; k++) b.g[k] = mk<float>((float)a.g[k].re, (float)a.g[k].im);
                r64.push_back(a);
                r32.push_back(b);
            }
            g.rcount[par] = (int)offs.size();
        }
    }
    const size_t nr = r64.size();
    QH_HIP(hipMalloc(&h->pc_roll64, std::max<size_t>(nr, 1) * sizeof(RTap<double>)));
    QH_HIP(hipMalloc(&h->pc_roll32, std::max<size_t>(nr, 1) * sizeof(RTap<float>)));
    if (nr) {
        QH_HIP(hipMemcpyAsync(h->pc_roll64, r64.data(), nr * sizeof(RTap<double>), hipMemcpyHostToDevice, h->stream));
        QH_HIP(hipMemcpyAsync(h->pc_roll32, r32.data(), nr * sizeof(RTap<float>), hipMemcpyHostToDevice, h->stream));
    }
    const size_t nt = t64.size();
    QH_HIP(hipMalloc(&h->pc_dev64, std::max<size_t>(nt, 1) * sizeof(PTap<double>)));
    QH_HIP(hipMalloc(&h->pc_dev32, std::max<size_t>(nt, 1) * sizeof(PTap<float>)));
    if (nt) {
        QH_HIP(hipMemcpyAsync(h->pc_dev64, t64.data(), nt * sizeof(PTap<double>), hipMemcpyHostToDevice, h->stream));
        QH_HIP(hipMemcpyAsync(h->pc_dev32, t32.data(), nt * sizeof(PTap<float>), hipMemcpyHostToDevice, h->stream));
    }
    QH_TRY(build_spectral(h, pass));
    QH_HIP(hipStreamSynchronize(h->stream));
    h->pc_ready = true;
    return QEDHMC_OK;
}

qedhmc_status ensure_paper_precond(qedhmc_ctx* h) {
    if (h->pc_ready) return QEDHMC_OK;
    return build_paper_precond(h);
}

// ---------------------------------------------------------------------------
// Stencil application, streamed along tau.  A workgroup owns one x parity of
// a band of TY rows (all x) and a run of Tc slices.  Its LDS holds a ring of
// nslot = amax - amin + 1 input slices over the band plus the rows and columns
// the taps reach (periodic in y and x, sign-flipped where the slice index
// leaves [0, Nt)), each slice stored as two planes of even and odd window
// columns, and a copy of the parity's taps.  Each step reads one new slice
// into the ring (prefetched into registers during the previous step); each
// output site is formed by a quad of lanes that split its taps (tap j to lane
// j mod 4 within each tau-offset group: an LDS read of the tap, an LDS read of
// the input at a fixed offset and four FMAs) and add their partial sums by
// DPP.  Four lanes per site give the workgroup four times the wavefronts to
// hide LDS latency with.
// stop (nullable): a scalar slot's stop flag; non-zero makes the launch a no-op.
// ---------------------------------------------------------------------------
struct PcGeo {
    int L, Nt, Vs;
    int TY, nband, Tc, nrun;
    int rows, cols, half, bmin, cmin, amin, nslot;
    int first[2], count[2];
    int gstart[2][kPcSlots + 1];  // per parity: start of each tau-offset group in the parity's list
};

// window elements per thread at most (the plan keeps rows x cols within
// kPcElems x threads)
static constexpr int kPcElems = 4;

template <typename R>
struct STap {
    R re, im;
    int toff;  // plane * plane size + off
    int pad;
};

__device__ __forceinline__ float dpp_f32_quad(float v, int sel) {
    const int i = __float_as_int(v);
    const int r = sel == 0 ? __builtin_amdgcn_update_dpp(0, i, 0xB1, 0xF, 0xF, false)
                           : __builtin_amdgcn_update_dpp(0, i, 0x4E, 0xF, 0xF, false);
    return __int_as_float(r);
}

template <typename R>
__device__ __forceinline__ R quad_sum(R v) {
    if constexpr (sizeof(R) == 8) {
        v += dpp_f64<0xB1, 0xF>(v);  // quad_perm [1,0,3,2]
        v += dpp_f64<0x4E, 0xF>(v);  // quad_perm [2,3,0,1]
    } else {
        v += dpp_f32_quad(v, 0);
        v += dpp_f32_quad(v, 1);
    }
    return v;
}

template <typename R>
__global__ __launch_bounds__(1024, 2) void k_pc_stream(PcGeo g, const PTap<R>* __restrict__ taps,
                                                       const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                                       const double* __restrict__ stop) {
    if (stop && *stop != 0.0) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<R>* win = reinterpret_cast<cplx<R>*>(smem);
    const int plane = g.rows * g.half;  // one column-parity plane of a slice
    const int slice_elems = 2 * plane;
    STap<R>* st = reinterpret_cast<STap<R>*>(win + (size_t)g.nslot * slice_elems);
    const int nwork = g.nband * g.nrun * 2;
    const int per = (nwork + 7) >> 3;
    const int w = (blockIdx.x & 7) * per + (blockIdx.x >> 3);  // runs of one XCD are contiguous
    if (w >= nwork) return;
    const int par = w & 1, band = (w >> 1) % g.nband, run = (w >> 1) / g.nband;
    const int y0 = band * g.TY;
    const int tau0 = run * g.Tc, tau1 = min(g.Nt, tau0 + g.Tc);
    const int hx = g.L / 2;
    const int q = threadIdx.x & 3, o = threadIdx.x >> 2;
    const int iy = o / hx, jx = o - iy * hx;
    const bool act = iy < g.TY && y0 + iy < g.L;
    const int base = act ? (iy - g.bmin) * g.half + jx : -g.bmin * g.half;  // idle lanes read the first site's window
    const int ntap = g.count[par];
    {
        const PTap<R>* tp = taps + g.first[par];
        for (int j = threadIdx.x; j < ntap; j += blockDim.x) {
            const PTap<R> t = tp[j];
            st[j] = STap<R>{t.g.re, t.g.im, t.plane * plane + t.off, 0};
        }
    }
    // this thread's window elements (the same for every slice): source site
    // inside a slice and LDS position inside a slot (-1: none)
    int soff[kPcElems], doff[kPcElems];
    {
        const int total = g.rows * g.cols;
#pragma unroll
        for (int k = 0; k < kPcElems; k++) {
            const int e = (int)threadIdx.x + k * (int)blockDim.x;
            doff[k] = -1;
            soff[k] = 0;
            if (e < total) {
                const int r = e / g.cols, c = e - r * g.cols;
                const int yy = (y0 + g.bmin + r + 8 * g.L) % g.L, xx = (g.cmin + c + 8 * g.L) % g.L;
                soff[k] = yy * g.L + xx;
                doff[k] = (c & 1) * plane + r * g.half + (c >> 1);
            }
        }
    }
    auto fetch = [&](int s, cplx<R> (&v)[kPcElems]) {
        const cplx<R>* src = in + (size_t)(((s % g.Nt) + g.Nt) % g.Nt) * g.Vs;
#pragma unroll
        for (int k = 0; k < kPcElems; k++) v[k] = src[soff[k]];  // unused entries read site 0
    };
    auto store = [&](int s, const cplx<R> (&v)[kPcElems]) {
        const R sg = (s < 0 || s >= g.Nt) ? R(-1) : R(1);
        cplx<R>* dst = win + (size_t)(((s % g.nslot) + g.nslot) % g.nslot) * slice_elems;
#pragma unroll
        for (int k = 0; k < kPcElems; k++)
            if (doff[k] >= 0) dst[doff[k]] = mk<R>(sg * v[k].re, sg * v[k].im);
    };
    cplx<R> nxt[kPcElems];
    for (int s = tau0 + g.amin; s < tau0 + g.amin + g.nslot - 1; s++) {
        fetch(s, nxt);
        store(s, nxt);
    }
    fetch(tau0 + g.amin + g.nslot - 1, nxt);
    const int* gs = g.gstart[par];
    for (int tau = tau0; tau < tau1; tau++) {
        store(tau + g.amin + g.nslot - 1, nxt);
        __syncthreads();
        if (tau + 1 < tau1) fetch(tau + g.amin + g.nslot, nxt);  // in flight during the taps
        const int r0 = (((tau + g.amin) % g.nslot) + g.nslot) % g.nslot;
        R ar = 0, ai = 0;
        for (int gg = 0; gg < g.nslot; gg++) {
            int sl = r0 + gg;
            sl = sl >= g.nslot ? sl - g.nslot : sl;
            const cplx<R>* ws = win + (size_t)sl * slice_elems + base;
            const int j1 = gs[gg + 1];
#pragma unroll 4
            for (int j = gs[gg] + q; j < j1; j += 4) {
                const STap<R> t = st[j];
                const cplx<R> v = ws[t.toff];
                // four FMAs into the running sums (a product formed first and
                // then added would cost two more instructions per tap)
                ar = fma(t.re, v.re, ar);
                ar = fma(-t.im, v.im, ar);
                ai = fma(t.re, v.im, ai);
                ai = fma(t.im, v.re, ai);
            }
        }
        ar = quad_sum(ar);
        ai = quad_sum(ai);
        if (act && q == 3) out[(size_t)tau * g.Vs + (y0 + iy) * g.L + 2 * jx + par] = mk<R>(ar, ai);
        __syncthreads();  // the next step overwrites the oldest slot
    }
}

// ---------------------------------------------------------------------------
// The same stencil pass rolled along tau.  The taps of a spatial offset
// (b, c) at the kRollNS tau offsets a = amin .. amax act on one input value
// in(s, y + b, x + c); a lane reads that value once per input slice s and
// adds its kRollNS products into the running sums of the outputs s - a, held
// in registers (output tau is complete once slice tau + amax has been read).
// A workgroup owns one x parity of a band of TY rows and a run of Tc output
// slices, reads Tc + kRollNS - 1 input slices one at a time into a double
// buffer in LDS (window of the band plus the rows and columns the taps reach,
// even and odd columns as two planes, sign-flipped where the slice index
// leaves [0, Nt)), and gives each output site Q lanes in Q different
// wavefronts, each taking every Q-th spatial offset: the offset index is
// uniform across a wavefront, so the taps come through scalar loads.  The
// Q partial sums of a completed output meet in LDS.  One barrier per slice.
// ---------------------------------------------------------------------------
struct PcRollGeo {
    int L, Nt, Vs;
    int TY, nband, Tc, nrun;
    int rows, cols, half, bmin, cmin, amin;
    int S, Q;  // lanes per copy of the band's sites (a multiple of 64) and copies
    int first[2], count[2];
};

static constexpr int kRollElems = 4;  // window elements per thread at most
// per application of G^dag G, FP32: L = 24 per-tap 53 us / rolled 63 us;
// L = 48 242 / 200 us; L = 66 603 / 450 us
static constexpr int kRollFromL = 40;

template <typename R>
__global__ __launch_bounds__(1024) void k_pc_roll(PcRollGeo g, const RTap<R>* __restrict__ taps,
                                                  const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                                  const double* __restrict__ stop) {
    if (stop && *stop != 0.0) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int plane = g.rows * g.half, slice_elems = 2 * plane;
    cplx<R>* win = reinterpret_cast<cplx<R>*>(smem);  // [2][slice_elems]
    cplx<R>* red = win + 2 * slice_elems;             // [2][Q][S] partial sums of completed outputs
    const int nwork = g.nband * g.nrun * 2;
    const int per = (nwork + 7) >> 3;
    const int w = (blockIdx.x & 7) * per + (blockIdx.x >> 3);  // runs of one XCD are contiguous
    if (w >= nwork) return;
    const int par = w & 1, band = (w >> 1) % g.nband, run = (w >> 1) / g.nband;
    const int y0 = band * g.TY;
    const int tau0 = run * g.Tc, tau1 = min(g.Nt, tau0 + g.Tc);
    const int hx = g.L / 2;
    const int o = (int)threadIdx.x % g.S;
    const int q = __builtin_amdgcn_readfirstlane((int)threadIdx.x / g.S);
    const int iy = o / hx, jx = o - iy * hx;
    const bool act = iy < g.TY && y0 + iy < g.L;
    const int base = act ? (iy - g.bmin) * g.half + jx : 0;  // idle lanes read a valid element
    int soff[kRollElems], doff[kRollElems];
    {
        const int total = g.rows * g.cols;
#pragma unroll
        for (int k = 0; k < kRollElems; k++) {
            const int e = (int)threadIdx.x + k * (int)blockDim.x;
            doff[k] = -1;
            soff[k] = 0;
            if (e < total) {
                const int r = e / g.cols, c = e - r * g.cols;
                const int yy = (y0 + g.bmin + r + 8 * g.L) % g.L, xx = (g.cmin + c + 8 * g.L) % g.L;
                soff[k] = yy * g.L + xx;
                doff[k] = (c & 1) * plane + r * g.half + (c >> 1);
            }
        }
    }
    auto fetch = [&](int s, cplx<R> (&v)[kRollElems]) {
        const cplx<R>* src = in + (size_t)(((s % g.Nt) + g.Nt) % g.Nt) * g.Vs;
#pragma unroll
        for (int k = 0; k < kRollElems; k++) v[k] = src[soff[k]];  // unused entries read site 0
    };
    auto store = [&](int buf, int s, const cplx<R> (&v)[kRollElems]) {
        const R sg = (s < 0 || s >= g.Nt) ? R(-1) : R(1);
        cplx<R>* dst = win + (size_t)buf * slice_elems;
#pragma unroll
        for (int k = 0; k < kRollElems; k++)
            if (doff[k] >= 0) dst[doff[k]] = mk<R>(sg * v[k].re, sg * v[k].im);
    };
    const RTap<R>* tp = taps + g.first[par];
    const int ntap = g.count[par];
    const int nsteps = (tau1 - tau0) + kRollNS - 1;
    const int s0 = tau0 + g.amin;
    cplx<R> acc[kRollNS];
#pragma unroll
    for (int k = 0; k < kRollNS; k++) acc[k] = mk<R>(R(0), R(0));
    cplx<R> nxt[kRollElems];
    fetch(s0, nxt);
    store(0, s0, nxt);
    __syncthreads();
    for (int j0 = 0; j0 < nsteps; j0 += kRollNS) {
#pragma unroll
        for (int u = 0; u < kRollNS; u++) {
            const int j = j0 + u;
            if (j >= nsteps) break;
            if (j + 1 < nsteps) fetch(s0 + j + 1, nxt);  // in flight during the taps
            const cplx<R>* ws = win + (size_t)(j & 1) * slice_elems + base;
            // wavefronts past the Q copies only help load the window
            for (int k = q; k < (q < g.Q ? ntap : 0); k += g.Q) {
                const RTap<R> t = tp[k];
                const cplx<R> v = ws[t.plane * plane + t.off];
                // input slice s0 + j feeds output tau0 + j - kk through the
                // tap of tau offset amin + kk (products for outputs outside
                // the run land in slots that are cleared unwritten: skipping
                // them measured slower)
#pragma unroll
                for (int kk = 0; kk < kRollNS; kk++) {
                    cplx<R>& A = acc[(u - kk + kRollNS) % kRollNS];
                    A.re = fma(t.g[kk].re, v.re, A.re);
                    A.re = fma(-t.g[kk].im, v.im, A.re);
                    A.im = fma(t.g[kk].re, v.im, A.im);
                    A.im = fma(t.g[kk].im, v.re, A.im);
                }
            }
            // output tau0 + j - (kRollNS - 1) is complete in slot (u + 1) mod kRollNS
            const int cs = (u + 1) % kRollNS;
            cplx<R>* rb = red + (size_t)(j & 1) * g.Q * g.S;
            if (g.Q > 1 && q < g.Q) rb[q * g.S + o] = acc[cs];
            if (j + 1 < nsteps) store((j + 1) & 1, s0 + j + 1, nxt);
            __syncthreads();
            const int tau = tau0 + j - (kRollNS - 1);
            if (q == 0 && act && tau >= tau0) {
                cplx<R> sum = acc[cs];
                if (g.Q > 1) {
                    sum = rb[o];
                    for (int k = 1; k < g.Q; k++) {
                        sum.re += rb[k * g.S + o].re;
                        sum.im += rb[k * g.S + o].im;
                    }
                }
                out[(size_t)tau * g.Vs + (y0 + iy) * g.L + 2 * jx + par] = sum;
            }
            acc[cs] = mk<R>(R(0), R(0));
        }
    }
}

template <typename R>
static const RTap<R>* rtaps_for(qedhmc_ctx* h) {
    if constexpr (sizeof(R) == 8)
        return (const RTap<double>*)h->pc_roll64;
    else
        return (const RTap<float>*)h->pc_roll32;
}

// Plan: a band of TY rows whose TY * L/2 output sites fill whole wavefronts
// best (at most 256 lanes per copy), Q = 2 copies for 256-lane bands and 4
// below, runs of 12 slices (each run reads kRollNS - 1 slices more than it
// writes).  QEDHMC_PC_TY, QEDHMC_PC_TC and QEDHMC_PC_Q (read per call)
// override the plan.
template <typename R>
static qedhmc_status launch_pc_roll(qedhmc_ctx* h, int ps, const cplx<R>* in, cplx<R>* out, const double* stop) {
    const PcPass& pp = h->pc_pass[ps];
    const Lat& lt = h->lat;
    PcRollGeo g{};
    g.L = lt.L;
    g.Nt = lt.Nt;
    g.Vs = lt.Vs;
    g.bmin = pp.bmin;
    g.cmin = pp.cmin;
    g.amin = pp.amin;
    g.cols = lt.L + pp.cmax - pp.cmin;
    g.half = (g.cols + 1) / 2;
    for (int par = 0; par < 2; par++) {
        g.first[par] = pp.rfirst[par];
        g.count[par] = pp.rcount[par];
    }
    const int hx = lt.L / 2;
    auto pad64 = [](int n) { return ((n + 63) / 64) * 64; };
    int TY = 1;
    double best = -1.0;
    for (int ty = 1; ty <= lt.L && pad64(ty * hx) <= 256; ty++) {
        const double eff = (double)(ty * hx) / pad64(ty * hx);
        if (eff >= best - 1e-9) {
            best = eff;
            TY = ty;
        }
    }
    const char* ety = std::getenv("QEDHMC_PC_TY");
    const char* etc = std::getenv("QEDHMC_PC_TC");
    const char* eq = std::getenv("QEDHMC_PC_Q");
    if (ety && std::atoi(ety) > 0) TY = std::min(lt.L, std::atoi(ety));
    g.nband = (lt.L + TY - 1) / TY;
    g.TY = (lt.L + g.nband - 1) / g.nband;
    g.rows = g.TY + pp.bmax - pp.bmin;
    g.S = pad64(g.TY * hx);
    g.Q = g.S >= 256 ? 2 : 4;  // measured best at L = 48 (4) and 66 (2)
    if (eq && std::atoi(eq) > 0) g.Q = std::atoi(eq);
    while (g.Q > 1 && g.Q * g.S > 1024) g.Q--;
    if (g.S > 1024) {
        set_error("paper preconditioner: a band row exceeds one workgroup at this L");
        return QEDHMC_EUNSUPPORTED;
    }
    // every window element of a slice has a thread (kRollElems each at most):
    // whole wavefronts past the Q copies only load
    const int need = ((g.rows * g.cols + kRollElems - 1) / kRollElems + 63) / 64 * 64;
    const int threads = std::max(g.Q * g.S, need);
    if (threads > 1024) {
        set_error("paper preconditioner: the stencil window exceeds the rolling kernel's workgroup");
        return QEDHMC_EUNSUPPORTED;
    }
    g.Tc = 12;  // a sweep of 6, 12, 24 at L = 48 and 66 put 12 first or within 1 %
    if (etc && std::atoi(etc) > 0) g.Tc = std::atoi(etc);
    g.Tc = std::min(g.Tc, lt.Nt);
    g.nrun = (lt.Nt + g.Tc - 1) / g.Tc;
    const size_t lds = (size_t)2 * 2 * g.rows * g.half * sizeof(cplx<R>) +
                       (g.Q > 1 ? (size_t)2 * g.Q * g.S * sizeof(cplx<R>) : 0);
    if (lds > h->max_lds) {
        set_error("paper preconditioner: the rolling kernel's window exceeds the LDS");
        return QEDHMC_EUNSUPPORTED;
    }
    if (lds > 65536) QH_TRY(allow_lds((const void*)k_pc_roll<R>, h->max_lds));
    const int nwork = g.nband * g.nrun * 2;
    hipLaunchKernelGGL(k_pc_roll<R>, dim3(8 * ((nwork + 7) / 8)), dim3(threads), lds, h->stream, g, rtaps_for<R>(h),
                       in, out, stop);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

template <typename R>
static const PTap<R>* taps_for(qedhmc_ctx* h) {
    if constexpr (sizeof(R) == 8)
        return (const PTap<double>*)h->pc_dev64;
    else
        return (const PTap<float>*)h->pc_dev32;
}

// Band height TY: four lanes per output site, about 448 lanes, and an LDS
// window within 64 KB (FP32) or 128 KB (FP64); runs of 2 .. 16 slices aiming
// at about 4096 workgroups.
template <typename R>
static qedhmc_status launch_pc(qedhmc_ctx* h, int ps, const cplx<R>* in, cplx<R>* out, const double* stop) {
    const PcPass& pp = h->pc_pass[ps];
    // the tau-rolling kernel from L = kRollFromL on (below it the per-tap
    // kernel measured as fast or faster: too few rolled work items to fill
    // the device); QEDHMC_PC_KERNEL=roll|stream (read per call) forces one
    const char* ek = std::getenv("QEDHMC_PC_KERNEL");
    const bool forced = ek && (std::strcmp(ek, "roll") == 0 || std::strcmp(ek, "stream") == 0);
    const bool roll = forced ? std::strcmp(ek, "roll") == 0 : h->lat.L >= kRollFromL;
    if (pp.rcount[0] > 0 && pp.rcount[1] > 0 && roll) return launch_pc_roll<R>(h, ps, in, out, stop);
    const Lat& lt = h->lat;
    PcGeo g{};
    g.L = lt.L;
    g.Nt = lt.Nt;
    g.Vs = lt.Vs;
    g.bmin = pp.bmin;
    g.cmin = pp.cmin;
    g.amin = pp.amin;
    g.nslot = pp.amax - pp.amin + 1;
    if (g.nslot > kPcSlots) {
        set_error("paper preconditioner: stencil reaches too many slices");
        return QEDHMC_EUNSUPPORTED;
    }
    g.cols = lt.L + pp.cmax - pp.cmin;
    g.half = (g.cols + 1) / 2;
    for (int par = 0; par < 2; par++) {
        g.first[par] = pp.first[par];
        g.count[par] = pp.count[par];
        for (int k = 0; k <= kPcSlots; k++) g.gstart[par][k] = pp.gstart[par][std::min(k, g.nslot)];
    }
    const int hx = lt.L / 2;
    const int maxtap = std::max(pp.count[0], pp.count[1]);
    const size_t tap_bytes = (size_t)maxtap * sizeof(STap<R>);
    const size_t budget = std::min<size_t>(sizeof(R) == 8 ? 131072 : 65536, h->max_lds);
    auto lds_of = [&](int ty) {
        return (size_t)g.nslot * (ty + pp.bmax - pp.bmin) * 2 * g.half * sizeof(cplx<R>) + tap_bytes;
    };
    // tuning overrides, read per call: QEDHMC_PC_TY (rows per band, at most
    // the plan's) and QEDHMC_PC_TC (slices per run); 0 or unset: automatic
    const char* ety = std::getenv("QEDHMC_PC_TY");
    const char* etc = std::getenv("QEDHMC_PC_TC");
    // about 448 lanes per workgroup: several small workgroups per compute
    // unit beat one large one (less barrier coupling; measured at L = 24,
    // 48, 66)
    int TY = std::max(1, std::min(lt.L, 448 / (4 * hx)));
    while (TY > 1 && lds_of(TY) > budget) TY--;
    if (ety && std::atoi(ety) > 0) TY = std::min(TY, std::atoi(ety));
    if (4 * hx > 1024 || lds_of(TY) > h->max_lds) {
        set_error("paper preconditioner: the stencil window exceeds one workgroup at this L");
        return QEDHMC_EUNSUPPORTED;
    }
    g.nband = (lt.L + TY - 1) / TY;
    g.TY = (lt.L + g.nband - 1) / g.nband;
    g.rows = g.TY + pp.bmax - pp.bmin;
    g.Tc = std::max(2, std::min(16, lt.Nt * g.nband * 2 / 4096));
    if (etc && std::atoi(etc) > 0) g.Tc = std::atoi(etc);
    g.Tc = std::min(g.Tc, lt.Nt);
    g.nrun = (lt.Nt + g.Tc - 1) / g.Tc;
    const size_t lds = lds_of(g.TY);
    int threads = ((4 * g.TY * hx + 63) / 64) * 64;
    // every window element of a slice has a thread (kPcElems each at most)
    const int need = (g.rows * g.cols + kPcElems - 1) / kPcElems;
    threads = std::max(threads, ((need + 63) / 64) * 64);
    if (threads > 1024) {
        set_error("paper preconditioner: stencil window too large for one workgroup at this L");
        return QEDHMC_EUNSUPPORTED;
    }
    const int nwork = g.nband * g.nrun * 2;
    if (lds > 65536) QH_TRY(allow_lds((const void*)k_pc_stream<R>, h->max_lds));
    hipLaunchKernelGGL(k_pc_stream<R>, dim3(8 * ((nwork + 7) / 8)), dim3(threads), lds, h->stream, g, taps_for<R>(h),
                       in, out, stop);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// ---------------------------------------------------------------------------
// Spectral application (the tables of build_spectral).  Momentum-space
// vectors use the memory of a site vector: slice tau holds the even plane
// [ny][nx] and then the odd one.
// ---------------------------------------------------------------------------
// acc += m v (complex), four FMAs
template <typename R>
__device__ __forceinline__ void v_cmac(cplx<R>& acc, cplx<R> m, cplx<R> v) {
    acc.re = fma(m.re, v.re, acc.re);
    acc.re = fma(-m.im, v.im, acc.re);
    acc.im = fma(m.re, v.im, acc.im);
    acc.im = fma(m.im, v.re, acc.im);
}

struct PcSpecGeo {
    int L, Lh, Nt, Vs, nk, a0, na;
};

// (slice, parity) of a workgroup of the per-plane spectral kernels: both
// planes of a slice on the XCD that slice_of_block gives the slice (so
// momentum planes written and read by consecutive launches stay in that
// XCD's L2); spec_grid(Nt) workgroups, the surplus ones get -1
__host__ __device__ __forceinline__ int spec_grid(int Nt) { return 16 * ((Nt + 7) / 8); }
__device__ __forceinline__ int spec_slice_of_block(int b, int Nt, int& p) {
    const int per = (Nt + 7) >> 3, j = b >> 3;
    const int tau = (b & 7) * per + (j >> 1);
    p = j & 1;
    return tau < Nt ? tau : -1;
}

// Workgroup size cap of the spectral kernels: FP64 takes at most 512
// threads (at 1024 its registers spill)
template <typename R>
constexpr int spec_max_threads() {
    return sizeof(R) == 8 ? 512 : 1024;
}

// 2D DFT of nplanes parity planes held in LDS (buf[plane][row][column],
// Lh columns), by the whole workgroup: a direct DFT over the column index
// (L/2 points) for every row, written back to buf, then one over the row
// index (L points) for every column, whose results go to
// emit(plane, kr * Lh + col, value).  Twiddles twx[Lh], twy[L] hold
// e^{-2 pi i j / n} (forward) or their conjugates (inverse).  Outputs per
// thread: at most kSpecE (nplanes * L * L/2 <= kSpecE * blockDim.x).
template <typename R, typename Emit>
__device__ __forceinline__ void dft_planes(cplx<R>* buf, const cplx<R>* twx, const cplx<R>* twy, int L, int Lh,
                                           int nplanes, Emit emit) {
    const int n = L * Lh, tot = nplanes * n;
    cplx<R> acc[kSpecE];
#pragma unroll
    for (int j = 0; j < kSpecE; j++) {
        const int ea = (int)threadIdx.x + j * (int)blockDim.x;
        if (ea < tot) {
            const int pl = ea / n, e = ea - pl * n;
            const int row = e / Lh, kc = e - row * Lh;
            const cplx<R>* src = buf + pl * n + row * Lh;
            R ar = 0, ai = 0;
            int idx = 0;
            for (int m = 0; m < Lh; m++) {
                const cplx<R> v = src[m], t = twx[idx];
                ar = fma(v.re, t.re, ar);
                ar = fma(-v.im, t.im, ar);
                ai = fma(v.re, t.im, ai);
                ai = fma(v.im, t.re, ai);
                idx += kc;
                idx = idx >= Lh ? idx - Lh : idx;
            }
            acc[j] = mk<R>(ar, ai);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSpecE; j++) {
        const int ea = (int)threadIdx.x + j * (int)blockDim.x;
        if (ea < tot) buf[ea] = acc[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSpecE; j++) {
        const int ea = (int)threadIdx.x + j * (int)blockDim.x;
        if (ea < tot) {
            const int pl = ea / n, e = ea - pl * n;
            const int kr = e / Lh, col = e - kr * Lh;
            const cplx<R>* src = buf + pl * n + col;
            R ar = 0, ai = 0;
            int idx = 0;
            for (int r = 0; r < L; r++) {
                const cplx<R> v = src[r * Lh], t = twy[idx];
                ar = fma(v.re, t.re, ar);
                ar = fma(-v.im, t.im, ar);
                ai = fma(v.re, t.im, ai);
                ai = fma(v.im, t.re, ai);
                idx += kr;
                idx = idx >= L ? idx - L : idx;
            }
            emit(pl, e, mk<R>(ar, ai));
        }
    }
}

// twiddles of both axes into LDS (twx then twy, contiguous), conjugated for
// the inverse
template <typename R, bool INV>
__device__ __forceinline__ void load_twiddles(const cplx<R>* __restrict__ tw, cplx<R>* twx, int n) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const cplx<R> t = tw[j];
        twx[j] = INV ? mk<R>(t.re, -t.im) : t;
    }
}

// Site vector <-> momentum planes, a workgroup per (slice, parity).
// Forward: in a site vector, out momentum planes (e^{-i k.r}); INV: the
// reverse with e^{+i k.r} (the normalisation sits in H).
template <typename R, bool INV>
__global__ __launch_bounds__(spec_max_threads<R>()) void k_pcs_dft(PcSpecGeo g, const cplx<R>* __restrict__ tw,
                                                  const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                                  const double* __restrict__ stop) {
    if (stop && *stop != 0.0) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = g.L, Lh = g.Lh, n = g.nk;
    cplx<R>* buf = reinterpret_cast<cplx<R>*>(smem);  // [row][column]
    cplx<R>* twx = buf + n;                           // [Lh], then twy [L]
    int p;
    const int tau = spec_slice_of_block(blockIdx.x, g.Nt, p);
    if (tau < 0) return;
    const size_t sbase = (size_t)tau * g.Vs;
    load_twiddles<R, INV>(tw, twx, Lh + L);
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int row = e / Lh, col = e - row * Lh;
        buf[e] = INV ? in[sbase + (size_t)p * n + e] : in[sbase + (size_t)row * L + 2 * col + p];
    }
    __syncthreads();
    dft_planes<R>(buf, twx, twx + Lh, L, Lh, 1, [&](int, int e, cplx<R> v) {
        if (INV) {
            const int y = e / Lh, m = e - y * Lh;
            out[sbase + (size_t)y * L + 2 * m + p] = v;
        } else {
            out[sbase + (size_t)p * n + e] = v;
        }
    });
}

// input slice s of the banded tau sum: its index in [0, N_tau) and the sign
// (-1 per wrap of the antiperiodic direction)
__device__ __forceinline__ int wrap_slice(int s, int Nt, int& flip) {
    const int q = s >= 0 ? s / Nt : -((-s + Nt - 1) / Nt);  // floor(s / Nt)
    flip = q & 1;
    return s - q * Nt;
}

// z^(k, tau) = sum_a sign H(k, a) v^(k, tau + a) on momentum planes: a thread
// per (momentum, run of TC slices) holds the TC + na - 1 input slices it
// needs in registers.  H is [a][entry][k] (coalesced across k).
template <typename R, int TC>
__global__ __launch_bounds__(256) void k_pcs_tconv(PcSpecGeo g, const cplx<R>* __restrict__ H,
                                                   const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                                   const double* __restrict__ stop) {
    if (stop && *stop != 0.0) return;
    const int nk = g.nk;
    const int nrun = (g.Nt + TC - 1) / TC;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nk * nrun) return;
    const int k = gid % nk, tau0 = (gid / nk) * TC;
    constexpr int NW = TC + kSpecNA - 1;
    // window slices past the last one needed read slice 0 with sign 0: no
    // branches, every load in flight together
    cplx<R> v0[NW], v1[NW];
    R sgw[NW];
#pragma unroll
    for (int j = 0; j < NW; j++) {
        int flip = 0;
        const bool on = j < TC + g.na - 1;
        const int sr = on ? wrap_slice(tau0 + g.a0 + j, g.Nt, flip) : 0;
        sgw[j] = on ? (flip ? R(-1) : R(1)) : R(0);
        const cplx<R>* src = in + (size_t)sr * g.Vs + k;
        v0[j] = src[0];
        v1[j] = src[nk];
    }
#pragma unroll
    for (int j = 0; j < NW; j++) {
        v0[j] = mk<R>(sgw[j] * v0[j].re, sgw[j] * v0[j].im);
        v1[j] = mk<R>(sgw[j] * v1[j].re, sgw[j] * v1[j].im);
    }
    cplx<R> z0[TC], z1[TC];
#pragma unroll
    for (int t = 0; t < TC; t++) z0[t] = z1[t] = mk<R>(R(0), R(0));
    // (guards rather than an early exit keep every window index a constant,
    // so the window stays in registers)
#pragma unroll
    for (int ia = 0; ia < kSpecNA; ia++) {
        if (ia < g.na) {
            const cplx<R>* hp = H + (size_t)ia * 4 * nk + k;
            const cplx<R> h00 = hp[0], h01 = hp[nk], h10 = hp[2 * nk], h11 = hp[3 * nk];
#pragma unroll
            for (int t = 0; t < TC; t++) {
                v_cmac(z0[t], h00, v0[t + ia]);
                v_cmac(z0[t], h01, v1[t + ia]);
                v_cmac(z1[t], h10, v0[t + ia]);
                v_cmac(z1[t], h11, v1[t + ia]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < TC; t++)
        if (tau0 + t < g.Nt) {
            cplx<R>* dst = out + (size_t)(tau0 + t) * g.Vs + k;
            dst[0] = z0[t];
            dst[nk] = z1[t];
        }
}

// The tau sum and the inverse DFT in one launch, a workgroup per (slice,
// parity): the plane z^_p(tau) is formed in LDS from the na input slices
// (read through the L2; used where a slice is small), then transformed back.
template <typename R>
__global__ __launch_bounds__(spec_max_threads<R>()) void k_pcs_tconv_idft(PcSpecGeo g, const cplx<R>* __restrict__ H,
                                                         const cplx<R>* __restrict__ tw,
                                                         const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                                         const double* __restrict__ stop) {
    if (stop && *stop != 0.0) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = g.L, Lh = g.Lh, n = g.nk;
    cplx<R>* buf = reinterpret_cast<cplx<R>*>(smem);
    cplx<R>* twx = buf + n;
    int p;
    const int tau = spec_slice_of_block(blockIdx.x, g.Nt, p);
    if (tau < 0) return;
    const int ntw = Lh + L;  // <= blockDim.x (spec_fits)
    const cplx<R> twv = (int)threadIdx.x < ntw ? tw[threadIdx.x] : mk<R>(R(0), R(0));
    // the tau offsets in chunks of kSpecChunk: per chunk, the slice offset,
    // H offset and sign of every offset (offsets past na read valid entries
    // with sign 0, so every load is unconditional and a chunk's loads are in
    // flight together)
    constexpr int CH = kSpecChunk;
    const int e0 = threadIdx.x;
    if (e0 < ntw) {
        twx[e0] = mk<R>(twv.re, -twv.im);  // inverse twiddles
    }
    for (int e = e0; e < n; e += blockDim.x) {
        cplx<R> z = mk<R>(R(0), R(0));
        for (int c0 = 0; c0 < g.na; c0 += CH) {
            cplx<R> h0[CH], h1[CH], v0[CH], v1[CH];
            R sgn[CH];
#pragma unroll
            for (int i = 0; i < CH; i++) {
                const int ia = c0 + i;
                int flip = 0;
                const bool on = ia < g.na;
                const size_t so = on ? (size_t)wrap_slice(tau + g.a0 + ia, g.Nt, flip) * g.Vs : 0;
                const size_t ho = ((size_t)(on ? ia : 0) * 4 + 2 * p) * n;
                sgn[i] = on ? (flip ? R(-1) : R(1)) : R(0);
                h0[i] = H[ho + e];
                h1[i] = H[ho + n + e];
                v0[i] = in[so + e];
                v1[i] = in[so + n + e];
            }
#pragma unroll
            for (int i = 0; i < CH; i++) {
                cplx<R> t = mk<R>(R(0), R(0));
                v_cmac(t, h0[i], v0[i]);
                v_cmac(t, h1[i], v1[i]);
                z.re = fma(sgn[i], t.re, z.re);
                z.im = fma(sgn[i], t.im, z.im);
            }
        }
        buf[e] = z;
    }
    __syncthreads();
    const size_t sbase = (size_t)tau * g.Vs;
    dft_planes<R>(buf, twx, twx + Lh, L, Lh, 1, [&](int, int e, cplx<R> v) {
        const int y = e / Lh, m = e - y * Lh;
        out[sbase + (size_t)y * L + 2 * m + p] = v;
    });
}

// whether apply_P_t takes the spectral form: built (L even, N_tau above the
// tau reach of a pass, L * L/2 <= 8192), a plane fits one workgroup of the
// precision, and not overridden by QEDHMC_PC_KERNEL=roll|stream (read per
// call)
template <typename R>
static bool spec_fits(const qedhmc_ctx* h, int nplanes, int& threads, size_t& lds);

template <typename R>
static bool use_spectral(const qedhmc_ctx* h) {
    if (h->pc_spec_na <= 0) return false;
    int threads;
    size_t lds;
    if (!spec_fits<R>(h, 1, threads, lds)) return false;
    const char* ek = std::getenv("QEDHMC_PC_KERNEL");
    return !ek || !*ek || std::strcmp(ek, "spectral") == 0;
}

// the tau sum fused into the inverse DFT up to this many momenta per plane
// (each workgroup then reads na input planes of both parities through the
// L2); QEDHMC_PC_FUSE=0|1 (read per call) forces either form
static constexpr int kSpecFuseNK = 1152;  // L = 48

static bool spec_fused(const qedhmc_ctx* h) {
    const char* ef = std::getenv("QEDHMC_PC_FUSE");
    if (ef && *ef) return std::atoi(ef) != 0;
    return h->lat.L * (h->lat.L / 2) <= kSpecFuseNK;
}

template <typename R>
static PcSpecGeo spec_geo(const qedhmc_ctx* h) {
    const Lat& lt = h->lat;
    return PcSpecGeo{lt.L, lt.L / 2, lt.Nt, lt.Vs, lt.L * (lt.L / 2), h->pc_spec_a0, h->pc_spec_na};
}

template <typename R>
static const cplx<R>* spec_tw(const qedhmc_ctx* h) {
    return (const cplx<R>*)(sizeof(R) == 8 ? h->pc_tw64 : h->pc_tw32);
}

template <typename R>
static const cplx<R>* spec_H(const qedhmc_ctx* h) {
    return (const cplx<R>*)(sizeof(R) == 8 ? h->pc_spec64 : h->pc_spec32);
}

// threads of a workgroup transforming nplanes planes (kSpecE outputs each at
// most) and its dynamic LDS; EUNSUPPORTED if the plan does not fit
template <typename R>
static bool spec_fits(const qedhmc_ctx* h, int nplanes, int& threads, size_t& lds) {
    const int L = h->lat.L, tot = nplanes * L * (L / 2);
    threads = std::min(spec_max_threads<R>(), (tot + 63) / 64 * 64);
    lds = (size_t)(tot + L / 2 + L) * sizeof(cplx<R>);
    // (room for the update kernel's static reduction scratch; one thread per
    // twiddle)
    return (tot + threads - 1) / threads <= kSpecE && lds + 2048 <= h->max_lds && L / 2 + L <= threads;
}

template <typename R>
static qedhmc_status spec_plan(qedhmc_ctx* h, int nplanes, int& threads, size_t& lds) {
    if (!spec_fits<R>(h, nplanes, threads, lds)) {
        set_error("paper preconditioner: the spectral plan does not fit one workgroup");
        return QEDHMC_EUNSUPPORTED;
    }
    return QEDHMC_OK;
}

// where the forward transform of r should land for launch_pcs_rest(z, tmp):
// tmp when the rest is fused (it reads neighbouring slices and writes z),
// z otherwise
template <typename R>
static cplx<R>* spec_vhat(const qedhmc_ctx* h, cplx<R>* z, cplx<R>* tmp) {
    return spec_fused(h) ? tmp : z;
}

template <typename R>
static qedhmc_status launch_pcs_fwd(qedhmc_ctx* h, const cplx<R>* r, cplx<R>* vhat, const double* stop) {
    int threads;
    size_t lds;
    QH_TRY(spec_plan<R>(h, 1, threads, lds));
    if (lds > 65536) QH_TRY(allow_lds((const void*)k_pcs_dft<R, false>, h->max_lds));
    hipLaunchKernelGGL((k_pcs_dft<R, false>), dim3(spec_grid(h->lat.Nt)), dim3(threads), lds, h->stream,
                       spec_geo<R>(h), spec_tw<R>(h), r, vhat, stop);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// z = P r from vhat = the forward transform of r (at spec_vhat(z, tmp))
template <typename R>
static qedhmc_status launch_pcs_rest(qedhmc_ctx* h, const cplx<R>* vhat, cplx<R>* z, cplx<R>* tmp,
                                     const double* stop) {
    const PcSpecGeo g = spec_geo<R>(h);
    int threads;
    size_t lds;
    QH_TRY(spec_plan<R>(h, 1, threads, lds));
    const dim3 dgrid(spec_grid(g.Nt));
    if (spec_fused(h)) {
        if (lds > 65536) QH_TRY(allow_lds((const void*)k_pcs_tconv_idft<R>, h->max_lds));
        hipEvent_t e0, e1;
        if (prof_sample(h, sizeof(R) == 4 ? QEDHMC_K_PC_SPEC_FP32 : QEDHMC_K_PC_SPEC_FP64, e0, e1))
            hipExtLaunchKernelGGL(k_pcs_tconv_idft<R>, dgrid, dim3(threads), lds, h->stream, e0, e1, 0, g,
                                  spec_H<R>(h), spec_tw<R>(h), vhat, z, stop);
        else
            hipLaunchKernelGGL(k_pcs_tconv_idft<R>, dgrid, dim3(threads), lds, h->stream, g, spec_H<R>(h),
                               spec_tw<R>(h), vhat, z, stop);
        QH_HIP(hipGetLastError());
        return QEDHMC_OK;
    }
    // longer runs once there are enough threads without them
    if (sizeof(R) == 4 && (size_t)g.nk * g.Nt >= ((size_t)1 << 20)) {
        const int nth = g.nk * ((g.Nt + 7) / 8);
        hipLaunchKernelGGL((k_pcs_tconv<R, 8>), dim3((nth + 255) / 256), dim3(256), 0, h->stream, g, spec_H<R>(h),
                           vhat, tmp, stop);
    } else {
        const int nth = g.nk * ((g.Nt + 3) / 4);
        hipLaunchKernelGGL((k_pcs_tconv<R, 4>), dim3((nth + 255) / 256), dim3(256), 0, h->stream, g, spec_H<R>(h),
                           vhat, tmp, stop);
    }
    QH_HIP(hipGetLastError());
    if (lds > 65536) QH_TRY(allow_lds((const void*)k_pcs_dft<R, true>, h->max_lds));
    hipLaunchKernelGGL((k_pcs_dft<R, true>), dgrid, dim3(threads), lds, h->stream, g, spec_tw<R>(h),
                       (const cplx<R>*)tmp, z, stop);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// z = G^dag (G r); tmp: scratch vector of the same precision (r, z and tmp
// distinct)
template <typename R>
static qedhmc_status apply_P_t(qedhmc_ctx* h, const cplx<R>* r, cplx<R>* z, cplx<R>* tmp, const double* stop) {
    if (use_spectral<R>(h)) {
        cplx<R>* vhat = spec_vhat<R>(h, z, tmp);
        QH_TRY(launch_pcs_fwd<R>(h, r, vhat, stop));
        return launch_pcs_rest<R>(h, vhat, z, tmp, stop);
    }
    QH_TRY(launch_pc<R>(h, 0, r, tmp, stop));
    return launch_pc<R>(h, 1, tmp, z, stop);
}

template <typename A, typename B>
__global__ void k_pc_convert(const cplx<A>* __restrict__ a, cplx<B>* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = mk<B>((B)a[i].re, (B)a[i].im);
}

// out = P in on FP64 vectors with the stencil passes in FP32 (the input
// rounded once, the result widened): for flexible CG, which tolerates an
// inexact preconditioner.  Scratch: ws[8] and ws[9].
qedhmc_status launch_apply_precond_fp32(qedhmc_ctx* h, const double* in, double* out) {
    QH_TRY(ensure_paper_precond(h));
    const size_t N = (size_t)h->lat.Nt * h->lat.Vs;
    cplx<float>* r32 = reinterpret_cast<cplx<float>*>(h->ws[9]);
    cplx<float>* t32 = r32 + N;
    cplx<float>* z32 = reinterpret_cast<cplx<float>*>(h->ws[8]);
    const int grid = (int)std::min<size_t>((N + 255) / 256, 4096);
    hipLaunchKernelGGL((k_pc_convert<double, float>), dim3(grid), dim3(256), 0, h->stream,
                       reinterpret_cast<const cplx<double>*>(in), r32, N);
    QH_HIP(hipGetLastError());
    QH_TRY(apply_P_t<float>(h, r32, z32, t32, nullptr));
    hipLaunchKernelGGL((k_pc_convert<float, double>), dim3(grid), dim3(256), 0, h->stream, (const cplx<float>*)z32,
                       reinterpret_cast<cplx<double>*>(out), N);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

qedhmc_status launch_apply_precond(qedhmc_ctx* h, qedhmc_precision prec, const void* in, void* out) {
    QH_TRY(ensure_paper_precond(h));
    if (prec == QEDHMC_FP64)
        return apply_P_t<double>(h, (const cplx<double>*)in, (cplx<double>*)out, (cplx<double>*)h->ws[9], nullptr);
    return apply_P_t<float>(h, (const cplx<float>*)in, (cplx<float>*)out, (cplx<float>*)h->ws[9], nullptr);
}

// ---------------------------------------------------------------------------
// PCG kernels
// ---------------------------------------------------------------------------
template <typename R>
struct PcgBufs {
    cplx<R>* r;
    cplx<R>* p;
    cplx<R>* s;
    cplx<R>* u;
    cplx<R>* w;
    cplx<R>* t;
    cplx<double>* x;
    const cplx<double>* rhs;
    const cplx<double>* Ox;
    double* part;   // [nparts][kNP7]: per slice, or per (slice, tile) for the tiled matvec
    double* partb;  // [Nt]: |rhs|^2 or the FP64 true |r|^2
    int nparts;
};

// r = rhs, x = p = s = 0; partb = |rhs|^2 per slice
template <typename R>
__global__ __launch_bounds__(256) void k_pcg_start(Lat lt, PcgBufs<R> B) {
    __shared__ double red[64];
    const size_t base = (size_t)blockIdx.x * lt.Vs;
    double b2 = 0.0;
    for (int k = threadIdx.x; k < lt.Vs; k += blockDim.x) {
        const cplx<double> b = B.rhs[base + k];
        B.r[base + k] = mk<R>((R)b.re, (R)b.im);
        B.p[base + k] = mk<R>(0, 0);
        B.s[base + k] = mk<R>(0, 0);
        B.x[base + k] = mk<double>(0, 0);
        b2 += b.re * b.re + b.im * b.im;
    }
    double v[1] = {b2};
    block_sumk<1>(v, red);
    if (threadIdx.x == 0) B.partb[blockIdx.x] = v[0];
}

// slot 0 from the |rhs|^2 partials
__global__ void k_pcg_init_slot(double* __restrict__ scal, const double* __restrict__ partb, int Nt, double tol2) {
    __shared__ double red[64];
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < Nt; t += blockDim.x) v[0] += partb[t];
    block_sumk<1>(v, red);
    if (threadIdx.x < S_NSLOT) {
        double val = 0.0;
        if (threadIdx.x == S_FIRST || threadIdx.x == S_GPREV || threadIdx.x == S_APREV) val = 1.0;
        scal[threadIdx.x] = val;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        scal[S_B2] = v[0];
        scal[S_TARGET] = tol2 * v[0];
        scal[S_RRUPD] = v[0];
    }
}

template <int K>
__device__ __forceinline__ void reduce_k(const double* __restrict__ part, int Nt, double* red, double* bc,
                                         double (&out)[K]) {
    double v[K];
#pragma unroll
    for (int k = 0; k < K; k++) v[k] = 0.0;
    for (int t = threadIdx.x; t < Nt; t += blockDim.x)
#pragma unroll
        for (int k = 0; k < K; k++) v[k] += part[K * t + k];
    block_sumk<K>(v, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; k++) bc[k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; k++) out[k] = bc[k];
}

// One slice per block (dealt to the XCDs as slice_of_block deals them):
// scalars from the partials, then the elementwise update.
// DFT: the block then also transforms the new r of its slice (both parity
// planes, through LDS) into vhat, the first step of the spectral P r; vhat
// may be u itself, whose slice only this block reads.
// Latency: once the slot says the solve runs, this block's share of the
// partials and the vectors of the thread's first kUpdPre sites are requested
// together (one round trip to memory instead of two in a row).
static constexpr int kUpdPre = 4;

template <typename R, bool DFT>
__global__ __launch_bounds__(spec_max_threads<R>()) void k_pcg_upd(Lat lt, PcgBufs<R> B, double* __restrict__ scal, int kpar,
                                                  int mixed, int maxit, PcSpecGeo sg, const cplx<R>* __restrict__ tw,
                                                  cplx<R>* __restrict__ vhat) {
    __shared__ double red[kNP7 * 16 + 16];
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<R>* buf = reinterpret_cast<cplx<R>*>(smem);  // [plane][row][column]: the new r by x parity
    cplx<R>* twx = buf + (DFT ? 2 * sg.nk : 0);
    const double* sin_ = scal + S_NSLOT * kpar;
    double* sout = scal + S_NSLOT * (kpar ^ 1);
    const int tau = slice_of_block(blockIdx.x, lt.Nt);
    const size_t base = (size_t)(tau < 0 ? 0 : tau) * lt.Vs;
    if (sin_[S_DONE] != 0.0) {
        if (blockIdx.x == 0 && threadIdx.x < S_NSLOT) sout[threadIdx.x] = sin_[threadIdx.x];
        return;
    }
    // requests, all in flight together: the vectors first (the partials'
    // loop waits inside)
    cplx<R> p0[kUpdPre], u0[kUpdPre], s0[kUpdPre], w0[kUpdPre], r0[kUpdPre];
    cplx<double> x0[kUpdPre];
#pragma unroll
    for (int j = 0; j < kUpdPre; j++) {
        const int k = (int)threadIdx.x + j * (int)blockDim.x;
        const size_t i = base + (k < lt.Vs ? k : 0);
        p0[j] = B.p[i];
        u0[j] = B.u[i];
        s0[j] = B.s[i];
        w0[j] = B.w[i];
        r0[j] = B.r[i];
        x0[j] = B.x[i];
    }
    const int ntw = DFT ? sg.Lh + sg.L : 0;  // <= blockDim.x (spec_fits)
    const cplx<R> twv = (int)threadIdx.x < ntw ? tw[threadIdx.x] : mk<R>(R(0), R(0));
    double sl[S_NSLOT];
#pragma unroll
    for (int k = 0; k < S_NSLOT; k++) sl[k] = sin_[k];
    double pv[kNP7];
#pragma unroll
    for (int k = 0; k < kNP7; k++) pv[k] = 0.0;
    for (int t = threadIdx.x; t < B.nparts; t += blockDim.x)
#pragma unroll
        for (int k = 0; k < kNP7; k++) pv[k] += B.part[kNP7 * t + k];
    double pr[kNP7];
    block_sumk<kNP7>(pv, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < kNP7; k++) red[kNP7 * 16 + k] = pv[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kNP7; k++) pr[k] = red[kNP7 * 16 + k];
    const double rr = pr[0], gam = pr[1], del = pr[2];
    const int it = (int)sl[S_ITERS];
    int stop = 0;
    double alpha = 0.0, beta = 0.0;
    const bool first = sl[S_FIRST] != 0.0;
    if (!isfinite(rr) || !isfinite(gam) || !isfinite(del))
        stop = 4;
    else if (rr <= sl[S_TARGET])
        stop = 1;
    else if (it >= maxit)
        stop = 2;  // the budget is used: the update decides
    else if (mixed && (rr <= kDecade2 * sl[S_RRUPD] || it - (int)sl[S_ITUPD] >= kCap))
        stop = 2;
    else {
        beta = first ? 0.0 : gam / sl[S_GPREV];
        const double den = first ? del : del + beta * (pr[3] + pr[4]) + beta * beta * pr[5];
        if (!(den > 0.0))
            stop = 3;
        else
            alpha = gam / den;
    }
    if (blockIdx.x == 0 && threadIdx.x < S_NSLOT) {
        double v = sin_[threadIdx.x];
        if (stop) {
            if (threadIdx.x == S_DONE) v = (double)stop;
            if (threadIdx.x == S_GCUR) v = rr;
        } else {
            if (threadIdx.x == S_GPREV) v = gam;
            if (threadIdx.x == S_APREV) v = alpha;
            if (threadIdx.x == S_ITERS) v = (double)(it + 1);
            if (threadIdx.x == S_FIRST) v = 0.0;
            if (threadIdx.x == S_GCUR) v = rr;
        }
        sout[threadIdx.x] = v;
    }
    if (stop || tau < 0) return;
    if (DFT && (int)threadIdx.x < ntw) twx[threadIdx.x] = twv;
    const R a = (R)alpha, b = (R)beta;
    auto update = [&](int k, cplx<R> pk, cplx<R> uk, cplx<R> sk, cplx<R> wk, cplx<R> rk, cplx<double> xv) {
        const size_t i = base + k;
        const cplx<R> pn = cfma(b, pk, uk);
        const cplx<R> sn = cfma(b, sk, wk);
        B.p[i] = pn;
        B.s[i] = sn;
        xv.re += alpha * (double)pn.re;
        xv.im += alpha * (double)pn.im;
        B.x[i] = xv;
        const cplx<R> rn = cfma(-a, sn, rk);
        B.r[i] = rn;
        if (DFT) {
            const int y = k / sg.L, x = k - y * sg.L;
            buf[(x & 1) * sg.nk + y * sg.Lh + (x >> 1)] = rn;
        }
    };
#pragma unroll
    for (int j = 0; j < kUpdPre; j++) {
        const int k = (int)threadIdx.x + j * (int)blockDim.x;
        if (k < lt.Vs) update(k, p0[j], u0[j], s0[j], w0[j], r0[j], x0[j]);
    }
    for (int k = (int)threadIdx.x + kUpdPre * (int)blockDim.x; k < lt.Vs; k += blockDim.x) {
        const size_t i = base + k;
        update(k, B.p[i], B.u[i], B.s[i], B.w[i], B.r[i], B.x[i]);
    }
    if (DFT) {
        __syncthreads();
        dft_planes<R>(buf, twx, twx + sg.Lh, sg.L, sg.Lh, 2,
                      [&](int pl, int e, cplx<R> v) { vhat[base + (size_t)pl * sg.nk + e] = v; });
    }
}

// w = O u (own slice) and the partials of the next iteration
template <typename R, int MC, int NB, int BS>
__global__ __launch_bounds__(BS) void k_pcg_mv(Lat lt, PcgBufs<R> B, const cplx<R>* __restrict__ gauge, Coef<R> co,
                                               const double* __restrict__ stop) {
    // (testing the flag only once the slice's data is in flight measured
    // slower: the launches after a pause then load everything too)
    if (stop && *stop != 0.0) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<R>* buf2 = reinterpret_cast<cplx<R>*>(smem);
    double* red = reinterpret_cast<double*>(smem + (size_t)NB * 2 * lt.Vs * sizeof(cplx<R>));
    const int tau = slice_of_block(blockIdx.x, lt.Nt);
    if (tau < 0) return;
    SliceCtx<MC> c;
    slice_ctx<MC>(lt, c, tau, whole_block_tile(smem, red));
    const size_t Vs = lt.Vs;
    cplx<R> hm[MC][12], ht[MC][12];
    hops_of<R, MC>(gauge, lt, c.tm, c.idx, co, hm);
    hops_of<R, MC>(gauge, lt, c.tau, c.idx, co, ht);
    Cells<R, MC> um, ut, un, w;
    load_cells<R, MC>(um, B.u + c.tm * Vs, c.g, c.own);
    load_cells<R, MC>(ut, B.u + c.tau * Vs, c.g, c.own);
    load_cells<R, MC>(un, B.u + c.tp * Vs, c.g, c.own);
    // the own-slice vectors of the inner products: with one cell a thread
    // and at most 512 threads requested with u (one round trip less);
    // otherwise after the matvec so they are not live across it (fewer
    // registers)
    Cells<R, MC> rt, pt, st;
    constexpr bool early = MC == 1 && BS <= 512;  // 1024-thread workgroups would spill
    if constexpr (early) {
        load_cells<R, MC>(rt, B.r + c.tau * Vs, c.g, c.own);
        load_cells<R, MC>(pt, B.p + c.tau * Vs, c.g, c.own);
        load_cells<R, MC>(st, B.s + c.tau * Vs, c.g, c.own);
    }
    mdagm_cells<R, MC, NB>(um, ut, un, hm, ht, c.g, c.own, co, c.tau == 0 ? R(-1) : R(1),
                           c.tau == lt.Nt - 1 ? R(-1) : R(1), buf2, lt.Vs, w);
    store_cells<R, MC>(w, B.w + c.tau * Vs, c.g, c.own);
    if constexpr (!early) {
        load_cells<R, MC>(rt, B.r + c.tau * Vs, c.g, c.own);
        load_cells<R, MC>(pt, B.p + c.tau * Vs, c.g, c.own);
        load_cells<R, MC>(st, B.s + c.tau * Vs, c.g, c.own);
    }
    const Cells<R, MC>& u0 = ut;  // the matvec reads its own slice without changing it
    double v[kNP7] = {dot_cells<R, MC>(rt, rt, c.own), dot_cells<R, MC>(rt, u0, c.own),
                      dot_cells<R, MC>(w, u0, c.own),  dot_cells<R, MC>(u0, st, c.own),
                      dot_cells<R, MC>(pt, w, c.own),  dot_cells<R, MC>(pt, st, c.own), 0.0};
    block_sumk<kNP7>(v, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < kNP7; k++) B.part[kNP7 * (size_t)c.tau + k] = v[k];
}

// r = rhs - O x from the FP64 O x; partb = FP64 |rhs - O x|^2 per slice.
// gate (nullable): a slot's stop flag; the launch is a no-op unless it asks
// for a reliable update.
template <typename R>
__global__ __launch_bounds__(256) void k_pcg_rep(Lat lt, PcgBufs<R> B, const double* __restrict__ gate) {
    if (gate && !gate_open(*gate)) return;
    __shared__ double red[64];
    const size_t base = (size_t)blockIdx.x * lt.Vs;
    double t2 = 0.0;
    for (int k = threadIdx.x; k < lt.Vs; k += blockDim.x) {
        const cplx<double> b = B.rhs[base + k], o = B.Ox[base + k];
        const double re = b.re - o.re, im = b.im - o.im;
        B.r[base + k] = mk<R>((R)re, (R)im);
        t2 += re * re + im * im;
    }
    double v[1] = {t2};
    block_sumk<1>(v, red);
    if (threadIdx.x == 0) B.partb[blockIdx.x] = v[0];
}

// After a replacement and a fresh u, w and partials: converged -> stop 1;
// otherwise resume (restart sets beta = 0 on the next iteration).
__global__ void k_pcg_check(double* __restrict__ scal, int kpar, const double* __restrict__ part, int nparts,
                            const double* __restrict__ partb, int Nt, int restart) {
    __shared__ double red[64];
    double v[2] = {0.0, 0.0};
    for (int t = threadIdx.x; t < Nt; t += blockDim.x) v[0] += partb[t];
    for (int t = threadIdx.x; t < nparts; t += blockDim.x) v[1] += part[kNP7 * t];
    block_sumk<2>(v, red);
    if (threadIdx.x == 0) {
        double* sl = scal + S_NSLOT * kpar;
        sl[S_TRUE] = v[0];
        if (v[0] <= sl[S_TARGET]) {
            sl[S_DONE] = 1.0;
        } else {
            sl[S_DONE] = 0.0;
            if (restart) sl[S_FIRST] = 1.0;
            sl[S_ITUPD] = sl[S_ITERS];
            sl[S_RRUPD] = v[1];
        }
    }
}

// skip = 0 when the slot's flag asks for a reliable update, else 1: the stop
// flag of the gated preconditioner and matvec of the update
__global__ void k_pcg_gate(const double* __restrict__ flag, double* __restrict__ skip) {
    if (threadIdx.x == 0) *skip = gate_open(*flag) ? 0.0 : 1.0;
}

// The reliable-update decision on the device (pipelined driver), after the
// gated replacement: converged (5) when the FP64 true residual meets the
// target; failed (4) on a non-finite residual, the iteration budget used or
// no progress across three updates, or a breakdown flagged by the recursion;
// otherwise resume (0; restart with beta = 0 after a non-positive
// denominator, and after every update with restart_all).  A solve already
// final is left as it is.  The record is mirrored to out (pinned host
// memory).
__global__ void k_pcg_check_dev(double* __restrict__ scal, int kpar, const double* __restrict__ part, int nparts,
                                const double* __restrict__ partb, int Nt, int maxit, int restart_all,
                                double* __restrict__ rec, double* __restrict__ out) {
    __shared__ double red[64];
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
        double v[2] = {0.0, 0.0};
        for (int t = threadIdx.x; t < Nt; t += blockDim.x) v[0] += partb[t];
        for (int t = threadIdx.x; t < nparts; t += blockDim.x) v[1] += part[kNP7 * t];
        block_sumk<2>(v, red);
        if (threadIdx.x == 0) {
            const double tr = v[0];
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
                sl[S_RRUPD] = v[1];
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

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
template <typename R>
static PcgBufs<R> pbufs_of(qedhmc_ctx* h, const double* rhs, double* x) {
    PcgBufs<R> B;
    const size_t N = (size_t)h->lat.Nt * h->lat.Vs;
    cplx<R>* base = reinterpret_cast<cplx<R>*>(h->cg_arena);
    B.r = base;
    B.p = base + N;
    B.s = base + 2 * N;
    B.u = base + 3 * N;
    B.w = base + 4 * N;
    B.t = base + 5 * N;
    B.x = reinterpret_cast<cplx<double>*>(x);
    B.rhs = reinterpret_cast<const cplx<double>*>(rhs);
    B.Ox = reinterpret_cast<const cplx<double>*>(h->ws[3]);
    if (h->lat.ncell > 1024) {
        // the tiled matvec writes one partial tuple per (slice, tile)
        B.nparts = h->lat.Nt * mdagm_tiled_tiles(h->lat, sizeof(R) == 8);
        B.part = h->tpart;
        B.partb = h->tpart + kNP7 * (size_t)h->lat.Nt * h->tpart_tiles;
    } else {
        B.nparts = h->lat.Nt;
        B.part = h->partial;
        B.partb = h->partial + kNP7 * (size_t)h->lat.Nt;
    }
    return B;
}

template <typename R>
static qedhmc_status launch_mv(qedhmc_ctx* h, const PcgBufs<R>& B, const double* stop, bool timed) {
    if (h->lat.ncell > 1024) return launch_mdagm_tiled_parts<R>(h, B.u, B.w, B.r, B.p, B.s, B.part, stop);
    return with_shape<R>(h, [&]<int MC, int NB, int BS>(int nt, size_t lds) -> qedhmc_status {
        QH_TRY(lds_attr(h, k_pcg_mv<R, MC, NB, BS>, lds));
        hipEvent_t e0, e1;
        const int cls = sizeof(R) == 4 ? QEDHMC_K_PCG_MV_FP32 : QEDHMC_K_PCG_MV_FP64;
        if (timed && prof_sample(h, cls, e0, e1))
            hipExtLaunchKernelGGL((k_pcg_mv<R, MC, NB, BS>), dim3(slice_grid(h->lat.Nt)), dim3(nt), lds, h->stream, e0, e1, 0,
                                  h->lat, B, gauge_for<R>(h), coef_of<R>(h->p), stop);
        else
            hipLaunchKernelGGL((k_pcg_mv<R, MC, NB, BS>), dim3(slice_grid(h->lat.Nt)), dim3(nt), lds, h->stream, h->lat, B,
                               gauge_for<R>(h), coef_of<R>(h->p), stop);
        QH_HIP(hipGetLastError());
        return QEDHMC_OK;
    });
}

// u = P r, w = O u, partials (stop: nullable slot flag); with the identity
// preconditioner u is r itself and only w = O r is launched
template <typename R>
static qedhmc_status pcg_tail(qedhmc_ctx* h, const PcgBufs<R>& B, const double* stop, bool identity) {
    if (!identity) QH_TRY(apply_P_t<R>(h, B.r, B.u, B.t, stop));
    return launch_mv<R>(h, B, stop, stop != nullptr);
}

// n iterations from launch parity kpar: update, then preconditioner and
// matvec, each gated on the slot's stop flag
// Spectral P with the update kernel doing its first step: the plan's
// threads and LDS for both planes of a slice, or false where it does not fit
template <typename R>
static bool upd_dft_plan(qedhmc_ctx* h, int& threads, size_t& lds) {
    return use_spectral<R>(h) && spec_fits<R>(h, 2, threads, lds);
}

template <typename R>
static qedhmc_status pcg_chunk(qedhmc_ctx* h, const PcgBufs<R>& B, int kpar, int n, bool mixed, bool identity,
                               int maxit) {
    int threads = 256;
    size_t lds = 0;
    const bool fdft = !identity && upd_dft_plan<R>(h, threads, lds);
    if (fdft && lds > 65536) QH_TRY(allow_lds((const void*)k_pcg_upd<R, true>, h->max_lds));
    const PcSpecGeo sg = fdft ? spec_geo<R>(h) : PcSpecGeo{};
    cplx<R>* vhat = fdft ? spec_vhat<R>(h, B.u, B.t) : nullptr;
    for (int k = 0; k < n; k++) {
        if (fdft)
            hipLaunchKernelGGL((k_pcg_upd<R, true>), dim3(slice_grid(h->lat.Nt)), dim3(threads), lds, h->stream, h->lat, B, h->scal,
                               kpar, mixed ? 1 : 0, maxit, sg, spec_tw<R>(h), vhat);
        else
            hipLaunchKernelGGL((k_pcg_upd<R, false>), dim3(slice_grid(h->lat.Nt)), dim3(256), 0, h->stream, h->lat, B, h->scal,
                               kpar, mixed ? 1 : 0, maxit, sg, (const cplx<R>*)nullptr, (cplx<R>*)nullptr);
        kpar ^= 1;
        const double* stop = h->scal + S_NSLOT * kpar + S_DONE;
        if (fdft) {
            QH_TRY(launch_pcs_rest<R>(h, vhat, B.u, B.t, stop));
            QH_TRY(launch_mv<R>(h, B, stop, true));
        } else {
            QH_TRY(pcg_tail<R>(h, B, stop, identity));
        }
    }
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// The same chunk replayed from a graph captured the first time this
// (buffers, mode, chunk) combination is seen on the handle; the launch
// shapes (and kernel attributes) are those of the solve's first matvec,
// made before any capture.
template <typename R>
static qedhmc_status pcg_chunk_graph(qedhmc_ctx* h, const PcgBufs<R>& B, int kpar, int n, bool mixed, bool identity,
                                     int maxit) {
    qedhmc_ctx::PcgGraph& gr = h->pcg_graph[sizeof(R) == 8 ? 1 : 0][identity ? 1 : 0][kpar];
    const int plan = identity ? 0 : (use_spectral<R>(h) ? 1 : 0) | (spec_fused(h) ? 2 : 0);
    if (gr.exec && (gr.x != B.x || gr.rhs != B.rhs || gr.mixed != (int)mixed || gr.count != n || gr.plan != plan ||
                    gr.maxit != maxit)) {
        QH_HIP(hipGraphExecDestroy(gr.exec));
        gr.exec = nullptr;
    }
    if (!gr.exec) {
        if (!h->cap_stream) QH_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        hipStream_t user = h->stream;
        const int prof = h->prof_every;
        h->stream = h->cap_stream;
        h->prof_every = 0;  // no event launches inside a graph
        hipGraph_t g = nullptr;
        qedhmc_status st = QEDHMC_OK;
        hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            st = pcg_chunk<R>(h, B, kpar, n, mixed, identity, maxit);
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
        gr.mixed = mixed ? 1 : 0;
        gr.count = n;
        gr.plan = plan;
        gr.maxit = maxit;
    }
    QH_HIP(hipGraphLaunch(gr.exec, h->stream));
    return QEDHMC_OK;
}

// One round of the pipelined PCG from launch parity kp: the chunk of n
// iterations (the mixed recursion pauses itself for a reliable update at a
// decade or after kCap iterations; FP64 pauses only to stop or restart, or
// at the budget), then the replacement gated on a pause in slot ke (FP64
// O x, r = rhs - O x, s = O p, u = P r, w = O u and the partials) and the
// decision, which mirrors the solve's record to out (pinned host memory).
template <typename R>
static qedhmc_status pcg_round(qedhmc_ctx* h, const PcgBufs<R>& B, double* x, int kp, int n, bool mixed, int maxit,
                               double* out) {
    const int ke = kp ^ (n & 1);
    double* skip = h->scal + kRecOff - 4;  // between the two slots and the record
    QH_TRY(pcg_chunk<R>(h, B, kp, n, mixed, false, maxit));
    const double* gate = h->scal + S_NSLOT * ke + S_DONE;
    QH_TRY(launch_mdagm(h, QEDHMC_FP64, x, h->ws[3], gate));
    hipLaunchKernelGGL(k_pcg_rep<R>, dim3(h->lat.Nt), dim3(256), 0, h->stream, h->lat, B, gate);
    QH_HIP(hipGetLastError());
    QH_TRY(launch_mdagm(h, mixed ? QEDHMC_FP32 : QEDHMC_FP64, B.p, B.s, gate));
    hipLaunchKernelGGL(k_pcg_gate, dim3(1), dim3(64), 0, h->stream, gate, skip);
    QH_HIP(hipGetLastError());
    QH_TRY(pcg_tail<R>(h, B, skip, false));
    hipLaunchKernelGGL(k_pcg_check_dev, dim3(1), dim3(256), 0, h->stream, h->scal, ke, (const double*)B.part,
                       B.nparts, (const double*)B.partb, h->lat.Nt, maxit, mixed ? 0 : 1, h->scal + kRecOff, out);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// The same round replayed from a graph captured the first time this
// (buffers, mode, round parity) combination is seen on the handle (every
// kernel attribute was set by an eager round before).
template <typename R>
static qedhmc_status pcg_round_graph(qedhmc_ctx* h, const PcgBufs<R>& B, double* x, int kp, int n, bool mixed,
                                     int maxit, int par, double* out) {
    qedhmc_ctx::PcgGraph& gr = h->pcg_round[sizeof(R) == 8 ? 1 : 0][par];
    const int plan = (use_spectral<R>(h) ? 1 : 0) | (spec_fused(h) ? 2 : 0);
    if (gr.exec && (gr.x != x || gr.rhs != B.rhs || gr.mixed != (int)mixed || gr.count != n || gr.plan != plan ||
                    gr.maxit != maxit || gr.kp != kp)) {
        QH_HIP(hipGraphExecDestroy(gr.exec));
        gr.exec = nullptr;
    }
    if (!gr.exec) {
        if (!h->cap_stream) QH_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        hipStream_t user = h->stream;
        const int prof = h->prof_every;
        h->stream = h->cap_stream;
        h->prof_every = 0;  // no event launches inside a graph
        hipGraph_t g = nullptr;
        qedhmc_status st = QEDHMC_OK;
        hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            st = pcg_round<R>(h, B, x, kp, n, mixed, maxit, out);
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
        gr.x = x;
        gr.rhs = B.rhs;
        gr.mixed = mixed ? 1 : 0;
        gr.count = n;
        gr.plan = plan;
        gr.maxit = maxit;
        gr.kp = kp;
    }
    QH_HIP(hipGraphLaunch(gr.exec, h->stream));
    return QEDHMC_OK;
}

// iterations per round of the mixed pipelined PCG: odd (so the launch parity
// alternates with the round parity) and shorter than the kCap + 1 of the
// unpreconditioned solver, since the paper's preconditioner reaches a decade,
// and with it a pause, within about 30 iterations (the launches of a round
// past its pause are no-ops).  QEDHMC_PCG_CHUNK (read per solve, made odd)
// overrides.
static constexpr int kPcgChunk = 9;

// Rounds queued on the device as in the pipelined CG: the host keeps the
// next round queued behind the running one and reads each round's record
// through an event; the round after the last is skipped when the residual
// estimates of the last two rounds, extrapolated geometrically, say the
// running round converges.  Rounds after the first replay a captured graph.
// Whole-slice lattices (the gated M^dag M has no tiled form).
template <typename R>
static qedhmc_status pcg_pipelined(qedhmc_ctx* h, const PcgBufs<R>& B, double* x, double tol, int maxit,
                                   qedhmc_precision prec, int* iters, double* true_rel, int* n_reliable) {
    const bool mixed = prec != QEDHMC_FP64;
    int chunk = mixed ? kPcgChunk : 64;
    if (const char* ec = std::getenv("QEDHMC_PCG_CHUNK"); ec && mixed && std::atoi(ec) > 0)
        chunk = std::atoi(ec) | 1;
    const int Nt = h->lat.Nt;
    for (auto& e : h->cg_ev)
        if (!e) QH_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipLaunchKernelGGL(k_pcg_start<R>, dim3(Nt), dim3(256), 0, h->stream, h->lat, B);
    hipLaunchKernelGGL(k_pcg_init_slot, dim3(1), dim3(256), 0, h->stream, h->scal, (const double*)B.partb, Nt,
                       tol * tol);
    QH_HIP(hipGetLastError());
    QH_TRY(pcg_tail<R>(h, B, nullptr, false));
    QH_HIP(hipMemsetAsync(h->scal + kRecOff, 0, CR_N * sizeof(double), h->stream));
    // the first round of a handle's first pipelined solve runs eagerly: it
    // sets every kernel attribute before any capture
    const bool eager0 = !h->pcg_round[sizeof(R) == 8 ? 1 : 0][0].exec;
    auto round = [&](long n) -> qedhmc_status {
        const int kp = (chunk & 1) ? (int)(n & 1) : 0, par = (int)(n & 1);
        double* out = h->h_pinned + 32 + 16 * par;
        if (n == 0 && eager0)
            QH_TRY(pcg_round<R>(h, B, x, kp, chunk, mixed, maxit, out));
        else
            QH_TRY(pcg_round_graph<R>(h, B, x, kp, chunk, mixed, maxit, par, out));
        QH_HIP(hipEventRecord(h->cg_ev[par], h->stream));
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
            set_error("PCG did not end within " + std::to_string(max_rounds) + " rounds");
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
            set_error("PCG breakdown: non-finite inner products after " + std::to_string(it) + " iterations");
            break;
        case WHY_NONFINITE:
            set_error("PCG breakdown: non-finite true residual after " + std::to_string(it) + " iterations");
            break;
        case WHY_STALL:
            set_error("PCG made no progress across reliable updates at iteration " + std::to_string(it));
            break;
        default:
            break;
    }
    return QEDHMC_ENOCONV;
}

// identity = true: plain CG in the same two-launch form (update, then
// M^dag M with the partials), the form used for lattices whose slices hold
// more than 1024 cells: there the fused one-launch iteration would need two
// cells per thread and more registers than a 576-thread workgroup has.
template <typename R>
static qedhmc_status pcg_t(qedhmc_ctx* h, const double* rhs, double* x, double tol, int maxit, qedhmc_precision prec,
                           int* iters, double* true_rel, int* n_reliable, bool identity) {
    if (!identity) QH_TRY(ensure_paper_precond(h));
    const bool mixed = prec != QEDHMC_FP64;
    PcgBufs<R> B = pbufs_of<R>(h, rhs, x);
    if (identity) B.u = B.r;
    const int Nt = h->lat.Nt;
    const int chunk = mixed ? kCap + 1 : 64;
    // QEDHMC_NO_GRAPH (read per solve) launches every chunk directly from the
    // host-driven loop below
    const bool no_graph = std::getenv("QEDHMC_NO_GRAPH") != nullptr;
    if (!identity && !no_graph && h->lat.ncell <= 1024)
        return pcg_pipelined<R>(h, B, x, tol, maxit, prec, iters, true_rel, n_reliable);
    int kpar = 0, nrel = 0, it = 0, stalled = 0, last_it = -1;
    double rel = 1.0;
    bool converged = false, broken = false;
    hipLaunchKernelGGL(k_pcg_start<R>, dim3(Nt), dim3(256), 0, h->stream, h->lat, B);
    hipLaunchKernelGGL(k_pcg_init_slot, dim3(1), dim3(256), 0, h->stream, h->scal, (const double*)B.partb, Nt,
                       tol * tol);
    QH_HIP(hipGetLastError());
    QH_TRY(pcg_tail<R>(h, B, nullptr, identity));
    while (true) {
        const int left = maxit - it;
        const int n = left < chunk ? left : chunk;
        if (n == chunk && !no_graph)
            QH_TRY(pcg_chunk_graph<R>(h, B, kpar, n, mixed, identity, maxit));
        else
            QH_TRY(pcg_chunk<R>(h, B, kpar, n, mixed, identity, maxit));
        if (n & 1) kpar ^= 1;
        QH_TRY(read_slot(h, kpar));
        it = (int)h->h_pinned[S_ITERS];
        const double flag = h->h_pinned[S_DONE];
        if (flag == 0.0 && it < maxit) continue;
        if (flag == 4.0) {
            broken = true;
            set_error("PCG breakdown: non-finite inner products after " + std::to_string(it) + " iterations");
            break;
        }
        stalled = (it == last_it) ? stalled + 1 : 0;
        last_it = it;
        if (stalled >= 3) {
            set_error("PCG made no progress across reliable updates at iteration " + std::to_string(it));
            break;
        }
        // FP64 true residual; r replaced, s = O p refreshed, u, w and partials recomputed
        QH_TRY(launch_mdagm(h, QEDHMC_FP64, x, h->ws[3], nullptr));
        hipLaunchKernelGGL(k_pcg_rep<R>, dim3(Nt), dim3(256), 0, h->stream, h->lat, B, (const double*)nullptr);
        QH_HIP(hipGetLastError());
        QH_TRY(launch_mdagm(h, prec == QEDHMC_FP64 ? QEDHMC_FP64 : QEDHMC_FP32, B.p, B.s, nullptr));
        QH_TRY(pcg_tail<R>(h, B, nullptr, identity));
        hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(256), 0, h->stream, h->scal, kpar, (const double*)B.part,
                           B.nparts, (const double*)B.partb, Nt, (!mixed || flag == 3.0) ? 1 : 0);
        QH_HIP(hipGetLastError());
        nrel++;
        QH_TRY(read_slot(h, kpar));
        const double b2 = h->h_pinned[S_B2];
        rel = b2 > 0.0 ? std::sqrt(h->h_pinned[S_TRUE] / b2) : 0.0;
        if (!std::isfinite(rel)) {
            broken = true;
            set_error("PCG breakdown: non-finite true residual after " + std::to_string(it) + " iterations");
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

qedhmc_status pcg_solve_impl(qedhmc_ctx* h, const double* rhs, double* x, double tol, int maxit,
                             qedhmc_precision prec, int* iters, double* true_rel, int* n_reliable) {
    if (prec == QEDHMC_FP64) return pcg_t<double>(h, rhs, x, tol, maxit, prec, iters, true_rel, n_reliable, false);
    return pcg_t<float>(h, rhs, x, tol, maxit, prec, iters, true_rel, n_reliable, false);
}

qedhmc_status cg2_solve_impl(qedhmc_ctx* h, const double* rhs, double* x, double tol, int maxit,
                             qedhmc_precision prec, int* iters, double* true_rel, int* n_reliable) {
    if (prec == QEDHMC_FP64) return pcg_t<double>(h, rhs, x, tol, maxit, prec, iters, true_rel, n_reliable, true);
    return pcg_t<float>(h, rhs, x, tol, maxit, prec, iters, true_rel, n_reliable, true);
}

}  // namespace qh
