// Host side of the NLOP hot path: plan tables, workspace layout, step and
// sweep drivers, binomial checkpoint schedule and the exported C ABI.
#include "npo_internal.h"
#include "../../include/npo.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

npo_status fail(npo_status s, const std::string& msg) {
    g_err = msg;
    return s;
}
npo_status hipfail(hipError_t e, const char* where) {
    return fail(NPO_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}
#define HIPCHK(expr)                                   \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hipfail(e_, #expr); \
    } while (0)

using ld = long double;

// roctx ranges around the plan, sweep, iteration and batch calls when the
// environment has NPO_TRACE=1.
bool trace_on() {
    static const bool on = [] {
        const char* e = std::getenv("NPO_TRACE");
        return e && e[0] == '1';
    }();
    return on;
}
struct Trace {
    bool on;
    explicit Trace(const char* name) : on(trace_on()) {
        if (on) roctxRangePushA(name);
    }
    ~Trace() {
        if (on) roctxRangePop();
    }
};

// ---------------------------------------------------------------- tables
// Radial nodes: positive half of a 2N-point Chebyshev-Gauss-Lobatto grid.
std::vector<ld> radial_nodes(int nr) {
    std::vector<ld> r(nr);
    const ld pi = acosl(-1.0L);
    for (int j = 0; j < nr; ++j) r[j] = cosl(pi * (ld)(nr - 1 - j) / (ld)(2 * nr - 1));
    r[nr - 1] = 1.0L;
    return r;
}

// Gaussian elimination with partial pivoting (small dense, long double).
std::vector<ld> dense_solve(std::vector<ld> A, std::vector<ld> b, int n) {
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (fabsl(A[i * n + k]) > fabsl(A[piv * n + k])) piv = i;
        if (piv != k) {
            for (int c = 0; c < n; ++c) std::swap(A[k * n + c], A[piv * n + c]);
            std::swap(b[k], b[piv]);
        }
        for (int i = k + 1; i < n; ++i) {
            const ld l = A[i * n + k] / A[k * n + k];
            for (int c = k; c < n; ++c) A[i * n + c] -= l * A[k * n + c];
            b[i] -= l * b[k];
        }
    }
    std::vector<ld> x(n);
    for (int i = n - 1; i >= 0; --i) {
        ld s = b[i];
        for (int c = i + 1; c < n; ++c) s -= A[i * n + c] * x[c];
        x[i] = s / A[i * n + i];
    }
    return x;
}

// Interpolatory weights of int_0^1 g(r) r dr on the nodes, exact for
// polynomials of degree < nr in s = r^2 (Chebyshev-moment formulation).
std::vector<ld> quad_weights(const std::vector<ld>& r) {
    const int n = (int)r.size();
    std::vector<ld> A(n * n), b(n);
    for (int k = 0; k < n; ++k) {
        for (int j = 0; j < n; ++j) {
            const ld x = 2.0L * r[j] * r[j] - 1.0L;
            // T_k(x) by recurrence
            ld t0 = 1.0L, t1 = x, tk = (k == 0) ? t0 : t1;
            for (int q = 2; q <= k; ++q) {
                tk = 2.0L * x * t1 - t0;
                t0 = t1;
                t1 = tk;
            }
            A[k * n + j] = tk;
        }
        b[k] = (k % 2 == 0) ? 1.0L / (1.0L - (ld)k * (ld)k) : 0.0L;   // int_0^1 T_k(2s-1) ds
    }
    std::vector<ld> W = dense_solve(A, b, n);
    for (auto& v : W) v *= 0.5L;
    return W;
}

// Fornberg's recursion for FD weights at x0 on nodes x[0..n-1], derivative
// orders 0..2; returns c[d][i].
void fornberg(ld x0, const ld* x, int n, ld c[3][7]) {
    ld c1 = 1.0L, c4 = x[0] - x0;
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i < n; ++i) c[d][i] = 0.0L;
    c[0][0] = 1.0L;
    for (int i = 1; i < n; ++i) {
        const int mn = std::min(i, 2);
        ld c2 = 1.0L;
        const ld c5 = c4;
        c4 = x[i] - x0;
        for (int j = 0; j < i; ++j) {
            const ld c3 = x[i] - x[j];
            c2 *= c3;
            if (j == i - 1) {
                for (int k = mn; k >= 1; --k) c[k][i] = c1 * (k * c[k - 1][i - 1] - c5 * c[k][i - 1]) / c2;
                c[0][i] = -c1 * c5 * c[0][i - 1] / c2;
            }
            for (int k = mn; k >= 1; --k) c[k][j] = (c4 * c[k][j] - k * c[k - 1][j]) / c3;
            c[0][j] = c4 * c[0][j] / c3;
        }
        c1 = c2;
    }
}

// Complex Bessel J0, J1 by their power series (|z| <= ~25 in long double).
void bessel01(std::complex<ld> z, std::complex<ld>& J0, std::complex<ld>& J1) {
    const std::complex<ld> q = -0.25L * z * z;
    std::complex<ld> t0 = 1.0L, t1 = 0.5L * z;
    J0 = t0;
    J1 = t1;
    for (int k = 1; k < 200; ++k) {
        t0 *= q / ((ld)k * (ld)k);
        t1 *= q / ((ld)k * (ld)(k + 1));
        J0 += t0;
        J1 += t1;
        if (std::abs(t0) < 1e-30L * std::abs(J0) && std::abs(t1) < 1e-30L * std::abs(J1) && k > 10) break;
    }
}

std::vector<int> radix_factors(int n) {
    std::vector<int> f;
    while (n % 4 == 0) { f.push_back(4); n /= 4; }
    while (n % 2 == 0) { f.push_back(2); n /= 2; }
    while (n % 3 == 0) { f.push_back(3); n /= 3; }
    if (n != 1) f.clear();
    return f;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }


// ------------------------------------------------- per-mode operator caches
// Interior operators (nodes 0..nr-2, wall column removed) from B = D2 + D1/r:
//   Helmholtz H_n = I/dt - (1/(2Re)) (B - n^2/r^2 - a^2),  Poisson P_n = B - n^2/r^2 - a^2.
// Factored without pivoting into rows of 9 values: l[0..4] (multipliers of
// columns i-5..i-1), 1/u_ii, u[i][i+1..i+3]; computed in long double.
struct BandOp {
    int nr;
    const std::vector<double>* B;   // [2][nr][7]
    const std::vector<double>* r;
};
void factor_ld(const BandOp& o, int helm, int n, ld a2, ld re, ld dt, ld* LU) {
    const int nr = o.nr, n1 = nr - 1, pi = n & 1;
    const ld re2 = 0.5L / re, idt = 1.0L / dt, nn = (ld)n * (ld)n;
    ld Uw[5][4] = {};
    for (int i = 0; i < n1; ++i) {
        const int c0 = std::min(std::max(i - 3, 0), nr - 7);
        const ld ri = (*o.r)[i];
        ld a[9];
        for (int t = 0; t < 9; ++t) {
            const int c = i - 5 + t, w = c - c0;
            const ld v = (c >= 0 && c < n1 && w >= 0 && w < 7) ? (ld)(*o.B)[(pi * nr + i) * 7 + w] : 0.0L;
            a[t] = helm ? -re2 * v : v;
        }
        const ld dg = nn / (ri * ri) + a2;
        a[5] += helm ? (idt + re2 * dg) : -dg;
        for (int t = 0; t < 5; ++t) {
            ld l = 0.0L;
            if (i - 5 + t >= 0) {
                l = a[t] * Uw[t][0];
                for (int q = 1; q <= 3; ++q) a[t + q] -= l * Uw[t][q];
            }
            LU[i * 9 + t] = l;
        }
        const ld inv = 1.0L / a[5];
        LU[i * 9 + 5] = inv;
        LU[i * 9 + 6] = a[6]; LU[i * 9 + 7] = a[7]; LU[i * 9 + 8] = a[8];
        for (int t = 0; t < 4; ++t)
            for (int q = 0; q < 4; ++q) Uw[t][q] = Uw[t + 1][q];
        Uw[4][0] = inv; Uw[4][1] = a[6]; Uw[4][2] = a[7]; Uw[4][3] = a[8];
    }
}
void subst_ld(const ld* LU, int n1, ld* x) {
    for (int i = 0; i < n1; ++i)
        for (int t = 0; t < 5; ++t)
            if (i - 5 + t >= 0) x[i] -= LU[i * 9 + t] * x[i - 5 + t];
    for (int i = n1 - 1; i >= 0; --i) {
        ld v = x[i];
        for (int q = 1; q <= 3; ++q)
            if (i + q < n1) v -= LU[i * 9 + 5 + q] * x[i + q];
        x[i] = v * LU[i * 9 + 5];
    }
}

// --------------------------------------------------- binomial checkpointing
// T(l, s): minimal forward advances to reverse l steps from a stored start
// with s slots in total (Sec. 2.4 closed form).
long long beta(long long n, long long s) {   // C(n + s, n), saturating
    long double v = 1.0L;
    for (long long i = 1; i <= s; ++i) {
        v = v * (long double)(n + i) / (long double)i;
        if (v > 9e18L) return (long long)9e18;
    }
    return (long long)(v + 0.5L);
}
long long adv_cost(long long l, long long s) {
    if (l <= 1) return 0;
    if (s <= 1) return l * (l - 1) / 2;
    long long r = 0;
    while (beta(s, r) < l) ++r;
    return r * l - beta(s + 1, r - 1);
}
// argmin over m in [1, l-1] of m + T(l-m, s-1) + T(m, s); convex in m.
long long best_split(long long l, long long s) {
    auto f = [&](long long m) { return m + adv_cost(l - m, s - 1) + adv_cost(m, s); };
    long long lo = 1, hi = l - 1;
    while (lo < hi) {
        const long long mid = lo + (hi - lo) / 2;
        if (f(mid + 1) < f(mid)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

enum ActKind { A_RESTORE = 0, A_ADV = 1, A_STORE = 2, A_ADJ = 3 };
struct Act { int kind; long long a, b; };

void reverse_sched(long long start, long long end, int slot, std::vector<int>& freeslots, std::vector<Act>& acts) {
    const long long l = end - start;
    if (l == 1) {
        acts.push_back({A_RESTORE, slot, start});
        acts.push_back({A_ADJ, start, 0});
        return;
    }
    const long long s = 1 + (long long)freeslots.size();
    if (s == 1) {
        for (long long i = end - 1; i >= start; --i) {
            acts.push_back({A_RESTORE, slot, start});
            if (i > start) acts.push_back({A_ADV, i - start, 0});
            acts.push_back({A_ADJ, i, 0});
        }
        return;
    }
    const long long m = best_split(l, s);
    acts.push_back({A_RESTORE, slot, start});
    acts.push_back({A_ADV, m, 0});
    const int sl = freeslots.back();
    freeslots.pop_back();
    acts.push_back({A_STORE, sl, start + m});
    reverse_sched(start + m, end, sl, freeslots, acts);
    freeslots.push_back(sl);
    reverse_sched(start, start + m, slot, freeslots, acts);
}

std::vector<Act> schedule(long long nsteps, int nck) {
    std::vector<Act> acts;
    std::vector<int> freeslots;
    for (int s = nck - 1; s >= 1; --s) freeslots.push_back(s);
    reverse_sched(0, nsteps, 0, freeslots, acts);
    return acts;
}
size_t first_adj(const std::vector<Act>& acts) {
    for (size_t i = 0; i < acts.size(); ++i)
        if (acts[i].kind == A_ADJ) return i;
    return acts.size();
}

// -------------------------------------------------------------- step drivers
struct WsPtrs {
    double2 *aux0, *nn, *ns, *muC, *muP, *yb, *zb2, *fa, *fb, *fa2, *fb2, *cur, *lam, *tmp, *g, *trial, *trialN, *r0;
    double2* st[npo::NCORR_MAX];
    double2* auxs[npo::NCORR_MAX];
    double* red;
    long long* step;
};
WsPtrs wsptrs(const npo_plan_s& p, void* ws) {
    char* b = static_cast<char*>(ws);
    auto F = [&](size_t off) { return reinterpret_cast<double2*>(b + off); };
    WsPtrs w;
    w.aux0 = F(p.ws.aux0); w.nn = F(p.ws.nn); w.ns = F(p.ws.ns);
    for (int c = 0; c < npo::NCORR_MAX; ++c) { w.st[c] = F(p.ws.st[c]); w.auxs[c] = F(p.ws.auxs[c]); }
    w.muC = F(p.ws.muC); w.muP = F(p.ws.muP); w.yb = F(p.ws.yb); w.zb2 = F(p.ws.zb2); w.r0 = F(p.ws.r0);
    w.step = reinterpret_cast<long long*>(b + p.ws.step);
    w.fa = F(p.ws.fa); w.fb = F(p.ws.fb); w.fa2 = F(p.ws.fa2); w.fb2 = F(p.ws.fb2);
    w.cur = F(p.ws.cur); w.lam = F(p.ws.lam); w.tmp = F(p.ws.tmp); w.g = F(p.ws.g);
    w.trial = F(p.ws.trial); w.trialN = F(p.ws.trialN);
    w.red = reinterpret_cast<double*>(b + p.ws.red);
    return w;
}

// Evaluation time t0 + (n + off) dt, with n from the device step index when
// dstep is given (captured graphs) and by value otherwise.
npo::TimeArg at_step(const long long* dstep, long long n, int off, unsigned long long* cfl = nullptr) {
    return npo::TimeArg{dstep, n, off, 0, 0.0, cfl};
}

// The device maximum of the CFL monitor sits 64 bytes after the step index.
unsigned long long* cfl_slot(const WsPtrs& w) { return reinterpret_cast<unsigned long long*>(w.step) + 8; }

// An injected failure (npo_plan_inject_fault) of this step driver.
bool injected(const npo_plan_s& p, int site) {
    if (p.fault_site != site) return false;
    return p.fault_after-- == 0;
}

// u_out = Phi(u_n).  If have_aux, w.aux0 already holds the vorticity parts of u_n.
// Stages: w_0 = S(E u + N(u)), w_c = S(E u + (N(u) + N(w_{c-1}))/2), u_out = w_ncorr;
// the predictor leaves R0 = E u + N(u)/2, and each corrector solves S(R0 + N(w_{c-1})/2).

hipError_t fwd_step(const npo_plan_s& p, void* ws, const double2* un, double2* uout, long long n, bool have_aux,
                    hipStream_t st, const long long* dstep = nullptr) {
    if (injected(p, 1)) return hipErrorLaunchFailure;
    WsPtrs w = wsptrs(p, ws);
    hipError_t e;
    const npo::TimeArg t0 = at_step(dstep, n, 0, p.cfl_monitor ? cfl_slot(w) : nullptr), t1 = at_step(dstep, n, 1);
    if (!have_aux && (e = npo::launch_curl_aux(p, un, w.aux0, st)) != hipSuccess) return e;
    if ((e = npo::launch_nl(p, 0, un, w.aux0, nullptr, t0, w.nn, nullptr, ws, st)) != hipSuccess) return e;
    if ((e = npo::launch_solve(p, 1, un, w.nn, w.st[0], w.auxs[0], st, w.r0)) != hipSuccess) return e;
    for (int c = 1; c <= p.ncorr; ++c) {
        if ((e = npo::launch_nl(p, 0, w.st[c - 1], w.auxs[c - 1], nullptr, t1, w.ns, nullptr, ws, st)) != hipSuccess)
            return e;
        const bool last = c == p.ncorr;
        if ((e = npo::launch_solve(p, 2, w.r0, w.ns, last ? uout : w.st[c], last ? w.aux0 : w.auxs[c], st)) !=
            hipSuccess)
            return e;
    }
    return hipSuccess;
}

// lam_out = Phi'(u_n)^dag lam_in:
//   mu_C = S^+ lam; mu_{c-1} = S^+ (N'(w_{c-1})^+ mu_c / 2), c = C..1;
//   lam_n = E^+ (sum mu_c) + N'(u_n)^+ (mu_0 + sum_{c>=1} mu_c / 2).
hipError_t adj_step(const npo_plan_s& p, void* ws, const double2* un, const double2* lamin, double2* lamout,
                    long long n, hipStream_t st, const long long* dstep = nullptr, bool have_aux = false) {
    if (injected(p, 2)) return hipErrorLaunchFailure;
    WsPtrs w = wsptrs(p, ws);
    hipError_t e;
    const npo::TimeArg t0 = at_step(dstep, n, 0), t1 = at_step(dstep, n, 1);
    const int C = p.ncorr;
    // stage recompute; the forward evaluations leave the axial transforms of
    // u^n (zst[0]) and of w_{c-1} (zst[c]) for the adjoint evaluations
    char* wb = static_cast<char*>(ws);
    auto zst = [&](int c) { return reinterpret_cast<double2*>(wb + p.ws.zst[c]); };
    if (!have_aux && (e = npo::launch_curl_aux(p, un, w.aux0, st)) != hipSuccess) return e;
    if ((e = npo::launch_nl(p, 0, un, w.aux0, nullptr, t0, w.nn, nullptr, ws, st, nullptr, zst(0))) != hipSuccess)
        return e;
    if ((e = npo::launch_solve(p, 1, un, w.nn, w.st[0], w.auxs[0], st, C > 1 ? w.r0 : nullptr)) !=
        hipSuccess)
        return e;
    for (int c = 1; c < C; ++c) {
        if ((e = npo::launch_nl(p, 0, w.st[c - 1], w.auxs[c - 1], nullptr, t1, w.ns, nullptr, ws, st, nullptr,
                                zst(c))) != hipSuccess)
            return e;
        if ((e = npo::launch_solve(p, 2, w.r0, w.ns, w.st[c], w.auxs[c], st)) != hipSuccess) return e;
    }
    double2* mu[2] = {w.muC, w.muP};
    // mu_C = S^+ lam; the accumulator Z starts as mu_C, which the solve of
    // stage C reads straight from mu_C
    if ((e = npo::launch_solve_adj(p, lamin, 1.0, nullptr, 0.0, mu[C & 1], nullptr, 0.0, nullptr, nullptr, 0.0,
                                   nullptr, st)) != hipSuccess)
        return e;
    for (int c = C; c >= 1; --c) {
        // w_{c-1} was evaluated forward above for c < C
        const double2* pre = c < C ? zst(c) : nullptr;
        if ((e = npo::launch_nl(p, 1, w.st[c - 1], w.auxs[c - 1], mu[c & 1], t1, w.fa, w.fb, ws, st, pre)) !=
            hipSuccess)
            return e;
        // Z accumulates mu_c (c = C..0); Y = mu_0 + sum_{c>=1} mu_c / 2 equals
        // (Z + mu_0) / 2, so only the last pass forms it, as Z_in / 2 + mu_0
        const double2* Zin = c == C ? mu[C & 1] : w.zb2;
        if (c > 1)
            e = npo::launch_solve_adj(p, w.fa, 0.5, w.fb, 0.5, mu[(c - 1) & 1], nullptr, 0.0, nullptr, Zin, 1.0, w.zb2,
                                      st);
        else
            e = npo::launch_solve_adj(p, w.fa, 0.5, w.fb, 0.5, nullptr, Zin, 1.0, w.yb, Zin, 1.0, w.zb2, st, 0.5, 1.0);
        if (e != hipSuccess) return e;
    }
    if ((e = npo::launch_nl(p, 1, un, w.aux0, w.yb, t0, w.fa2, w.fb2, ws, st, zst(0))) != hipSuccess) return e;
    return npo::launch_final(p, w.zb2, w.fa2, w.fb2, lamout, st);
}

// One backward step of the continuous adjoint (the paper's adjoint equations,
// integrated backwards with the direct stepper): lam^{n+1} at t_{n+1} ->
// lam^n at t_n, with the direct fields u^n and u^{n+1} and the convective term
// Nc(u; y) = P_K F[Omega x Y] + curl P_K F[Y x V]:
//   v_0 = S(E lam + Nc(u^{n+1}, t_{n+1}; lam)),
//   v_c = S(E lam + (Nc(u^{n+1}, t_{n+1}; lam) + Nc(u^n, t_n; v_{c-1})) / 2),
//   lam^n = v_C.
// lamout may alias lamin (lam is read by the predictor only).
hipError_t adj_step_cont(const npo_plan_s& p, void* ws, const double2* un, const double2* unp1, const double2* lamin,
                         double2* lamout, long long n, hipStream_t st) {
    if (injected(p, 2)) return hipErrorLaunchFailure;
    WsPtrs w = wsptrs(p, ws);
    hipError_t e;
    const npo::TimeArg t0 = at_step(nullptr, n, 0), t1 = at_step(nullptr, n, 1);
    // vorticity parts: u^{n+1} into auxs[0], u^n into aux0
    if ((e = npo::launch_curl_aux(p, unp1, w.auxs[0], st)) != hipSuccess) return e;
    if ((e = npo::launch_curl_aux(p, un, w.aux0, st)) != hipSuccess) return e;
    if ((e = npo::launch_nl(p, 1, unp1, w.auxs[0], lamin, t1, w.fa, w.fb, ws, st)) != hipSuccess) return e;
    if ((e = npo::launch_curl_add(p, w.fa, w.fb, w.nn, st)) != hipSuccess) return e;
    if ((e = npo::launch_solve(p, 1, lamin, w.nn, p.ncorr > 0 ? w.st[0] : lamout, nullptr, st, w.r0)) != hipSuccess)
        return e;
    for (int c = 1; c <= p.ncorr; ++c) {
        if ((e = npo::launch_nl(p, 1, un, w.aux0, w.st[c - 1], t0, w.fa, w.fb, ws, st)) != hipSuccess) return e;
        if ((e = npo::launch_curl_add(p, w.fa, w.fb, w.ns, st)) != hipSuccess) return e;
        if ((e = npo::launch_solve(p, 2, w.r0, w.ns, c == p.ncorr ? lamout : w.st[c], nullptr, st)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------- captured step graphs
// The forward advance (cur -> cur, vorticity parts of cur present, then
// step += 1) and the adjoint step (lam -> lam at u = cur, vorticity parts of
// cur present) read their step index from the workspace, so one capture per
// workspace serves every step.
void drop_graphs(npo_plan_s& p) {
    if (p.g_fwd) (void)hipGraphExecDestroy(p.g_fwd);
    if (p.g_adj) (void)hipGraphExecDestroy(p.g_adj);
    p.g_fwd = p.g_adj = nullptr;
    p.graph_ws = nullptr;
}

hipError_t capture(npo_plan_s& p, void* ws, bool adjoint, hipGraphExec_t* exec) {
    WsPtrs w = wsptrs(p, ws);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(p.graph_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t e1 = adjoint ? adj_step(p, ws, w.cur, w.lam, w.lam, 0, p.graph_stream, w.step, true)
                            : fwd_step(p, ws, w.cur, w.cur, 0, true, p.graph_stream, w.step);
    if (e1 == hipSuccess && !adjoint) e1 = npo::launch_step_index(w.step, 1, 1, p.graph_stream);
    e = hipStreamEndCapture(p.graph_stream, &g);
    if (e == hipSuccess) e = e1;
    if (e == hipSuccess) e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

hipError_t build_graphs(npo_plan_s& p, void* ws) {
    drop_graphs(p);
    hipError_t e = hipSuccess;
    if (!p.graph_stream) e = hipStreamCreateWithFlags(&p.graph_stream, hipStreamNonBlocking);
    const bool prof = p.prof.on;
    p.prof.on = false;                    // no profiler events inside a graph
    if (e == hipSuccess) e = capture(p, ws, false, &p.g_fwd);
    if (e == hipSuccess) e = capture(p, ws, true, &p.g_adj);
    p.prof.on = prof;
    if (e != hipSuccess) {
        drop_graphs(p);
        return e;
    }
    p.graph_ws = ws;
    return hipSuccess;
}

npo_status check_plan(npo_plan p) {
    if (!p) return fail(NPO_EINVAL, "null plan");
    return NPO_OK;
}

}  // namespace


namespace npo {
void prof_begin(const npo_plan_s& p, int kid, hipStream_t st) {
    Profiler& f = p.prof;
    if (!f.on || recorder()) return;
    const long long n = f.launches[kid];
    if (n % f.stride == 0 && f.used[kid] < PROF_SLOTS)
        (void)hipEventRecord(f.ev[(kid * PROF_SLOTS + f.used[kid]) * 2], st);
}
void prof_end(const npo_plan_s& p, int kid, hipStream_t st) {
    Profiler& f = p.prof;
    if (!f.on || recorder()) return;
    const long long n = f.launches[kid]++;
    if (n % f.stride == 0 && f.used[kid] < PROF_SLOTS) {
        (void)hipEventRecord(f.ev[(kid * PROF_SLOTS + f.used[kid]) * 2 + 1], st);
        f.used[kid]++;
    }
}
}  // namespace npo

// ===================================================================== ABI
extern "C" {

const char* npo_last_error(void) { return g_err.c_str(); }

npo_status npo_plan_create(const npo_grid* grid, const npo_flow* flow, const npo_time* time, uint32_t flags,
                           npo_plan* out) {
    Trace trace_("npo_plan_create");
    g_err.clear();
    if (!grid || !flow || !time || !out) return fail(NPO_EINVAL, "null argument");
    if (flags != 0) return fail(NPO_EINVAL, "flags must be 0");
    const int nr = grid->nr, nt = grid->ntheta, nz = grid->nz;
    if (nr < 8 || nr > npo::NR_MAX) return fail(NPO_EUNSUPPORTED, "nr must be in [8, 64]");
    if (nt < 6 || nt > 128 || radix_factors(nt).empty()) return fail(NPO_EUNSUPPORTED, "ntheta must be 2^a 3^b in [6,128]");
    if (nz < 6 || nz > 2048 || nz % 2 || radix_factors(nz).empty())
        return fail(NPO_EUNSUPPORTED, "nz must be even and 2^a 3^b in [6,2048]");
    if (!(grid->lz > 0) || !(flow->re > 0) || !(flow->wo > 0) || !(time->dt > 0) || time->nsteps < 1)
        return fail(NPO_EINVAL, "lz, re, wo, dt must be positive and nsteps >= 1");
    if (flow->amp < 0) return fail(NPO_EINVAL, "amp must be >= 0");
    if (time->ncorr < 1 || time->ncorr > npo::NCORR_MAX) return fail(NPO_EINVAL, "ncorr must be in [1, 3]");

    auto* p = new npo_plan_s();
    p->nr = nr; p->nt = nt; p->nz = nz;
    p->M = (nt - 1) / 3; p->K = (nz - 1) / 3; p->nk = 2 * p->K + 1; p->mp1 = p->M + 1;
    p->lz = grid->lz; p->k0 = 2.0 * M_PI / grid->lz;
    p->re = flow->re; p->wo = flow->wo; p->amp = flow->amp;
    p->dt = time->dt; p->t0 = time->t0; p->nsteps = time->nsteps; p->ncorr = time->ncorr;
    p->omega = flow->wo * flow->wo / flow->re;
    (void)hipGetDevice(&p->device);
    // once per device: the address of the fixed workspace of the no-allocation
    // forward step (a failure is reported by that entry point, not here)
    (void)npo::scratch_setup(p->device);

    // radial tables
    std::vector<ld> r = radial_nodes(nr);
    std::vector<ld> w = quad_weights(r);
    p->r.resize(nr); p->w.resize(nr);
    for (int j = 0; j < nr; ++j) { p->r[j] = (double)r[j]; p->w[j] = (double)w[j]; }
    p->col0.resize(nr);
    p->D1.assign(2 * nr * 7, 0.0);
    p->D2.assign(2 * nr * 7, 0.0);
    for (int j = 0; j < nr; ++j) {
        const int c0 = std::min(std::max(j - 3, 0), nr - 7);
        p->col0[j] = c0;
        // stencil nodes in the mirrored numbering
        int cols[7];
        if (j >= nr - 3) for (int t = 0; t < 7; ++t) cols[t] = nr - 7 + t;
        else for (int t = 0; t < 7; ++t) cols[t] = j - 3 + t;
        ld xs[7];
        for (int t = 0; t < 7; ++t) xs[t] = cols[t] >= 0 ? r[cols[t]] : -r[-cols[t] - 1];
        ld c[3][7];
        fornberg(r[j], xs, 7, c);
        for (int pi = 0; pi < 2; ++pi) {
            const ld par = pi == 0 ? 1.0L : -1.0L;
            ld a1[7] = {0}, a2[7] = {0};
            for (int t = 0; t < 7; ++t) {
                const int cc = cols[t] >= 0 ? cols[t] : -cols[t] - 1;
                const ld s = cols[t] >= 0 ? 1.0L : par;
                a1[cc - c0] += s * c[1][t];
                a2[cc - c0] += s * c[2][t];
            }
            for (int t = 0; t < 7; ++t) {
                p->D1[(pi * nr + j) * 7 + t] = (double)a1[t];
                p->D2[(pi * nr + j) * 7 + t] = (double)a2[t];
            }
        }
    }
    // Womersley profile: Ut = b [1 - J0(k r)/J0(k)] / [1 - 2 J1(k)/(k J0(k))], k = Wo e^{3 i pi/4}, b = -i A/2
    p->ut_re.assign(nr, 0.0); p->ut_im.assign(nr, 0.0); p->dut_re.assign(nr, 0.0); p->dut_im.assign(nr, 0.0);
    if (flow->amp != 0.0) {
        const ld pi = acosl(-1.0L);
        const std::complex<ld> kap = (ld)flow->wo * std::polar(1.0L, 0.75L * pi);
        const std::complex<ld> b(0.0L, -0.5L * (ld)flow->amp);
        std::complex<ld> J0k, J1k;
        bessel01(kap, J0k, J1k);
        const std::complex<ld> den = 1.0L - 2.0L * J1k / (kap * J0k);
        for (int j = 0; j < nr; ++j) {
            std::complex<ld> J0r, J1r;
            bessel01(kap * r[j], J0r, J1r);
            const std::complex<ld> ut = b * (1.0L - J0r / J0k) / den;
            const std::complex<ld> dut = b * kap * J1r / J0k / den;
            p->ut_re[j] = (double)ut.real(); p->ut_im[j] = (double)ut.imag();
            p->dut_re[j] = (double)dut.real(); p->dut_im[j] = (double)dut.imag();
        }
    }
    // FFT factors
    std::vector<int> fz = radix_factors(nz), ft = radix_factors(nt);
    if ((int)fz.size() > npo::NFAC_MAX || (int)ft.size() > npo::NFAC_MAX) {
        delete p;
        return fail(NPO_EUNSUPPORTED, "too many FFT factors");
    }
    // device tables: r, w, D1, D2, B (doubles), their transposed 13-tap forms,
    // Ut, dUt, twz, twt (double2), col0 (int)
    const size_t nd = nr + nr + 3 * (2 * nr * 7) + 3 * (2 * nr * npo::TAPS);
    const size_t nc = nr + nr + nz + nt;
    const size_t bytes = align256(nd * 8) + align256(nc * 16) + align256(nr * 4);
    if (hipMalloc(&p->d_tables, bytes) != hipSuccess) {
        delete p;
        return fail(NPO_ENOMEM, "hipMalloc of plan tables failed");
    }
    std::vector<char> host(bytes, 0);
    double* hd = reinterpret_cast<double*>(host.data());
    size_t o = 0;
    std::memcpy(hd + o, p->r.data(), nr * 8); const size_t o_r = o; o += nr;
    std::memcpy(hd + o, p->w.data(), nr * 8); const size_t o_w = o; o += nr;
    std::memcpy(hd + o, p->D1.data(), 2 * nr * 7 * 8); const size_t o_d1 = o; o += 2 * nr * 7;
    std::memcpy(hd + o, p->D2.data(), 2 * nr * 7 * 8); const size_t o_d2 = o; o += 2 * nr * 7;
    const size_t o_b = o;
    for (int pi = 0; pi < 2; ++pi)
        for (int j = 0; j < nr; ++j)
            for (int t = 0; t < 7; ++t)
                hd[o_b + (pi * nr + j) * 7 + t] = p->D2[(pi * nr + j) * 7 + t] + p->D1[(pi * nr + j) * 7 + t] / p->r[j];
    o += 2 * nr * 7;
    // transposed stencils: entry s of column j is the weight of row i = j - 6 + s
    // (zero where row i's stencil does not reach j); D1T plain, D1WT and BWT
    // with the row's quadrature weight w_i folded in.
    const size_t o_d1t = o, o_d1wt = o + 2 * nr * npo::TAPS, o_bwt = o + 4 * nr * npo::TAPS;
    for (int pi = 0; pi < 2; ++pi)
        for (int j = 0; j < nr; ++j)
            for (int s = 0; s < npo::TAPS; ++s) {
                const int i = j - 6 + s;
                double d1 = 0.0, bb = 0.0;
                if (i >= 0 && i < nr) {
                    const int t = j - p->col0[i];
                    if (t >= 0 && t < 7) {
                        d1 = p->D1[(pi * nr + i) * 7 + t];
                        bb = hd[o_b + (pi * nr + i) * 7 + t];
                    }
                }
                const size_t e = (size_t)(pi * nr + j) * npo::TAPS + s;
                hd[o_d1t + e] = d1;
                hd[o_d1wt + e] = (i >= 0 && i < nr) ? d1 * p->w[i] : 0.0;
                hd[o_bwt + e] = (i >= 0 && i < nr) ? bb * p->w[i] : 0.0;
            }
    o += 6 * nr * npo::TAPS;
    const size_t cbase = align256(nd * 8);
    double2* hc = reinterpret_cast<double2*>(host.data() + cbase);
    const ld pi = acosl(-1.0L);
    for (int j = 0; j < nr; ++j) {
        hc[j] = make_double2(p->ut_re[j], p->ut_im[j]);
        hc[nr + j] = make_double2(p->dut_re[j], p->dut_im[j]);
    }
    for (int t = 0; t < nz; ++t) hc[2 * nr + t] = make_double2((double)cosl(2 * pi * t / nz), (double)-sinl(2 * pi * t / nz));
    for (int t = 0; t < nt; ++t)
        hc[2 * nr + nz + t] = make_double2((double)cosl(2 * pi * t / nt), (double)-sinl(2 * pi * t / nt));
    const size_t ibase = cbase + align256(nc * 16);
    std::memcpy(host.data() + ibase, p->col0.data(), nr * 4);
    if (hipMemcpy(p->d_tables, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(p->d_tables);
        delete p;
        return fail(NPO_EHIP, "upload of plan tables failed");
    }
    const double* dd = reinterpret_cast<const double*>(p->d_tables);
    const double2* dc = reinterpret_cast<const double2*>(reinterpret_cast<const char*>(p->d_tables) + cbase);
    npo::KP& kp = p->kp;
    kp.nr = nr; kp.nt = nt; kp.nz = nz; kp.M = p->M; kp.K = p->K; kp.nk = p->nk; kp.mp1 = p->mp1;
    kp.k0 = p->k0; kp.re = p->re; kp.dt = p->dt; kp.lz = p->lz; kp.t0 = p->t0; kp.omega = p->omega;
    kp.r = dd + o_r; kp.w = dd + o_w; kp.D1 = dd + o_d1; kp.D2 = dd + o_d2; kp.B = dd + o_b;
    kp.D1T = dd + o_d1t; kp.D1WT = dd + o_d1wt; kp.BWT = dd + o_bwt;
    kp.col0 = reinterpret_cast<const int*>(reinterpret_cast<const char*>(p->d_tables) + ibase);
    kp.Ut = dc; kp.dUt = dc + nr; kp.twz = dc + 2 * nr; kp.twt = dc + 2 * nr + nz;
    kp.nfz = (int)fz.size(); kp.nft = (int)ft.size();
    for (int i = 0; i < npo::NFAC_MAX; ++i) {
        kp.fz[i] = i < kp.nfz ? fz[i] : 1;
        kp.ft[i] = i < kp.nft ? ft[i] : 1;
    }

    // per-mode operator caches: Helmholtz factors for n = 0..M+1, Poisson
    // factors for m = 0..M, and the homogeneous (influence) solutions
    {
        const int n1 = nr - 1, M = p->M, K = p->K;
        std::vector<double> Btab(2 * nr * 7);
        for (int pi = 0; pi < 2; ++pi)
            for (int j = 0; j < nr; ++j)
                for (int t = 0; t < 7; ++t)
                    Btab[(pi * nr + j) * 7 + t] = p->D2[(pi * nr + j) * 7 + t] + p->D1[(pi * nr + j) * 7 + t] / p->r[j];
        BandOp bo{nr, &Btab, &p->r};
        const size_t opsz = (size_t)n1 * 9;
        const size_t homsz = (size_t)3 * nr + 1;
        std::vector<double> hlu((size_t)(K + 1) * (M + 2) * opsz), plu((size_t)(K + 1) * (M + 1) * opsz);
        std::vector<double> hom((size_t)(K + 1) * (M + 1) * homsz, 0.0);
        std::vector<ld> LUh((size_t)(M + 2) * opsz), LUp(opsz), x(nr), y(nr), z(nr), ph(nr);
        for (int ka = 0; ka <= K; ++ka) {
            const ld al = (ld)ka * (2.0L * acosl(-1.0L) / (ld)p->lz);
            const ld a2 = al * al;
            for (int n = 0; n <= M + 1; ++n) {
                factor_ld(bo, 1, n, a2, p->re, p->dt, &LUh[n * opsz]);
                for (size_t e = 0; e < opsz; ++e) hlu[((size_t)ka * (M + 2) + n) * opsz + e] = (double)LUh[n * opsz + e];
            }
            for (int m = 0; m <= M; ++m) {
                double* hm = &hom[((size_t)ka * (M + 1) + m) * homsz];
                factor_ld(bo, 0, m, a2, p->re, p->dt, LUp.data());
                for (size_t e = 0; e < opsz; ++e) plu[((size_t)ka * (M + 1) + m) * opsz + e] = (double)LUp[e];
                if (m == 0 && ka == 0) {
                    // mean mode: g = H_0^{-1} 1 and sum_i w_i g_i
                    for (int i = 0; i < n1; ++i) x[i] = 1.0L;
                    subst_ld(&LUh[0], n1, x.data());
                    ld wg = 0.0L;
                    for (int i = 0; i < n1; ++i) { hm[i] = (double)x[i]; wg += (ld)p->w[i] * x[i]; }
                    hm[3 * nr] = (double)wg;
                    continue;
                }
                const int pe = m & 1, po = (m + 1) & 1;
                for (int i = 0; i < n1; ++i) {
                    const int w = n1 - p->col0[i];
                    ph[i] = (w >= 0 && w < 7) ? -(ld)Btab[(pe * nr + i) * 7 + w] : 0.0L;
                }
                subst_ld(LUp.data(), n1, ph.data());
                ph[n1] = 1.0L;
                for (int i = 0; i < n1; ++i) {
                    ld d = 0.0L;
                    for (int t = 0; t < 7; ++t) d += (ld)p->D1[(pe * nr + i) * 7 + t] * ph[p->col0[i] + t];
                    const ld mr = (ld)m / (ld)p->r[i];
                    x[i] = -(d - mr * ph[i]);
                    y[i] = -(d + mr * ph[i]);
                    z[i] = -ph[i];
                }
                subst_ld(&LUh[(m + 1) * opsz], n1, x.data());
                subst_ld(&LUh[std::abs(m - 1) * opsz], n1, y.data());
                subst_ld(&LUh[m * opsz], n1, z.data());
                ld sh = 0.0L;
                const int cw = p->col0[n1];
                for (int t = 0; t < 7; ++t)
                    if (cw + t < n1) sh += (ld)p->D1[(po * nr + n1) * 7 + t] * (x[cw + t] + y[cw + t]);
                for (int i = 0; i < n1; ++i) {
                    hm[i] = (double)x[i];
                    hm[nr + i] = (double)y[i];
                    hm[2 * nr + i] = (double)z[i];
                }
                hm[3 * nr] = (double)sh;
            }
        }
        const size_t cbytes = (hlu.size() + plu.size() + hom.size()) * 8;
        if (hipMalloc(&p->d_cache, cbytes) != hipSuccess) {
            (void)hipFree(p->d_tables);
            delete p;
            return fail(NPO_ENOMEM, "hipMalloc of operator caches failed");
        }
        double* dcache = p->d_cache;
        if (hipMemcpy(dcache, hlu.data(), hlu.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(dcache + hlu.size(), plu.data(), plu.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(dcache + hlu.size() + plu.size(), hom.data(), hom.size() * 8, hipMemcpyHostToDevice) !=
                hipSuccess) {
            (void)hipFree(p->d_cache);
            (void)hipFree(p->d_tables);
            delete p;
            return fail(NPO_EHIP, "upload of operator caches failed");
        }
        p->kp.HLU = dcache;
        p->kp.PLU = dcache + hlu.size();
        p->kp.HOM = dcache + hlu.size() + plu.size();
        p->cache_bytes = cbytes;
    }
    // launch shapes: LDS budget 64 KiB per block for the FFT kernels
    const size_t lds = 64 * 1024;
    if (npo::zpass_lds(*p, 1) > 160 * 1024) {
        (void)hipFree(p->d_cache);
        (void)hipFree(p->d_tables);
        delete p;
        return fail(NPO_EUNSUPPORTED, "nz too large for one LDS-resident axial transform");
    }
    p->zgroup = 1;
    for (int g : {3, 2, 1})
        if (npo::zpass_lds(*p, g) <= lds) { p->zgroup = g; break; }
    p->zb_theta_fwd = p->zb_theta_adj = 2;
    for (int ZB : {8, 4, 2}) {
        if (nz % ZB == 0 && npo::theta_lds(*p, ZB, 0) <= lds) { p->zb_theta_fwd = ZB; break; }
    }
    for (int ZB : {8, 4, 2}) {
        if (nz % ZB == 0 && npo::theta_lds(*p, ZB, 1) <= lds) { p->zb_theta_adj = ZB; break; }
    }
    // workspace layout
    const size_t fb = (size_t)3 * nr * p->mp1 * p->nk * 16;
    const size_t f2 = (size_t)2 * nr * p->mp1 * p->nk * 16;
    const size_t gb = (size_t)nr * p->mp1 * nz * 16;
    size_t off = 0;
    auto take = [&](size_t n) { size_t at = off; off += align256(n); return at; };
    npo::WsLayout& L = p->ws;
    L.aux0 = take(f2);
    for (int c = 0; c < npo::NCORR_MAX; ++c) { L.auxs[c] = take(f2); L.st[c] = take(fb); }
    L.nn = take(fb); L.ns = take(fb);
    L.muC = take(fb); L.muP = take(fb); L.yb = take(fb); L.zb2 = take(fb); L.r0 = take(fb);
    L.fa = take(fb); L.fb = take(fb); L.fa2 = take(fb); L.fb2 = take(fb);
    L.cur = take(fb); L.lam = take(fb); L.tmp = take(fb); L.g = take(fb);
    L.trial = take(fb); L.trialN = take(fb);
    L.zbuf = take(9 * gb); L.tbuf = take(6 * gb);
    for (int c = 0; c < npo::NCORR_MAX; ++c) L.zst[c] = c < p->ncorr ? take(6 * gb) : 0;
    L.red = take((npo::NR_MAX * 4 + 512 + 5 * 256) * 8);   // reductions, scalars, diagnostics partials
    L.step = take(256);
    L.total = off;
    *out = p;
    return NPO_OK;
}

npo_status npo_plan_destroy(npo_plan p) {
    if (!p) return NPO_OK;
    drop_graphs(*p);
    if (p->graph_stream) (void)hipStreamDestroy(p->graph_stream);
    if (p->d_tables) (void)hipFree(p->d_tables);
    if (p->d_cache) (void)hipFree(p->d_cache);
    delete p;
    return NPO_OK;
}

npo_status npo_plan_info(npo_plan p, npo_info* out) {
    if (check_plan(p) || !out) return fail(NPO_EINVAL, "null argument");
    out->nr = p->nr; out->ntheta = p->nt; out->nz = p->nz; out->M = p->M; out->K = p->K; out->nk = p->nk;
    out->field_elems = (int64_t)3 * p->nr * p->mp1 * p->nk;
    out->field_bytes = out->field_elems * 16;
    out->workspace_bytes = (int64_t)p->ws.total;
    out->scalars_bytes = 256;
    out->period = 2.0 * M_PI * p->re / (p->wo * p->wo);
    out->k0 = p->k0; out->dt = p->dt; out->t0 = p->t0; out->nsteps = p->nsteps;
    return NPO_OK;
}

npo_status npo_plan_tables(npo_plan p, double* r, double* w, double* D1, double* D2, int32_t* col0) {
    if (check_plan(p)) return NPO_EINVAL;
    if (r) std::memcpy(r, p->r.data(), p->nr * 8);
    if (w) std::memcpy(w, p->w.data(), p->nr * 8);
    if (D1) std::memcpy(D1, p->D1.data(), p->D1.size() * 8);
    if (D2) std::memcpy(D2, p->D2.data(), p->D2.size() * 8);
    if (col0) for (int j = 0; j < p->nr; ++j) col0[j] = p->col0[j];
    return NPO_OK;
}


#define ST(s) reinterpret_cast<hipStream_t>(s)
#define CF(x) reinterpret_cast<const double2*>(x)
#define F(x) reinterpret_cast<double2*>(x)

npo_status npo_base_flow(npo_plan p, double t, double* U_dev, double* dUdr_dev, void* stream) {
    if (check_plan(p) || !U_dev || !dUdr_dev) return fail(NPO_EINVAL, "null argument");
    if (!std::isfinite(t)) return fail(NPO_EINVAL, "t must be finite");
    HIPCHK(npo::launch_base_flow(*p, t, U_dev, dUdr_dev, ST(stream)));
    return NPO_OK;
}

npo_status npo_nonlinear(npo_plan p, void* ws, const void* u, double t, void* out, void* stream) {
    if (check_plan(p) || !ws || !u || !out) return fail(NPO_EINVAL, "null argument");
    WsPtrs w = wsptrs(*p, ws);
    HIPCHK(npo::launch_curl_aux(*p, CF(u), w.aux0, ST(stream)));
    HIPCHK(npo::launch_nl(*p, 0, CF(u), w.aux0, nullptr, npo::TimeArg{nullptr, 0, 0, 1, t, nullptr}, F(out), nullptr, ws,
                          ST(stream)));
    return NPO_OK;
}

npo_status npo_nonlinear_adj(npo_plan p, void* ws, const void* u, double t, const void* y, void* out, void* stream) {
    if (check_plan(p) || !ws || !u || !y || !out) return fail(NPO_EINVAL, "null argument");
    WsPtrs w = wsptrs(*p, ws);
    HIPCHK(npo::launch_curl_aux(*p, CF(u), w.aux0, ST(stream)));
    HIPCHK(npo::launch_nl(*p, 1, CF(u), w.aux0, CF(y), npo::TimeArg{nullptr, 0, 0, 1, t, nullptr}, w.fa, w.fb, ws,
                          ST(stream)));
    HIPCHK(npo::launch_final(*p, nullptr, w.fa, w.fb, F(out), ST(stream)));
    return NPO_OK;
}

npo_status npo_nonlinear_adj_cont(npo_plan p, void* ws, const void* u, double t, const void* y, void* out,
                                  void* stream) {
    if (check_plan(p) || !ws || !u || !y || !out) return fail(NPO_EINVAL, "null argument");
    if (!std::isfinite(t)) return fail(NPO_EINVAL, "t must be finite");
    WsPtrs w = wsptrs(*p, ws);
    HIPCHK(npo::launch_curl_aux(*p, CF(u), w.aux0, ST(stream)));
    HIPCHK(npo::launch_nl(*p, 1, CF(u), w.aux0, CF(y), npo::TimeArg{nullptr, 0, 0, 1, t, nullptr}, w.fa, w.fb, ws,
                          ST(stream)));
    HIPCHK(npo::launch_curl_add(*p, w.fa, w.fb, F(out), ST(stream)));
    return NPO_OK;
}

npo_status npo_adjoint_step_cont(npo_plan p, void* ws, const void* un, const void* unp1, const void* lam_in,
                                 void* lam_out, int64_t n, void* stream) {
    if (check_plan(p) || !ws || !un || !unp1 || !lam_in || !lam_out) return fail(NPO_EINVAL, "null argument");
    if (n < 0) return fail(NPO_EINVAL, "n must be >= 0");
    HIPCHK(adj_step_cont(*p, ws, CF(un), CF(unp1), CF(lam_in), F(lam_out), n, ST(stream)));
    return NPO_OK;
}

npo_status npo_plan_set_adjoint(npo_plan p, int32_t kind) {
    if (check_plan(p)) return NPO_EINVAL;
    if (kind != 0 && kind != 1) return fail(NPO_EINVAL, "kind must be 0 (discrete) or 1 (continuous)");
    p->adjoint_kind = kind;
    drop_graphs(*p);
    return NPO_OK;
}

npo_status npo_solve(npo_plan p, void* ws, const void* R, void* out, void* stream) {
    if (check_plan(p) || !R || !out) return fail(NPO_EINVAL, "null argument");
    (void)ws;
    HIPCHK(npo::launch_solve(*p, 0, CF(R), nullptr, F(out), nullptr, ST(stream)));
    return NPO_OK;
}

npo_status npo_solve_adj(npo_plan p, void* ws, const void* y, void* out, void* stream) {
    if (check_plan(p) || !y || !out) return fail(NPO_EINVAL, "null argument");
    (void)ws;
    HIPCHK(npo::launch_solve_adj(*p, CF(y), 1.0, nullptr, 0.0, F(out), nullptr, 0.0, nullptr, nullptr, 0.0, nullptr,
                                 ST(stream)));
    return NPO_OK;
}

npo_status npo_forward_step(npo_plan p, void* ws, const void* un, void* unp1, int64_t n, void* stream) {
    if (check_plan(p) || !ws || !un || !unp1) return fail(NPO_EINVAL, "null argument");
    HIPCHK(fwd_step(*p, ws, CF(un), F(unp1), n, false, ST(stream)));
    return NPO_OK;
}

npo_status npo_forward_step_noalloc(npo_plan p, const void* un, void* unp1, int64_t n, void* stream) {
    if (check_plan(p) || !un || !unp1) return fail(NPO_EINVAL, "null argument");
    if (p->ws.total > (size_t)NPO_SCRATCH_BYTES)
        return fail(NPO_EINVAL, "npo_forward_step_noalloc: this grid needs " + std::to_string(p->ws.total) +
                                    " workspace bytes, the fixed scratch holds " +
                                    std::to_string((long long)NPO_SCRATCH_BYTES) + "; use npo_forward_step");
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != p->device) return fail(NPO_EINVAL, "npo_forward_step_noalloc: current device is not the plan's");
    hipError_t se = hipSuccess;
    void* ws = npo::scratch_ptr(dev, &se);
    if (!ws) return hipfail(se, "npo_forward_step_noalloc: device address of the fixed scratch");
    HIPCHK(fwd_step(*p, ws, CF(un), F(unp1), n, false, ST(stream)));
    return NPO_OK;
}

npo_status npo_adjoint_step(npo_plan p, void* ws, const void* un, const void* lnp1, void* ln, int64_t n,
                            void* stream) {
    if (check_plan(p) || !ws || !un || !lnp1 || !ln) return fail(NPO_EINVAL, "null argument");
    HIPCHK(adj_step(*p, ws, CF(un), CF(lnp1), F(ln), n, ST(stream)));
    return NPO_OK;
}

npo_status npo_ckpt_count(int64_t nsteps, int32_t n_ckpt, int64_t* n_recompute) {
    if (nsteps < 1 || n_ckpt < 1 || !n_recompute) return fail(NPO_EINVAL, "bad argument");
    std::vector<Act> acts = schedule(nsteps, n_ckpt);
    int64_t c = 0;
    for (size_t i = first_adj(acts); i < acts.size(); ++i)
        if (acts[i].kind == A_ADV) c += acts[i].a;
    *n_recompute = c;
    return NPO_OK;
}

// Diagnostics partials sit after the reduction partials and scalars.
static double* diag_partial(const WsPtrs& w) { return w.red + npo::NR_MAX * 4 + 512; }

// The forward sweep; with hist, the energy diagnostics of u^n are written to
// row n / stride of hist (5 doubles a row) for n = 0, stride, 2 stride, ... < N,
// and those of u^N to row (N - 1) / stride + 1.
// The sweep covers steps n0 .. n0 + nseg - 1 of the plan's horizon (the whole
// horizon for the exported runs, one interval of the hybrid tier otherwise);
// with last_step false the final step (whose result only the forward output
// needs) is skipped.
static npo_status forward_run(npo_plan p, void* ws, void* ckpt, int32_t nck, const void* u0, void* uN,
                              double* hist, int32_t stride, void* stream, long long n0 = 0, long long nseg = -1,
                              bool last_step = true) {
    if (check_plan(p) || !ws || !ckpt || !u0 || (!uN && last_step)) return fail(NPO_EINVAL, "null argument");
    if (nck < 1) return fail(NPO_EINVAL, "n_ckpt must be >= 1");
    if (nseg < 0) nseg = p->nsteps;
    const hipStream_t st = ST(stream);
    const size_t fb = (size_t)3 * p->nr * p->mp1 * p->nk * 16;
    WsPtrs w = wsptrs(*p, ws);
    auto slot = [&](long long s) { return reinterpret_cast<double2*>(static_cast<char*>(ckpt) + s * fb); };
    std::vector<Act> acts = schedule(nseg, nck);
    const size_t fa = first_adj(acts);
    const bool gr = p->use_graphs && !p->prof.on;
    if (gr && p->graph_ws != ws) HIPCHK(build_graphs(*p, ws));
    // Slot 0 holds u0.  The state lives at `where` (a slot or cur): a step
    // whose result the schedule stores next writes it straight into the slot,
    // and the step after reads it from there, so states are not copied between
    // buffers.
    HIPCHK(hipMemcpyAsync(slot(0), u0, fb, hipMemcpyDeviceToDevice, st));
    const double2* where = slot(0);
    long long pos = 0;
    auto record = [&](const double2* u, long long n) -> hipError_t {
        if (!hist || n0 != 0 || nseg != p->nsteps) return hipSuccess;
        if (n != p->nsteps && n % stride) return hipSuccess;
        const long long row = n == p->nsteps ? (p->nsteps - 1) / stride + 1 : n / stride;
        return npo::launch_diag(*p, u, diag_partial(w), hist + 5 * row, nullptr, st);
    };
    HIPCHK(record(where, 0));
    bool aux = false, synced = false;   // synced: the device step index equals pos
    for (size_t i = 0; i < fa; ++i) {
        const Act& a = acts[i];
        if (a.kind == A_ADV) {
            for (long long k = 0; k < a.a; ++k) {
                double2* out = w.cur;
                if (k + 1 == a.a && i + 1 < fa && acts[i + 1].kind == A_STORE) out = slot(acts[i + 1].a);
                if (gr && aux && where == w.cur && out == w.cur) {
                    if (!synced) HIPCHK(npo::launch_step_index(w.step, n0 + pos, 0, st));
                    HIPCHK(hipGraphLaunch(p->g_fwd, st));
                    synced = true;
                } else {
                    HIPCHK(fwd_step(*p, ws, where, out, n0 + pos, aux, st));
                    synced = false;
                }
                where = out;
                aux = true;
                ++pos;
                HIPCHK(record(where, pos));
            }
        } else if (a.kind == A_STORE) {
            if (a.b != pos) return fail(NPO_ESTATE, "schedule store position mismatch");
            if (where != slot(a.a)) HIPCHK(hipMemcpyAsync(slot(a.a), where, fb, hipMemcpyDeviceToDevice, st));
            where = slot(a.a);
        }
    }
    if (pos != nseg - 1) return fail(NPO_ESTATE, "schedule descent did not reach the last step");
    // u^{N-1} is left in cur for the first adjoint step; the last step goes to uN
    if (where != w.cur) HIPCHK(hipMemcpyAsync(w.cur, where, fb, hipMemcpyDeviceToDevice, st));
    if (!last_step) return NPO_OK;
    HIPCHK(fwd_step(*p, ws, w.cur, F(uN), n0 + pos, aux, st));
    HIPCHK(record(CF(uN), p->nsteps));
    return NPO_OK;
}

npo_status npo_forward_run(npo_plan p, void* ws, void* ckpt, int32_t nck, const void* u0, void* uN, void* stream) {
    Trace trace_("npo_forward_run");
    return forward_run(p, ws, ckpt, nck, u0, uN, nullptr, 1, stream);
}

npo_status npo_forward_run_diag(npo_plan p, void* ws, void* ckpt, int32_t nck, const void* u0, void* uN,
                                double* hist_dev, int32_t stride, void* stream) {
    if (!hist_dev || stride < 1) return fail(NPO_EINVAL, "hist_dev must be given and stride >= 1");
    return forward_run(p, ws, ckpt, nck, u0, uN, hist_dev, stride, stream);
}

npo_status npo_energy_diag(npo_plan p, void* ws, const void* u, double* out_dev, double* spec_dev, void* stream) {
    if (check_plan(p) || !ws || !u || !out_dev) return fail(NPO_EINVAL, "null argument");
    WsPtrs w = wsptrs(*p, ws);
    HIPCHK(npo::launch_diag(*p, CF(u), diag_partial(w), out_dev, spec_dev, ST(stream)));
    return NPO_OK;
}

static npo_status adjoint_run(npo_plan p, void* ws, void* ckpt, int32_t nck, const void* lamN, void* lam0,
                              int64_t* n_recompute, void* stream, long long n0 = 0, long long nseg = -1) {
    if (check_plan(p) || !ws || !ckpt || !lamN || !lam0) return fail(NPO_EINVAL, "null argument");
    if (nck < 1) return fail(NPO_EINVAL, "n_ckpt must be >= 1");
    if (nseg < 0) nseg = p->nsteps;
    const hipStream_t st = ST(stream);
    const size_t fb = (size_t)3 * p->nr * p->mp1 * p->nk * 16;
    WsPtrs w = wsptrs(*p, ws);
    auto slot = [&](long long s) { return reinterpret_cast<double2*>(static_cast<char*>(ckpt) + s * fb); };
    std::vector<Act> acts = schedule(nseg, nck);
    const bool gr = p->use_graphs && !p->prof.on;
    if (gr && p->graph_ws != ws) HIPCHK(build_graphs(*p, ws));
    HIPCHK(hipMemcpyAsync(w.lam, lamN, fb, hipMemcpyDeviceToDevice, st));
    // the state lives at `where` (cur or a slot), as in the forward sweep: a
    // restore only points at its slot
    const double2* where = w.cur;
    long long pos = nseg - 1, adv = 0;
    bool aux = false, synced = false;   // synced: the device step index equals pos
    // continuous adjoint: w.tmp holds u^{pos+1} (the state of the step after
    // this one), made by one forward step for the first step of the segment
    const bool cont = p->adjoint_kind == 1;
    bool have_next = false;
    for (size_t i = first_adj(acts); i < acts.size(); ++i) {
        const Act& a = acts[i];
        if (a.kind == A_RESTORE) {
            where = slot(a.a);
            pos = a.b;
            aux = false;
            synced = false;
        } else if (a.kind == A_ADV) {
            for (long long k = 0; k < a.a; ++k) {
                double2* out = w.cur;
                if (k + 1 == a.a && i + 1 < acts.size() && acts[i + 1].kind == A_STORE) out = slot(acts[i + 1].a);
                if (gr && aux && where == w.cur && out == w.cur) {
                    if (!synced) HIPCHK(npo::launch_step_index(w.step, n0 + pos, 0, st));
                    HIPCHK(hipGraphLaunch(p->g_fwd, st));
                    synced = true;
                } else {
                    HIPCHK(fwd_step(*p, ws, where, out, n0 + pos, aux, st));
                    synced = false;
                }
                where = out;
                aux = true;
                ++pos;
            }
            adv += a.a;
        } else if (a.kind == A_STORE) {
            if (a.b != pos) return fail(NPO_ESTATE, "schedule store position mismatch");
            if (where != slot(a.a)) HIPCHK(hipMemcpyAsync(slot(a.a), where, fb, hipMemcpyDeviceToDevice, st));
            where = slot(a.a);
        } else {
            if (a.a != pos) return fail(NPO_ESTATE, "schedule adjoint position mismatch");
            if (cont) {
                if (!have_next) HIPCHK(fwd_step(*p, ws, where, w.tmp, n0 + pos, aux, st));
                HIPCHK(adj_step_cont(*p, ws, where, w.tmp, w.lam, w.lam, n0 + pos, st));
                HIPCHK(hipMemcpyAsync(w.tmp, where, fb, hipMemcpyDeviceToDevice, st));
                have_next = true;
                aux = false;
                synced = false;
                continue;
            }
            // after an advance aux0 already holds the vorticity parts of u^pos
            if (gr && where == w.cur) {
                if (!aux) HIPCHK(npo::launch_curl_aux(*p, w.cur, w.aux0, st));
                if (!synced) HIPCHK(npo::launch_step_index(w.step, n0 + pos, 0, st));
                HIPCHK(hipGraphLaunch(p->g_adj, st));
                synced = true;
            } else {
                HIPCHK(adj_step(*p, ws, where, w.lam, w.lam, n0 + pos, st, nullptr, aux));
                synced = false;
            }
            aux = false;   // the adjoint step reuses aux0 for its own work
        }
    }
    HIPCHK(hipMemcpyAsync(lam0, w.lam, fb, hipMemcpyDeviceToDevice, st));
    if (n_recompute) *n_recompute = adv;
    return NPO_OK;
}

npo_status npo_adjoint_run(npo_plan p, void* ws, void* ckpt, int32_t nck, const void* lamN, void* lam0,
                           int64_t* n_recompute, void* stream) {
    Trace trace_("npo_adjoint_run");
    return adjoint_run(p, ws, ckpt, nck, lamN, lam0, n_recompute, stream);
}

// ------------------------------------------------ hybrid (host-tier) checkpoints
// Interval i of n_file + 1 equispaced intervals: steps [bound(i), bound(i + 1)).
static long long hybrid_bound(long long nsteps, int n_file, int i) {
    return (long long)((__int128)nsteps * i / (n_file + 1));
}

npo_status npo_forward_run_hybrid(npo_plan p, void* ws, void* ckpt, int32_t nck, void* host_tier, int32_t n_file,
                                  const void* u0, void* uN, void* stream) {
    Trace trace_("npo_forward_run_hybrid");
    if (check_plan(p) || !ws || !ckpt || !u0 || !uN || (n_file > 0 && !host_tier))
        return fail(NPO_EINVAL, "null argument");
    if (n_file < 0 || n_file >= p->nsteps) return fail(NPO_EINVAL, "n_file must be in [0, nsteps)");
    const hipStream_t st = ST(stream);
    const size_t fb = (size_t)3 * p->nr * p->mp1 * p->nk * 16;
    const void* in = u0;
    for (int i = 0; i <= n_file; ++i) {
        const long long b0 = hybrid_bound(p->nsteps, n_file, i), b1 = hybrid_bound(p->nsteps, n_file, i + 1);
        if (i < n_file) {
            // the interval's start state goes to the host tier; the interval is
            // advanced without device checkpoints (one slot)
            HIPCHK(hipMemcpyAsync(static_cast<char*>(host_tier) + (size_t)i * fb, in, fb, hipMemcpyDeviceToHost,
                                  st));
            npo_status s = forward_run(p, ws, ckpt, 1, in, uN, nullptr, 1, stream, b0, b1 - b0);
            if (s) return s;
        } else {
            // the last interval keeps its binomial device checkpoints for the adjoint sweep
            npo_status s = forward_run(p, ws, ckpt, nck, in, uN, nullptr, 1, stream, b0, b1 - b0);
            if (s) return s;
        }
        in = uN;
    }
    return NPO_OK;
}

npo_status npo_adjoint_run_hybrid(npo_plan p, void* ws, void* ckpt, int32_t nck, const void* host_tier,
                                  int32_t n_file, const void* lamN, void* lam0, int64_t* n_recompute, void* stream) {
    Trace trace_("npo_adjoint_run_hybrid");
    if (check_plan(p) || !ws || !ckpt || !lamN || !lam0 || (n_file > 0 && !host_tier))
        return fail(NPO_EINVAL, "null argument");
    if (n_file < 0 || n_file >= p->nsteps) return fail(NPO_EINVAL, "n_file must be in [0, nsteps)");
    const hipStream_t st = ST(stream);
    const size_t fb = (size_t)3 * p->nr * p->mp1 * p->nk * 16;
    WsPtrs w = wsptrs(*p, ws);
    int64_t total = 0;
    const void* lin = lamN;
    for (int i = n_file; i >= 0; --i) {
        const long long b0 = hybrid_bound(p->nsteps, n_file, i), b1 = hybrid_bound(p->nsteps, n_file, i + 1);
        if (i < n_file) {
            // restore the interval's start state from the host tier and place its
            // device checkpoints (the interval's last step is not needed)
            HIPCHK(hipMemcpyAsync(w.tmp, static_cast<const char*>(host_tier) + (size_t)i * fb, fb,
                                  hipMemcpyHostToDevice, st));
            npo_status s = forward_run(p, ws, ckpt, nck, w.tmp, nullptr, nullptr, 1, stream, b0, b1 - b0, false);
            if (s) return s;
            total += b1 - b0 - 1;
        }
        int64_t rec = 0;
        npo_status s = adjoint_run(p, ws, ckpt, nck, lin, lam0, &rec, stream, b0, b1 - b0);
        if (s) return s;
        total += rec;
        lin = lam0;
    }
    if (n_recompute) *n_recompute = total;
    return NPO_OK;
}

// Forward advances of the hybrid adjoint sweep: every interval but the last
// is re-advanced to place its device checkpoints (its length less one step),
// and each interval's adjoint sweep re-advances from them.
static long long hybrid_advances(long long nsteps, int n_ckpt, int n_file) {
    auto advances = [&](long long l) -> long long {      // advances to reverse l steps with n_ckpt slots
        if (l <= 1) return 0;
        std::vector<Act> acts = schedule(l, n_ckpt);
        long long c = 0;
        for (size_t i = first_adj(acts); i < acts.size(); ++i)
            if (acts[i].kind == A_ADV) c += acts[i].a;
        return c;
    };
    long long steps = 0;
    for (int i = 0; i <= n_file; ++i) {
        const long long l = hybrid_bound(nsteps, n_file, i + 1) - hybrid_bound(nsteps, n_file, i);
        steps += advances(l) + (i < n_file ? l - 1 : 0);
    }
    return steps;
}

npo_status npo_hybrid_count(int64_t nsteps, int32_t n_ckpt, int32_t n_file, int64_t* n_recompute) {
    if (nsteps < 1 || n_ckpt < 1 || n_file < 0 || n_file >= nsteps || !n_recompute)
        return fail(NPO_EINVAL, "bad argument");
    *n_recompute = hybrid_advances(nsteps, n_ckpt, n_file);
    return NPO_OK;
}

npo_status npo_hybrid_plan(int64_t nsteps, int32_t n_ckpt, double t_io, double t_step, int32_t max_file,
                           int32_t* n_file, double* t_rec) {
    if (nsteps < 1 || n_ckpt < 1 || max_file < 0 || !(t_io >= 0) || !(t_step > 0) || !n_file)
        return fail(NPO_EINVAL, "bad argument");
    double best = std::numeric_limits<double>::infinity();
    int bestf = 0;
    const int top = (int)std::min<long long>(max_file, nsteps - 1);
    for (int f = 0; f <= top; ++f) {
        const double t = f * t_io + (double)hybrid_advances(nsteps, n_ckpt, f) * t_step;
        if (t < best) { best = t; bestf = f; }
    }
    *n_file = bestf;
    if (t_rec) *t_rec = best;
    return NPO_OK;
}

npo_status npo_inner(npo_plan p, void* ws, const void* a, const void* b, double* out_dev, void* stream) {
    if (check_plan(p) || !ws || !a || !b || !out_dev) return fail(NPO_EINVAL, "null argument");
    WsPtrs w = wsptrs(*p, ws);
    HIPCHK(npo::launch_wdot(*p, CF(a), CF(b), w.red, out_dev, ST(stream)));
    return NPO_OK;
}

npo_status npo_project(npo_plan p, void* ws, const void* u, void* out, void* stream) {
    if (check_plan(p) || !u || !out) return fail(NPO_EINVAL, "null argument");
    (void)ws;
    HIPCHK(npo::launch_project(*p, CF(u), F(out), ST(stream)));
    return NPO_OK;
}

static double lambda_plus(double al, double E0, double E0d, double C0) {
    const double a = (al * C0 - 2.0 * E0) / (2.0 * al * E0);
    const double q = (-al * C0 + 2.0 * E0) / (2.0 * al * E0);
    const double disc = q * q - (al * E0d - C0) / (al * E0);
    return a + std::sqrt(disc > 0.0 ? disc : 0.0);
}

// The gradient step with host scalars (the line search of npo_iterate, which
// needs E0dag and C0 on the host anyway for alpha_max).
static npo_status update_host(npo_plan p, void* ws, const void* u0, const void* udag, double e0, double alpha,
                              double e0dag, double c0, void* u_new, void* stream) {
    if (check_plan(p) || !ws || !u0 || !udag || !u_new) return fail(NPO_EINVAL, "null argument");
    if (!(e0 > 0) || !(alpha > 0)) return fail(NPO_EINVAL, "e0 and alpha must be positive");
    WsPtrs w = wsptrs(*p, ws);
    const hipStream_t st = ST(stream);
    const double lam = lambda_plus(alpha, e0, e0dag, c0);
    HIPCHK(npo::launch_axpby(*p, 1.0 + lam * alpha, CF(u0), -alpha, CF(udag), F(u_new), st));
    double* en = w.red + npo::NR_MAX * 4 + 256;
    HIPCHK(npo::launch_wdot(*p, CF(u_new), CF(u_new), w.red, en, st));
    // energy = <u,u>/2
    HIPCHK(npo::launch_rescale(*p, F(u_new), en, 2.0 * e0, st));
    return NPO_OK;
}

npo_status npo_update(npo_plan p, void* ws, const void* u0, const void* g, double e0, double alpha, void* u_new,
                      double* info_dev, void* stream) {
    if (check_plan(p) || !ws || !u0 || !g || !u_new || !info_dev) return fail(NPO_EINVAL, "null argument");
    if (!(e0 > 0)) return fail(NPO_EINVAL, "e0 must be positive");
    if (!std::isfinite(alpha)) return fail(NPO_EINVAL, "alpha must be finite (<= 0 selects alpha_max)");
    if (u_new == u0 || u_new == g) return fail(NPO_EINVAL, "u_new must not alias u0 or g");
    WsPtrs w = wsptrs(*p, ws);
    const hipStream_t st = ST(stream);
    double* sc = w.red + npo::NR_MAX * 4 + 256 + 16;     // sc[0..1] inner products, sc[2..3] coefficients
    HIPCHK(npo::launch_wdot(*p, CF(g), CF(g), w.red, sc, st));
    HIPCHK(npo::launch_wdot(*p, CF(u0), CF(g), w.red, sc + 1, st));
    HIPCHK(npo::launch_update_dev(*p, sc, e0, alpha, info_dev, sc + 2, CF(u0), CF(g), F(u_new), st));
    double* en = sc + 4;
    HIPCHK(npo::launch_wdot(*p, CF(u_new), CF(u_new), w.red, en, st));
    HIPCHK(npo::launch_half(en, info_dev, st));
    // energy = <u,u>/2
    HIPCHK(npo::launch_rescale(*p, F(u_new), en, 2.0 * e0, st));
    return NPO_OK;
}

npo_status npo_iterate(npo_plan p, void* ws, void* ckpt, int32_t nck, void* u0, void* uN, double e0, double tol,
                       int32_t max_halvings, double* stats, void* stream) {
    Trace trace_("npo_iterate");
    if (check_plan(p) || !ws || !ckpt || !u0 || !uN || !stats) return fail(NPO_EINVAL, "null argument");
    if (!(e0 > 0) || max_halvings < 0) return fail(NPO_EINVAL, "bad e0 or max_halvings");
    const hipStream_t st = ST(stream);
    const size_t fb = (size_t)3 * p->nr * p->mp1 * p->nk * 16;
    WsPtrs w = wsptrs(*p, ws);
    double* sc = w.red + npo::NR_MAX * 4 + 256 + 8;
    auto read = [&](double* dev, double* host, int n) -> hipError_t {
        hipError_t e = hipMemcpyAsync(host, dev, n * 8, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(st);
    };
    double h[4];
    HIPCHK(npo::launch_wdot(*p, CF(uN), CF(uN), w.red, sc, st));
    HIPCHK(read(sc, h, 1));
    const double Gold = 0.5 * h[0] / e0;
    int64_t nrec = 0;
    npo_status s = npo_adjoint_run(p, ws, ckpt, nck, uN, w.g, &nrec, stream);
    if (s) return s;
    HIPCHK(npo::launch_project(*p, w.g, w.g, st));
    // udag = -g:  E0dag = <g,g>/2, C0 = <u0, udag> = -<u0, g>
    HIPCHK(npo::launch_wdot(*p, w.g, w.g, w.red, sc, st));
    HIPCHK(npo::launch_wdot(*p, CF(u0), w.g, w.red, sc + 1, st));
    HIPCHK(read(sc, h, 2));
    const double E0d = 0.5 * h[0], C0 = -h[1];
    const double q = E0d / e0 - C0 * C0 / (4.0 * e0 * e0);
    const double amax = q > 0 ? 1.0 / std::sqrt(q) : std::numeric_limits<double>::infinity();
    stats[0] = Gold; stats[1] = Gold; stats[2] = 0.0; stats[3] = amax; stats[4] = E0d; stats[5] = C0;
    stats[6] = 0.0; stats[7] = 0.0;
    if (!std::isfinite(Gold) || !std::isfinite(E0d) || !std::isfinite(C0)) return NPO_OK;   // blown-up state
    if (!std::isfinite(amax)) return NPO_OK;
    // udag into w.tmp
    HIPCHK(npo::launch_axpby(*p, -1.0, w.g, 0.0, nullptr, w.tmp, st));
    double al = amax;
    for (int hv = 0; hv <= max_halvings; ++hv) {
        s = update_host(p, ws, u0, w.tmp, e0, al, E0d, C0, w.trial, stream);
        if (s) return s;
        s = npo_forward_run(p, ws, ckpt, nck, w.trial, w.trialN, stream);
        if (s) return s;
        stats[7] += 1.0;
        HIPCHK(npo::launch_wdot(*p, w.trialN, w.trialN, w.red, sc, st));
        HIPCHK(read(sc, h, 1));
        const double Gn = 0.5 * h[0] / e0;
        if (Gn > Gold) {
            HIPCHK(hipMemcpyAsync(u0, w.trial, fb, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(uN, w.trialN, fb, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
            stats[1] = Gn; stats[2] = al; stats[6] = 1.0;
            return NPO_OK;
        }
        if (std::fabs((Gn - Gold) / Gn) < tol) break;
        al *= 0.5;
    }
    return NPO_OK;
}

npo_status npo_plan_set_tuning(npo_plan p, int32_t zgroup, int32_t zb_fwd, int32_t zb_adj) {
    if (check_plan(p)) return NPO_EINVAL;
    auto ok_zb = [&](int zb, int adj) {
        if (zb < 0) return npo::theta_wave_ok(p->nt, p->nz, -zb);   // the wave-resident kernels
        if (zb != 2 && zb != 4 && zb != 8) return false;
        if (p->nz % zb) return false;
        return npo::theta_lds(*p, zb, adj) <= 160 * 1024;
    };
    if (zgroup < 1 || zgroup > 3 || npo::zpass_lds(*p, zgroup) > 160 * 1024)
        return fail(NPO_EINVAL, "zgroup must be 1..3 and fit 160 KiB of LDS");
    if (!ok_zb(zb_fwd, 0) || !ok_zb(zb_adj, 1)) return fail(NPO_EINVAL, "bad azimuthal z-block");
    p->zgroup = zgroup;
    p->zb_theta_fwd = zb_fwd;
    p->zb_theta_adj = zb_adj;
    drop_graphs(*p);          // launch shapes are baked into captured graphs
    return NPO_OK;
}

npo_status npo_plan_set_cfl_monitor(npo_plan p, int32_t enable) {
    if (check_plan(p)) return NPO_EINVAL;
    if (enable != 0 && enable != 1) return fail(NPO_EINVAL, "enable must be 0 or 1");
    p->cfl_monitor = enable != 0;
    drop_graphs(*p);          // the monitor's pointer is part of the captured launches
    return NPO_OK;
}

npo_status npo_cfl_read(npo_plan p, void* ws, double* out_dev, int32_t reset, void* stream) {
    if (check_plan(p) || !ws || !out_dev) return fail(NPO_EINVAL, "null argument");
    WsPtrs w = wsptrs(*p, ws);
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    HIPCHK(hipMemcpyAsync(out_dev, cfl_slot(w), 8, hipMemcpyDeviceToDevice, st));
    if (reset) HIPCHK(npo::launch_fill_u64(cfl_slot(w), 0ull, st));
    return NPO_OK;
}

npo_status npo_plan_inject_fault(npo_plan p, int32_t site, int64_t after) {
    if (check_plan(p)) return NPO_EINVAL;
    if (site < 0 || site > 2 || after < 0) return fail(NPO_EINVAL, "site must be 0, 1 or 2 and after >= 0");
    p->fault_site = site;
    p->fault_after = after;
    return NPO_OK;
}

npo_status npo_plan_set_graphs(npo_plan p, int32_t enable) {
    if (check_plan(p)) return NPO_EINVAL;
    if (enable != 0 && enable != 1) return fail(NPO_EINVAL, "enable must be 0 or 1");
    p->use_graphs = enable != 0;
    if (!p->use_graphs) drop_graphs(*p);
    return NPO_OK;
}

npo_status npo_plan_get_tuning(npo_plan p, int32_t* zgroup, int32_t* zb_fwd, int32_t* zb_adj) {
    if (check_plan(p) || !zgroup || !zb_fwd || !zb_adj) return fail(NPO_EINVAL, "null argument");
    *zgroup = p->zgroup;
    *zb_fwd = p->zb_theta_fwd;
    *zb_adj = p->zb_theta_adj;
    return NPO_OK;
}

npo_status npo_plan_set_radial_block(npo_plan p, int32_t rg) {
    if (check_plan(p)) return NPO_EINVAL;
    if (rg != 4 && rg != 8 && rg != 16) return fail(NPO_EINVAL, "rg must be 4, 8 or 16");
    p->rg = rg;
    drop_graphs(*p);          // launch shapes are baked into captured graphs
    return NPO_OK;
}

npo_status npo_plan_get_radial_block(npo_plan p, int32_t* rg) {
    if (check_plan(p) || !rg) return fail(NPO_EINVAL, "null argument");
    *rg = p->rg;
    return NPO_OK;
}

npo_status npo_euclid_grad(npo_plan p, const void* lam, double scale, void* out, void* stream) {
    if (check_plan(p) || !lam || !out) return fail(NPO_EINVAL, "null argument");
    HIPCHK(npo::launch_wscale(*p, CF(lam), F(out), scale, ST(stream)));
    return NPO_OK;
}

npo_status npo_profile_begin(npo_plan p, int32_t stride) {
    if (check_plan(p) || stride < 1) return fail(NPO_EINVAL, "bad argument");
    npo::Profiler& f = p->prof;
    if (f.ev.empty()) {
        f.ev.resize((size_t)npo::KID_COUNT * npo::PROF_SLOTS * 2);
        for (auto& e : f.ev) HIPCHK(hipEventCreate(&e));
    }
    for (int k = 0; k < npo::KID_COUNT; ++k) { f.launches[k] = 0; f.used[k] = 0; }
    f.stride = stride;
    f.on = true;
    return NPO_OK;
}

npo_status npo_profile_read(npo_plan p, int64_t* launches, int64_t* sampled, double* avg_ms) {
    if (check_plan(p) || !launches || !sampled || !avg_ms) return fail(NPO_EINVAL, "null argument");
    npo::Profiler& f = p->prof;
    for (int k = 0; k < npo::KID_COUNT; ++k) {
        launches[k] = f.on || f.launches[k] ? f.launches[k] : 0;
        sampled[k] = f.used[k];
        double tot = 0.0;
        for (int s = 0; s < f.used[k]; ++s) {
            hipEvent_t a = f.ev[(k * npo::PROF_SLOTS + s) * 2], b = f.ev[(k * npo::PROF_SLOTS + s) * 2 + 1];
            HIPCHK(hipEventSynchronize(b));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, a, b));
            tot += ms;
        }
        avg_ms[k] = f.used[k] ? tot / f.used[k] : 0.0;
    }
    f.on = false;
    return NPO_OK;
}

npo_status npo_normalize(npo_plan p, void* ws, void* u, double e0, void* stream) {
    if (check_plan(p) || !ws || !u) return fail(NPO_EINVAL, "null argument");
    if (!(e0 > 0)) return fail(NPO_EINVAL, "e0 must be positive");
    WsPtrs w = wsptrs(*p, ws);
    double* en = w.red + npo::NR_MAX * 4 + 256;
    HIPCHK(npo::launch_wdot(*p, CF(u), CF(u), w.red, en, ST(stream)));
    HIPCHK(npo::launch_rescale(*p, F(u), en, 2.0 * e0, ST(stream)));
    return NPO_OK;
}

// ================================================================ batches
// Instances of uneven shape advanced together (one launch per kernel for
// every instance of a shape class, each instance's constants, buffers and
// evaluation time read from a device work-descriptor table).
}  // extern "C"

struct npo_batch_s {
    std::vector<npo_plan> plans;
    std::vector<std::vector<int>> classes;      // instance indices per shape class
    struct Phase {
        std::vector<void*> key;                 // workspace pointers the tables were built for
        // per class: recorded launch sequence, descriptor table [site][instance], step table
        std::vector<std::vector<std::function<void(const npo::BDesc*, int, hipStream_t)>>> launch;
        std::vector<npo::BDesc*> dtab;
        std::vector<char> batched;              // 0: the class falls back to per-instance launches
        hipGraphExec_t graph = nullptr;
    } ph[2];
    std::vector<npo::BDesc*> steptab;           // per class: one descriptor per instance (step index)
    std::vector<void*> step_key;
    hipStream_t cap = nullptr;
    // class branches of the captured step: one stream per class forked from
    // and joined back to the capture stream, so the graph runs the classes
    // concurrently
    std::vector<hipStream_t> cs;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    int launches = 0;                           // kernel launches of the last batched step
};

namespace {

bool same_class(const npo_plan_s& a, const npo_plan_s& b) {
    return a.nr == b.nr && a.nt == b.nt && a.nz == b.nz && a.ncorr == b.ncorr && a.zgroup == b.zgroup &&
           a.zb_theta_fwd == b.zb_theta_fwd && a.zb_theta_adj == b.zb_theta_adj && a.device == b.device &&
           a.cfl_monitor == b.cfl_monitor && a.rg == b.rg;
}

void drop_phase(npo_batch_s::Phase& f) {
    for (npo::BDesc* d : f.dtab)
        if (d) (void)hipFree(d);
    f.dtab.clear();
    f.launch.clear();
    f.batched.clear();
    f.key.clear();
    if (f.graph) (void)hipGraphExecDestroy(f.graph);
    f.graph = nullptr;
}

// The per-instance buffers of the batched steps: the state advances in the
// workspace's `cur`, the adjoint field in its `lam`, the step index in `step`.
npo_status batch_tables(npo_batch_s& b, void* const* ws, hipStream_t st) {
    std::vector<void*> key(ws, ws + b.plans.size());
    if (b.step_key == key && b.ph[0].key == key && b.ph[1].key == key) return NPO_OK;
    for (auto& f : b.ph) drop_phase(f);
    for (npo::BDesc* d : b.steptab)
        if (d) (void)hipFree(d);
    b.steptab.clear();
    for (int phase = 0; phase < 2; ++phase) {
        npo_batch_s::Phase& f = b.ph[phase];
        for (const std::vector<int>& cl : b.classes) {
            std::vector<npo::Recorder> rec(cl.size());
            bool ok = true;
            for (size_t q = 0; q < cl.size(); ++q) {
                const npo_plan_s& p = *b.plans[cl[q]];
                WsPtrs w = wsptrs(p, ws[cl[q]]);
                npo::recorder() = &rec[q];
                hipError_t e = phase == 0 ? fwd_step(p, ws[cl[q]], w.cur, w.cur, 0, false, st, w.step)
                                          : adj_step(p, ws[cl[q]], w.cur, w.lam, w.lam, 0, st, w.step, false);
                npo::recorder() = nullptr;
                if (e != hipSuccess) return hipfail(e, "recording a batched step");
                ok = ok && rec[q].ok && rec[q].desc.size() == rec[0].desc.size();
            }
            f.batched.push_back(ok ? 1 : 0);
            f.launch.push_back(ok ? rec[0].launch : decltype(rec[0].launch){});
            npo::BDesc* dt = nullptr;
            if (ok) {
                const size_t ns = rec[0].desc.size(), nb = cl.size();
                std::vector<npo::BDesc> host(ns * nb);
                for (size_t sidx = 0; sidx < ns; ++sidx)
                    for (size_t q = 0; q < nb; ++q) host[sidx * nb + q] = rec[q].desc[sidx];
                HIPCHK(hipMalloc(&dt, host.size() * sizeof(npo::BDesc)));
                HIPCHK(hipMemcpy(dt, host.data(), host.size() * sizeof(npo::BDesc), hipMemcpyHostToDevice));
            }
            f.dtab.push_back(dt);
        }
        f.key = key;
    }
    for (const std::vector<int>& cl : b.classes) {
        std::vector<npo::BDesc> host(cl.size());
        for (size_t q = 0; q < cl.size(); ++q) host[q].step = wsptrs(*b.plans[cl[q]], ws[cl[q]]).step;
        npo::BDesc* dt = nullptr;
        HIPCHK(hipMalloc(&dt, host.size() * sizeof(npo::BDesc)));
        HIPCHK(hipMemcpy(dt, host.data(), host.size() * sizeof(npo::BDesc), hipMemcpyHostToDevice));
        b.steptab.push_back(dt);
    }
    b.step_key = key;
    return NPO_OK;
}

// One batched step on stream st (phase 0: forward advance of cur, then every
// step index + 1; phase 1: adjoint step of lam at u = cur, then step index - 1).
// The launches of one class of one phase on stream st; nl counts them.
hipError_t batch_issue_class(npo_batch_s& b, void* const* ws, int phase, size_t c, hipStream_t st, int& nl) {
    npo_batch_s::Phase& f = b.ph[phase];
    const std::vector<int>& cl = b.classes[c];
    const int nb = (int)cl.size();
    if (f.batched[c]) {
        for (size_t sidx = 0; sidx < f.launch[c].size(); ++sidx) {
            f.launch[c][sidx](f.dtab[c] + sidx * nb, nb, st);
            ++nl;
        }
    } else {
        for (int i : cl) {
            const npo_plan_s& p = *b.plans[i];
            WsPtrs w = wsptrs(p, ws[i]);
            hipError_t e = phase == 0 ? fwd_step(p, ws[i], w.cur, w.cur, 0, false, st, w.step)
                                      : adj_step(p, ws[i], w.cur, w.lam, w.lam, 0, st, w.step, false);
            if (e != hipSuccess) return e;
            nl += 1;
        }
    }
    hipError_t e = npo::launch_step_index_batched(b.steptab[c], nb, phase == 0 ? 1 : -1, 1, st);
    if (e != hipSuccess) return e;
    ++nl;
    return hipGetLastError();
}

// Every class one after another on st.
hipError_t batch_issue(npo_batch_s& b, void* const* ws, int phase, hipStream_t st, int* launches) {
    int nl = 0;
    for (size_t c = 0; c < b.classes.size(); ++c) {
        hipError_t e = batch_issue_class(b, ws, phase, c, st, nl);
        if (e != hipSuccess) return e;
    }
    if (launches) *launches = nl;
    return hipGetLastError();
}

// Every class on its own stream, forked from st and joined back to it (inside
// a capture this makes the classes parallel branches of the graph).
hipError_t batch_issue_forked(npo_batch_s& b, void* const* ws, int phase, hipStream_t st, int* launches) {
    const size_t nc = b.classes.size();
    hipError_t e = hipSuccess;
    if (!b.fork) e = hipEventCreateWithFlags(&b.fork, hipEventDisableTiming);
    while (e == hipSuccess && b.cs.size() < nc) {
        hipStream_t s = nullptr;
        hipEvent_t j = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) b.cs.push_back(s);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
        if (e == hipSuccess) b.join.push_back(j);
    }
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(b.fork, st)) != hipSuccess) return e;
    int nl = 0;
    for (size_t c = 0; c < nc; ++c) {
        if ((e = hipStreamWaitEvent(b.cs[c], b.fork, 0)) != hipSuccess) return e;
        if ((e = batch_issue_class(b, ws, phase, c, b.cs[c], nl)) != hipSuccess) return e;
        if ((e = hipEventRecord(b.join[c], b.cs[c])) != hipSuccess) return e;
    }
    for (size_t c = 0; c < nc; ++c)
        if ((e = hipStreamWaitEvent(st, b.join[c], 0)) != hipSuccess) return e;
    if (launches) *launches = nl;
    return hipGetLastError();
}

npo_status batch_step(npo_batch_s& b, void* const* ws, int phase, hipStream_t st, bool use_graph) {
    npo_status s = batch_tables(b, ws, st);
    if (s) return s;
    npo_batch_s::Phase& f = b.ph[phase];
    if (!use_graph) {
        HIPCHK(batch_issue(b, ws, phase, st, &b.launches));
        return NPO_OK;
    }
    if (!f.graph) {
        if (!b.cap) HIPCHK(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
        hipError_t e1 = b.classes.size() > 1 ? batch_issue_forked(b, ws, phase, b.cap, &b.launches)
                                             : batch_issue(b, ws, phase, b.cap, &b.launches);
        hipError_t e = hipStreamEndCapture(b.cap, &g);
        if (e == hipSuccess) e = e1;
        if (e == hipSuccess) e = hipGraphInstantiate(&f.graph, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hipfail(e, "capturing the batched step");
    }
    HIPCHK(hipGraphLaunch(f.graph, st));
    return NPO_OK;
}

npo_status batch_set_steps(npo_batch_s& b, void* const* ws, long long v, hipStream_t st) {
    npo_status s = batch_tables(b, ws, st);
    if (s) return s;
    for (size_t c = 0; c < b.classes.size(); ++c)
        HIPCHK(npo::launch_step_index_batched(b.steptab[c], (int)b.classes[c].size(), v, 0, st));
    return NPO_OK;
}

npo_status batch_check(npo_batch b, void* const* ws) {
    if (!b || !ws) return fail(NPO_EINVAL, "null argument");
    for (size_t i = 0; i < b->plans.size(); ++i) {
        if (!ws[i]) return fail(NPO_EINVAL, "null workspace");
        if (b->plans[i]->adjoint_kind != 0)
            return fail(NPO_EUNSUPPORTED, "batched sweeps take the exact discrete adjoint only");
    }
    return NPO_OK;
}

}  // namespace

extern "C" {

npo_status npo_batch_create(const npo_plan* plans, int32_t n, npo_batch* out) {
    if (!plans || n < 1 || !out) return fail(NPO_EINVAL, "null argument or n < 1");
    auto* b = new npo_batch_s();
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) {
            delete b;
            return fail(NPO_EINVAL, "null plan");
        }
        b->plans.push_back(plans[i]);
        if (plans[i]->nsteps != plans[0]->nsteps) {
            delete b;
            return fail(NPO_EINVAL, "batched instances share the horizon nsteps (one checkpoint schedule)");
        }
        bool placed = false;
        for (std::vector<int>& cl : b->classes)
            if (same_class(*plans[cl[0]], *plans[i])) {
                cl.push_back(i);
                placed = true;
                break;
            }
        if (!placed) b->classes.push_back({i});
    }
    *out = b;
    return NPO_OK;
}

npo_status npo_batch_destroy(npo_batch b) {
    if (!b) return NPO_OK;
    for (auto& f : b->ph) drop_phase(f);
    for (npo::BDesc* d : b->steptab)
        if (d) (void)hipFree(d);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (hipStream_t c : b->cs) (void)hipStreamDestroy(c);
    for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
    return NPO_OK;
}

npo_status npo_batch_info(npo_batch b, int32_t* n_classes, int32_t* n_batched, int32_t* launches) {
    if (!b) return fail(NPO_EINVAL, "null batch");
    if (n_classes) *n_classes = (int32_t)b->classes.size();
    if (n_batched) {
        int nb = 0;
        for (size_t c = 0; c < b->classes.size(); ++c)
            if (!b->ph[0].batched.empty() && b->ph[0].batched[c] && b->ph[1].batched[c]) nb += (int)b->classes[c].size();
        *n_batched = nb;
    }
    if (launches) *launches = b->launches;
    return NPO_OK;
}

npo_status npo_batch_step(npo_batch b, void* const* states, void* const* ws, int32_t phase, void* stream) {
    Trace trace_("npo_batch_step");
    npo_status s = batch_check(b, ws);
    if (s) return s;
    if (!states || (phase != 0 && phase != 1)) return fail(NPO_EINVAL, "states must be given and phase 0 or 1");
    const hipStream_t st = ST(stream);
    const size_t n = b->plans.size();
    for (size_t i = 0; i < (phase ? 2 * n : n); ++i)
        if (!states[i]) return fail(NPO_EINVAL, "null state");
    // the batched launches work on each workspace's cur (and lam)
    for (size_t i = 0; i < n; ++i) {
        const npo_plan_s& p = *b->plans[i];
        const size_t fb = (size_t)3 * p.nr * p.mp1 * p.nk * 16;
        WsPtrs w = wsptrs(p, ws[i]);
        const void* u = phase ? states[2 * i] : states[i];
        if (u != w.cur) HIPCHK(hipMemcpyAsync(w.cur, u, fb, hipMemcpyDeviceToDevice, st));
        if (phase && states[2 * i + 1] != w.lam)
            HIPCHK(hipMemcpyAsync(w.lam, states[2 * i + 1], fb, hipMemcpyDeviceToDevice, st));
    }
    s = batch_step(*b, ws, phase, st, false);
    if (s) return s;
    for (size_t i = 0; i < n; ++i) {
        const npo_plan_s& p = *b->plans[i];
        const size_t fb = (size_t)3 * p.nr * p.mp1 * p.nk * 16;
        WsPtrs w = wsptrs(p, ws[i]);
        void* o = phase ? states[2 * i + 1] : states[i];
        if (o != (phase ? (void*)w.lam : (void*)w.cur))
            HIPCHK(hipMemcpyAsync(o, phase ? w.lam : w.cur, fb, hipMemcpyDeviceToDevice, st));
    }
    return NPO_OK;
}

npo_status npo_batch_set_steps(npo_batch b, void* const* ws, int64_t n, void* stream) {
    npo_status s = batch_check(b, ws);
    if (s) return s;
    return batch_set_steps(*b, ws, n, ST(stream));
}

// Checkpointed sweeps of every instance in lockstep: one schedule (the
// instances share nsteps and n_ckpt); advances and adjoint steps are batched
// steps (replayed from one captured graph per phase), stores and restores are
// per-instance device copies between the workspace's cur and the slots.
npo_status npo_batch_forward_run(npo_batch b, void* const* ws, void* const* ckpt, int32_t nck, void* const* u0,
                                 void* const* uN, void* stream) {
    Trace trace_("npo_batch_forward_run");
    npo_status s = batch_check(b, ws);
    if (s) return s;
    if (!ckpt || !u0 || !uN || nck < 1) return fail(NPO_EINVAL, "null argument or n_ckpt < 1");
    const size_t n = b->plans.size();
    for (size_t i = 0; i < n; ++i)
        if (!ckpt[i] || !u0[i] || !uN[i]) return fail(NPO_EINVAL, "null buffer");
    const hipStream_t st = ST(stream);
    const long long N = b->plans[0]->nsteps;
    auto fbytes = [&](size_t i) { const npo_plan_s& p = *b->plans[i]; return (size_t)3 * p.nr * p.mp1 * p.nk * 16; };
    auto slot = [&](size_t i, long long sl) { return static_cast<char*>(ckpt[i]) + sl * fbytes(i); };
    auto cur = [&](size_t i) { return (void*)wsptrs(*b->plans[i], ws[i]).cur; };
    for (size_t i = 0; i < n; ++i) {
        HIPCHK(hipMemcpyAsync(slot(i, 0), u0[i], fbytes(i), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(cur(i), u0[i], fbytes(i), hipMemcpyDeviceToDevice, st));
    }
    s = batch_set_steps(*b, ws, 0, st);
    if (s) return s;
    std::vector<Act> acts = schedule(N, nck);
    const size_t fa = first_adj(acts);
    long long pos = 0;
    for (size_t a = 0; a < fa; ++a) {
        if (acts[a].kind == A_ADV) {
            for (long long k = 0; k < acts[a].a; ++k) {
                s = batch_step(*b, ws, 0, st, true);
                if (s) return s;
                ++pos;
            }
        } else if (acts[a].kind == A_STORE) {
            for (size_t i = 0; i < n; ++i)
                HIPCHK(hipMemcpyAsync(slot(i, acts[a].a), cur(i), fbytes(i), hipMemcpyDeviceToDevice, st));
        }
    }
    if (pos != N - 1) return fail(NPO_ESTATE, "schedule descent did not reach the last step");
    // cur keeps u^{N-1} for the adjoint sweep; the last step goes to uN
    for (size_t i = 0; i < n; ++i) {
        const npo_plan_s& p = *b->plans[i];
        WsPtrs w = wsptrs(p, ws[i]);
        HIPCHK(fwd_step(p, ws[i], w.cur, static_cast<double2*>(uN[i]), N - 1, false, st));
    }
    return NPO_OK;
}

npo_status npo_batch_adjoint_run(npo_batch b, void* const* ws, void* const* ckpt, int32_t nck, void* const* lamN,
                                 void* const* lam0, int64_t* n_recompute, void* stream) {
    Trace trace_("npo_batch_adjoint_run");
    npo_status s = batch_check(b, ws);
    if (s) return s;
    if (!ckpt || !lamN || !lam0 || nck < 1) return fail(NPO_EINVAL, "null argument or n_ckpt < 1");
    const size_t n = b->plans.size();
    for (size_t i = 0; i < n; ++i)
        if (!ckpt[i] || !lamN[i] || !lam0[i]) return fail(NPO_EINVAL, "null buffer");
    const hipStream_t st = ST(stream);
    const long long N = b->plans[0]->nsteps;
    auto fbytes = [&](size_t i) { const npo_plan_s& p = *b->plans[i]; return (size_t)3 * p.nr * p.mp1 * p.nk * 16; };
    auto slot = [&](size_t i, long long sl) { return static_cast<char*>(ckpt[i]) + sl * fbytes(i); };
    for (size_t i = 0; i < n; ++i) {
        WsPtrs w = wsptrs(*b->plans[i], ws[i]);
        HIPCHK(hipMemcpyAsync(w.lam, lamN[i], fbytes(i), hipMemcpyDeviceToDevice, st));
    }
    s = batch_set_steps(*b, ws, N - 1, st);
    if (s) return s;
    std::vector<Act> acts = schedule(N, nck);
    long long adv = 0;
    for (size_t a = first_adj(acts); a < acts.size(); ++a) {
        const Act& x = acts[a];
        if (x.kind == A_RESTORE) {
            for (size_t i = 0; i < n; ++i) {
                WsPtrs w = wsptrs(*b->plans[i], ws[i]);
                HIPCHK(hipMemcpyAsync(w.cur, slot(i, x.a), fbytes(i), hipMemcpyDeviceToDevice, st));
            }
            s = batch_set_steps(*b, ws, x.b, st);
            if (s) return s;
        } else if (x.kind == A_ADV) {
            for (long long k = 0; k < x.a; ++k) {
                s = batch_step(*b, ws, 0, st, true);
                if (s) return s;
            }
            adv += x.a;
        } else if (x.kind == A_STORE) {
            for (size_t i = 0; i < n; ++i) {
                WsPtrs w = wsptrs(*b->plans[i], ws[i]);
                HIPCHK(hipMemcpyAsync(slot(i, x.a), w.cur, fbytes(i), hipMemcpyDeviceToDevice, st));
            }
        } else {
            // the adjoint step at u^pos = cur; the step index then moves to pos - 1
            s = batch_step(*b, ws, 1, st, true);
            if (s) return s;
        }
    }
    for (size_t i = 0; i < n; ++i) {
        WsPtrs w = wsptrs(*b->plans[i], ws[i]);
        HIPCHK(hipMemcpyAsync(lam0[i], w.lam, fbytes(i), hipMemcpyDeviceToDevice, st));
    }
    if (n_recompute) *n_recompute = adv;
    return NPO_OK;
}

}  // extern "C"
