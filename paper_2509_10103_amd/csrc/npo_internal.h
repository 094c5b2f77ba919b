// Internal declarations shared by the host driver (npo_host.cpp) and the
// device kernels (npo_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

namespace npo {

// Kernel families timed by the sampling profiler (ids of npo_profile_read).
enum KernelId {
    KID_CURL = 0, KID_ZINV_F, KID_THETA_F, KID_ZFWD_F, KID_ZINV_A, KID_THETA_A, KID_ZFWD_A,
    KID_SOLVE_P, KID_SOLVE_C, KID_SOLVE_R, KID_SOLVE_ADJ, KID_FINAL, KID_WDOT, KID_PROJECT, KID_AXPBY,
    KID_SOLVE_ADJ2, KID_ZINV_Y, KID_COUNT
};
constexpr int PROF_SLOTS = 256;   // sampled launches kept per kernel family

struct Profiler {
    bool on = false;
    int stride = 1;
    long long launches[KID_COUNT] = {0};
    int used[KID_COUNT] = {0};
    std::vector<hipEvent_t> ev;   // KID_COUNT * PROF_SLOTS * 2
};

constexpr int NR_MAX = 64;     // radial nodes handled by one workgroup
constexpr int NFAC_MAX = 8;    // radix factors of an FFT length
constexpr int TAPS = 13;       // taps of a transposed 7-point stencil (rows j-6 .. j+6)

// Per-plan constants handed to every kernel by value.
struct KP {
    int nr, nt, nz, M, K, nk, mp1;
    double k0, re, dt;
    double lz;
    double t0, omega;     // start time and base-flow angular frequency
    const double* r;      // [nr]
    const double* w;      // [nr]
    const double* D1;     // [2][nr][7] parity 0 = even, 1 = odd
    const double* D2;     // [2][nr][7]
    const double* B;      // [2][nr][7] D2 + D1 / r_j
    const double* D1T;    // [2][nr][TAPS] D1 transposed: tap s of column j = D1[i][j], i = j - 6 + s
    const double* D1WT;   // [2][nr][TAPS] the same with w_i folded in
    const double* BWT;    // [2][nr][TAPS] B transposed with w_i folded in
    const int* col0;      // [nr] first column of each 7-point row
    const double2* Ut;    // [nr] Womersley amplitude
    const double2* dUt;   // [nr] its radial derivative
    const double2* twz;   // [nz] exp(-2 pi i t / nz)
    const double2* twt;   // [nt] exp(-2 pi i t / nt)
    const double* HLU;    // [K+1][M+2][nr-1][9] Helmholtz factors
    const double* PLU;    // [K+1][M+1][nr-1][9] Poisson factors
    const double* HOM;    // [K+1][M+1][3 nr + 1] homogeneous solutions and s_h
    int nfz, nft;
    int fz[NFAC_MAX];
    int ft[NFAC_MAX];
};

// Time of a nonlinear-term evaluation: either `t` itself (direct), or
// t0 + (n + off) dt with the step index n read from device memory (`dstep`,
// when not null: captured graphs replay at any step) or given by value.
struct TimeArg {
    const long long* dstep;
    long long n;
    int off;
    int direct;
    double t;
    // CFL monitor (optional): the evaluation folds the largest
    // dt (|u_z + U| / dz + |u_theta| / (r dtheta) + |u_r| / dr) over its
    // physical points into *cfl (a non-negative double's bit pattern, so an
    // unsigned integer maximum orders it)
    unsigned long long* cfl;
};

// Work descriptor of one instance in a batched launch: one launch per kernel
// serves every instance of a shape class, blockIdx.z selecting the instance;
// the kernel takes its plan constants, buffers, scalars and evaluation time
// from its descriptor instead of its by-value arguments.
struct BDesc {
    KP kp;
    const double2* in[4];
    double2* out[3];
    double s[6];
    TimeArg ta;
    long long* step;
};

// Workspace carve-up (byte offsets into the caller's workspace).
constexpr int NCORR_MAX = 3;

struct WsLayout {
    size_t aux0;                // 2-component vorticity parts of u^n
    size_t auxs[NCORR_MAX];     // ... of the stage iterates w_c
    size_t st[NCORR_MAX];       // stage iterates w_0 .. w_{ncorr-1}
    size_t nn, ns;              // N(u^n), N(w_c)
    size_t muC, muP, yb, zb2;   // adjoint temporaries
    size_t r0;                  // E u^n + N(u^n)/2 of the current step, read by the corrector passes
    size_t fa, fb;              // adjoint convective outputs (A, B)
    size_t fa2, fb2;
    size_t cur, lam, tmp;       // checkpoint-run state buffers
    size_t g, trial, trialN;    // iterate buffers
    size_t zbuf, tbuf;          // z-transformed and theta-pass intermediates
    size_t zst[NCORR_MAX];      // z-transformed u, w of the stage states kept for the adjoint
    size_t red;                 // reduction partials + scalars
    size_t step;                // device step index read by captured step graphs
    size_t total;
};

}  // namespace npo

struct npo_plan_s {
    int nr, nt, nz, M, K, nk, mp1;
    double lz, k0, re, wo, amp, dt, t0, omega;
    int64_t nsteps;
    int ncorr = 2;
    std::vector<double> r, w, D1, D2;
    std::vector<int> col0;
    std::vector<double> ut_re, ut_im, dut_re, dut_im;
    double* d_tables = nullptr;   // one device allocation for all tables
    double* d_cache = nullptr;    // per-mode operator factors and homogeneous solutions
    size_t cache_bytes = 0;
    npo::KP kp;
    npo::WsLayout ws;
    int device = 0;
    // launch shapes
    int zb_theta_fwd = 4, zb_theta_adj = 4;
    int zgroup = 1;
    int rg = 16;          // |k| per radial block (4, 8 or 16)
    mutable npo::Profiler prof;
    // CFL monitor of the forward steps (npo_plan_set_cfl_monitor)
    bool cfl_monitor = false;
    // adjoint of the sweeps (npo_plan_set_adjoint): 0 the exact discrete
    // adjoint, 1 the continuous adjoint equations with the direct stepper
    int adjoint_kind = 0;
    // injected failure of the step drivers (npo_plan_inject_fault): site 1
    // forward steps, 2 adjoint steps; the call after `fault_after` more calls fails
    int fault_site = 0;
    mutable long long fault_after = 0;
    // captured step graphs (see npo_plan_set_graphs); rebuilt for a new workspace
    bool use_graphs = false;
    void* graph_ws = nullptr;
    hipStream_t graph_stream = nullptr;
    hipGraphExec_t g_fwd = nullptr;   // forward advance cur -> cur (aux of cur present), then step += 1
    hipGraphExec_t g_adj = nullptr;   // adjoint step lam -> lam at u = cur
};

#include <functional>

namespace npo {

// Batched launches.  While a Recorder is installed on the calling thread, the
// step-path launchers enqueue nothing: each appends the launch (a closure that
// launches its kernel for nb instances with a descriptor table) and the
// descriptor of the instance being recorded.  Recording the same step for
// every instance of a shape class yields the same launch sequence, which the
// batch then issues once per launch with the instances' descriptors.
struct Recorder {
    std::vector<std::function<void(const BDesc*, int, hipStream_t)>> launch;
    std::vector<BDesc> desc;
    bool ok = true;       // false: a launch without a batched form was met
};
Recorder*& recorder();

// Sampling profiler hooks around one launch on stream st.
void prof_begin(const npo_plan_s& p, int kid, hipStream_t st);
void prof_end(const npo_plan_s& p, int kid, hipStream_t st);

// Enqueue a launch now, or record it (with the descriptor of the instance
// being recorded) while a Recorder is installed.  fn(bd, nb, st) launches the
// kernel for nb instances with descriptor table bd (bd = null: the call's own
// arguments); kid is the profiler family (-1: none).
template <class F>
hipError_t issue(const npo_plan_s& p, int kid, const BDesc& d, hipStream_t st, F fn) {
    if (Recorder* r = recorder()) {
        r->launch.emplace_back(fn);
        r->desc.push_back(d);
        return hipSuccess;
    }
    if (kid >= 0) prof_begin(p, kid, st);
    fn(nullptr, 1, st);
    if (kid >= 0) prof_end(p, kid, st);
    return hipGetLastError();
}
inline BDesc desc_of(const npo_plan_s& p) {
    BDesc d{};
    d.kp = p.kp;
    return d;
}

// Kernel launchers (npo_kernels.hip).  All enqueue on `st` and return the
// hipGetLastError() of the launch.
// Dynamic LDS bytes of the axial passes (G fields per round) and of the
// azimuthal pass (z-block ZB) for this plan's transform lengths.
size_t zpass_lds(const npo_plan_s& p, int G);
size_t theta_lds(const npo_plan_s& p, int ZB, int adj);
// Whether the wave-resident forward azimuthal kernel with L lanes per column
// (tuning value zb_fwd = -L) supports these transform lengths.
bool theta_wave_ok(int nt, int nz, int L);
hipError_t launch_curl_aux(const npo_plan_s& p, const double2* u, double2* aux, hipStream_t st);
// out = a + curl b (continuous-adjoint convective term); no batched form
hipError_t launch_curl_add(const npo_plan_s& p, const double2* a, const double2* b, double2* out, hipStream_t st);
// uw_pre (adjoint only): the axial transforms of the six u, w fields of this
// state, left by an earlier forward evaluation (then only y is transformed);
// uw_save (forward only): where the forward evaluation leaves them (default:
// the workspace's shared buffer).
hipError_t launch_nl(const npo_plan_s& p, int adjoint, const double2* u, const double2* aux,
                     const double2* y, const TimeArg& ta, double2* out0, double2* out1, void* ws, hipStream_t st,
                     const double2* uw_pre = nullptr, double2* uw_save = nullptr);
// *d = v (set) or *d += v (add), one thread.
hipError_t launch_step_index(long long* d, long long v, int add, hipStream_t st);
// *d = v (one 64-bit word).
hipError_t launch_fill_u64(unsigned long long* d, unsigned long long v, hipStream_t st);
// The same for the step index of every instance of a descriptor table.
hipError_t launch_step_index_batched(const BDesc* bd, int nb, long long v, int add, hipStream_t st);

// solve kinds: 0 = out = S(R) with R = a (raw); 1 = predictor S(E a + b),
// which also stores R0 = E a + b/2 in the (+, -, z) basis when r0_out is given;
// 2 = corrector S(R0 + b/2) with a = R0.  aux_out may be null.
hipError_t launch_solve(const npo_plan_s& p, int kind, const double2* a, const double2* b, double2* u_out,
                        double2* aux_out, hipStream_t st, double2* r0_out = nullptr);
// mu = S^dag(ca*A + cb*curl^dag(B)); out0 = mu; Yout = sy*Yin + qy*mu; Zout = sz*Zin + qz*mu
// (B, out0, Yin, Yout, Zin, Zout optional; Yin may alias Yout and Zin Zout).
hipError_t launch_solve_adj(const npo_plan_s& p, const double2* A, double ca, const double2* B, double cb,
                            double2* out0, const double2* Yin, double qy, double2* Yout, const double2* Zin,
                            double qz, double2* Zout, hipStream_t st, double sy = 1.0, double sz = 1.0);
// out = E^dag Z + A + curl^dag B
hipError_t launch_final(const npo_plan_s& p, const double2* Z, const double2* A, const double2* B,
                        double2* out, hipStream_t st);
hipError_t launch_wdot(const npo_plan_s& p, const double2* a, const double2* b, double* partial,
                       double* out, hipStream_t st);
hipError_t launch_project(const npo_plan_s& p, const double2* u, double2* out, hipStream_t st);
// Energy diagnostics of u: out[0..4] = E_r, E_theta, E_z, the energy in the
// modes m = M and in the modes |k| = K; spec (optional) = energy per (m, kk).
// partial: 5 * 256 doubles of scratch.
hipError_t launch_diag(const npo_plan_s& p, const double2* u, double* partial, double* out, double* spec,
                       hipStream_t st);
// out = ca*a + cb*b
hipError_t launch_axpby(const npo_plan_s& p, double ca, const double2* a, double cb, const double2* b,
                        double2* out, hipStream_t st);
// Fixed workspace of npo_forward_step_noalloc (npo_noalloc.hip): resolve the
// device address of the static array on `device` (the current device) once;
// scratch_ptr returns it (null with *err set if it was never resolved or failed).
hipError_t scratch_setup(int device);
void* scratch_ptr(int device, hipError_t* err);

// out = s * 2 pi L_z c_m w_j * x
hipError_t launch_wscale(const npo_plan_s& p, const double2* x, double2* out, double s, hipStream_t st);
// Device-scalar gradient step: from sc[0] = <g,g>_W, sc[1] = <u0,g>_W write
// info[0..3] = E0dag, C0, alpha_max, lambda_+ and out = (1 + lambda_+ al) u0 + al g
// (al = alpha, or alpha_max when alpha <= 0); coef holds 2 doubles of scratch.
hipError_t launch_update_dev(const npo_plan_s& p, const double* sc, double e0, double alpha, double* info,
                             double* coef, const double2* u0, const double2* g, double2* out, hipStream_t st);
// U[j] = U(r_j, t), dUdr[j] = dU/dr(r_j, t) of the laminar base flow (device arrays of nr)
hipError_t launch_base_flow(const npo_plan_s& p, double t, double* U, double* dUdr, hipStream_t st);
// info[4] = en[0] / 2
hipError_t launch_half(const double* en, double* info, hipStream_t st);
// x *= sqrt(e0 / energy_dev[0])
hipError_t launch_rescale(const npo_plan_s& p, double2* x, const double* energy_dev, double e0,
                          hipStream_t st);

}  // namespace npo
