// Device kernels of the NLOP hot path for gfx950 (CDNA4), FP64 throughout.
//
// The time step of the perturbation equations (Keuchel & Avila, Sec. 2 and
// 2.3) factors into three kinds of work with three natural data groupings:
//   * axial FFTs: independent per (radial node j, azimuthal index m) column;
//   * azimuthal FFTs + pointwise products: independent per (j, z) row;
//   * radial solves: independent per Fourier mode (k, m) over all j.
// Each grouping is one kernel family; fields move between them through HBM
// in layouts chosen so every kernel reads and writes contiguous runs.
//
// Spectral field layout: complex [c][j][m][kk], kk in FFT order.
// Intermediate layout (after the axial transform): complex [j][f][m][z].
#include "npo_device.h"

namespace npo {

// ------------------------------------------------------------ vorticity aux
// aux[0] = w_theta = i a u_r - D1 u_z ; aux[1] = w_z = D1 u_theta + u_theta/r - (i m / r) u_r
// Grid: x over kk in tiles of CURL_T, y over (j, m) = j (M + 1) + m, so every
// row offset is uniform over the block and no thread divides its index.
constexpr int CURL_T = 128;
__global__ __launch_bounds__(CURL_T) void k_curl_aux(KP p, const double2* __restrict__ u, double2* __restrict__ aux,
                                                   const BDesc* bd) {
    if (bd) {
        const BDesc& d = bd[blockIdx.z];
        p = d.kp; globalize(p, bd); u = rebase(bd, d.in[0]); aux = rebase(bd, d.out[0]);
    }
    const int kk = blockIdx.x * CURL_T + threadIdx.x;
    const int jm = blockIdx.y, j = jm / p.mp1, m = jm - j * p.mp1;
    if (kk >= p.nk) return;
    const size_t comp = (size_t)p.nr * p.mp1 * p.nk;      // one component
    const size_t rrow = (size_t)p.mp1 * p.nk;             // one radial row of a component
    const double2* ur0 = u + (size_t)jm * p.nk + kk;      // u_r at (j, m, kk)
    const double a = alpha_of(p, kk), r = p.r[j];
    const int c0 = p.col0[j];
    const double* d1e = p.D1 + ((m & 1) * p.nr + j) * 7;
    const double* d1o = p.D1 + (((m + 1) & 1) * p.nr + j) * 7;
    const double2* ut0 = ur0 + comp + (ptrdiff_t)(c0 - j) * (ptrdiff_t)rrow;
    const double2* uz0 = ut0 + comp;
    double2 duz = czero(), dut = czero();
#pragma unroll
    for (int t = 0; t < 7; ++t) {
        duz = caxpy(duz, d1e[t], uz0[(size_t)t * rrow]);
        dut = caxpy(dut, d1o[t], ut0[(size_t)t * rrow]);
    }
    const double2 ur = ur0[0], ut = ur0[comp];
    double2* o = aux + (size_t)jm * p.nk + kk;
    o[0] = csub(cscale(cmuli(ur), a), duz);
    o[comp] = csub(caxpy(dut, 1.0 / r, ut), cscale(cmuli(ur), m / r));
}

// ------------------------------------------------ continuous-adjoint term
// out = a + curl b (the continuous-adjoint convective term from the two
// product fields of the adjoint evaluation: a = Omega x y, b = y x V):
//   (curl b)_r = (i m / r) b_z - i a b_theta
//   (curl b)_theta = i a b_r - D1 b_z
//   (curl b)_z = D1 b_theta + b_theta / r - (i m / r) b_r
__global__ void k_curl_add(KP p, const double2* __restrict__ a, const double2* __restrict__ b,
                           double2* __restrict__ out) {
    const size_t per = (size_t)p.nr * p.mp1 * p.nk;
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per) return;
    const int kk = idx % p.nk;
    const int m = (idx / p.nk) % p.mp1;
    const int j = idx / ((size_t)p.nk * p.mp1);
    const double al = alpha_of(p, kk), r = p.r[j];
    const int c0 = p.col0[j];
    const double* d1e = p.D1 + ((m & 1) * p.nr + j) * 7;
    const double* d1o = p.D1 + (((m + 1) & 1) * p.nr + j) * 7;
    double2 dbz = czero(), dbt = czero();
    for (int t = 0; t < 7; ++t) {
        dbz = caxpy(dbz, d1e[t], b[fidx(p, 2, c0 + t, m, kk)]);
        dbt = caxpy(dbt, d1o[t], b[fidx(p, 1, c0 + t, m, kk)]);
    }
    const double2 br = b[fidx(p, 0, j, m, kk)], bt = b[fidx(p, 1, j, m, kk)], bz = b[fidx(p, 2, j, m, kk)];
    const double mr = m / r;
    out[fidx(p, 0, j, m, kk)] = cadd(a[fidx(p, 0, j, m, kk)], csub(cscale(cmuli(bz), mr), cscale(cmuli(bt), al)));
    out[fidx(p, 1, j, m, kk)] = cadd(a[fidx(p, 1, j, m, kk)], csub(cscale(cmuli(br), al), dbz));
    out[fidx(p, 2, j, m, kk)] =
        cadd(a[fidx(p, 2, j, m, kk)], csub(caxpy(dbt, 1.0 / r, bt), cscale(cmuli(br), mr)));
}

// ------------------------------------------------------ banded operators
// Interior operators on nodes 0..nr-2 (the wall node carries a Dirichlet value
// and its column is removed):
//   Helmholtz H_n = I/dt - (1/(2Re)) (D2 + D1/r - n^2/r^2 - a^2)
//   Poisson   P_n = D2 + D1/r - n^2/r^2 - a^2
// They depend on the plan only, so the host factors each one once (no
// pivoting; growth factor <= 1 for every operator of these grids) into rows of
// 9 doubles: l[0..4] (multipliers of columns i-5..i-1), 1/u_ii,
// u[i][i+1..i+3] (tables p.HLU, p.PLU).  One lane runs one substitution on a
// real vector x[i*s] in LDS; entries needed from earlier rows ride in shift
// registers so no load is on the dependence chain.
constexpr int LUW = 9;
// radial sizes with compile-time substitution chains (others use the loops)
#define NPO_NR_SIZES(X) X(16) X(24) X(32) X(48) X(64)

// (L U) x = b in place.
__device__ void gsubst(const double* __restrict__ LU, int n1, double* x, int s) {
    double y1 = 0.0, y2 = 0.0, y3 = 0.0, y4 = 0.0, y5 = 0.0;   // y_{i-1} .. y_{i-5}
#pragma unroll 4
    for (int i = 0; i < n1; ++i) {
        const double* L = LU + i * LUW;
        double y = x[i * s];
        y = fma(-L[0], y5, y);
        y = fma(-L[1], y4, y);
        y = fma(-L[2], y3, y);
        y = fma(-L[3], y2, y);
        y = fma(-L[4], y1, y);
        x[i * s] = y;
        y5 = y4; y4 = y3; y3 = y2; y2 = y1; y1 = y;
    }
    double x1 = 0.0, x2 = 0.0, x3 = 0.0;                       // x_{i+1} .. x_{i+3}
#pragma unroll 4
    for (int i = n1 - 1; i >= 0; --i) {
        const double* U = LU + i * LUW;
        double v = x[i * s];
        v = fma(-U[8], x3, v);
        v = fma(-U[7], x2, v);
        v = fma(-U[6], x1, v);
        v *= U[5];
        x[i * s] = v;
        x3 = x2; x2 = x1; x1 = v;
    }
}

// (L U)^T x = b in place: U^T z = b forward, then L^T x = z backward.
__device__ void gsubst_T(const double* __restrict__ LU, int n1, double* x, int s) {
    double z1 = 0.0, z2 = 0.0, z3 = 0.0;                       // z_{i-1} .. z_{i-3}
    double u61 = 0.0, u71 = 0.0, u72 = 0.0, u81 = 0.0, u82 = 0.0, u83 = 0.0;
#pragma unroll 4
    for (int i = 0; i < n1; ++i) {
        const double* R = LU + i * LUW;
        const double inv = R[5], r6 = R[6], r7 = R[7], r8 = R[8];
        double v = x[i * s];
        v = fma(-u83, z3, v);
        v = fma(-u72, z2, v);
        v = fma(-u61, z1, v);
        v *= inv;
        x[i * s] = v;
        z3 = z2; z2 = z1; z1 = v;
        u83 = u82; u82 = u81; u81 = r8;
        u72 = u71; u71 = r7;
        u61 = r6;
    }
    double x1 = 0.0, x2 = 0.0, x3 = 0.0, x4 = 0.0, x5 = 0.0;   // x_{i+1} .. x_{i+5}
    double l41 = 0.0, l31 = 0.0, l32 = 0.0, l21 = 0.0, l22 = 0.0, l23 = 0.0;
    double l11 = 0.0, l12 = 0.0, l13 = 0.0, l14 = 0.0, l01 = 0.0, l02 = 0.0, l03 = 0.0, l04 = 0.0, l05 = 0.0;
#pragma unroll 4
    for (int i = n1 - 1; i >= 0; --i) {
        const double* R = LU + i * LUW;
        const double r0 = R[0], r1 = R[1], r2 = R[2], r3 = R[3], r4 = R[4];
        double v = x[i * s];
        v = fma(-l05, x5, v);
        v = fma(-l14, x4, v);
        v = fma(-l23, x3, v);
        v = fma(-l32, x2, v);
        v = fma(-l41, x1, v);
        x[i * s] = v;
        x5 = x4; x4 = x3; x3 = x2; x2 = x1; x1 = v;
        l05 = l04; l04 = l03; l03 = l02; l02 = l01; l01 = r0;
        l14 = l13; l13 = l12; l12 = l11; l11 = r1;
        l23 = l22; l22 = l21; l21 = r2;
        l32 = l31; l31 = r3;
        l41 = r4;
    }
}

// Fully unrolled substitutions for a compile-time size N1.  Factor rows reach
// the chain through a ring of PF rows in registers: the row used at step i is
// refilled with row i + PF, and a scheduling barrier after every step keeps
// those loads where they are written, so PF rows' loads stay in flight and the
// cache latency is paid once per PF rows rather than once per few rows (without
// unrolling, loads carried around a loop are drained at every iteration).  The
// entries of x are read DB steps ahead into a second ring, so no LDS read is on
// the dependence chain either (a row of x is read before its own step writes
// it; the arithmetic and its order are unchanged).  The last PF steps of the
// first pass, which have no rows of their own left to load, load the first PF
// rows of the second pass, so its ring starts full instead of waiting once
// for the whole latency.
template <int N1, int PF, int DB = 4>
__device__ __forceinline__ void gsubst_u(const double* __restrict__ LU, double* x, int s) {
    double y1 = 0.0, y2 = 0.0, y3 = 0.0, y4 = 0.0, y5 = 0.0;   // y_{i-1} .. y_{i-5}
    double Lr[PF][5];
    double Ur[PF][4];                  // ring of the back substitution
#pragma unroll
    for (int r = 0; r < PF; ++r)
        if (r < N1)
#pragma unroll
            for (int c = 0; c < 5; ++c) Lr[r][c] = LU[r * LUW + c];
    double xb[DB];
#pragma unroll
    for (int r = 0; r < DB; ++r)
        if (r < N1) xb[r] = x[r * s];
#pragma unroll
    for (int i = 0; i < N1; ++i) {
        const int r = i % PF;
        double y = xb[i % DB];
        if (i + DB < N1) xb[i % DB] = x[(i + DB) * s];
        y = fma(-Lr[r][0], y5, y);
        y = fma(-Lr[r][1], y4, y);
        y = fma(-Lr[r][2], y3, y);
        y = fma(-Lr[r][3], y2, y);
        y = fma(-Lr[r][4], y1, y);
        x[i * s] = y;
        y5 = y4; y4 = y3; y3 = y2; y2 = y1; y1 = y;
        if (i + PF < N1) {
#pragma unroll
            for (int c = 0; c < 5; ++c) Lr[r][c] = LU[(i + PF) * LUW + c];
        } else if (N1 >= PF) {
            const int kb = i + PF - N1;            // back-substitution step of this row
#pragma unroll
            for (int c = 0; c < 4; ++c) Ur[kb][c] = LU[(N1 - 1 - kb) * LUW + 5 + c];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    double x1 = 0.0, x2 = 0.0, x3 = 0.0;                       // x_{i+1} .. x_{i+3}
    if (N1 < PF) {
#pragma unroll
        for (int r = 0; r < PF; ++r)
            if (r < N1)
#pragma unroll
                for (int c = 0; c < 4; ++c) Ur[r][c] = LU[(N1 - 1 - r) * LUW + 5 + c];
    }
#pragma unroll
    for (int r = 0; r < DB; ++r)
        if (r < N1) xb[r] = x[(N1 - 1 - r) * s];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        const int i = N1 - 1 - k, r = k % PF;
        double v = xb[k % DB];
        if (k + DB < N1) xb[k % DB] = x[(i - DB) * s];
        v = fma(-Ur[r][3], x3, v);
        v = fma(-Ur[r][2], x2, v);
        v = fma(-Ur[r][1], x1, v);
        v *= Ur[r][0];
        x[i * s] = v;
        x3 = x2; x2 = x1; x1 = v;
        if (k + PF < N1)
#pragma unroll
            for (int c = 0; c < 4; ++c) Ur[r][c] = LU[(i - PF) * LUW + 5 + c];
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int N1, int PF, int DB = 4>
__device__ __forceinline__ void gsubst_T_u(const double* __restrict__ LU, double* x, int s) {
    double z1 = 0.0, z2 = 0.0, z3 = 0.0;                       // z_{i-1} .. z_{i-3}
    double u61 = 0.0, u71 = 0.0, u72 = 0.0, u81 = 0.0, u82 = 0.0, u83 = 0.0;
    double Ur[PF][4];
    double Lr[PF][5];                  // ring of the second pass, started in the first
#pragma unroll
    for (int r = 0; r < PF; ++r)
        if (r < N1)
#pragma unroll
            for (int c = 0; c < 4; ++c) Ur[r][c] = LU[r * LUW + 5 + c];
    double xb[DB];
#pragma unroll
    for (int r = 0; r < DB; ++r)
        if (r < N1) xb[r] = x[r * s];
#pragma unroll
    for (int i = 0; i < N1; ++i) {
        const int r = i % PF;
        const double inv = Ur[r][0], r6 = Ur[r][1], r7 = Ur[r][2], r8 = Ur[r][3];
        double v = xb[i % DB];
        if (i + DB < N1) xb[i % DB] = x[(i + DB) * s];
        v = fma(-u83, z3, v);
        v = fma(-u72, z2, v);
        v = fma(-u61, z1, v);
        v *= inv;
        x[i * s] = v;
        z3 = z2; z2 = z1; z1 = v;
        u83 = u82; u82 = u81; u81 = r8;
        u72 = u71; u71 = r7;
        u61 = r6;
        if (i + PF < N1) {
#pragma unroll
            for (int c = 0; c < 4; ++c) Ur[r][c] = LU[(i + PF) * LUW + 5 + c];
        } else if (N1 >= PF) {
            const int kb = i + PF - N1;            // second-pass step of this row
#pragma unroll
            for (int c = 0; c < 5; ++c) Lr[kb][c] = LU[(N1 - 1 - kb) * LUW + c];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    double x1 = 0.0, x2 = 0.0, x3 = 0.0, x4 = 0.0, x5 = 0.0;   // x_{i+1} .. x_{i+5}
    double l41 = 0.0, l31 = 0.0, l32 = 0.0, l21 = 0.0, l22 = 0.0, l23 = 0.0;
    double l11 = 0.0, l12 = 0.0, l13 = 0.0, l14 = 0.0, l01 = 0.0, l02 = 0.0, l03 = 0.0, l04 = 0.0, l05 = 0.0;
    if (N1 < PF) {
#pragma unroll
        for (int r = 0; r < PF; ++r)
            if (r < N1)
#pragma unroll
                for (int c = 0; c < 5; ++c) Lr[r][c] = LU[(N1 - 1 - r) * LUW + c];
    }
#pragma unroll
    for (int r = 0; r < DB; ++r)
        if (r < N1) xb[r] = x[(N1 - 1 - r) * s];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        const int i = N1 - 1 - k, r = k % PF;
        double v = xb[k % DB];
        if (k + DB < N1) xb[k % DB] = x[(i - DB) * s];
        v = fma(-l05, x5, v);
        v = fma(-l14, x4, v);
        v = fma(-l23, x3, v);
        v = fma(-l32, x2, v);
        v = fma(-l41, x1, v);
        x[i * s] = v;
        x5 = x4; x4 = x3; x3 = x2; x2 = x1; x1 = v;
        l05 = l04; l04 = l03; l03 = l02; l02 = l01; l01 = Lr[r][0];
        l14 = l13; l13 = l12; l12 = l11; l11 = Lr[r][1];
        l23 = l22; l22 = l21; l21 = Lr[r][2];
        l32 = l31; l31 = Lr[r][3];
        l41 = Lr[r][4];
        if (k + PF < N1)
#pragma unroll
            for (int c = 0; c < 5; ++c) Lr[r][c] = LU[(i - PF) * LUW + c];
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Substitutions for a compile-time interior size N1C (0: the size n1 given at
// run time).  Ring depths: 12 rows in both solves (about 220 VGPRs of the 256
// that two waves per SIMD allow; 16 would spill).
constexpr int PF_FWD = 12, PF_ADJ = 12;
template <int N1C>
__device__ __forceinline__ void subst(const double* __restrict__ LU, int n1, double* x, int s) {
    if constexpr (N1C > 0) gsubst_u<N1C, PF_FWD>(LU, x, s);
    else gsubst(LU, n1, x, s);
}
template <int N1C>
__device__ __forceinline__ void subst_T(const double* __restrict__ LU, int n1, double* x, int s) {
    if constexpr (N1C > 0) gsubst_T_u<N1C, PF_ADJ>(LU, x, s);
    else gsubst_T(LU, n1, x, s);
}

// -(Poisson wall column) at interior row j: right-hand side of the
// homogeneous pressure with p(1) = 1.
__device__ __forceinline__ double poisson_wall_rhs(const KP& p, int m, int j) {
    const int n1 = p.nr - 1;
    const int w = n1 - p.col0[j];
    return (w >= 0 && w < 7) ? -p.B[((m & 1) * p.nr + j) * 7 + w] : 0.0;
}

// Sum over the 7-point row j of FD table D (parity pi) applied to x[col].
__device__ __forceinline__ double2 fd_apply(const KP& p, const double* D, int pi, int j, const double2* x) {
    const double* d = D + (pi * p.nr + j) * 7;
    const int c0 = p.col0[j];
    double2 s = czero();
#pragma unroll
    for (int t = 0; t < 7; ++t) s = caxpy(s, d[t], x[c0 + t]);
    return s;
}
__device__ __forceinline__ double fd_apply_r(const KP& p, const double* D, int pi, int j, const double* x) {
    const double* d = D + (pi * p.nr + j) * 7;
    const int c0 = p.col0[j];
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < 7; ++t) s = fma(d[t], x[c0 + t], s);
    return s;
}

// Transposed stencil from a 13-tap table T ([2][nr][TAPS]): sum over rows
// i = j - 6 + s inside [0, nr) of T[pi][j][s] * x[i * st].
__device__ __forceinline__ double2 taps13(const KP& p, const double* T, int pi, int j, const double2* x, int st) {
    const double* t = T + (size_t)(pi * p.nr + j) * TAPS;
    const int lo = j < 6 ? 6 - j : 0;
    const int hi = j + 6 >= p.nr ? p.nr + 5 - j : TAPS - 1;
    double2 s = czero();
    for (int k = lo; k <= hi; ++k) s = caxpy(s, t[k], x[(j - 6 + k) * st]);
    return s;
}

// Radial kernels: a block owns one azimuthal index m and RG consecutive |k|
// (RQ = 2*RG modes: +k and -k).  Lanes run over modes, so global loads and
// stores of a radial row touch contiguous runs of kk; the block count is
// padded to a multiple of 8 and consecutive logical blocks are placed on one
// XCD.  Logical blocks run over bands of GB consecutive |k| groups, m outer,
// group inner, so the blocks resident on an XCD at once cover a few groups
// times a few m: neighbouring groups share the 128-byte lines their runs
// straddle (a row is 8176 bytes at K = 255, so most runs are not line
// aligned), and neighbouring m share Helmholtz operators (n = m +- 1).
// RG |k| per block is the plan's tuning value rg (4, 8 or 16; RQ = 2 RG
// modes, 32 RG threads, RJ = 16 radial rows at a time): sixteen (256-byte
// runs, eight waves, one block per CU by LDS) measured 7-10% faster than eight
// (two blocks of four waves per CU) and 30% faster than four at 64 x 96 x 768,
// but a small grid then has few blocks (a 32 x 24 x 96 instance: 16).
constexpr int RJ = 16;     // radial rows handled concurrently
constexpr int GB = 8;      // |k| groups per band of logical blocks

__host__ __device__ __forceinline__ int radial_groups(int K, int rg) { return (K + 1 + rg - 1) / rg; }

template <int RG>
__device__ __forceinline__ bool block_group(const KP& p, int& g, int& m) {
    const int ng = radial_groups(p.K, RG);
    const int nb = ng * p.mp1;
    const int per = (nb + 7) / 8;
    const int b = blockIdx.x;
    const int L = (b % 8) * per + b / 8;
    if (L >= nb) return false;
    // band gb holds groups gb*GB .. gb*GB + gw - 1 (the last band may be narrower)
    const int gb = L / (GB * p.mp1), rem = L - gb * GB * p.mp1;
    const int gw = ng - gb * GB < GB ? ng - gb * GB : GB;
    m = rem / gw;
    g = gb * GB + rem % gw;
    return true;
}

struct Slot {
    int ka, kk;
    double al;
    bool valid, mean;
};
template <int RG>
__device__ __forceinline__ Slot slot_of(const KP& p, int g, int m, int q) {
    Slot s;
    s.ka = g * RG + (q >> 1);
    const int neg = q & 1;
    s.valid = s.ka <= p.K && !(s.ka == 0 && neg);
    s.kk = neg ? p.nk - s.ka : s.ka;
    s.al = (neg ? -s.ka : s.ka) * p.k0;
    s.mean = s.valid && m == 0 && s.ka == 0;
    return s;
}

// ------------------------------------------------------------ forward solve
// Lanes are (radial row, mode) in the pointwise phases and independent real
// right-hand sides (operator, mode, re/im) in the substitution phases.
template <int kind, int NRC, int RG>
__global__ __launch_bounds__(32 * RG) void k_solve(KP p, const double2* __restrict__ ain,
                                              const double2* __restrict__ bin, double2* __restrict__ uout,
                                              double2* __restrict__ auxout, double2* __restrict__ r0out,
                                              const BDesc* bd) {
    if (bd) {
        const BDesc& d = bd[blockIdx.z];
        p = d.kp; globalize(p, bd); ain = rebase(bd, d.in[0]); bin = rebase(bd, d.in[1]); uout = rebase(bd, d.out[0]); auxout = rebase(bd, d.out[1]); r0out = rebase(bd, d.out[2]);
    }
    int g, m;
    constexpr int RQ = 2 * RG;
    if (!block_group<RG>(p, g, m)) return;
    const int t = threadIdx.x, q = t % RQ, jg = t / RQ;
    const int nr = p.nr, N1 = nr - 1;
    const double re2 = 0.5 / p.re, idt = 1.0 / p.dt;
    const int pe = m & 1, po = (m + 1) & 1;
    const size_t opsz = (size_t)N1 * LUW;
    const Slot sl = slot_of<RG>(p, g, m, q);
    const double a2 = sl.al * sl.al;
    __shared__ double2 sR[3][NR_MAX][RQ];
    __shared__ double2 sp[NR_MAX][RQ];
    __shared__ double2 sa[RQ];

    // u (kind 0: R; kind 2: R0 + N/2) in the (+, -, z) basis, staged in LDS; the homogeneous
    // solutions the combine step needs are requested at the same time
    constexpr int NJ = NR_MAX / RJ;
    const double* hom = p.HOM + ((size_t)sl.ka * p.mp1 + m) * (3 * nr + 1);
    double hv[NJ][3];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = jg + jj * RJ;
        hv[jj][0] = hv[jj][1] = hv[jj][2] = 0.0;
        if (j < N1 && sl.valid) {
            hv[jj][0] = hom[j];
            hv[jj][1] = hom[nr + j];
            hv[jj][2] = hom[2 * nr + j];
        }
    }
    for (int j = jg; j < nr; j += RJ) {
        double2 up = czero(), um = czero(), uz = czero();
        if (sl.valid) {
            if constexpr (kind == 2) {
                // R = R0 + N/2 with R0 = E u^n + N(u^n)/2 stored in the (+, -, z) basis
                const double2 nr_ = bin[fidx(p, 0, j, m, sl.kk)], nt_ = bin[fidx(p, 1, j, m, sl.kk)];
                up = caxpy(ain[fidx(p, 0, j, m, sl.kk)], 0.5, cadd(nr_, cmuli(nt_)));
                um = caxpy(ain[fidx(p, 1, j, m, sl.kk)], 0.5, csub(nr_, cmuli(nt_)));
                uz = caxpy(ain[fidx(p, 2, j, m, sl.kk)], 0.5, bin[fidx(p, 2, j, m, sl.kk)]);
            } else {
                const double2 ur = ain[fidx(p, 0, j, m, sl.kk)], ut = ain[fidx(p, 1, j, m, sl.kk)];
                uz = ain[fidx(p, 2, j, m, sl.kk)];
                up = cadd(ur, cmuli(ut));
                um = csub(ur, cmuli(ut));
            }
        }
        sR[0][j][q] = up;
        sR[1][j][q] = um;
        sR[2][j][q] = uz;
    }
    __syncthreads();
    if constexpr (kind == 1) {
        // R = E u^n + N: stencils read from LDS, results held in registers
        // until every lane has read its neighbours
        double2 Rv[NJ][3];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int j = jg + jj * RJ;
            Rv[jj][0] = Rv[jj][1] = Rv[jj][2] = czero();
            if (j < nr && sl.valid) {
                const int kk = sl.kk;
                const double rj = p.r[j];
                const int c0 = p.col0[j];
                const double* bo = p.B + (po * nr + j) * 7;
                const double* be = p.B + (pe * nr + j) * 7;
                double2 lp = czero(), lm = czero(), lz = czero();
#pragma unroll
                for (int s = 0; s < 7; ++s) {
                    lp = caxpy(lp, bo[s], sR[0][c0 + s][q]);
                    lm = caxpy(lm, bo[s], sR[1][c0 + s][q]);
                    lz = caxpy(lz, be[s], sR[2][c0 + s][q]);
                }
                const double2 up = sR[0][j][q], um = sR[1][j][q], uz = sR[2][j][q];
                const double ia = 1.0 / (rj * rj);
                lp = caxpy(lp, -((double)((m + 1) * (m + 1)) * ia + a2), up);
                lm = caxpy(lm, -((double)((m - 1) * (m - 1)) * ia + a2), um);
                lz = caxpy(lz, -((double)(m * m) * ia + a2), uz);
                double2 Nr = bin[fidx(p, 0, j, m, kk)];
                double2 Nt = bin[fidx(p, 1, j, m, kk)];
                double2 Nz = bin[fidx(p, 2, j, m, kk)];
                const double2 Ep = caxpy(cscale(up, idt), re2, lp), Em = caxpy(cscale(um, idt), re2, lm),
                              Ez = caxpy(cscale(uz, idt), re2, lz);
                Rv[jj][0] = cadd(Ep, cadd(Nr, cmuli(Nt)));
                Rv[jj][1] = cadd(Em, csub(Nr, cmuli(Nt)));
                Rv[jj][2] = cadd(Ez, Nz);
                // R0 = E u^n + N(u^n)/2 for the corrector passes of this step
                if (r0out) {
                    r0out[fidx(p, 0, j, m, kk)] = caxpy(Ep, 0.5, cadd(Nr, cmuli(Nt)));
                    r0out[fidx(p, 1, j, m, kk)] = caxpy(Em, 0.5, csub(Nr, cmuli(Nt)));
                    r0out[fidx(p, 2, j, m, kk)] = caxpy(Ez, 0.5, Nz);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < NR_MAX / RJ; ++jj) {
            const int j = jg + jj * RJ;
            if (j < nr) {
                sR[0][j][q] = Rv[jj][0];
                sR[1][j][q] = Rv[jj][1];
                sR[2][j][q] = Rv[jj][2];
            }
        }
        __syncthreads();
    }
    // particular pressure: P_m p = div R on interior nodes, p(1) = 0 (zero for the mean mode)
    for (int j = jg; j < nr; j += RJ) {
        double2 d = czero();
        if (j < N1 && sl.valid && !sl.mean) {
            const double rj = p.r[j];
            const double* d1 = p.D1 + (po * nr + j) * 7;
            const int c0 = p.col0[j];
            double2 dsum = czero();
            for (int s = 0; s < 7; ++s) dsum = caxpy(dsum, d1[s], cadd(sR[0][c0 + s][q], sR[1][c0 + s][q]));
            d = cscale(dsum, 0.5);
            d = caxpy(d, 0.5 * (1 + m) / rj, sR[0][j][q]);
            d = caxpy(d, 0.5 * (1 - m) / rj, sR[1][j][q]);
            d = cadd(d, cscale(cmuli(sR[2][j][q]), sl.al));
        }
        sp[j][q] = d;
    }
    __syncthreads();
    if (t < 2 * RQ) {
        const int qq = t % RQ, part = t / RQ;
        const Slot s2 = slot_of<RG>(p, g, m, qq);
        if (s2.valid && !s2.mean)
            subst<NRC ? NRC - 1 : 0>(p.PLU + ((size_t)s2.ka * p.mp1 + m) * opsz, N1,
                                     reinterpret_cast<double*>(&sp[0][qq]) + part, 2 * RQ);
    }
    __syncthreads();
    // Helmholtz right-hand sides R - grad p; the mean mode keeps (R_theta, R_z)
    for (int j = jg; j < N1; j += RJ) {
        if (sl.mean) {
            sR[1][j][q] = cscale(cmuli(csub(sR[1][j][q], sR[0][j][q])), 0.5);   // (R+ - R-)/(2i)
        } else if (sl.valid) {
            const double mr = m / p.r[j];
            const double* d1 = p.D1 + (pe * nr + j) * 7;
            const int c0 = p.col0[j];
            double2 Dp = czero();
            for (int s = 0; s < 7; ++s) Dp = caxpy(Dp, d1[s], sp[c0 + s][q]);
            const double2 pj = sp[j][q];
            sR[0][j][q] = csub(sR[0][j][q], caxpy(Dp, -mr, pj));
            sR[1][j][q] = csub(sR[1][j][q], caxpy(Dp, mr, pj));
            sR[2][j][q] = csub(sR[2][j][q], cscale(cmuli(pj), sl.al));
        }
    }
    __syncthreads();
    if (t < 6 * RQ) {
        // lane = (operator, mode, re/im): H_{m+1} u+, H_{|m-1|} u-, H_m u_z (mean mode: H_1 u_theta, H_0 u_z)
        const int qq = t % RQ, part = (t / RQ) & 1, op = t / (2 * RQ);
        const Slot s2 = slot_of<RG>(p, g, m, qq);
        if (s2.valid && !(s2.mean && op == 0)) {
            const int n = op == 0 ? m + 1 : (op == 1 ? abs(m - 1) : m);
            subst<NRC ? NRC - 1 : 0>(p.HLU + ((size_t)s2.ka * (p.M + 2) + n) * opsz, N1,
                   reinterpret_cast<double*>(&sR[op][0][qq]) + part, 2 * RQ);
        }
    }
    __syncthreads();
    if (t < RQ && sl.valid) {
        if (sl.mean) {
            // zero flux: u_z += c g with c = -sum w u_z / sum w g
            double2 s = czero();
            for (int i = 0; i < N1; ++i) s = caxpy(s, p.w[i], sR[2][i][q]);
            sa[q] = cscale(s, -1.0 / hom[3 * nr]);
        } else {
            // influence coefficient: zero discrete wall divergence
            const double* dw = p.D1 + (po * nr + N1) * 7;
            const int c0 = p.col0[N1];
            double2 s = czero();
            for (int i = 0; i < 7; ++i)
                if (c0 + i < N1) s = caxpy(s, dw[i], cadd(sR[0][c0 + i][q], sR[1][c0 + i][q]));
            sa[q] = cscale(s, -1.0 / hom[3 * nr]);
        }
    }
    __syncthreads();
    // combine and store (each lane touches only its own (row, mode) here)
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = jg + jj * RJ;
        if (j >= nr) continue;
        double2 ur = czero(), ut = czero(), uz = czero();
        if (j < N1 && sl.valid) {
            const double2 a = sa[q];
            if (sl.mean) {
                ut = sR[1][j][q];
                uz = cadd(sR[2][j][q], cscale(a, hv[jj][0]));
            } else {
                const double2 up = cadd(sR[0][j][q], cscale(a, hv[jj][0]));
                const double2 um = cadd(sR[1][j][q], cscale(a, hv[jj][1]));
                uz = cadd(sR[2][j][q], cscale(cmuli(a), sl.al * hv[jj][2]));
                ur = cscale(cadd(up, um), 0.5);
                ut = cscale(cmuli(csub(um, up)), 0.5);   // (up - um)/(2i)
            }
        }
        sR[0][j][q] = ur;
        sR[1][j][q] = ut;
        sR[2][j][q] = uz;
        if (sl.valid) {
            uout[fidx(p, 0, j, m, sl.kk)] = ur;
            uout[fidx(p, 1, j, m, sl.kk)] = ut;
            uout[fidx(p, 2, j, m, sl.kk)] = uz;
        }
    }
    if (!auxout) return;
    __syncthreads();
    if (!sl.valid) return;
    for (int j = jg; j < nr; j += RJ) {
        const double rj = p.r[j];
        const double* d1e = p.D1 + (pe * nr + j) * 7;
        const double* d1o = p.D1 + (po * nr + j) * 7;
        const int c0 = p.col0[j];
        double2 duz = czero(), dut = czero();
        for (int s = 0; s < 7; ++s) {
            duz = caxpy(duz, d1e[s], sR[2][c0 + s][q]);
            dut = caxpy(dut, d1o[s], sR[1][c0 + s][q]);
        }
        const double2 ur = sR[0][j][q], ut = sR[1][j][q];
        auxout[fidx(p, 0, j, m, sl.kk)] = csub(cscale(cmuli(ur), sl.al), duz);
        auxout[fidx(p, 1, j, m, sl.kk)] = csub(caxpy(dut, 1.0 / rj, ut), cscale(cmuli(ur), m / rj));
    }
}



// curl^H (W b) at row j for b in LDS (rows strided by st), mode index m and
// axial wavenumber al.
__device__ __forceinline__ void curlH_row(const KP& p, int m, double al, int j, const double2* br, const double2* bt,
                                          const double2* bz, int st, double2& cr, double2& ct, double2& cz) {
    const double rj = p.r[j], wj = p.w[j];
    const int pe = m & 1, po = (m + 1) & 1;
    const double2 wr = cscale(br[j * st], wj), wt = cscale(bt[j * st], wj), wz = cscale(bz[j * st], wj);
    cr = cadd(cscale(cmuli(wt), -al), cscale(cmuli(wz), m / rj));
    ct = cadd(cadd(cscale(cmuli(wr), al), taps13(p, p.D1WT, po, j, bz, st)), cscale(wz, 1.0 / rj));
    cz = csub(cscale(cmuli(wr), -m / rj), taps13(p, p.D1WT, pe, j, bt, st));
}

// ------------------------------------------------------------ adjoint solve
// mu = S^dag(ca*A + cb*curl^dag B); out0 = mu; Yout = sy*Yin + qy*mu;
// Zout = sz*Zin + qz*mu.  S^dag = W^{-1} S^H W is applied as the reversed chain
// of conjugate-transposed steps of the forward solve.
struct AdjOut {
    double2* out0;
    const double2* Yin;
    double2* Yout;
    const double2* Zin;
    double2* Zout;
    double qy, qz, sy, sz;
};
template <bool useB, int NRC, int RG>
__global__ __launch_bounds__(32 * RG) void k_solve_adj(KP p, const double2* Ain, double ca, const double2* Bin, double cb,
                                                  AdjOut ao, const BDesc* bd) {
    if (bd) {
        const BDesc& d = bd[blockIdx.z];
        p = d.kp; globalize(p, bd); Ain = rebase(bd, d.in[0]); Bin = rebase(bd, d.in[1]); ao.Yin = rebase(bd, d.in[2]); ao.Zin = rebase(bd, d.in[3]);
        ao.out0 = rebase(bd, d.out[0]); ao.Yout = rebase(bd, d.out[1]); ao.Zout = rebase(bd, d.out[2]);
        ca = d.s[0]; cb = d.s[1]; ao.qy = d.s[2]; ao.qz = d.s[3]; ao.sy = d.s[4]; ao.sz = d.s[5];
    }
    int g, m;
    constexpr int RQ = 2 * RG;
    if (!block_group<RG>(p, g, m)) return;
    const int t = threadIdx.x, q = t % RQ, jg = t / RQ;
    const int nr = p.nr, N1 = nr - 1;
    const int pe = m & 1, po = (m + 1) & 1;
    const size_t opsz = (size_t)N1 * LUW;
    const Slot sl = slot_of<RG>(p, g, m, q);
    constexpr int NJ = NR_MAX / RJ;
    __shared__ double2 sy[3][NR_MAX][RQ];
    __shared__ double2 sphi[NR_MAX][RQ];
    __shared__ double2 sa[RQ];
    __shared__ double2 sred[RJ][RQ];
    // A, B (staged in LDS for the curl stencils) and the homogeneous solutions
    // are requested up front; the accumulators Y, Z only after the
    // substitutions (held across the chains they would take some 100 VGPRs and
    // leave the factor ring 6 rows deep)
    const double* hom = p.HOM + ((size_t)sl.ka * p.mp1 + m) * (3 * nr + 1);
    double2 V[NJ][3], Yv[NJ][3], Zv[NJ][3];
    double hv[NJ][3];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = jg + jj * RJ;
#pragma unroll
        for (int c = 0; c < 3; ++c) V[jj][c] = Yv[jj][c] = Zv[jj][c] = czero();
        hv[jj][0] = hv[jj][1] = hv[jj][2] = 0.0;
        if (j < nr && sl.valid) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const size_t id = fidx(p, c, j, m, sl.kk);
                V[jj][c] = cscale(Ain[id], ca);
                if constexpr (useB) sy[c][j][q] = Bin[id];
            }
            if (j < N1) {
                hv[jj][0] = hom[j];
                hv[jj][1] = hom[nr + j];
                hv[jj][2] = hom[2 * nr + j];
            }
        } else if (useB && j < nr) {
#pragma unroll
            for (int c = 0; c < 3; ++c) sy[c][j][q] = czero();
        }
    }
    if constexpr (useB) {
        // v = ca A + cb W^{-1} curl^H (W B)
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int j = jg + jj * RJ;
            if (j < nr && sl.valid) {
                double2 cr, ct, cz;
                curlH_row(p, m, sl.al, j, &sy[0][0][q], &sy[1][0][q], &sy[2][0][q], RQ, cr, ct, cz);
                const double iw = cb / p.w[j];
                V[jj][0] = caxpy(V[jj][0], iw, cr);
                V[jj][1] = caxpy(V[jj][1], iw, ct);
                V[jj][2] = caxpy(V[jj][2], iw, cz);
            }
        }
        __syncthreads();
    }
    // y = W v on interior rows in the (+, -, z) basis (the solve's wall output
    // is identically zero), and each thread's share of the transposed
    // influence (for the mean mode, flux) sum over its rows
    double2 pr = czero();
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = jg + jj * RJ;
        if (j >= nr) continue;
        const double wj = (j < N1) ? p.w[j] : 0.0;
        const double2 yr = cscale(V[jj][0], wj), yt = cscale(V[jj][1], wj), yz = cscale(V[jj][2], wj);
        double2 y0, y1;
        if (sl.mean) {
            y0 = czero();
            y1 = yt;
            pr = caxpy(pr, hv[jj][0], yz);
        } else {
            y0 = cscale(cadd(yr, cmuli(yt)), 0.5);
            y1 = cscale(csub(yr, cmuli(yt)), 0.5);
            pr = caxpy(pr, hv[jj][0], y0);
            pr = caxpy(pr, hv[jj][1], y1);
            pr = cadd(pr, cscale(cmuli(yz), -sl.al * hv[jj][2]));   // conj(i a uhz) = -i a uhz
        }
        sy[0][j][q] = y0;
        sy[1][j][q] = y1;
        sy[2][j][q] = yz;
    }
    sred[jg][q] = pr;
    __syncthreads();
    if (t < RQ && sl.valid) {
        double2 s = czero();
        for (int i = 0; i < RJ; ++i) s = cadd(s, sred[i][q]);
        sa[q] = cscale(s, 1.0 / hom[3 * nr]);
    }
    __syncthreads();
    if (sl.valid) {
        const double* dw = p.D1 + (po * nr + N1) * 7;
        const int cw0 = p.col0[N1];
        for (int j = jg; j < N1; j += RJ) {
            if (sl.mean) {
                sy[2][j][q] = caxpy(sy[2][j][q], -p.w[j], sa[q]);
            } else {
                const int s = j - cw0;
                if (s >= 0 && s < 7) {
                    sy[0][j][q] = caxpy(sy[0][j][q], -dw[s], sa[q]);
                    sy[1][j][q] = caxpy(sy[1][j][q], -dw[s], sa[q]);
                }
            }
        }
    }
    __syncthreads();
    if (t < 6 * RQ) {
        const int qq = t % RQ, part = (t / RQ) & 1, op = t / (2 * RQ);
        const Slot s2 = slot_of<RG>(p, g, m, qq);
        if (s2.valid && !(s2.mean && op == 0)) {
            const int n = op == 0 ? m + 1 : (op == 1 ? abs(m - 1) : m);
            subst_T<NRC ? NRC - 1 : 0>(p.HLU + ((size_t)s2.ka * (p.M + 2) + n) * opsz, N1,
                     reinterpret_cast<double*>(&sy[op][0][qq]) + part, 2 * RQ);
        }
    }
    __syncthreads();
    // q = G^H w on interior rows (into sphi)
    for (int j = jg; j < nr; j += RJ) {
        double2 qv = czero();
        if (j < N1 && sl.valid && !sl.mean) {
            const double mr = m / p.r[j];
            // rows >= N1 of sy are zero, so the full transposed stencil applies
            qv = cadd(taps13(p, p.D1T, pe, j, &sy[0][0][q], RQ), taps13(p, p.D1T, pe, j, &sy[1][0][q], RQ));
            qv = caxpy(qv, -mr, csub(sy[0][j][q], sy[1][j][q]));
            qv = csub(qv, cscale(cmuli(sy[2][j][q]), sl.al));
        }
        sphi[j][q] = qv;
    }
    __syncthreads();
    if (t < 2 * RQ) {
        const int qq = t % RQ, part = t / RQ;
        const Slot s2 = slot_of<RG>(p, g, m, qq);
        if (s2.valid && !s2.mean)
            subst_T<NRC ? NRC - 1 : 0>(p.PLU + ((size_t)s2.ka * p.mp1 + m) * opsz, N1,
                                       reinterpret_cast<double*>(&sphi[0][qq]) + part,
                     2 * RQ);
    }
    if (sl.valid) {
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int j = jg + jj * RJ;
            if (j < nr) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const size_t id = fidx(p, c, j, m, sl.kk);
                    if (ao.Yout && ao.Yin) Yv[jj][c] = cscale(ao.Yin[id], ao.sy);
                    if (ao.Zout && ao.Zin) Zv[jj][c] = cscale(ao.Zin[id], ao.sz);
                }
            }
        }
    }
    __syncthreads();
    if (!sl.valid) return;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = jg + jj * RJ;
        if (j >= nr) continue;
        const double rj = p.r[j];
        const double iw = 1.0 / p.w[j];
        double2 mv[3];
        if (sl.mean) {
            mv[0] = czero();
            mv[1] = (j < N1) ? cscale(sy[1][j][q], iw) : czero();
            mv[2] = (j < N1) ? cscale(sy[2][j][q], iw) : czero();
        } else {
            const double2 DT = taps13(p, p.D1T, po, j, &sphi[0][q], RQ);   // sphi[N1] = 0
            const double2 ph = (j < N1) ? sphi[j][q] : czero();
            const double2 wp = (j < N1) ? sy[0][j][q] : czero();
            const double2 wm = (j < N1) ? sy[1][j][q] : czero();
            const double2 wz = (j < N1) ? sy[2][j][q] : czero();
            const double2 Rp = csub(wp, cscale(caxpy(DT, (1 + m) / rj, ph), 0.5));
            const double2 Rm = csub(wm, cscale(caxpy(DT, (1 - m) / rj, ph), 0.5));
            const double2 Rz = cadd(wz, cscale(cmuli(ph), sl.al));
            mv[0] = cscale(cadd(Rp, Rm), iw);
            mv[1] = cscale(cmuli(csub(Rm, Rp)), iw);
            mv[2] = cscale(Rz, iw);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t id = fidx(p, c, j, m, sl.kk);
            if (ao.out0) ao.out0[id] = mv[c];
            if (ao.Yout) ao.Yout[id] = caxpy(Yv[jj][c], ao.qy, mv[c]);
            if (ao.Zout) ao.Zout[id] = caxpy(Zv[jj][c], ao.qz, mv[c]);
        }
    }
}

// ----------------------------------------------- adjoint combine (E^dag etc.)
// out = E^dag Z + A + curl^dag B  (Z, A, B optional).  All inputs are
// requested up front; Z, then B, is staged in LDS and every transposed
// stencil reads it there through the 13-tap tables.
template <int RG>
__global__ __launch_bounds__(32 * RG) void k_final(KP p, const double2* __restrict__ Z, const double2* __restrict__ Ain,
                                              const double2* __restrict__ Bin, double2* __restrict__ out,
                                              const BDesc* bd) {
    if (bd) {
        const BDesc& d = bd[blockIdx.z];
        p = d.kp; globalize(p, bd); Z = rebase(bd, d.in[0]); Ain = rebase(bd, d.in[1]); Bin = rebase(bd, d.in[2]); out = rebase(bd, d.out[0]);
    }
    int g, m;
    constexpr int RQ = 2 * RG;
    if (!block_group<RG>(p, g, m)) return;
    const int t = threadIdx.x, q = t % RQ, jg = t / RQ;
    const int nr = p.nr;
    const Slot sl = slot_of<RG>(p, g, m, q);
    const int kk = sl.kk;
    const double a2 = sl.al * sl.al;
    const double re2 = 0.5 / p.re, idt = 1.0 / p.dt;
    const int pe = m & 1, po = (m + 1) & 1;
    constexpr int NJ = NR_MAX / RJ;
    __shared__ double2 s3[3][NR_MAX][RQ];
    double2 E[NJ][3], Av[NJ][3], Bv[NJ][3];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = jg + jj * RJ;
#pragma unroll
        for (int c = 0; c < 3; ++c) E[jj][c] = Av[jj][c] = Bv[jj][c] = czero();
        if (j >= nr) continue;
        double2 zp = czero(), zm = czero(), zz = czero();
        if (sl.valid) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const size_t id = fidx(p, c, j, m, kk);
                if (Ain) Av[jj][c] = Ain[id];
                if (Bin) Bv[jj][c] = Bin[id];
            }
            if (Z) {
                const double2 zr = Z[fidx(p, 0, j, m, kk)], zt = Z[fidx(p, 1, j, m, kk)];
                zz = Z[fidx(p, 2, j, m, kk)];
                zp = cadd(zr, cmuli(zt));
                zm = csub(zr, cmuli(zt));
            }
        }
        if (Z) {
            // E_n^T is applied to W Z in the (+, -, z) basis
            s3[0][j][q] = zp;
            s3[1][j][q] = zm;
            s3[2][j][q] = zz;
        }
    }
    if (Z) {
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int j = jg + jj * RJ;
            if (j < nr && sl.valid) {
                const double rc = p.r[j], wj = p.w[j];
                const double ia = 1.0 / (rc * rc);
                double2 ep = cscale(taps13(p, p.BWT, po, j, &s3[0][0][q], RQ), 0.5 * re2);
                double2 em = cscale(taps13(p, p.BWT, po, j, &s3[1][0][q], RQ), 0.5 * re2);
                double2 ez = cscale(taps13(p, p.BWT, pe, j, &s3[2][0][q], RQ), re2);
                ep = caxpy(ep, 0.5 * wj * (idt - re2 * ((double)((m + 1) * (m + 1)) * ia + a2)), s3[0][j][q]);
                em = caxpy(em, 0.5 * wj * (idt - re2 * ((double)((m - 1) * (m - 1)) * ia + a2)), s3[1][j][q]);
                ez = caxpy(ez, wj * (idt - re2 * ((double)(m * m) * ia + a2)), s3[2][j][q]);
                E[jj][0] = cadd(ep, em);
                E[jj][1] = cmuli(csub(em, ep));     // -i (ep - em)
                E[jj][2] = ez;
            }
        }
        if (Bin) __syncthreads();
    }
    if (Bin) {
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int j = jg + jj * RJ;
            if (j < nr)
#pragma unroll
                for (int c = 0; c < 3; ++c) s3[c][j][q] = Bv[jj][c];
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int j = jg + jj * RJ;
            if (j < nr && sl.valid) {
                double2 cr, ct, cz;
                curlH_row(p, m, sl.al, j, &s3[0][0][q], &s3[1][0][q], &s3[2][0][q], RQ, cr, ct, cz);
                E[jj][0] = cadd(E[jj][0], cr);
                E[jj][1] = cadd(E[jj][1], ct);
                E[jj][2] = cadd(E[jj][2], cz);
            }
        }
    }
    if (!sl.valid) return;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = jg + jj * RJ;
        if (j >= nr) continue;
        const double iw = 1.0 / p.w[j];
#pragma unroll
        for (int c = 0; c < 3; ++c) out[fidx(p, c, j, m, kk)] = caxpy(Av[jj][c], iw, E[jj][c]);
    }
}

// ------------------------------------------------------------ W inner product
constexpr int RED_BLOCKS = 256;
__global__ __launch_bounds__(256) void k_wdot_partial(KP p, const double2* __restrict__ a,
                                                      const double2* __restrict__ b, double* __restrict__ part) {
    __shared__ double s[256];
    const size_t total = (size_t)3 * p.nr * p.mp1 * p.nk;
    double acc = 0.0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)RED_BLOCKS * 256) {
        const int m = (e / p.nk) % p.mp1;
        const int j = (e / ((size_t)p.nk * p.mp1)) % p.nr;
        const double wt = p.w[j] * (m == 0 ? 1.0 : 2.0);
        const double2 x = a[e], y = b[e];
        acc = fma(wt, x.x * y.x + x.y * y.y, acc);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}
// Energy diagnostics of a field (the growth decompositions of Sec. 3-4 and
// the resolution criterion of Sec. 2.3), fixed-order block partials of
//   0..2  <u_c, u_c>_W for c = r, theta, z (twice the component energies),
//   3     the same summed over the modes m = M (the highest azimuthal mode),
//   4     the same summed over the modes |k| = K (the highest axial modes);
// part is [5][RED_BLOCKS].
__global__ __launch_bounds__(256) void k_diag_partial(KP p, const double2* __restrict__ u, double* __restrict__ part) {
    __shared__ double s[5][256];
    const size_t total = (size_t)3 * p.nr * p.mp1 * p.nk;
    const size_t per_c = (size_t)p.nr * p.mp1 * p.nk;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)RED_BLOCKS * 256) {
        const int kk = e % p.nk;
        const int m = (e / p.nk) % p.mp1;
        const int j = (e / ((size_t)p.nk * p.mp1)) % p.nr;
        const int c = (int)(e / per_c);
        const double2 x = u[e];
        const double v = p.w[j] * (m == 0 ? 1.0 : 2.0) * (x.x * x.x + x.y * x.y);
        acc[0] += c == 0 ? v : 0.0;
        acc[1] += c == 1 ? v : 0.0;
        acc[2] += c == 2 ? v : 0.0;
        acc[3] += m == p.M ? v : 0.0;
        acc[4] += (kk == p.K || kk == p.nk - p.K) ? v : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) s[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < 5; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 5) part[threadIdx.x * RED_BLOCKS + blockIdx.x] = s[threadIdx.x][0];
}
// out[q] = scale * sum of the partials of quantity q (q = blockIdx.x)
__global__ __launch_bounds__(256) void k_diag_final(const double* __restrict__ part, double scale,
                                                    double* __restrict__ out) {
    __shared__ double s[256];
    s[threadIdx.x] = part[blockIdx.x * RED_BLOCKS + threadIdx.x];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = s[0] * scale;
}
// Energy of each stored mode (m, kk): 1/2 * 2 pi L_z c_m sum_j w_j sum_c |u|^2.
__global__ void k_mode_energy(KP p, const double2* __restrict__ u, double* __restrict__ spec) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.mp1 * p.nk) return;
    const int m = t / p.nk, kk = t - m * p.nk;
    double acc = 0.0;
    for (int c = 0; c < 3; ++c)
        for (int j = 0; j < p.nr; ++j) {
            const double2 x = u[fidx(p, c, j, m, kk)];
            acc = fma(p.w[j], x.x * x.x + x.y * x.y, acc);
        }
    spec[t] = M_PI * p.lz * (m == 0 ? 1.0 : 2.0) * acc;
}

__global__ __launch_bounds__(256) void k_wdot_final(const double* __restrict__ part, double scale,
                                                    double* __restrict__ out) {
    __shared__ double s[256];
    s[threadIdx.x] = part[threadIdx.x];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0] * scale;
}

// ------------------------------------------------------------ projection
// W-orthogonal projection onto {wall = 0, D u = 0 at every node}; the normal
// matrix D W^-1 D^T (real, SPD) is Cholesky-factored in LDS, and the
// projection is applied twice (one refinement step).
__global__ __launch_bounds__(64) void k_project(KP p, const double2* __restrict__ uin, double2* __restrict__ uout) {
    const int ka = blockIdx.x, m = blockIdx.y, tid = threadIdx.x;
    const int nr = p.nr, N1 = nr - 1;
    const int ncol = ka == 0 ? 1 : 2;
    const int kkc[2] = {ka, ka == 0 ? 0 : p.nk - ka};
    const double alc[2] = {ka * p.k0, -ka * p.k0};
    const double a2 = alc[0] * alc[0];
    const int po = (m + 1) & 1;
    __shared__ double Mx[NR_MAX][NR_MAX + 1];
    __shared__ double2 su[3][2][NR_MAX];
    __shared__ double2 sd[2][NR_MAX];
    __shared__ double2 sc[2];
    if (tid < nr) {
        for (int col = 0; col < 2; ++col)
            for (int c = 0; c < 3; ++c)
                su[c][col][tid] = (col < ncol && tid < N1) ? uin[fidx(p, c, tid, m, kkc[col])] : czero();
    }
    __syncthreads();
    if (m == 0 && ka == 0) {
        if (tid == 0) {
            double2 s = czero();
            double ws = 0.0;
            for (int i = 0; i < N1; ++i) {
                s = caxpy(s, p.w[i], su[2][0][i]);
                ws += p.w[i];
            }
            sc[0] = cscale(s, 1.0 / ws);
        }
        __syncthreads();
        if (tid < nr) {
            uout[fidx(p, 0, tid, 0, 0)] = czero();
            uout[fidx(p, 1, tid, 0, 0)] = su[1][0][tid];
            uout[fidx(p, 2, tid, 0, 0)] = (tid < N1) ? csub(su[2][0][tid], sc[0]) : czero();
        }
        return;
    }
    // Ar[i][c] = D1o[i][c] + delta_ic / r_i on columns c < N1
    for (int e = tid; e < nr * nr; e += blockDim.x) {
        const int i = e / nr, k = e - i * nr;
        double s = 0.0;
        if (k >= i) {
            const int lo = max(p.col0[i], p.col0[k]);
            const int hi = min(min(p.col0[i], p.col0[k]) + 6, N1 - 1);
            for (int c = lo; c <= hi; ++c) {
                const double ai = fdw(p.D1, po, nr, p.col0, i, c) + (c == i ? 1.0 / p.r[i] : 0.0);
                const double ak = fdw(p.D1, po, nr, p.col0, k, c) + (c == k ? 1.0 / p.r[k] : 0.0);
                s += ai * ak / p.w[c];
            }
            if (i == k && i < N1) s += ((double)(m * m) / (p.r[i] * p.r[i]) + a2) / p.w[i];
            Mx[i][k] = s;
            Mx[k][i] = s;
        }
    }
    __syncthreads();
    // Cholesky (lower) in place
    for (int k = 0; k < nr; ++k) {
        if (tid == 0) Mx[k][k] = sqrt(Mx[k][k]);
        __syncthreads();
        for (int i = k + 1 + tid; i < nr; i += blockDim.x) Mx[i][k] /= Mx[k][k];
        __syncthreads();
        for (int e = tid; e < (nr - k - 1) * (nr - k - 1); e += blockDim.x) {
            const int i = k + 1 + e / (nr - k - 1), c = k + 1 + e % (nr - k - 1);
            if (c <= i) Mx[i][c] -= Mx[i][k] * Mx[c][k];
        }
        __syncthreads();
    }
    for (int pass = 0; pass < 2; ++pass) {
        // d = D u
        if (tid < nr) {
            const double ri = p.r[tid];
            for (int col = 0; col < 2; ++col) {
                double2 d = czero();
                const int c0 = p.col0[tid];
                for (int t = 0; t < 7; ++t) {
                    const int c = c0 + t;
                    if (c < N1) d = caxpy(d, p.D1[(po * nr + tid) * 7 + t], su[0][col][c]);
                }
                if (tid < N1) {
                    d = caxpy(d, 1.0 / ri, su[0][col][tid]);
                    d = cadd(d, cscale(cmuli(su[1][col][tid]), m / ri));
                    d = cadd(d, cscale(cmuli(su[2][col][tid]), alc[col]));
                }
                sd[col][tid] = d;
            }
        }
        __syncthreads();
        // L L^T phi = d
        for (int k = 0; k < nr; ++k) {
            if (tid < 2) sd[tid][k] = cscale(sd[tid][k], 1.0 / Mx[k][k]);
            __syncthreads();
            for (int i = k + 1 + tid; i < nr; i += blockDim.x)
                for (int col = 0; col < 2; ++col) sd[col][i] = caxpy(sd[col][i], -Mx[i][k], sd[col][k]);
            __syncthreads();
        }
        for (int k = nr - 1; k >= 0; --k) {
            if (tid < 2) sd[tid][k] = cscale(sd[tid][k], 1.0 / Mx[k][k]);
            __syncthreads();
            for (int i = tid; i < k; i += blockDim.x)
                for (int col = 0; col < 2; ++col) sd[col][i] = caxpy(sd[col][i], -Mx[k][i], sd[col][k]);
            __syncthreads();
        }
        // u -= W^-1 D^H phi on interior rows
        if (tid < N1) {
            const double rc = p.r[tid], iw = 1.0 / p.w[tid];
            for (int col = 0; col < 2; ++col) {
                double2 dr = cscale(sd[col][tid], 1.0 / rc);
                const int lo = max(0, tid - 6), hi = min(nr - 1, tid + 6);
                for (int i = lo; i <= hi; ++i) dr = caxpy(dr, fdw(p.D1, po, nr, p.col0, i, tid), sd[col][i]);
                const double2 dt = cscale(cmuli(sd[col][tid]), -m / rc);
                const double2 dz = cscale(cmuli(sd[col][tid]), -alc[col]);
                su[0][col][tid] = caxpy(su[0][col][tid], -iw, dr);
                su[1][col][tid] = caxpy(su[1][col][tid], -iw, dt);
                su[2][col][tid] = caxpy(su[2][col][tid], -iw, dz);
            }
        }
        __syncthreads();
    }
    if (tid < nr) {
        for (int col = 0; col < ncol; ++col)
            for (int c = 0; c < 3; ++c) uout[fidx(p, c, tid, m, kkc[col])] = su[c][col][tid];
    }
}

__global__ void k_axpby(size_t n, double ca, const double2* __restrict__ a, double cb, const double2* __restrict__ b,
                        double2* __restrict__ out) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 v = cscale(a[i], ca);
    if (b) v = caxpy(v, cb, b[i]);
    out[i] = v;
}
// out = s * q (.) x with q = 2 pi L_z c_m w_j: the W-gradient as a Euclidean
// gradient in the (Re, Im) coordinates of the stored coefficients.
__global__ void k_wscale(KP p, const double2* __restrict__ x, double2* __restrict__ out, double s) {
    const size_t total = (size_t)3 * p.nr * p.mp1 * p.nk;
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int m = (e / p.nk) % p.mp1;
    const int j = (e / ((size_t)p.nk * p.mp1)) % p.nr;
    const double q = s * 2.0 * M_PI * p.lz * p.w[j] * (m == 0 ? 1.0 : 2.0);
    out[e] = cscale(x[e], q);
}
__global__ void k_rescale(size_t n, double2* __restrict__ x, const double* __restrict__ en, double e0) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = sqrt(e0 / en[0]);
    x[i] = cscale(x[i], s);
}

// Scalars of the gradient step (Sec. 2.2) from sc[0] = <g,g>_W and
// sc[1] = <u0,g>_W, with udag = -g: E0dag = <g,g>/2, C0 = <u0,udag> = -<u0,g>,
// alpha_max from the reality condition of the multiplier, lambda_+ the '+' root
// of the energy constraint at step al (alpha, or alpha_max when alpha <= 0; the
// discriminant is clamped at 0, where it sits at alpha_max).  Writes
// info[0..3] = E0dag, C0, alpha_max, lambda_+ and coef[0..1] such that
// u_new = coef[0] u0 + coef[1] g.  With alpha_max infinite (g parallel to u0)
// and alpha <= 0 the step is empty: coef = (1, 0), lambda_+ = 0.
__global__ void k_update_coef(const double* __restrict__ sc, double e0, double alpha, double* __restrict__ info,
                              double* __restrict__ coef) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double E0d = 0.5 * sc[0], C0 = -sc[1];
    const double q = E0d / e0 - C0 * C0 / (4.0 * e0 * e0);
    const double amax = q > 0.0 ? 1.0 / sqrt(q) : __builtin_inf();
    const double al = alpha > 0.0 ? alpha : amax;
    double lam = 0.0, c0 = 1.0, c1 = 0.0;
    if (al < __builtin_inf()) {
        const double a = (al * C0 - 2.0 * e0) / (2.0 * al * e0);
        const double disc = a * a - (al * E0d - C0) / (al * e0);
        lam = a + sqrt(disc > 0.0 ? disc : 0.0);
        c0 = 1.0 + lam * al;
        c1 = al;
    }
    info[0] = E0d; info[1] = C0; info[2] = amax; info[3] = lam;
    coef[0] = c0; coef[1] = c1;
}

// out = coef[0] a + coef[1] b with the coefficients read from device memory.
__global__ void k_axpby_dev(size_t n, const double* __restrict__ coef, const double2* __restrict__ a,
                            const double2* __restrict__ b, double2* __restrict__ out) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = caxpy(cscale(a[i], coef[0]), coef[1], b[i]);
}

// Laminar base flow at time t (Sec. 2, Sexl-Womersley profile): U(r_j, t) and
// dU/dr = -Omega_theta at every radial node, from the same device helper the
// transform kernels use.
__global__ void k_base_flow(KP p, double t, double* __restrict__ U, double* __restrict__ dUdr) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p.nr) return;
    double sw, cw, u, om;
    sincos(p.omega * t, &sw, &cw);
    base_at(p, j, cw, sw, u, om);
    U[j] = u;
    dUdr[j] = -om;
}

// info[4] = <u,u>_W / 2 (the energy of the updated iterate before rescaling).
__global__ void k_half(const double* __restrict__ en, double* __restrict__ info) {
    if (threadIdx.x == 0 && blockIdx.x == 0) info[4] = 0.5 * en[0];
}

// Device step index of captured step graphs: *d = v or *d += v.
__global__ void k_step_index(long long* d, long long v, int add, const BDesc* bd) {
    if (bd) d = bd[blockIdx.z].step;
    if (threadIdx.x == 0) *d = add ? *d + v : v;
}

// ---------------------------------------------------------------- launchers
static inline size_t field_elems(const npo_plan_s& p) { return (size_t)3 * p.nr * p.mp1 * p.nk; }

Recorder*& recorder() {
    static thread_local Recorder* r = nullptr;
    return r;
}


// *d = v for one 64-bit word (a fill kernel, so that capture-safe clears need no memset node).
__global__ void k_fill_u64(unsigned long long* d, unsigned long long v) {
    if (threadIdx.x == 0) *d = v;
}
hipError_t launch_fill_u64(unsigned long long* d, unsigned long long v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, d, v);
    return hipGetLastError();
}

hipError_t launch_step_index(long long* d, long long v, int add, hipStream_t st) {
    if (recorder()) return hipErrorInvalidValue;     // the batch advances its step indices itself
    hipLaunchKernelGGL(k_step_index, dim3(1), dim3(64), 0, st, d, v, add, nullptr);
    return hipGetLastError();
}
hipError_t launch_step_index_batched(const BDesc* bd, int nb, long long v, int add, hipStream_t st) {
    hipLaunchKernelGGL(k_step_index, dim3(1, 1, nb), dim3(64), 0, st, nullptr, v, add, bd);
    return hipGetLastError();
}
hipError_t launch_curl_aux(const npo_plan_s& p, const double2* u, double2* aux, hipStream_t st) {
    BDesc d = desc_of(p);
    d.in[0] = u;
    d.out[0] = aux;
    const KP kp = p.kp;
    const unsigned gx = (unsigned)((p.nk + CURL_T - 1) / CURL_T), gy = (unsigned)(p.nr * p.mp1);
    return issue(p, KID_CURL, d, st, [=](const BDesc* bd, int nb, hipStream_t s) {
        hipLaunchKernelGGL(k_curl_aux, dim3(gx, gy, nb), dim3(CURL_T), 0, s, kp, u, aux, bd);
    });
}
hipError_t launch_curl_add(const npo_plan_s& p, const double2* a, const double2* b, double2* out, hipStream_t st) {
    if (Recorder* r = recorder()) r->ok = false;     // no batched form
    const size_t per = (size_t)p.nr * p.mp1 * p.nk;
    const unsigned gx = (unsigned)((per + 255) / 256);
    hipLaunchKernelGGL(k_curl_add, dim3(gx), dim3(256), 0, st, p.kp, a, b, out);
    return hipGetLastError();
}
// Radial launches: blocks of 32 RG threads over radial_groups(K, RG) |k|
// groups times M + 1 azimuthal indices (padded to a multiple of 8 for the
// XCD placement), RG the plan's rg.
static unsigned radial_grid(const npo_plan_s& p) {
    return (unsigned)((radial_groups(p.K, p.rg) * p.mp1 + 7) / 8 * 8);
}
template <int R, int G>
static hipError_t launch_solve_r(const npo_plan_s& p, int kid, int kind, unsigned gx, const BDesc& d,
                                 const double2* a, const double2* b, double2* u_out, double2* aux_out,
                                 double2* r0_out, hipStream_t st) {
    const KP kp = p.kp;
    return issue(p, kid, d, st, [=](const BDesc* bd, int nb, hipStream_t s) {
        const dim3 grid(gx, 1, nb), blk(32 * G);
        if (kind == 1) hipLaunchKernelGGL((k_solve<1, R, G>), grid, blk, 0, s, kp, a, b, u_out, aux_out, r0_out, bd);
        else if (kind == 2)
            hipLaunchKernelGGL((k_solve<2, R, G>), grid, blk, 0, s, kp, a, b, u_out, aux_out, r0_out, bd);
        else hipLaunchKernelGGL((k_solve<0, R, G>), grid, blk, 0, s, kp, a, b, u_out, aux_out, r0_out, bd);
    });
}
template <int G>
static hipError_t launch_solve_g(const npo_plan_s& p, int kid, int kind, unsigned gx, const BDesc& d,
                                 const double2* a, const double2* b, double2* u_out, double2* aux_out,
                                 double2* r0_out, hipStream_t st) {
    switch (p.nr) {
#define NPO_CASE(R)                                                                          \
    case R:                                                                                  \
        return launch_solve_r<R, G>(p, kid, kind, gx, d, a, b, u_out, aux_out, r0_out, st);
        NPO_NR_SIZES(NPO_CASE)
#undef NPO_CASE
    default:
        return launch_solve_r<0, G>(p, kid, kind, gx, d, a, b, u_out, aux_out, r0_out, st);
    }
}
hipError_t launch_solve(const npo_plan_s& p, int kind, const double2* a, const double2* b, double2* u_out,
                        double2* aux_out, hipStream_t st, double2* r0_out) {
    const int kid = kind == 1 ? KID_SOLVE_P : (kind == 2 ? KID_SOLVE_C : KID_SOLVE_R);
    const unsigned gx = radial_grid(p);
    BDesc d = desc_of(p);
    d.in[0] = a; d.in[1] = b;
    d.out[0] = u_out; d.out[1] = aux_out; d.out[2] = r0_out;
    if (p.rg == 4) return launch_solve_g<4>(p, kid, kind, gx, d, a, b, u_out, aux_out, r0_out, st);
    if (p.rg == 8) return launch_solve_g<8>(p, kid, kind, gx, d, a, b, u_out, aux_out, r0_out, st);
    return launch_solve_g<16>(p, kid, kind, gx, d, a, b, u_out, aux_out, r0_out, st);
}
template <int R, int G>
static hipError_t launch_solve_adj_r(const npo_plan_s& p, unsigned gx, const BDesc& d, const double2* A, double ca,
                                     const double2* B, double cb, AdjOut ao, hipStream_t st) {
    const KP kp = p.kp;
    return issue(p, B ? KID_SOLVE_ADJ2 : KID_SOLVE_ADJ, d, st, [=](const BDesc* bd, int nb, hipStream_t s) {
        const dim3 grid(gx, 1, nb), blk(32 * G);
        if (B) hipLaunchKernelGGL((k_solve_adj<true, R, G>), grid, blk, 0, s, kp, A, ca, B, cb, ao, bd);
        else hipLaunchKernelGGL((k_solve_adj<false, R, G>), grid, blk, 0, s, kp, A, ca, B, cb, ao, bd);
    });
}
template <int G>
static hipError_t launch_solve_adj_g(const npo_plan_s& p, unsigned gx, const BDesc& d, const double2* A, double ca,
                                     const double2* B, double cb, AdjOut ao, hipStream_t st) {
    switch (p.nr) {
#define NPO_CASE(R)                                                               \
    case R:                                                                       \
        return launch_solve_adj_r<R, G>(p, gx, d, A, ca, B, cb, ao, st);
        NPO_NR_SIZES(NPO_CASE)
#undef NPO_CASE
    default:
        return launch_solve_adj_r<0, G>(p, gx, d, A, ca, B, cb, ao, st);
    }
}
hipError_t launch_solve_adj(const npo_plan_s& p, const double2* A, double ca, const double2* B, double cb,
                            double2* out0, const double2* Yin, double qy, double2* Yout, const double2* Zin,
                            double qz, double2* Zout, hipStream_t st, double sy, double sz) {
    AdjOut ao{out0, Yin, Yout, Zin, Zout, qy, qz, sy, sz};
    const unsigned gx = radial_grid(p);
    BDesc d = desc_of(p);
    d.in[0] = A; d.in[1] = B; d.in[2] = Yin; d.in[3] = Zin;
    d.out[0] = out0; d.out[1] = Yout; d.out[2] = Zout;
    d.s[0] = ca; d.s[1] = cb; d.s[2] = qy; d.s[3] = qz; d.s[4] = sy; d.s[5] = sz;
    if (p.rg == 4) return launch_solve_adj_g<4>(p, gx, d, A, ca, B, cb, ao, st);
    if (p.rg == 8) return launch_solve_adj_g<8>(p, gx, d, A, ca, B, cb, ao, st);
    return launch_solve_adj_g<16>(p, gx, d, A, ca, B, cb, ao, st);
}
template <int G>
static hipError_t launch_final_g(const npo_plan_s& p, unsigned gx, const BDesc& d, const double2* Z,
                                 const double2* A, const double2* B, double2* out, hipStream_t st) {
    const KP kp = p.kp;
    return issue(p, KID_FINAL, d, st, [=](const BDesc* bd, int nb, hipStream_t s) {
        hipLaunchKernelGGL((k_final<G>), dim3(gx, 1, nb), dim3(32 * G), 0, s, kp, Z, A, B, out, bd);
    });
}
hipError_t launch_final(const npo_plan_s& p, const double2* Z, const double2* A, const double2* B, double2* out,
                        hipStream_t st) {
    BDesc d = desc_of(p);
    d.in[0] = Z; d.in[1] = A; d.in[2] = B;
    d.out[0] = out;
    const unsigned gx = radial_grid(p);
    if (p.rg == 4) return launch_final_g<4>(p, gx, d, Z, A, B, out, st);
    if (p.rg == 8) return launch_final_g<8>(p, gx, d, Z, A, B, out, st);
    return launch_final_g<16>(p, gx, d, Z, A, B, out, st);
}

hipError_t launch_wdot(const npo_plan_s& p, const double2* a, const double2* b, double* partial, double* out,
                       hipStream_t st) {
    prof_begin(p, KID_WDOT, st);
    hipLaunchKernelGGL(k_wdot_partial, dim3(RED_BLOCKS), dim3(256), 0, st, p.kp, a, b, partial);
    prof_end(p, KID_WDOT, st);
    hipLaunchKernelGGL(k_wdot_final, dim3(1), dim3(256), 0, st, partial, 2.0 * M_PI * p.lz, out);
    return hipGetLastError();
}

hipError_t launch_diag(const npo_plan_s& p, const double2* u, double* partial, double* out, double* spec,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_diag_partial, dim3(RED_BLOCKS), dim3(256), 0, st, p.kp, u, partial);
    hipLaunchKernelGGL(k_diag_final, dim3(5), dim3(256), 0, st, partial, M_PI * p.lz, out);   // energies: <.,.>/2
    if (spec) {
        const int n = p.mp1 * p.nk;
        hipLaunchKernelGGL(k_mode_energy, dim3((n + 255) / 256), dim3(256), 0, st, p.kp, u, spec);
    }
    return hipGetLastError();
}

hipError_t launch_project(const npo_plan_s& p, const double2* u, double2* out, hipStream_t st) {
    prof_begin(p, KID_PROJECT, st);
    hipLaunchKernelGGL(k_project, dim3(p.K + 1, p.mp1), dim3(64), 0, st, p.kp, u, out);
    prof_end(p, KID_PROJECT, st);
    return hipGetLastError();
}

hipError_t launch_axpby(const npo_plan_s& p, double ca, const double2* a, double cb, const double2* b, double2* out,
                        hipStream_t st) {
    const size_t n = field_elems(p);
    prof_begin(p, KID_AXPBY, st);
    hipLaunchKernelGGL(k_axpby, dim3((n + 255) / 256), dim3(256), 0, st, n, ca, a, cb, b, out);
    prof_end(p, KID_AXPBY, st);
    return hipGetLastError();
}

hipError_t launch_wscale(const npo_plan_s& p, const double2* x, double2* out, double s, hipStream_t st) {
    const size_t n = field_elems(p);
    hipLaunchKernelGGL(k_wscale, dim3((n + 255) / 256), dim3(256), 0, st, p.kp, x, out, s);
    return hipGetLastError();
}

hipError_t launch_update_dev(const npo_plan_s& p, const double* sc, double e0, double alpha, double* info,
                             double* coef, const double2* u0, const double2* g, double2* out, hipStream_t st) {
    const size_t n = field_elems(p);
    hipLaunchKernelGGL(k_update_coef, dim3(1), dim3(64), 0, st, sc, e0, alpha, info, coef);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_axpby_dev, dim3((n + 255) / 256), dim3(256), 0, st, n, coef, u0, g, out);
    return hipGetLastError();
}

hipError_t launch_base_flow(const npo_plan_s& p, double t, double* U, double* dUdr, hipStream_t st) {
    hipLaunchKernelGGL(k_base_flow, dim3(1), dim3(64), 0, st, p.kp, t, U, dUdr);
    return hipGetLastError();
}

hipError_t launch_half(const double* en, double* info, hipStream_t st) {
    hipLaunchKernelGGL(k_half, dim3(1), dim3(64), 0, st, en, info);
    return hipGetLastError();
}

hipError_t launch_rescale(const npo_plan_s& p, double2* x, const double* en, double e0, hipStream_t st) {
    const size_t n = field_elems(p);
    hipLaunchKernelGGL(k_rescale, dim3((n + 255) / 256), dim3(256), 0, st, n, x, en, e0);
    return hipGetLastError();
}

}  // namespace npo
