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
#include "npo_internal.h"

namespace npo {

// ------------------------------------------------------------------ complex
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cmuli(double2 a) { return make_double2(-a.y, a.x); }   // i*a
__device__ __forceinline__ double2 czero() { return make_double2(0.0, 0.0); }
// a + s*b (s real)
__device__ __forceinline__ double2 caxpy(double2 a, double s, double2 b) {
    return make_double2(fma(s, b.x, a.x), fma(s, b.y, a.y));
}

__device__ __forceinline__ double alpha_of(const KP& p, int kk) {
    return (kk <= p.K ? kk : kk - p.nk) * p.k0;
}
__device__ __forceinline__ size_t fidx(const KP& p, int c, int j, int m, int kk) {
    return ((size_t)(c * p.nr + j) * p.mp1 + m) * p.nk + kk;
}
// 7-point FD weight of row `row` at column `col` (0 outside the stencil).
__device__ __forceinline__ double fdw(const double* D, int pi, int nr, const int* col0, int row, int col) {
    int t = col - col0[row];
    return (t >= 0 && t < 7) ? D[(pi * nr + row) * 7 + t] : 0.0;
}

// Base flow at node j: U and Omega_theta = -dU/dr, with (cw, sw) = (cos wt, sin wt).
__device__ __forceinline__ void base_at(const KP& p, int j, double cw, double sw, double& U, double& Om) {
    double r = p.r[j];
    double2 a = p.Ut[j], b = p.dUt[j];
    U = 1.0 - r * r + (a.x * cw - a.y * sw);
    Om = 2.0 * r - (b.x * cw - b.y * sw);
}

// ---------------------------------------------------------------- LDS FFTs
// Batched Stockham autosort FFT of B transforms of length n held in LDS
// (a: input, b: scratch); radices 2, 3, 4.  sg = -1 forward, +1 inverse,
// no scaling.  tw[t] = exp(-2 pi i t / n).  Returns the buffer with the result.
__device__ double2* fft_lds(double2* a, double2* b, int B, int n, const int* fac, int nfac,
                            const double2* __restrict__ tw, double sg) {
    int Ns = 1;
    for (int s = 0; s < nfac; ++s) {
        const int R = fac[s];
        const int nb = n / R;
        const int total = B * nb;
        const int tws = n / (Ns * R);
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            const int bi = t / nb;
            const int jj = t - bi * nb;
            const double2* x = a + bi * n;
            double2* y = b + bi * n;
            const int k = jj % Ns;
            const int base = (jj / Ns) * Ns * R + k;
            if (R == 4) {
                double2 v0 = x[jj], v1 = x[jj + nb], v2 = x[jj + 2 * nb], v3 = x[jj + 3 * nb];
                if (k) {
                    double2 w1 = tw[k * tws], w2 = tw[2 * k * tws], w3 = tw[3 * k * tws];
                    if (sg > 0) { w1.y = -w1.y; w2.y = -w2.y; w3.y = -w3.y; }
                    v1 = cmul(v1, w1); v2 = cmul(v2, w2); v3 = cmul(v3, w3);
                }
                double2 s02 = cadd(v0, v2), d02 = csub(v0, v2);
                double2 s13 = cadd(v1, v3), d13 = csub(v1, v3);
                // w = exp(sg * 2 pi i / 4) = sg * i
                double2 wd = cmuli(d13);
                if (sg < 0) wd = make_double2(-wd.x, -wd.y);
                y[base] = cadd(s02, s13);
                y[base + Ns] = cadd(d02, wd);
                y[base + 2 * Ns] = csub(s02, s13);
                y[base + 3 * Ns] = csub(d02, wd);
            } else if (R == 2) {
                double2 v0 = x[jj], v1 = x[jj + nb];
                if (k) {
                    double2 w1 = tw[k * tws];
                    if (sg > 0) w1.y = -w1.y;
                    v1 = cmul(v1, w1);
                }
                y[base] = cadd(v0, v1);
                y[base + Ns] = csub(v0, v1);
            } else {  // R == 3
                double2 v0 = x[jj], v1 = x[jj + nb], v2 = x[jj + 2 * nb];
                if (k) {
                    double2 w1 = tw[k * tws], w2 = tw[2 * k * tws];
                    if (sg > 0) { w1.y = -w1.y; w2.y = -w2.y; }
                    v1 = cmul(v1, w1); v2 = cmul(v2, w2);
                }
                const double c = -0.5, s3 = 0.86602540378443864676 * sg;
                double2 s12 = cadd(v1, v2), d12 = csub(v1, v2);
                double2 t0 = caxpy(v0, c, s12);
                double2 t1 = cscale(cmuli(d12), s3);
                y[base] = cadd(v0, s12);
                y[base + Ns] = cadd(t0, t1);
                y[base + 2 * Ns] = csub(t0, t1);
            }
        }
        __syncthreads();
        double2* tmp = a; a = b; b = tmp;
        Ns *= R;
    }
    return a;
}

// ------------------------------------------------------------ vorticity aux
// aux[0] = w_theta = i a u_r - D1 u_z ; aux[1] = w_z = D1 u_theta + u_theta/r - (i m / r) u_r
__global__ void k_curl_aux(KP p, const double2* __restrict__ u, double2* __restrict__ aux) {
    const size_t per = (size_t)p.nr * p.mp1 * p.nk;
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per) return;
    const int kk = idx % p.nk;
    const int m = (idx / p.nk) % p.mp1;
    const int j = idx / ((size_t)p.nk * p.mp1);
    const double a = alpha_of(p, kk), r = p.r[j];
    const int c0 = p.col0[j];
    const double* d1e = p.D1 + ((m & 1) * p.nr + j) * 7;
    const double* d1o = p.D1 + (((m + 1) & 1) * p.nr + j) * 7;
    double2 duz = czero(), dut = czero();
    for (int t = 0; t < 7; ++t) {
        duz = caxpy(duz, d1e[t], u[fidx(p, 2, c0 + t, m, kk)]);
        dut = caxpy(dut, d1o[t], u[fidx(p, 1, c0 + t, m, kk)]);
    }
    const double2 ur = u[fidx(p, 0, j, m, kk)], ut = u[fidx(p, 1, j, m, kk)];
    aux[fidx(p, 0, j, m, kk)] = csub(cscale(cmuli(ur), a), duz);
    aux[fidx(p, 1, j, m, kk)] = csub(caxpy(dut, 1.0 / r, ut), cscale(cmuli(ur), m / r));
}

// ------------------------------------------------------ axial inverse FFT
// Block (m, j).  Fields: 0..2 u, 3 w_r (built from u), 4..5 aux, 6..8 y.
__global__ void k_zinv(KP p, int nf, int G, const double2* __restrict__ u, const double2* __restrict__ aux,
                       const double2* __restrict__ y, double2* __restrict__ zb) {
    extern __shared__ double2 sh[];
    const int m = blockIdx.x, j = blockIdx.y;
    const int nz = p.nz, nk = p.nk, K = p.K;
    const double r = p.r[j];
    double2* A = sh;
    double2* Bf = sh + G * nz;
    for (int f0 = 0; f0 < nf; f0 += G) {
        const int g = min(G, nf - f0);
        for (int t = threadIdx.x; t < g * nz; t += blockDim.x) A[t] = czero();
        __syncthreads();
        for (int t = threadIdx.x; t < g * nk; t += blockDim.x) {
            const int fi = t / nk, kk = t - fi * nk, f = f0 + fi;
            double2 v;
            if (f < 3) {
                v = u[fidx(p, f, j, m, kk)];
            } else if (f == 3) {
                const double a = alpha_of(p, kk);
                v = csub(cscale(cmuli(u[fidx(p, 2, j, m, kk)]), m / r), cscale(cmuli(u[fidx(p, 1, j, m, kk)]), a));
            } else if (f < 6) {
                v = aux[fidx(p, f - 4, j, m, kk)];
            } else {
                v = y[fidx(p, f - 6, j, m, kk)];
            }
            const int pos = kk <= K ? kk : nz - (nk - kk);
            A[fi * nz + pos] = v;
        }
        __syncthreads();
        double2* res = fft_lds(A, Bf, g, nz, p.fz, p.nfz, p.twz, 1.0);
        for (int t = threadIdx.x; t < g * nz; t += blockDim.x) {
            const int fi = t / nz, z = t - fi * nz;
            zb[((size_t)(j * nf + f0 + fi) * p.mp1 + m) * nz + z] = res[t];
        }
        __syncthreads();
    }
}

// ------------------------------------------- azimuthal FFTs and products
// Block (z-block, j).  Forward (adj = 0): 6 inputs (u, w) -> 3 outputs N.
// Adjoint (adj = 1): 9 inputs (u, w, y) -> 6 outputs A = (Om + w) x Y, B = Y x (U + u).
__device__ __forceinline__ void place_pair(double2* s, int nt, int m, double2 xa, double2 xb) {
    if (m == 0) {
        s[0] = make_double2(xa.x, xb.x);
    } else {
        s[m] = make_double2(xa.x - xb.y, xa.y + xb.x);          // xa + i xb
        s[nt - m] = make_double2(xa.x + xb.y, -xa.y + xb.x);    // conj(xa) + i conj(xb)
    }
}

__global__ void k_theta(KP p, int adj, int ZB, const double2* __restrict__ zb, double2* __restrict__ tb,
                        double cw, double sw) {
    extern __shared__ double2 sh[];
    const int j = blockIdx.y, z0 = blockIdx.x * ZB;
    const int nt = p.nt, mp1 = p.mp1, nz = p.nz;
    const int nf = adj ? 9 : 6, nfo = adj ? 6 : 3;
    const int H = ZB / 2;
    const int nin = adj ? 4 * ZB + H : 3 * ZB;
    const int nout = adj ? 3 * ZB : ZB + H;
    const int nseq = nin > nout ? nin : nout;
    double2* A = sh;
    double2* Bf = sh + nseq * nt;
    for (int t = threadIdx.x; t < nin * nt; t += blockDim.x) A[t] = czero();
    __syncthreads();
    const int npair = adj ? 4 : 3;
    for (int t = threadIdx.x; t < npair * ZB * mp1; t += blockDim.x) {
        const int zi = t % ZB, m = (t / ZB) % mp1, pi = t / (ZB * mp1);
        const double2 xa = zb[((size_t)(j * nf + 2 * pi) * mp1 + m) * nz + z0 + zi];
        const double2 xb = zb[((size_t)(j * nf + 2 * pi + 1) * mp1 + m) * nz + z0 + zi];
        place_pair(A + (pi * ZB + zi) * nt, nt, m, xa, xb);
    }
    if (adj) {
        for (int t = threadIdx.x; t < H * mp1; t += blockDim.x) {
            const int zi = t % H, m = t / H;
            const double2 xa = zb[((size_t)(j * nf + 8) * mp1 + m) * nz + z0 + zi];
            const double2 xb = zb[((size_t)(j * nf + 8) * mp1 + m) * nz + z0 + zi + H];
            place_pair(A + (4 * ZB + zi) * nt, nt, m, xa, xb);
        }
    }
    __syncthreads();
    double2* R1 = fft_lds(A, Bf, nin, nt, p.ft, p.nft, p.twt, 1.0);
    double2* O = (R1 == A) ? Bf : A;
    double* Od = reinterpret_cast<double*>(O);
    double U, Om;
    base_at(p, j, cw, sw, U, Om);
    for (int t = threadIdx.x; t < ZB * nt; t += blockDim.x) {
        const int zi = t / nt, th = t - zi * nt;
        const double2 s0 = R1[(0 * ZB + zi) * nt + th];
        const double2 s1 = R1[(1 * ZB + zi) * nt + th];
        const double2 s2 = R1[(2 * ZB + zi) * nt + th];
        const double ur = s0.x, ut = s0.y, uz = s1.x, wr = s1.y, wt = s2.x, wz = s2.y;
        if (!adj) {
            const double uzU = uz + U;
            const double Nr = ut * wz - uzU * wt - uz * Om;
            const double Nt = uzU * wr - ur * wz;
            const double Nz = ur * (wt + Om) - ut * wr;
            O[zi * nt + th] = make_double2(Nr, Nt);
            const int q = ZB + (zi < H ? zi : zi - H);
            Od[2 * (q * nt + th) + (zi < H ? 0 : 1)] = Nz;
        } else {
            const double2 s3 = R1[(3 * ZB + zi) * nt + th];
            const double2 s4 = R1[(4 * ZB + (zi < H ? zi : zi - H)) * nt + th];
            const double yr = s3.x, yt = s3.y, yz = (zi < H) ? s4.x : s4.y;
            const double wtO = wt + Om, uzU = uz + U;
            const double Ar = wtO * yz - wz * yt;
            const double At = wz * yr - wr * yz;
            const double Az = wr * yt - wtO * yr;
            const double Br = yt * uzU - yz * ut;
            const double Bt = yz * ur - yr * uzU;
            const double Bz = yr * ut - yt * ur;
            O[zi * nt + th] = make_double2(Ar, At);
            O[(ZB + zi) * nt + th] = make_double2(Az, Br);
            O[(2 * ZB + zi) * nt + th] = make_double2(Bt, Bz);
        }
    }
    __syncthreads();
    double2* R2 = fft_lds(O, R1, nout, nt, p.ft, p.nft, p.twt, -1.0);
    for (int t = threadIdx.x; t < nfo * mp1 * ZB; t += blockDim.x) {
        const int zi = t % ZB, m = (t / ZB) % mp1, f = t / (ZB * mp1);
        int q, half;
        if (!adj) {
            if (f < 2) { q = zi; half = f; }
            else { q = ZB + (zi < H ? zi : zi - H); half = (zi < H) ? 0 : 1; }
        } else {
            q = (f >> 1) * ZB + zi;
            half = f & 1;
        }
        const double2 a = R2[q * nt + m];
        const double2 b = cconj(R2[q * nt + (m == 0 ? 0 : nt - m)]);
        double2 v;
        if (half == 0) v = cscale(cadd(a, b), 0.5);
        else v = cscale(cmuli(csub(b, a)), 0.5);          // (a - b) / (2i)
        tb[((size_t)(j * nfo + f) * mp1 + m) * nz + z0 + zi] = v;
    }
}

// ------------------------------------------------------ axial forward FFT
__global__ void k_zfwd(KP p, int nfo, int G, const double2* __restrict__ tb, double2* __restrict__ out0,
                       double2* __restrict__ out1, double scale) {
    extern __shared__ double2 sh[];
    const int m = blockIdx.x, j = blockIdx.y;
    const int nz = p.nz, nk = p.nk, K = p.K;
    double2* A = sh;
    double2* Bf = sh + G * nz;
    for (int f0 = 0; f0 < nfo; f0 += G) {
        const int g = min(G, nfo - f0);
        for (int t = threadIdx.x; t < g * nz; t += blockDim.x) {
            const int fi = t / nz, z = t - fi * nz;
            A[t] = tb[((size_t)(j * nfo + f0 + fi) * p.mp1 + m) * nz + z];
        }
        __syncthreads();
        double2* res = fft_lds(A, Bf, g, nz, p.fz, p.nfz, p.twz, -1.0);
        for (int t = threadIdx.x; t < g * nk; t += blockDim.x) {
            const int fi = t / nk, kk = t - fi * nk, f = f0 + fi;
            const int pos = kk <= K ? kk : nz - (nk - kk);
            const double2 v = cscale(res[fi * nz + pos], scale);
            if (f < 3) out0[fidx(p, f, j, m, kk)] = v;
            else out1[fidx(p, f - 3, j, m, kk)] = v;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------ banded operators
// Operator kinds on the interior nodes 0..nr-2 (the wall node carries a
// Dirichlet value and its column is removed):
//   Helmholtz H_n = I/dt - (1/(2Re)) (D2 + D1/r - n^2/r^2 - a^2)
//   Poisson   P_n = D2 + D1/r - n^2/r^2 - a^2
struct OpDesc {
    int helm;   // 1 = Helmholtz, 0 = Poisson
    int n;      // azimuthal index of the scalar
    double a2;  // alpha^2
};

// Entry (row, col) of the full-width scalar Laplacian (no column restriction).
__device__ __forceinline__ double lap_entry(const KP& p, int n, double a2, int row, int col) {
    const int pi = n & 1;
    const double ri = p.r[row];
    double v = fdw(p.D2, pi, p.nr, p.col0, row, col) + fdw(p.D1, pi, p.nr, p.col0, row, col) / ri;
    if (row == col) v -= (double)(n * n) / (ri * ri) + a2;
    return v;
}

__device__ __forceinline__ double op_entry(const KP& p, const OpDesc& o, int row, int col) {
    const int n1 = p.nr - 1;
    if (row < 0 || col < 0 || row >= n1 || col >= n1) return 0.0;
    const double l = lap_entry(p, o.n, o.a2, row, col);
    if (!o.helm) return l;
    double v = -l / (2.0 * p.re);
    if (row == col) v += 1.0 / p.dt;
    return v;
}

// Banded LU without pivoting, factor + forward elimination in one sweep and
// back substitution, run by ONE thread.  The operator (or its transpose) is
// generated row by row from the FD tables.  NC complex right-hand sides
// rc[c*ldc + i] and NRR real right-hand sides rr[c*ldr + i] are solved in
// place.  Uf (LDS, n*(KU+1) doubles) holds U with the inverse diagonal.
template <int KL, int KU, int NC, int NRR, bool TRANS>
__device__ void band_solve(const KP& p, const OpDesc& o, int n, double* Uf, double2* rc, int ldc, double* rr,
                           int ldr) {
    double Uw[KL][KU + 1];
    double2 yc[KL][NC > 0 ? NC : 1];
    double yr[KL][NRR > 0 ? NRR : 1];
#pragma unroll
    for (int t = 0; t < KL; ++t) {
#pragma unroll
        for (int q = 0; q <= KU; ++q) Uw[t][q] = 0.0;
#pragma unroll
        for (int c = 0; c < (NC > 0 ? NC : 1); ++c) yc[t][c] = czero();
#pragma unroll
        for (int c = 0; c < (NRR > 0 ? NRR : 1); ++c) yr[t][c] = 0.0;
    }
    for (int i = 0; i < n; ++i) {
        double a[KL + KU + 1];
#pragma unroll
        for (int t = 0; t <= KL + KU; ++t) {
            const int col = i - KL + t;
            a[t] = TRANS ? op_entry(p, o, col, i) : op_entry(p, o, i, col);
        }
        double2 bc[NC > 0 ? NC : 1];
        double br[NRR > 0 ? NRR : 1];
#pragma unroll
        for (int c = 0; c < NC; ++c) bc[c] = rc[c * ldc + i];
#pragma unroll
        for (int c = 0; c < NRR; ++c) br[c] = rr[c * ldr + i];
#pragma unroll
        for (int t = 0; t < KL; ++t) {
            if (i - KL + t >= 0) {
                const double l = a[t] * Uw[t][0];
#pragma unroll
                for (int q = 1; q <= KU; ++q) a[t + q] = fma(-l, Uw[t][q], a[t + q]);
#pragma unroll
                for (int c = 0; c < NC; ++c) bc[c] = caxpy(bc[c], -l, yc[t][c]);
#pragma unroll
                for (int c = 0; c < NRR; ++c) br[c] = fma(-l, yr[t][c], br[c]);
            }
        }
        const double inv = 1.0 / a[KL];
        Uf[i * (KU + 1)] = inv;
#pragma unroll
        for (int q = 1; q <= KU; ++q) Uf[i * (KU + 1) + q] = a[KL + q];
#pragma unroll
        for (int c = 0; c < NC; ++c) rc[c * ldc + i] = bc[c];
#pragma unroll
        for (int c = 0; c < NRR; ++c) rr[c * ldr + i] = br[c];
#pragma unroll
        for (int t = 0; t < KL - 1; ++t) {
#pragma unroll
            for (int q = 0; q <= KU; ++q) Uw[t][q] = Uw[t + 1][q];
#pragma unroll
            for (int c = 0; c < NC; ++c) yc[t][c] = yc[t + 1][c];
#pragma unroll
            for (int c = 0; c < NRR; ++c) yr[t][c] = yr[t + 1][c];
        }
        Uw[KL - 1][0] = inv;
#pragma unroll
        for (int q = 1; q <= KU; ++q) Uw[KL - 1][q] = a[KL + q];
#pragma unroll
        for (int c = 0; c < NC; ++c) yc[KL - 1][c] = bc[c];
#pragma unroll
        for (int c = 0; c < NRR; ++c) yr[KL - 1][c] = br[c];
    }
    double2 xc[KU][NC > 0 ? NC : 1];
    double xr[KU][NRR > 0 ? NRR : 1];
#pragma unroll
    for (int q = 0; q < KU; ++q) {
#pragma unroll
        for (int c = 0; c < (NC > 0 ? NC : 1); ++c) xc[q][c] = czero();
#pragma unroll
        for (int c = 0; c < (NRR > 0 ? NRR : 1); ++c) xr[q][c] = 0.0;
    }
    for (int i = n - 1; i >= 0; --i) {
        double2 bc[NC > 0 ? NC : 1];
        double br[NRR > 0 ? NRR : 1];
#pragma unroll
        for (int c = 0; c < NC; ++c) bc[c] = rc[c * ldc + i];
#pragma unroll
        for (int c = 0; c < NRR; ++c) br[c] = rr[c * ldr + i];
#pragma unroll
        for (int q = 1; q <= KU; ++q) {
            if (i + q < n) {
                const double uq = Uf[i * (KU + 1) + q];
#pragma unroll
                for (int c = 0; c < NC; ++c) bc[c] = caxpy(bc[c], -uq, xc[q - 1][c]);
#pragma unroll
                for (int c = 0; c < NRR; ++c) br[c] = fma(-uq, xr[q - 1][c], br[c]);
            }
        }
        const double inv = Uf[i * (KU + 1)];
#pragma unroll
        for (int c = 0; c < NC; ++c) { bc[c] = cscale(bc[c], inv); rc[c * ldc + i] = bc[c]; }
#pragma unroll
        for (int c = 0; c < NRR; ++c) { br[c] *= inv; rr[c * ldr + i] = br[c]; }
#pragma unroll
        for (int q = KU - 1; q > 0; --q) {
#pragma unroll
            for (int c = 0; c < NC; ++c) xc[q][c] = xc[q - 1][c];
#pragma unroll
            for (int c = 0; c < NRR; ++c) xr[q][c] = xr[q - 1][c];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) xc[0][c] = bc[c];
#pragma unroll
        for (int c = 0; c < NRR; ++c) xr[0][c] = br[c];
    }
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
// (D^T x)[j] restricted to rows i < rows_lim of D.
__device__ __forceinline__ double2 fd_apply_T(const KP& p, const double* D, int pi, int j, const double2* x,
                                              int rows_lim) {
    double2 s = czero();
    const int lo = j - 6 < 0 ? 0 : j - 6;
    const int hi = j + 6 < rows_lim - 1 ? j + 6 : rows_lim - 1;
    for (int i = lo; i <= hi; ++i) {
        const int t = j - p.col0[i];
        if (t >= 0 && t < 7) s = caxpy(s, D[(pi * p.nr + i) * 7 + t], x[i]);
    }
    return s;
}

// ------------------------------------------------------------ forward solve
// Block (ka, m): modes (k, m) and (-k, m) share every operator.
__global__ __launch_bounds__(64) void k_solve(KP p, int kind, const double2* __restrict__ ain,
                                              const double2* __restrict__ bin, const double2* __restrict__ cin,
                                              double2* __restrict__ uout, double2* __restrict__ auxout) {
    const int ka = blockIdx.x, m = blockIdx.y, j = threadIdx.x;
    const int nr = p.nr, N1 = nr - 1;
    const int ncol = ka == 0 ? 1 : 2;
    const int kkc[2] = {ka, ka == 0 ? 0 : p.nk - ka};
    const double alc[2] = {ka * p.k0, -ka * p.k0};
    const double a2 = alc[0] * alc[0];
    const double re2 = 0.5 / p.re, idt = 1.0 / p.dt;
    const int pe = m & 1, po = (m + 1) & 1;
    __shared__ double2 su[3][2][NR_MAX];
    __shared__ double2 sR[3][2][NR_MAX];
    __shared__ double2 sp[2][NR_MAX];
    __shared__ double sph[NR_MAX];
    __shared__ double shv[3][NR_MAX];
    __shared__ double sUf[3][NR_MAX * 4];
    __shared__ double2 sa[2];

    if (j < nr) {
        for (int col = 0; col < 2; ++col)
            for (int c = 0; c < 3; ++c)
                su[c][col][j] = (col < ncol) ? ain[fidx(p, c, j, m, kkc[col])] : czero();
    }
    __syncthreads();
    if (j < nr) {
        const double rj = p.r[j];
        for (int col = 0; col < 2; ++col) {
            const double2 ur = su[0][col][j], ut = su[1][col][j], uz = su[2][col][j];
            double2 Rp, Rm, Rz;
            if (kind == 0) {
                Rp = cadd(ur, cmuli(ut));
                Rm = csub(ur, cmuli(ut));
                Rz = uz;
            } else {
                // E u = u/dt + (1/(2Re)) lap u, vector Laplacian in the +- basis
                const double* d1 = p.D1 + (po * nr + j) * 7;
                const double* d2 = p.D2 + (po * nr + j) * 7;
                const double* d1z = p.D1 + (pe * nr + j) * 7;
                const double* d2z = p.D2 + (pe * nr + j) * 7;
                const int c0 = p.col0[j];
                double2 lp = czero(), lm = czero(), lz = czero();
                for (int t = 0; t < 7; ++t) {
                    const double2 vr = su[0][col][c0 + t], vt = su[1][col][c0 + t], vz = su[2][col][c0 + t];
                    const double wgt = d2[t] + d1[t] / rj;
                    lp = caxpy(lp, wgt, cadd(vr, cmuli(vt)));
                    lm = caxpy(lm, wgt, csub(vr, cmuli(vt)));
                    lz = caxpy(lz, d2z[t] + d1z[t] / rj, vz);
                }
                const double2 up = cadd(ur, cmuli(ut)), um = csub(ur, cmuli(ut));
                const double np2 = (double)((m + 1) * (m + 1)), nm2 = (double)((m - 1) * (m - 1));
                const double ia = 1.0 / (rj * rj);
                lp = caxpy(lp, -(np2 * ia + a2), up);
                lm = caxpy(lm, -(nm2 * ia + a2), um);
                lz = caxpy(lz, -((double)(m * m) * ia + a2), uz);
                double2 Nr, Nt, Nz;
                if (col < ncol) {
                    const int kk = kkc[col];
                    Nr = bin[fidx(p, 0, j, m, kk)];
                    Nt = bin[fidx(p, 1, j, m, kk)];
                    Nz = bin[fidx(p, 2, j, m, kk)];
                    if (kind == 2) {
                        Nr = cscale(cadd(Nr, cin[fidx(p, 0, j, m, kk)]), 0.5);
                        Nt = cscale(cadd(Nt, cin[fidx(p, 1, j, m, kk)]), 0.5);
                        Nz = cscale(cadd(Nz, cin[fidx(p, 2, j, m, kk)]), 0.5);
                    }
                } else {
                    Nr = Nt = Nz = czero();
                }
                Rp = cadd(caxpy(cscale(up, idt), re2, lp), cadd(Nr, cmuli(Nt)));
                Rm = cadd(caxpy(cscale(um, idt), re2, lm), csub(Nr, cmuli(Nt)));
                Rz = cadd(caxpy(cscale(uz, idt), re2, lz), Nz);
            }
            sR[0][col][j] = Rp;
            sR[1][col][j] = Rm;
            sR[2][col][j] = Rz;
        }
    }
    __syncthreads();

    if (m == 0 && ka == 0) {
        // mean mode: u_r = 0, swirl H_1 u_theta = R_theta, axial H_0 u_z = R_z - f_z with zero flux
        double2 rt = czero();
        if (j < N1) rt = cscale(cmuli(csub(sR[1][0][j], sR[0][0][j])), 0.5);   // (R+ - R-)/(2i)
        __syncthreads();
        if (j < N1) {
            sR[1][0][j] = rt;
            shv[1][j] = 1.0;
        }
        __syncthreads();
        if (j < 2) {
            OpDesc o{1, j == 0 ? 1 : 0, 0.0};
            band_solve<5, 3, 2, 1, false>(p, o, N1, sUf[j], &sR[j + 1][0][0], NR_MAX, shv[j], NR_MAX);
        }
        __syncthreads();
        if (j == 0) {
            double2 s = czero();
            double g = 0.0;
            for (int i = 0; i < N1; ++i) {
                s = caxpy(s, p.w[i], sR[2][0][i]);
                g = fma(p.w[i], shv[1][i], g);
            }
            sa[0] = cscale(s, -1.0 / g);
        }
        __syncthreads();
        if (j < nr) {
            double2 ut = czero(), uz = czero();
            if (j < N1) {
                ut = sR[1][0][j];
                uz = caxpy(sR[2][0][j], shv[1][j], sa[0]);
                uz = cadd(sR[2][0][j], cscale(sa[0], shv[1][j]));
            }
            su[0][0][j] = czero();
            su[1][0][j] = ut;
            su[2][0][j] = uz;
            uout[fidx(p, 0, j, 0, 0)] = czero();
            uout[fidx(p, 1, j, 0, 0)] = ut;
            uout[fidx(p, 2, j, 0, 0)] = uz;
        }
        __syncthreads();
    } else {
        // particular pressure: P_m p = div R on interior nodes, p(1) = 0
        if (j < N1) {
            const double rj = p.r[j];
            for (int col = 0; col < 2; ++col) {
                double2 dsum = czero();
                const double* d1 = p.D1 + (po * nr + j) * 7;
                const int c0 = p.col0[j];
                for (int t = 0; t < 7; ++t) dsum = caxpy(dsum, d1[t], cadd(sR[0][col][c0 + t], sR[1][col][c0 + t]));
                double2 d = cscale(dsum, 0.5);
                d = caxpy(d, 0.5 * (1 + m) / rj, sR[0][col][j]);
                d = caxpy(d, 0.5 * (1 - m) / rj, sR[1][col][j]);
                d = cadd(d, cscale(cmuli(sR[2][col][j]), alc[col]));
                sp[col][j] = d;
            }
            sph[j] = -lap_entry(p, m, a2, j, N1);
        }
        __syncthreads();
        if (j == 0) {
            OpDesc o{0, m, a2};
            band_solve<5, 3, 2, 1, false>(p, o, N1, sUf[0], &sp[0][0], NR_MAX, sph, NR_MAX);
            sp[0][N1] = czero();
            sp[1][N1] = czero();
            sph[N1] = 1.0;
        }
        __syncthreads();
        if (j < N1) {
            const double rj = p.r[j];
            const double mr = m / rj;
            for (int col = 0; col < 2; ++col) {
                const double2 Dp = fd_apply(p, p.D1, pe, j, sp[col]);
                const double2 pj = sp[col][j];
                sR[0][col][j] = csub(sR[0][col][j], caxpy(Dp, -mr, pj));
                sR[1][col][j] = csub(sR[1][col][j], caxpy(Dp, mr, pj));
                sR[2][col][j] = csub(sR[2][col][j], cscale(cmuli(pj), alc[col]));
            }
            const double Dph = fd_apply_r(p, p.D1, pe, j, sph);
            shv[0][j] = -(Dph - mr * sph[j]);
            shv[1][j] = -(Dph + mr * sph[j]);
            shv[2][j] = -sph[j];
        }
        __syncthreads();
        if (j < 3) {
            const int n = (j == 0) ? m + 1 : (j == 1 ? m - 1 : m);
            OpDesc o{1, n, a2};
            band_solve<5, 3, 2, 1, false>(p, o, N1, sUf[j], &sR[j][0][0], NR_MAX, shv[j], NR_MAX);
        }
        __syncthreads();
        if (j == 0) {
            const double* dw = p.D1 + (po * nr + N1) * 7;
            const int c0 = p.col0[N1];
            double shs = 0.0;
            double2 s[2] = {czero(), czero()};
            for (int t = 0; t < 7; ++t) {
                const int c = c0 + t;
                if (c >= N1) continue;
                shs = fma(dw[t], shv[0][c] + shv[1][c], shs);
                for (int col = 0; col < 2; ++col) s[col] = caxpy(s[col], dw[t], cadd(sR[0][col][c], sR[1][col][c]));
            }
            for (int col = 0; col < 2; ++col) sa[col] = cscale(s[col], -1.0 / shs);
        }
        __syncthreads();
        if (j < nr) {
            for (int col = 0; col < ncol; ++col) {
                double2 up = czero(), um = czero(), uz = czero();
                if (j < N1) {
                    const double2 a = sa[col];
                    up = cadd(sR[0][col][j], cscale(a, shv[0][j]));
                    um = cadd(sR[1][col][j], cscale(a, shv[1][j]));
                    uz = cadd(sR[2][col][j], cscale(cmuli(a), alc[col] * shv[2][j]));
                }
                const double2 ur = cscale(cadd(up, um), 0.5);
                const double2 ut = cscale(cmuli(csub(um, up)), 0.5);   // (up - um)/(2i)
                su[0][col][j] = ur;
                su[1][col][j] = ut;
                su[2][col][j] = uz;
                const int kk = kkc[col];
                uout[fidx(p, 0, j, m, kk)] = ur;
                uout[fidx(p, 1, j, m, kk)] = ut;
                uout[fidx(p, 2, j, m, kk)] = uz;
            }
        }
        __syncthreads();
    }
    if (auxout && j < nr) {
        const double rj = p.r[j];
        for (int col = 0; col < ncol; ++col) {
            const int kk = kkc[col];
            const double2 ur = su[0][col][j], ut = su[1][col][j];
            const double2 duz = fd_apply(p, p.D1, pe, j, su[2][col]);
            const double2 dut = fd_apply(p, p.D1, po, j, su[1][col]);
            auxout[fidx(p, 0, j, m, kk)] = csub(cscale(cmuli(ur), alc[col]), duz);
            auxout[fidx(p, 1, j, m, kk)] = csub(caxpy(dut, 1.0 / rj, ut), cscale(cmuli(ur), m / rj));
        }
    }
}

// curl^H b at row j (b already W-weighted), for mode index m and axial wavenumber al.
__device__ __forceinline__ void curlH_row(const KP& p, int m, double al, int j, const double2* br, const double2* bt,
                                          const double2* bz, double2& cr, double2& ct, double2& cz) {
    const double rj = p.r[j];
    const int pe = m & 1, po = (m + 1) & 1;
    cr = cadd(cscale(cmuli(bt[j]), -al), cscale(cmuli(bz[j]), m / rj));
    ct = cadd(cadd(cscale(cmuli(br[j]), al), fd_apply_T(p, p.D1, po, j, bz, p.nr)), cscale(bz[j], 1.0 / rj));
    cz = csub(cscale(cmuli(br[j]), -m / rj), fd_apply_T(p, p.D1, pe, j, bt, p.nr));
}

// ------------------------------------------------------------ adjoint solve
// mu = S^dag(ca*A + cb*curl^dag B); out0 = mu + q0*Q; out1 = mu + q1*Q.
__global__ __launch_bounds__(64) void k_solve_adj(KP p, const double2* __restrict__ Ain, double ca,
                                                  const double2* __restrict__ Bin, double cb,
                                                  const double2* __restrict__ Qin, double q0, double q1,
                                                  double2* __restrict__ out0, double2* __restrict__ out1) {
    const int ka = blockIdx.x, m = blockIdx.y, j = threadIdx.x;
    const int nr = p.nr, N1 = nr - 1;
    const int ncol = ka == 0 ? 1 : 2;
    const int kkc[2] = {ka, ka == 0 ? 0 : p.nk - ka};
    const double alc[2] = {ka * p.k0, -ka * p.k0};
    const double a2 = alc[0] * alc[0];
    const int pe = m & 1, po = (m + 1) & 1;
    __shared__ double2 sy[3][2][NR_MAX];
    __shared__ double2 sb[3][2][NR_MAX];
    __shared__ double2 sp[2][NR_MAX];
    __shared__ double sph[NR_MAX];
    __shared__ double shv[3][NR_MAX];
    __shared__ double sUf[3][NR_MAX * 4];
    __shared__ double2 sa[2];
    const bool useB = Bin != nullptr;

    if (j < nr) {
        const double wj = p.w[j];
        for (int col = 0; col < 2; ++col)
            for (int c = 0; c < 3; ++c) {
                const bool ok = col < ncol;
                const size_t id = fidx(p, c, j, m, kkc[col]);
                sy[c][col][j] = ok ? cscale(Ain[id], ca) : czero();
                sb[c][col][j] = (ok && useB) ? cscale(Bin[id], wj) : czero();
            }
    }
    __syncthreads();
    if (useB && j < nr) {
        const double iw = cb / p.w[j];
        for (int col = 0; col < 2; ++col) {
            double2 cr, ct, cz;
            curlH_row(p, m, alc[col], j, sb[0][col], sb[1][col], sb[2][col], cr, ct, cz);
            sy[0][col][j] = caxpy(sy[0][col][j], iw, cr);
            sy[1][col][j] = caxpy(sy[1][col][j], iw, ct);
            sy[2][col][j] = caxpy(sy[2][col][j], iw, cz);
        }
    }
    __syncthreads();
    // y = W lambda on interior rows (the solve's wall output is identically zero)
    const bool mean = (m == 0 && ka == 0);
    if (j < nr) {
        const double wj = (j < N1) ? p.w[j] : 0.0;
        for (int col = 0; col < 2; ++col) {
            const double2 yr = cscale(sy[0][col][j], wj), yt = cscale(sy[1][col][j], wj);
            const double2 yz = cscale(sy[2][col][j], wj);
            if (mean) {
                sy[0][col][j] = yr;
                sy[1][col][j] = yt;
            } else {
                sy[0][col][j] = cscale(cadd(yr, cmuli(yt)), 0.5);
                sy[1][col][j] = cscale(csub(yr, cmuli(yt)), 0.5);
            }
            sy[2][col][j] = yz;
        }
    }
    __syncthreads();

    if (mean) {
        if (j < N1) shv[1][j] = 1.0;
        __syncthreads();
        if (j == 0) {
            OpDesc o{1, 0, 0.0};
            band_solve<5, 3, 0, 1, false>(p, o, N1, sUf[0], nullptr, 0, shv[1], NR_MAX);
            double wg = 0.0;
            double2 pr = czero();
            for (int i = 0; i < N1; ++i) {
                wg = fma(p.w[i], shv[1][i], wg);
                pr = caxpy(pr, shv[1][i], sy[2][0][i]);
            }
            sa[0] = cscale(pr, 1.0 / wg);
        }
        __syncthreads();
        if (j < N1) sy[2][0][j] = caxpy(sy[2][0][j], -p.w[j], sa[0]);
        __syncthreads();
        if (j < 2) {
            OpDesc o{1, j == 0 ? 1 : 0, 0.0};
            band_solve<3, 5, 2, 0, true>(p, o, N1, sUf[j], &sy[j + 1][0][0], NR_MAX, nullptr, 0);
        }
        __syncthreads();
        if (j < nr) {
            const double iw = 1.0 / p.w[j];
            const double2 mt = (j < N1) ? cscale(sy[1][0][j], iw) : czero();
            const double2 mz = (j < N1) ? cscale(sy[2][0][j], iw) : czero();
            const double2 mv[3] = {czero(), mt, mz};
            for (int c = 0; c < 3; ++c) {
                const size_t id = fidx(p, c, j, 0, 0);
                const double2 qv = Qin ? Qin[id] : czero();
                out0[id] = caxpy(mv[c], q0, qv);
                if (out1) out1[id] = caxpy(mv[c], q1, qv);
            }
        }
        return;
    }

    // homogeneous pair (forward operators)
    if (j < N1) sph[j] = -lap_entry(p, m, a2, j, N1);
    __syncthreads();
    if (j == 0) {
        OpDesc o{0, m, a2};
        band_solve<5, 3, 0, 1, false>(p, o, N1, sUf[0], nullptr, 0, sph, NR_MAX);
        sph[N1] = 1.0;
    }
    __syncthreads();
    if (j < N1) {
        const double mr = m / p.r[j];
        const double Dph = fd_apply_r(p, p.D1, pe, j, sph);
        shv[0][j] = -(Dph - mr * sph[j]);
        shv[1][j] = -(Dph + mr * sph[j]);
        shv[2][j] = -sph[j];
    }
    __syncthreads();
    if (j < 3) {
        const int n = (j == 0) ? m + 1 : (j == 1 ? m - 1 : m);
        OpDesc o{1, n, a2};
        band_solve<5, 3, 0, 1, false>(p, o, N1, sUf[j], nullptr, 0, shv[j], NR_MAX);
    }
    __syncthreads();
    // transposed influence correction: ybar_pm -= s * (u_h^H ybar) / s_h
    const double* dw = p.D1 + (po * nr + N1) * 7;
    const int cw0 = p.col0[N1];
    if (j == 0) {
        double shs = 0.0;
        for (int t = 0; t < 7; ++t) {
            const int c = cw0 + t;
            if (c < N1) shs = fma(dw[t], shv[0][c] + shv[1][c], shs);
        }
        for (int col = 0; col < 2; ++col) {
            double2 pr = czero();
            for (int i = 0; i < N1; ++i) {
                pr = caxpy(pr, shv[0][i], sy[0][col][i]);
                pr = caxpy(pr, shv[1][i], sy[1][col][i]);
                // conj(i a uhz) = -i a uhz
                pr = cadd(pr, cscale(cmuli(sy[2][col][i]), -alc[col] * shv[2][i]));
            }
            sa[col] = cscale(pr, 1.0 / shs);
        }
    }
    __syncthreads();
    if (j < N1) {
        const int t = j - cw0;
        if (t >= 0 && t < 7) {
            for (int col = 0; col < 2; ++col) {
                sy[0][col][j] = caxpy(sy[0][col][j], -dw[t], sa[col]);
                sy[1][col][j] = caxpy(sy[1][col][j], -dw[t], sa[col]);
            }
        }
    }
    __syncthreads();
    if (j < 3) {
        const int n = (j == 0) ? m + 1 : (j == 1 ? m - 1 : m);
        OpDesc o{1, n, a2};
        band_solve<3, 5, 2, 0, true>(p, o, N1, sUf[j], &sy[j][0][0], NR_MAX, nullptr, 0);
    }
    __syncthreads();
    // q = G^H w on interior rows
    if (j < N1) {
        const double mr = m / p.r[j];
        for (int col = 0; col < 2; ++col) {
            // sum of w+ and w- stored temporarily in sb[0]
            sb[0][col][j] = cadd(sy[0][col][j], sy[1][col][j]);
        }
    } else if (j == N1) {
        sb[0][0][j] = czero();
        sb[0][1][j] = czero();
    }
    __syncthreads();
    if (j < N1) {
        const double mr = m / p.r[j];
        for (int col = 0; col < 2; ++col) {
            double2 q = fd_apply_T(p, p.D1, pe, j, sb[0][col], N1);
            q = caxpy(q, -mr, csub(sy[0][col][j], sy[1][col][j]));
            q = csub(q, cscale(cmuli(sy[2][col][j]), alc[col]));
            sp[col][j] = q;
        }
    }
    __syncthreads();
    if (j == 0) {
        OpDesc o{0, m, a2};
        band_solve<3, 5, 2, 0, true>(p, o, N1, sUf[0], &sp[0][0], NR_MAX, nullptr, 0);
        sp[0][N1] = czero();
        sp[1][N1] = czero();
    }
    __syncthreads();
    if (j < nr) {
        const double rj = p.r[j];
        const double iw = 1.0 / p.w[j];
        for (int col = 0; col < ncol; ++col) {
            const double2 DT = fd_apply_T(p, p.D1, po, j, sp[col], N1);
            const double2 ph = sp[col][j];
            const double2 wp = (j < N1) ? sy[0][col][j] : czero();
            const double2 wm = (j < N1) ? sy[1][col][j] : czero();
            const double2 wz = (j < N1) ? sy[2][col][j] : czero();
            const double2 Rp = csub(wp, cscale(caxpy(DT, (1 + m) / rj, ph), 0.5));
            const double2 Rm = csub(wm, cscale(caxpy(DT, (1 - m) / rj, ph), 0.5));
            const double2 Rz = cadd(wz, cscale(cmuli(ph), alc[col]));
            const double2 mv[3] = {cscale(cadd(Rp, Rm), iw), cscale(cmuli(csub(Rm, Rp)), iw), cscale(Rz, iw)};
            const int kk = kkc[col];
            for (int c = 0; c < 3; ++c) {
                const size_t id = fidx(p, c, j, m, kk);
                const double2 qv = Qin ? Qin[id] : czero();
                out0[id] = caxpy(mv[c], q0, qv);
                if (out1) out1[id] = caxpy(mv[c], q1, qv);
            }
        }
    }
}

// ----------------------------------------------- adjoint combine (E^dag etc.)
// out = E^dag Z + A + curl^dag B
__global__ __launch_bounds__(64) void k_final(KP p, const double2* __restrict__ Z, const double2* __restrict__ Ain,
                                              const double2* __restrict__ Bin, double2* __restrict__ out) {
    const int ka = blockIdx.x, m = blockIdx.y, j = threadIdx.x;
    const int nr = p.nr;
    const int ncol = ka == 0 ? 1 : 2;
    const int kkc[2] = {ka, ka == 0 ? 0 : p.nk - ka};
    const double alc[2] = {ka * p.k0, -ka * p.k0};
    const double a2 = alc[0] * alc[0];
    const double re2 = 0.5 / p.re, idt = 1.0 / p.dt;
    const int pe = m & 1, po = (m + 1) & 1;
    __shared__ double2 sz[3][2][NR_MAX];
    __shared__ double2 sb[3][2][NR_MAX];
    if (j < nr) {
        const double wj = p.w[j];
        for (int col = 0; col < 2; ++col) {
            const bool ok = col < ncol;
            double2 zr = czero(), zt = czero(), zz = czero();
            if (ok && Z) {
                zr = cscale(Z[fidx(p, 0, j, m, kkc[col])], wj);
                zt = cscale(Z[fidx(p, 1, j, m, kkc[col])], wj);
                zz = cscale(Z[fidx(p, 2, j, m, kkc[col])], wj);
            }
            sz[0][col][j] = cscale(cadd(zr, cmuli(zt)), 0.5);
            sz[1][col][j] = cscale(csub(zr, cmuli(zt)), 0.5);
            sz[2][col][j] = zz;
            for (int c = 0; c < 3; ++c)
                sb[c][col][j] = (ok && Bin) ? cscale(Bin[fidx(p, c, j, m, kkc[col])], wj) : czero();
        }
    }
    __syncthreads();
    if (j >= nr) return;
    const double rc = p.r[j];
    const double iw = 1.0 / p.w[j];
    const int lo = j - 6 < 0 ? 0 : j - 6;
    const int hi = j + 6 < nr - 1 ? j + 6 : nr - 1;
    for (int col = 0; col < ncol; ++col) {
        // E_n^T column j: sum_i E_n[i][j] v_i
        double2 ep = czero(), em = czero(), ez = czero();
        for (int i = lo; i <= hi; ++i) {
            const int t = j - p.col0[i];
            if (t < 0 || t >= 7) continue;
            const double ri = p.r[i];
            const double wo = re2 * (p.D2[(po * nr + i) * 7 + t] + p.D1[(po * nr + i) * 7 + t] / ri);
            const double we = re2 * (p.D2[(pe * nr + i) * 7 + t] + p.D1[(pe * nr + i) * 7 + t] / ri);
            ep = caxpy(ep, wo, sz[0][col][i]);
            em = caxpy(em, wo, sz[1][col][i]);
            ez = caxpy(ez, we, sz[2][col][i]);
        }
        const double ia = 1.0 / (rc * rc);
        ep = caxpy(ep, idt - re2 * ((double)((m + 1) * (m + 1)) * ia + a2), sz[0][col][j]);
        em = caxpy(em, idt - re2 * ((double)((m - 1) * (m - 1)) * ia + a2), sz[1][col][j]);
        ez = caxpy(ez, idt - re2 * ((double)(m * m) * ia + a2), sz[2][col][j]);
        double2 er = cadd(ep, em);
        double2 et = cmuli(csub(em, ep));     // -i (ep - em)
        if (Bin) {
            double2 cr, ct, cz;
            curlH_row(p, m, alc[col], j, sb[0][col], sb[1][col], sb[2][col], cr, ct, cz);
            er = cadd(er, cr);
            et = cadd(et, ct);
            ez = cadd(ez, cz);
        }
        const int kk = kkc[col];
        const double2 ev[3] = {er, et, ez};
        for (int c = 0; c < 3; ++c) {
            const size_t id = fidx(p, c, j, m, kk);
            const double2 av = Ain ? Ain[id] : czero();
            out[id] = caxpy(av, iw, ev[c]);
        }
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
__global__ void k_rescale(size_t n, double2* __restrict__ x, const double* __restrict__ en, double e0) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = sqrt(e0 / en[0]);
    x[i] = cscale(x[i], s);
}

// ---------------------------------------------------------------- launchers
static inline size_t field_elems(const npo_plan_s& p) { return (size_t)3 * p.nr * p.mp1 * p.nk; }

hipError_t launch_curl_aux(const npo_plan_s& p, const double2* u, double2* aux, hipStream_t st) {
    const size_t per = (size_t)p.nr * p.mp1 * p.nk;
    prof_begin(p, KID_CURL, st);
    hipLaunchKernelGGL(k_curl_aux, dim3((per + 255) / 256), dim3(256), 0, st, p.kp, u, aux);
    prof_end(p, KID_CURL, st);
    return hipGetLastError();
}

hipError_t launch_nl(const npo_plan_s& p, int adj, const double2* u, const double2* aux, const double2* y,
                     double t, double2* out0, double2* out1, void* ws, hipStream_t st) {
    char* base = static_cast<char*>(ws);
    double2* zb = reinterpret_cast<double2*>(base + p.ws.zbuf);
    double2* tb = reinterpret_cast<double2*>(base + p.ws.tbuf);
    const int nf = adj ? 9 : 6, nfo = adj ? 6 : 3;
    const int G = p.zgroup;
    const size_t shz = (size_t)2 * G * p.nz * sizeof(double2);
    prof_begin(p, adj ? KID_ZINV_A : KID_ZINV_F, st);
    hipLaunchKernelGGL(k_zinv, dim3(p.mp1, p.nr), dim3(256), shz, st, p.kp, nf, G, u, aux, y, zb);
    prof_end(p, adj ? KID_ZINV_A : KID_ZINV_F, st);
    const int ZB = adj ? p.zb_theta_adj : p.zb_theta_fwd;
    const int H = ZB / 2;
    const int nin = adj ? 4 * ZB + H : 3 * ZB, nout = adj ? 3 * ZB : ZB + H;
    const size_t sht = (size_t)2 * (nin > nout ? nin : nout) * p.nt * sizeof(double2);
    const double cw = cos(p.omega * t), sw = sin(p.omega * t);
    prof_begin(p, adj ? KID_THETA_A : KID_THETA_F, st);
    hipLaunchKernelGGL(k_theta, dim3(p.nz / ZB, p.nr), dim3(256), sht, st, p.kp, adj, ZB, zb, tb, cw, sw);
    prof_end(p, adj ? KID_THETA_A : KID_THETA_F, st);
    const double scale = 1.0 / ((double)p.nt * p.nz);
    prof_begin(p, adj ? KID_ZFWD_A : KID_ZFWD_F, st);
    hipLaunchKernelGGL(k_zfwd, dim3(p.mp1, p.nr), dim3(256), shz, st, p.kp, nfo, G, tb, out0, out1, scale);
    prof_end(p, adj ? KID_ZFWD_A : KID_ZFWD_F, st);
    return hipGetLastError();
}

hipError_t launch_solve(const npo_plan_s& p, int kind, const double2* a, const double2* b, const double2* c,
                        double2* u_out, double2* aux_out, hipStream_t st) {
    prof_begin(p, kind == 1 ? KID_SOLVE_P : (kind == 2 ? KID_SOLVE_C : KID_SOLVE_R), st);
    hipLaunchKernelGGL(k_solve, dim3(p.K + 1, p.mp1), dim3(64), 0, st, p.kp, kind, a, b, c, u_out, aux_out);
    prof_end(p, kind == 1 ? KID_SOLVE_P : (kind == 2 ? KID_SOLVE_C : KID_SOLVE_R), st);
    return hipGetLastError();
}

hipError_t launch_solve_adj(const npo_plan_s& p, const double2* A, double ca, const double2* B, double cb,
                            const double2* Q, double q0, double q1, double2* out0, double2* out1, hipStream_t st) {
    prof_begin(p, B ? KID_SOLVE_ADJ2 : KID_SOLVE_ADJ, st);
    hipLaunchKernelGGL(k_solve_adj, dim3(p.K + 1, p.mp1), dim3(64), 0, st, p.kp, A, ca, B, cb, Q, q0, q1, out0,
                       out1);
    prof_end(p, B ? KID_SOLVE_ADJ2 : KID_SOLVE_ADJ, st);
    return hipGetLastError();
}

hipError_t launch_final(const npo_plan_s& p, const double2* Z, const double2* A, const double2* B, double2* out,
                        hipStream_t st) {
    prof_begin(p, KID_FINAL, st);
    hipLaunchKernelGGL(k_final, dim3(p.K + 1, p.mp1), dim3(64), 0, st, p.kp, Z, A, B, out);
    prof_end(p, KID_FINAL, st);
    return hipGetLastError();
}

hipError_t launch_wdot(const npo_plan_s& p, const double2* a, const double2* b, double* partial, double* out,
                       hipStream_t st) {
    prof_begin(p, KID_WDOT, st);
    hipLaunchKernelGGL(k_wdot_partial, dim3(RED_BLOCKS), dim3(256), 0, st, p.kp, a, b, partial);
    prof_end(p, KID_WDOT, st);
    hipLaunchKernelGGL(k_wdot_final, dim3(1), dim3(256), 0, st, partial, 2.0 * M_PI * p.lz, out);
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

hipError_t launch_rescale(const npo_plan_s& p, double2* x, const double* en, double e0, hipStream_t st) {
    const size_t n = field_elems(p);
    hipLaunchKernelGGL(k_rescale, dim3((n + 255) / 256), dim3(256), 0, st, n, x, en, e0);
    return hipGetLastError();
}

}  // namespace npo
