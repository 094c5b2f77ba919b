// Nonlinear-term kernels: axial FFTs, azimuthal FFTs and the pointwise
// products of the rotational form (Sec. 2.3: pseudo-spectral evaluation with
// 3/2-rule dealiasing), for gfx950 in FP64.
//
// Three kernels per evaluation, one per data grouping:
//   k_zinv   block (m, j): inverse axial FFTs of the spectral inputs, zero
//            padded from 2K+1 retained modes to N_z points;
//   k_theta  block (z-block, j): inverse azimuthal FFTs (two real fields packed
//            per complex transform), products, forward azimuthal FFTs;
//   k_zfwd   block (m, j): forward axial FFTs, truncation to the retained band.
// Intermediates live in HBM as complex [j][f][m][z].
//
// Each kernel exists in two forms: a compile-time-sized one for the common
// transform lengths (radix sequence, loop bounds and index arithmetic fixed at
// compile time, twiddles staged in LDS, LDS index padded against bank
// conflicts) and a generic one with run-time radices for every other length.
#include "npo_device.h"

namespace npo {

// ====================================================== generic transforms
// Run-time radices (factors p.fz / p.ft), for lengths without a compiled size.
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

// ------------------------------------------------------ axial inverse FFT
// Block (m, j).  Fields: 0..2 u, 3 w_r (built from u), 4..5 aux, 6..8 y.
__global__ void k_zinv(KP p, int fbase, int nf, int G, const double2* __restrict__ u, const double2* __restrict__ aux,
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
            const int fi = t / nk, kk = t - fi * nk, f = fbase + f0 + fi;
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

// cos and sin of the base-flow phase at the evaluation time
__device__ __forceinline__ void phase_of(const KP& p, const TimeArg& ta, double& cw, double& sw) {
    const double t = ta.direct ? ta.t : p.t0 + (double)((ta.dstep ? *ta.dstep : ta.n) + ta.off) * p.dt;
    sincos(p.omega * t, &sw, &cw);
}

// CFL monitor pieces shared by the azimuthal kernels: the scales dt / dz,
// dt / (r dtheta) and dt / dr at radial node j (dr: the smaller neighbour gap;
// the axis gap of the first node is 2 r_0), and the fold of a thread's maximum
// into *dst: a wave maximum, then one atomic maximum per wave (non-negative
// doubles order as their bit patterns).  Every lane of the wave must call it.
__device__ __forceinline__ void cfl_scales(const KP& p, int j, int nt, double& cz, double& cth, double& cr) {
    const double rj = p.r[j];
    const double gl = j > 0 ? rj - p.r[j - 1] : 2.0 * rj;
    const double gr = j + 1 < p.nr ? p.r[j + 1] - rj : gl;
    cz = p.dt * p.nz / p.lz;
    cth = p.dt * nt / (2.0 * M_PI * rj);
    cr = p.dt / fmin(gl, gr);
}
// The running maximum only grows between resets, and a device-scope load never
// returns more than it holds, so a wave whose maximum does not exceed the value
// read skips the atomic: after the first blocks almost every wave does, instead
// of some ten thousand atomics per launch queueing on one address.
__device__ __forceinline__ void cfl_fold(double cmax, unsigned long long* dst) {
    for (int off = 32; off > 0; off >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, off));
    if ((threadIdx.x & 63) == 0) {
        const unsigned long long v = (unsigned long long)__double_as_longlong(cmax);
        if (v > __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(dst, v);
    }
}

__global__ void k_theta(KP p, int adj, int ZB, const double2* __restrict__ zu, int nfu, const double2* __restrict__ zy,
                        int nfy, double2* __restrict__ tb, TimeArg ta) {
    extern __shared__ double2 sh[];
    const int j = blockIdx.y, z0 = blockIdx.x * ZB;
    const int nt = p.nt, mp1 = p.mp1, nz = p.nz;
    const int nfo = adj ? 6 : 3;
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
        // u, w pairs from zu (nfu fields per node), y pairs from zy (nfy per node)
        const double2* src = pi < 3 ? zu + (size_t)j * nfu * mp1 * nz : zy + (size_t)j * nfy * mp1 * nz;
        const int fl = pi < 3 ? 2 * pi : 2 * pi - 6;
        const double2 xa = src[((size_t)fl * mp1 + m) * nz + z0 + zi];
        const double2 xb = src[((size_t)(fl + 1) * mp1 + m) * nz + z0 + zi];
        place_pair(A + (pi * ZB + zi) * nt, nt, m, xa, xb);
    }
    if (adj) {
        for (int t = threadIdx.x; t < H * mp1; t += blockDim.x) {
            const int zi = t % H, m = t / H;
            const double2* src = zy + ((size_t)j * nfy + 2) * mp1 * nz;
            const double2 xa = src[(size_t)m * nz + z0 + zi];
            const double2 xb = src[(size_t)m * nz + z0 + zi + H];
            place_pair(A + (4 * ZB + zi) * nt, nt, m, xa, xb);
        }
    }
    __syncthreads();
    double2* R1 = fft_lds(A, Bf, nin, nt, p.ft, p.nft, p.twt, 1.0);
    double2* O = (R1 == A) ? Bf : A;
    double* Od = reinterpret_cast<double*>(O);
    double U, Om, cw, sw;
    phase_of(p, ta, cw, sw);
    base_at(p, j, cw, sw, U, Om);
    double cmax = 0.0, cz = 0.0, cth = 0.0, cr = 0.0;
    if (ta.cfl) cfl_scales(p, j, nt, cz, cth, cr);
    for (int t = threadIdx.x; t < ZB * nt; t += blockDim.x) {
        const int zi = t / nt, th = t - zi * nt;
        const double2 s0 = R1[(0 * ZB + zi) * nt + th];
        const double2 s1 = R1[(1 * ZB + zi) * nt + th];
        const double2 s2 = R1[(2 * ZB + zi) * nt + th];
        const double ur = s0.x, ut = s0.y, uz = s1.x, wr = s1.y, wt = s2.x, wz = s2.y;
        if (!adj) {
            const double uzU = uz + U;
            if (ta.cfl) cmax = fmax(cmax, fabs(uzU) * cz + fabs(ut) * cth + fabs(ur) * cr);
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
    if (ta.cfl) cfl_fold(cmax, ta.cfl);
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


// ============================================ compile-time-sized transforms
constexpr int TB = 256;   // threads per block of the transform kernels
// Radix ceiling of the azimuthal transforms: the adjoint pass (4.5 sequences
// per axial point) gains from fewer LDS passes, the forward pass (1.5-3) from
// more butterflies per pass (both measured at 96 x 768).
template <int ADJ>
constexpr int theta_maxr() { return ADJ ? 16 : 8; }

// Padded LDS index: one complex of padding per 16, so that the strided
// accesses of the early Stockham passes spread over the LDS banks.
__device__ __forceinline__ int lp(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lp_size(int n) { return n + (n >> 4) + 1; }

// Radix plans.  With a ceiling of 4 or 8 (few sequences per block:
// parallelism per pass matters) the radices are taken greedily from {8, 4, 3,
// 2} or {4, 3, 2}; with a
// ceiling of 16 (many sequences per block: fewer LDS passes matter) the plan
// has the fewest passes over {16, 12, 8, 6, 4, 3, 2}, the largest first radix
// among such plans.
constexpr int kRadices[7] = {16, 12, 8, 6, 4, 3, 2};
__host__ __device__ constexpr int min_passes(int n) {
    if (n == 1) return 0;
    int best = 1 << 20;
    for (int i = 0; i < 7; ++i)
        if (n % kRadices[i] == 0) {
            const int c = 1 + min_passes(n / kRadices[i]);
            if (c < best) best = c;
        }
    return best;
}
template <int MAXR>
__host__ __device__ constexpr int pick_radix(int rem) {
    if (MAXR <= 4) return rem % 4 == 0 ? 4 : (rem % 3 == 0 ? 3 : 2);
    if (MAXR <= 8) return rem % 8 == 0 ? 8 : (rem % 4 == 0 ? 4 : (rem % 3 == 0 ? 3 : 2));
    const int target = min_passes(rem);
    for (int i = 0; i < 7; ++i)
        if (rem % kRadices[i] == 0 && 1 + min_passes(rem / kRadices[i]) == target) return kRadices[i];
    return 2;
}

// a * w (forward) or a * conj(w) (inverse)
template <bool INV>
__device__ __forceinline__ double2 tw_mul(double2 a, double2 w) {
    if (INV) return make_double2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
    return make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}
// a * (-i) forward, a * i inverse: the quarter-turn of the length-4 DFT
template <bool INV>
__device__ __forceinline__ double2 qturn(double2 a) {
    return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(double2& a, double2& b) {
    const double2 s = cadd(a, b), d = csub(a, b);
    a = s; b = d;
}
template <bool INV>
__device__ __forceinline__ void dft3(double2& a, double2& b, double2& c) {
    constexpr double h = 0.86602540378443864676;   // sin(pi/3)
    const double2 s = cadd(b, c), d = csub(b, c);
    const double2 t0 = caxpy(a, -0.5, s);
    const double2 t1 = cscale(qturn<INV>(d), h);     // -+ i sqrt(3)/2 (b - c)
    a = cadd(a, s); b = cadd(t0, t1); c = csub(t0, t1);
}
template <bool INV>
__device__ __forceinline__ void dft4(double2& a, double2& b, double2& c, double2& d) {
    const double2 s02 = cadd(a, c), d02 = csub(a, c);
    const double2 s13 = cadd(b, d), t13 = qturn<INV>(csub(b, d));
    a = cadd(s02, s13); c = csub(s02, s13);
    b = cadd(d02, t13); d = csub(d02, t13);
}
// length-8 DFT: two length-4 DFTs of the even and odd samples, odd half
// rotated by w8^k = exp(-+ i pi k / 4)
template <bool INV>
__device__ __forceinline__ void dft8(double2* v) {
    constexpr double s = 0.70710678118654752440;
    dft4<INV>(v[0], v[2], v[4], v[6]);
    dft4<INV>(v[1], v[3], v[5], v[7]);
    const double2 o1 = v[3], o2 = v[5], o3 = v[7];
    const double2 r1 = INV ? make_double2((o1.x - o1.y) * s, (o1.x + o1.y) * s)
                           : make_double2((o1.x + o1.y) * s, (o1.y - o1.x) * s);
    const double2 r2 = qturn<INV>(o2);
    const double2 r3 = INV ? make_double2(-(o3.x + o3.y) * s, (o3.x - o3.y) * s)
                           : make_double2((o3.y - o3.x) * s, -(o3.x + o3.y) * s);
    const double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1];
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, r1); v[5] = csub(e1, r1);
    v[2] = cadd(e2, r2); v[6] = csub(e2, r2);
    v[3] = cadd(e3, r3); v[7] = csub(e3, r3);
}

// exp(-2 pi i k / R) for the constant twiddles inside the composite radices
template <int R>
__device__ __forceinline__ double2 unit_root(int k);
template <>
__device__ __forceinline__ double2 unit_root<16>(int k) {
    constexpr double c[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                              0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                              -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                              0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
    return make_double2(c[k & 15], -c[(k + 12) & 15]);   // sin(x) = cos(x - pi/2)
}
template <>
__device__ __forceinline__ double2 unit_root<12>(int k) {
    constexpr double c[12] = {1.0, 0.86602540378443864676, 0.5, 0.0, -0.5, -0.86602540378443864676,
                              -1.0, -0.86602540378443864676, -0.5, 0.0, 0.5, 0.86602540378443864676};
    return make_double2(c[k % 12], -c[(k + 9) % 12]);
}
template <>
__device__ __forceinline__ double2 unit_root<6>(int k) {
    constexpr double c[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
    constexpr double s[6] = {0.0, 0.86602540378443864676, 0.86602540378443864676, 0.0,
                             -0.86602540378443864676, -0.86602540378443864676};
    return make_double2(c[k % 6], -s[k % 6]);
}

template <int R, bool INV>
__device__ __forceinline__ void dft(double2* v);

// Composite length R = R1 * R2 (Cooley-Tukey in registers): length-R2 DFTs
// over n2 of v[n1 + R1 n2], twiddles w_R^(n1 k2), length-R1 DFTs over n1;
// output k = k2 + R2 k1 in natural order.
template <int R1, int R2, bool INV>
__device__ __forceinline__ void dft_split(double2* v) {
    constexpr int R = R1 * R2;
    double2 y[R1][R2];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
        double2 c[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) c[n2] = v[n1 + R1 * n2];
        dft<R2, INV>(c);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) y[n1][k2] = (n1 * k2) ? tw_mul<INV>(c[k2], unit_root<R>(n1 * k2)) : c[k2];
    }
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
        double2 c[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) c[n1] = y[n1][k2];
        dft<R1, INV>(c);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) v[k2 + R2 * k1] = c[k1];
    }
}

template <int R, bool INV>
__device__ __forceinline__ void dft(double2* v) {
    if constexpr (R == 2) dft2<INV>(v[0], v[1]);
    else if constexpr (R == 3) dft3<INV>(v[0], v[1], v[2]);
    else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8<INV>(v);
    else if constexpr (R == 6) dft_split<2, 3, INV>(v);
    else if constexpr (R == 12) dft_split<4, 3, INV>(v);
    else dft_split<4, 4, INV>(v);   // 16
}

// One Stockham autosort pass of radix R over B sequences of length N stored
// back to back (padded index); NS = product of the radices already applied.
// tw[t] = exp(-2 pi i t / N) in LDS.
template <int N, int R, int NS, bool INV>
__device__ __forceinline__ void stockham_pass(const double2* __restrict__ x, double2* __restrict__ y, int B,
                                              const double2* __restrict__ tw) {
    constexpr int nb = N / R;
    constexpr int tws = N / (NS * R);
    const int total = B * nb;
    for (int t = threadIdx.x; t < total; t += TB) {
        const int bi = t / nb;
        const int jj = t - bi * nb;
        const int k = jj % NS;
        const int ib = bi * N + jj;
        const int ob = bi * N + (jj - k) * R + k;
        double2 v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = x[lp(ib + q * nb)];
        if constexpr (NS > 1) {
#pragma unroll
            for (int q = 1; q < R; ++q) v[q] = tw_mul<INV>(v[q], tw[q * k * tws]);
        }
        dft<R, INV>(v);
#pragma unroll
        for (int q = 0; q < R; ++q) y[lp(ob + q * NS)] = v[q];
    }
}

// B transforms of length N in LDS (a: data, b: scratch, both padded); the
// passes end with a barrier.  Returns the buffer holding the result.
template <int N, bool INV, int MAXR, int NS = 1>
__device__ __forceinline__ double2* fft_ct(double2* a, double2* b, int B, const double2* tw) {
    if constexpr (NS == N) {
        return a;
    } else {
        constexpr int R = pick_radix<MAXR>(N / NS);
        stockham_pass<N, R, NS, INV>(a, b, B, tw);
        __syncthreads();
        return fft_ct<N, INV, MAXR, NS * R>(b, a, B, tw);
    }
}

// Stockham passes of length N (radices pick_radix<MAXR>) from stride NS up to
// stride STOP, each ending with a barrier; returns the buffer with the result.
template <int N, bool INV, int MAXR, int NS, int STOP>
__device__ __forceinline__ double2* fft_span(double2* a, double2* b, int B, const double2* tw) {
    if constexpr (NS == STOP) {
        return a;
    } else {
        constexpr int R = pick_radix<MAXR>(STOP / NS);
        stockham_pass<N, R, NS, INV>(a, b, B, tw);
        __syncthreads();
        return fft_span<N, INV, MAXR, NS * R, STOP>(b, a, B, tw);
    }
}

// Inverse axial transforms of fields F0 .. F0+NF-1 of the list 0..2 u, 3 w_r
// (built from u), 4..5 aux, 6..8 y (forward term 0..5, adjoint term 0..8, or
// the adjoint field alone 6..8), written as NF fields per node.  One field per round;
// the next field's inputs are loaded into registers while the current one is
// transformed, so the global-load latency overlaps the LDS passes.
template <int NZ, int F0, int NF>
__global__ __launch_bounds__(TB) void k_zinv_t(KP p, const double2* __restrict__ u, const double2* __restrict__ aux,
                                              const double2* __restrict__ y, double2* __restrict__ zb) {
    constexpr int K = (NZ - 1) / 3, NK = 2 * K + 1;
    constexpr int PER = (NZ + TB - 1) / TB;
    extern __shared__ double2 sh[];
    double2* tw = sh;
    double2* A = sh + NZ;
    double2* Bf = A + lp_size(NZ);
    const int m = blockIdx.x, j = blockIdx.y, mp1 = p.mp1;
    const double mr = m / p.r[j];
    for (int t = threadIdx.x; t < NZ; t += TB) tw[t] = p.twz[t];
    double2 v[PER];
    auto fetch = [&](int f) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int z = threadIdx.x + i * TB;
            const int kk = z <= K ? z : (z >= NZ - K ? z - NZ + NK : -1);
            v[i] = czero();
            if (z < NZ && kk >= 0) {
                if (f < 3) {
                    v[i] = u[fidx(p, f, j, m, kk)];
                } else if (f == 3) {
                    v[i] = csub(cscale(cmuli(u[fidx(p, 2, j, m, kk)]), mr),
                                cscale(cmuli(u[fidx(p, 1, j, m, kk)]), alpha_of(p, kk)));
                } else if (f < 6) {
                    v[i] = aux[fidx(p, f - 4, j, m, kk)];
                } else {
                    v[i] = y[fidx(p, f - 6, j, m, kk)];
                }
            }
        }
    };
    fetch(F0);
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int z = threadIdx.x + i * TB;
            if (z < NZ) A[lp(z)] = v[i];
        }
        __syncthreads();
        if (f + 1 < NF) fetch(F0 + f + 1);
        // radix <= 4 for the six- and nine-field passes (more butterflies per
        // pass beat fewer passes there; measured at N_z = 768)
        const double2* res = fft_ct<NZ, true, (NF >= 6 ? 4 : 8)>(A, Bf, 1, tw);
        double2* row = zb + ((size_t)(j * NF + f) * mp1 + m) * NZ;
        for (int z = threadIdx.x; z < NZ; z += TB) row[z] = res[lp(z)];
        __syncthreads();
    }
}

// Inverse axial transforms for N_z = 3P (then K = P - 1), same fields and
// output as k_zinv_t.  Plan: radix 3 (stride P), pick_radix<8> passes, radix 4
// (stride N_z / 4).  The first pass runs on the modes in registers: its
// butterfly jj reads z = jj (mode jj), z = P + jj (in the zero band) and
// z = 2P + jj (mode jj - P, zero for jj = 0), so nothing is placed in LDS
// beforehand; the last pass stores its outputs straight to the row.  Two LDS
// round trips and two barriers fewer per field than k_zinv_t.
template <int NZ, int F0, int NF, int MB>
__global__ __launch_bounds__(TB) void k_zinv_p(KP p, const double2* __restrict__ u, const double2* __restrict__ aux,
                                              const double2* __restrict__ y, double2* __restrict__ zb,
                                              const BDesc* bd) {
    static_assert(NZ % 12 == 0, "N_z = 3P with P a multiple of 4");
    if (bd) {
        const BDesc& d = bd[blockIdx.z];
        p = d.kp; globalize(p, bd); u = rebase(bd, d.in[0]); aux = rebase(bd, d.in[1]); y = rebase(bd, d.in[2]); zb = rebase(bd, d.out[0]);
    }
    constexpr int P = NZ / 3, NK = 2 * P - 1;
    constexpr int PB = (P + TB - 1) / TB;             // first-pass butterflies per thread
    constexpr int NB4 = NZ / 4;                       // last-pass butterflies
    extern __shared__ double2 sh[];
    double2* tw = sh;
    double2* A = sh + NZ;
    double2* Bf = A + lp_size(NZ);
    // MB consecutive m per block, NF fields each: rounds rd = (m - m0) NF + f
    const int m0 = blockIdx.x * MB, j = blockIdx.y, mp1 = p.mp1;
    const int nround = MB == 1 ? NF : (mp1 - m0 < MB ? mp1 - m0 : MB) * NF;
    const double rj = p.r[j];
    for (int t = threadIdx.x; t < NZ; t += TB) tw[t] = p.twz[t];
    auto load = [&](int m, int f, int kk) -> double2 {
        if (f < 3) return u[fidx(p, f, j, m, kk)];
        if (f == 3)
            return csub(cscale(cmuli(u[fidx(p, 2, j, m, kk)]), m / rj), cscale(cmuli(u[fidx(p, 1, j, m, kk)]), alpha_of(p, kk)));
        if (f < 6) return aux[fidx(p, f - 4, j, m, kk)];
        return y[fidx(p, f - 6, j, m, kk)];
    };
    // modes jj (z = jj) and jj - P (z = 2P + jj, stored at kk = jj + NK - P)
    double2 v0[PB], v2[PB];
    // u_theta of the current m, kept from its round for omega_r (field 3), which
    // is formed from it and from u_z (still in v0, v2 from the round before)
    double2 s0[PB], s2[PB];
    auto fetch = [&](int rd) {
        const int m = m0 + rd / NF, f = F0 + rd % NF;
        if (f == 3 && rd % NF == 3) {
#pragma unroll
            for (int b = 0; b < PB; ++b) {
                const int jj = threadIdx.x + b * TB;
                v0[b] = csub(cscale(cmuli(v0[b]), m / rj), cscale(cmuli(s0[b]), alpha_of(p, jj)));
                v2[b] = csub(cscale(cmuli(v2[b]), m / rj), cscale(cmuli(s2[b]), alpha_of(p, jj + NK - P)));
            }
            return;
        }
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const int jj = threadIdx.x + b * TB;
            v0[b] = v2[b] = czero();
            if (jj < P) {
                v0[b] = load(m, f, jj);
                if (jj) v2[b] = load(m, f, jj + NK - P);
            }
            if (f == 1) {
                s0[b] = v0[b];
                s2[b] = v2[b];
            }
        }
    };
    fetch(0);
    // unrolled: the field of each round is known at compile time
#pragma unroll
    for (int rd = 0; rd < MB * NF; ++rd) {
        if (rd >= nround) break;
        const int m = m0 + rd / NF, f = rd % NF;
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const int jj = threadIdx.x + b * TB;
            if (jj < P) {
                double2 a = v0[b], c = czero(), d = v2[b];
                dft3<true>(a, c, d);
                A[lp(3 * jj)] = a;
                A[lp(3 * jj + 1)] = c;
                A[lp(3 * jj + 2)] = d;
            }
        }
        __syncthreads();
        if (rd + 1 < nround) fetch(rd + 1);
        const double2* X = fft_span<NZ, true, 8, 3, NB4>(A, Bf, 1, tw);
        double2* row = zb + ((size_t)(j * NF + f) * mp1 + m) * NZ;
        for (int jj = threadIdx.x; jj < NB4; jj += TB) {
            double2 v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = X[lp(jj + q * NB4)];
#pragma unroll
            for (int q = 1; q < 4; ++q) v[q] = tw_mul<true>(v[q], tw[q * jj]);
            dft4<true>(v[0], v[1], v[2], v[3]);
#pragma unroll
            for (int q = 0; q < 4; ++q) row[jj + q * NB4] = v[q];
        }
        __syncthreads();
    }
}

// Forward axial transforms of NFO theta-pass outputs, truncated to the band;
// one field per round with the next field prefetched into registers.
template <int NZ, int NFO>
__global__ __launch_bounds__(TB) void k_zfwd_t(KP p, const double2* __restrict__ tb, double2* __restrict__ out0,
                                              double2* __restrict__ out1, double scale) {
    constexpr int K = (NZ - 1) / 3, NK = 2 * K + 1;
    constexpr int PER = (NZ + TB - 1) / TB;
    extern __shared__ double2 sh[];
    double2* tw = sh;
    double2* A = sh + NZ;
    double2* Bf = A + lp_size(NZ);
    const int m = blockIdx.x, j = blockIdx.y, mp1 = p.mp1;
    for (int t = threadIdx.x; t < NZ; t += TB) tw[t] = p.twz[t];
    double2 v[PER];
    auto fetch = [&](int f) {
        const double2* row = tb + ((size_t)(j * NFO + f) * mp1 + m) * NZ;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int z = threadIdx.x + i * TB;
            v[i] = z < NZ ? row[z] : czero();
        }
    };
    fetch(0);
    for (int f = 0; f < NFO; ++f) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int z = threadIdx.x + i * TB;
            if (z < NZ) A[lp(z)] = v[i];
        }
        __syncthreads();
        if (f + 1 < NFO) fetch(f + 1);
        const double2* res = fft_ct<NZ, false, 8>(A, Bf, 1, tw);
        double2* out = f < 3 ? out0 : out1;
        const int c = f < 3 ? f : f - 3;
        for (int kk = threadIdx.x; kk < NK; kk += TB) {
            const int pos = kk <= K ? kk : NZ - (NK - kk);
            out[fidx(p, c, j, m, kk)] = cscale(res[lp(pos)], scale);
        }
        __syncthreads();
    }
}

// Forward axial transforms for N_z = 3P (then K = P - 1), same inputs and
// outputs as k_zfwd_t.  Plan: radix 4 (stride N_z / 4), pick_radix<8> passes,
// radix 3 (stride P).  The first pass runs on the row in registers, and the
// last pass computes only the outputs that survive the truncation (z = jj and
// z = 2P + jj of butterfly jj; z = P + jj lies outside the band) and stores
// them to the spectral field.
template <int NZ, int NFO, int MB>
__global__ __launch_bounds__(TB) void k_zfwd_p(KP p, const double2* __restrict__ tb, double2* __restrict__ out0,
                                              double2* __restrict__ out1, double scale, const BDesc* bd) {
    static_assert(NZ % 12 == 0, "N_z = 3P with P a multiple of 4");
    if (bd) {
        const BDesc& d = bd[blockIdx.z];
        p = d.kp; globalize(p, bd); tb = rebase(bd, d.in[0]); out0 = rebase(bd, d.out[0]); out1 = rebase(bd, d.out[1]);
    }
    constexpr int P = NZ / 3, NK = 2 * P - 1;
    constexpr int NB4 = NZ / 4;
    constexpr int PB = (NB4 + TB - 1) / TB;           // first-pass butterflies per thread
    extern __shared__ double2 sh[];
    double2* tw = sh;
    double2* A = sh + NZ;
    double2* Bf = A + lp_size(NZ);
    // MB consecutive m per block, NFO fields each: rounds rd = (m - m0) NFO + f
    const int m0 = blockIdx.x * MB, j = blockIdx.y, mp1 = p.mp1;
    const int nround = MB == 1 ? NFO : (mp1 - m0 < MB ? mp1 - m0 : MB) * NFO;
    for (int t = threadIdx.x; t < NZ; t += TB) tw[t] = p.twz[t];
    double2 v[PB][4];
    auto fetch = [&](int rd) {
        const int m = m0 + rd / NFO, f = rd % NFO;
        const double2* row = tb + ((size_t)(j * NFO + f) * mp1 + m) * NZ;
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const int jj = threadIdx.x + b * TB;
#pragma unroll
            for (int q = 0; q < 4; ++q) v[b][q] = jj < NB4 ? row[jj + q * NB4] : czero();
        }
    };
    fetch(0);
    // unrolled: the field of each round is known at compile time
#pragma unroll
    for (int rd = 0; rd < MB * NFO; ++rd) {
        if (rd >= nround) break;
        const int m = m0 + rd / NFO, f = rd % NFO;
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const int jj = threadIdx.x + b * TB;
            if (jj < NB4) {
                dft4<false>(v[b][0], v[b][1], v[b][2], v[b][3]);
#pragma unroll
                for (int q = 0; q < 4; ++q) A[lp(4 * jj + q)] = v[b][q];
            }
        }
        __syncthreads();
        if (rd + 1 < nround) fetch(rd + 1);
        const double2* X = fft_span<NZ, false, 8, 4, P>(A, Bf, 1, tw);
        double2* out = f < 3 ? out0 : out1;
        const int c = f < 3 ? f : f - 3;
        for (int jj = threadIdx.x; jj < P; jj += TB) {
            double2 a = X[lp(jj)], b = X[lp(jj + P)], d = X[lp(jj + 2 * P)];
            b = tw_mul<false>(b, tw[jj]);
            d = tw_mul<false>(d, tw[2 * jj]);
            dft3<false>(a, b, d);
            out[fidx(p, c, j, m, jj)] = cscale(a, scale);
            if (jj) out[fidx(p, c, j, m, jj + NK - P)] = cscale(d, scale);
        }
        __syncthreads();
    }
}

// Azimuthal transforms and products.  A block owns Q tiles of ZB axial points
// at node j (nq tiles apart) and walks through them, loading the next tile's
// inputs into registers while the current one is transformed.  Blocks are
// placed so that consecutive tiles of one j run on the same XCD (hardware
// round-robin over 8 XCDs by workgroup id), where they share L2 lines of the
// [j][f][m][z] intermediates.
// CFL (forward only): also fold the CFL number of u into *ta.cfl, as a
// separate instance so that the plain kernel keeps its registers.
template <int NT, int ADJ, int ZB, bool CFL = false>
__global__ __launch_bounds__(TB) void k_theta_t(KP p, int nq, int Q, const double2* __restrict__ zu, int nfu,
                                               const double2* __restrict__ zy, int nfy, double2* __restrict__ tb,
                                               TimeArg ta) {
    constexpr int M = (NT - 1) / 3, MP1 = M + 1;
    constexpr int NFO = ADJ ? 6 : 3;
    constexpr int H = ZB / 2;
    constexpr int NIN = ADJ ? 4 * ZB + H : 3 * ZB;
    constexpr int NOUT = ADJ ? 3 * ZB : ZB + H;
    constexpr int NSEQ = NIN > NOUT ? NIN : NOUT;
    constexpr int NPAIR = ADJ ? 4 : 3;
    constexpr int NP = NPAIR * MP1 * ZB;              // paired-field loads per tile
    constexpr int NL = NP + (ADJ ? H * MP1 : 0);       // + paired z columns of y_z
    constexpr int PER = (NL + TB - 1) / TB;
    constexpr int NGAP = NT - 2 * M - 1;
    const int nblk = nq * p.nr;
    const int per = (nblk + 7) >> 3;
    const int L = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (L >= nblk) return;
    const int j = L / nq, zq = L - j * nq, nz = p.nz;
    extern __shared__ double2 sh[];
    double2* tw = sh;
    double2* A = sh + NT;
    double2* Bf = A + lp_size(NSEQ * NT);
    for (int t = threadIdx.x; t < NT; t += TB) tw[t] = p.twt[t];
    double U, Om, cw, sw;
    phase_of(p, ta, cw, sw);
    base_at(p, j, cw, sw, U, Om);
    double cmax = 0.0, cz = 0.0, cth = 0.0, cr = 0.0;
    if constexpr (CFL) cfl_scales(p, j, NT, cz, cth, cr);
    // u, w pairs from zu (nfu fields per node), y pairs from zy (nfy per node)
    const double2* bu = zu + (size_t)j * nfu * MP1 * nz;
    const double2* by = ADJ ? zy + (size_t)j * nfy * MP1 * nz : nullptr;
    double2 xa[PER], xb[PER];
    auto fetch = [&](int z0) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = threadIdx.x + i * TB;
            if (e < NP) {
                const int zi = e % ZB, q = e / ZB;
                const int pi = q / MP1, m = q - pi * MP1;
                const double2* src = pi < 3 ? bu : by;
                const int fl = pi < 3 ? 2 * pi : 2 * pi - 6;
                xa[i] = src[(size_t)(fl * MP1 + m) * nz + z0 + zi];
                xb[i] = src[(size_t)((fl + 1) * MP1 + m) * nz + z0 + zi];
            } else if (ADJ && e < NL) {
                const int e2 = e - NP, m = e2 / H, zi = e2 - m * H;
                xa[i] = by[(size_t)(2 * MP1 + m) * nz + z0 + zi];
                xb[i] = by[(size_t)(2 * MP1 + m) * nz + z0 + zi + H];
            }
        }
    };
    // pairs of real fields packed as xa + i xb into the Hermitian halves
    auto place = [&]() {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = threadIdx.x + i * TB;
            if (e >= NL) continue;
            int s, m;
            if (e < NP) {
                const int zi = e % ZB, q = e / ZB;
                const int pi = q / MP1;
                m = q - pi * MP1;
                s = (pi * ZB + zi) * NT;
            } else {
                const int e2 = e - NP;
                m = e2 / H;
                s = (4 * ZB + (e2 - m * H)) * NT;
            }
            if (m == 0) {
                A[lp(s)] = make_double2(xa[i].x, xb[i].x);
            } else {
                A[lp(s + m)] = make_double2(xa[i].x - xb[i].y, xa[i].y + xb[i].x);
                A[lp(s + NT - m)] = make_double2(xa[i].x + xb[i].y, -xa[i].y + xb[i].x);
            }
        }
    };
    // tiles zq, zq + nq, ...: neighbouring blocks (same XCD, same time) hold
    // neighbouring tiles, so the halves of a 128-byte line are read and
    // written together in L2
    int z0 = zq * ZB;
    fetch(z0);
    for (int tile = 0; tile < Q; ++tile, z0 += nq * ZB) {
        if constexpr (NGAP > 0) {
            for (int t = threadIdx.x; t < NIN * NGAP; t += TB) {
                const int s = t / NGAP, q = t - s * NGAP;
                A[lp(s * NT + M + 1 + q)] = czero();
            }
        }
        place();
        __syncthreads();
        if (tile + 1 < Q) fetch(z0 + nq * ZB);
        double2* R1 = fft_ct<NT, true, theta_maxr<ADJ>()>(A, Bf, NIN, tw);
        double2* O = (R1 == A) ? Bf : A;
        for (int t = threadIdx.x; t < ZB * NT; t += TB) {
            const int zi = t / NT, th = t - zi * NT;
            const double2 s0 = R1[lp((0 * ZB + zi) * NT + th)];
            const double2 s1 = R1[lp((1 * ZB + zi) * NT + th)];
            const double2 s2 = R1[lp((2 * ZB + zi) * NT + th)];
            const double ur = s0.x, ut = s0.y, uz = s1.x, wr = s1.y, wt = s2.x, wz = s2.y;
            if constexpr (!ADJ) {
                const double uzU = uz + U;
                if constexpr (CFL) cmax = fmax(cmax, fabs(uzU) * cz + fabs(ut) * cth + fabs(ur) * cr);
                const double Nr = ut * wz - uzU * wt - uz * Om;
                const double Nt = uzU * wr - ur * wz;
                const double Nz = ur * (wt + Om) - ut * wr;
                O[lp(zi * NT + th)] = make_double2(Nr, Nt);
                // N_z of columns zi and zi + H share one complex sequence
                const int q = ZB + (zi < H ? zi : zi - H);
                double* slot = reinterpret_cast<double*>(&O[lp(q * NT + th)]);
                slot[zi < H ? 0 : 1] = Nz;
            } else {
                const double2 s3 = R1[lp((3 * ZB + zi) * NT + th)];
                const double2 s4 = R1[lp((4 * ZB + (zi < H ? zi : zi - H)) * NT + th)];
                const double yr = s3.x, yt = s3.y, yz = (zi < H) ? s4.x : s4.y;
                const double wtO = wt + Om, uzU = uz + U;
                const double Ar = wtO * yz - wz * yt;
                const double At = wz * yr - wr * yz;
                const double Az = wr * yt - wtO * yr;
                const double Br = yt * uzU - yz * ut;
                const double Bt = yz * ur - yr * uzU;
                const double Bz = yr * ut - yt * ur;
                O[lp(zi * NT + th)] = make_double2(Ar, At);
                O[lp((ZB + zi) * NT + th)] = make_double2(Az, Br);
                O[lp((2 * ZB + zi) * NT + th)] = make_double2(Bt, Bz);
            }
        }
        __syncthreads();
        const double2* R2 = fft_ct<NT, false, theta_maxr<ADJ>()>(O, R1, NOUT, tw);
        for (int t = threadIdx.x; t < NFO * MP1 * ZB; t += TB) {
            const int zi = t % ZB, q0 = t / ZB;
            const int f = q0 / MP1, m = q0 - f * MP1;
            int q, half;
            if constexpr (!ADJ) {
                if (f < 2) { q = zi; half = f; }
                else { q = ZB + (zi < H ? zi : zi - H); half = (zi < H) ? 0 : 1; }
            } else {
                q = (f >> 1) * ZB + zi;
                half = f & 1;
            }
            // unpack the two real transforms sharing sequence q
            const double2 a = R2[lp(q * NT + m)];
            const double2 b = cconj(R2[lp(q * NT + (m == 0 ? 0 : NT - m))]);
            const double2 v = half == 0 ? cscale(cadd(a, b), 0.5) : cscale(cmuli(csub(b, a)), 0.5);
            tb[((size_t)(j * NFO + f) * MP1 + m) * nz + z0 + zi] = v;
        }
        __syncthreads();
    }
    if constexpr (CFL) cfl_fold(cmax, ta.cfl);
}

// Pieces shared by the pruned azimuthal kernels (N_theta = 3P, sequences of
// length NT back to back in padded LDS; see k_theta_p for the plan).

// First inverse pass of one packed sequence (base sb), butterflies jj and
// P - jj: xa + i xb of mode jj sits at position jj and its conjugate pair at
// 2P + jj (and symmetrically for mode P - jj); position P + jj is in the
// zero band.  (a1, b1) are modes jj of the two real fields, (a2, b2) modes
// P - jj (unused for jj = 0).
template <int NT>
__device__ __forceinline__ void theta_first_pair(double2* A, int sb, int jj, double2 a1, double2 b1, double2 a2,
                                                 double2 b2) {
    constexpr int P = NT / 3;
    if (jj == 0) {
        double2 v0 = make_double2(a1.x, b1.x), v1 = czero(), v2 = czero();
        dft3<true>(v0, v1, v2);
        A[lp(sb)] = v0;
        A[lp(sb + 1)] = v1;
        A[lp(sb + 2)] = v2;
        return;
    }
    const double2 m1 = make_double2(a1.x - b1.y, a1.y + b1.x);    // mode jj
    const double2 c1 = make_double2(a1.x + b1.y, -a1.y + b1.x);   // its conjugate pair
    const double2 m2 = make_double2(a2.x - b2.y, a2.y + b2.x);    // mode P - jj
    const double2 c2 = make_double2(a2.x + b2.y, -a2.y + b2.x);
    double2 v0 = m1, v1 = czero(), v2 = c2;
    dft3<true>(v0, v1, v2);
    A[lp(sb + 3 * jj)] = v0;
    A[lp(sb + 3 * jj + 1)] = v1;
    A[lp(sb + 3 * jj + 2)] = v2;
    if (2 * jj != P) {
        double2 u0 = m2, u1 = czero(), u2 = c1;
        dft3<true>(u0, u1, u2);
        A[lp(sb + 3 * (P - jj))] = u0;
        A[lp(sb + 3 * (P - jj) + 1)] = u1;
        A[lp(sb + 3 * (P - jj) + 2)] = u2;
    }
}

// Last inverse pass (radix 4, stride NT / 4) of sequence s, butterfly jj,
// twiddled by w[1..3] = tw[q jj]: v[q] = values at theta = jj + q NT / 4.
template <int NT>
__device__ __forceinline__ void theta_inv_tail(const double2* X, int s, int jj, const double2* w, double2* v) {
    constexpr int NBL = NT / 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = X[lp(s * NT + jj + q * NBL)];
#pragma unroll
    for (int q = 1; q < 4; ++q) v[q] = tw_mul<true>(v[q], w[q]);
    dft4<true>(v[0], v[1], v[2], v[3]);
}

// First forward pass (radix 4, stride 1, no twiddles) of output sequence s,
// butterfly jj, on the values at theta = jj + q NT / 4.
template <int NT>
__device__ __forceinline__ void theta_fwd_head(double2* Y, int s, int jj, double2* v) {
    dft4<false>(v[0], v[1], v[2], v[3]);
#pragma unroll
    for (int q = 0; q < 4; ++q) Y[lp(s * NT + 4 * jj + q)] = v[q];
}

// Outputs 0 and 2 of the last forward butterfly jx (radix 3, stride P) of
// sequence s: X[jx] and X[2P + jx].
template <int NT>
__device__ __forceinline__ void theta_last_pair(const double2* R, const double2* tw, int s, int jx, double2& y0,
                                                double2& y2) {
    constexpr int P = NT / 3;
    double2 v0 = R[lp(s * NT + jx)], v1 = R[lp(s * NT + jx + P)], v2 = R[lp(s * NT + jx + 2 * P)];
    v1 = tw_mul<false>(v1, tw[jx]);
    v2 = tw_mul<false>(v2, tw[2 * jx]);
    dft3<false>(v0, v1, v2);
    y0 = v0;
    y2 = v2;
}

// Forward azimuthal pass for N_theta = 3P (then M = P - 1), with the first
// and last passes of both transforms pruned and fused.  Plan: inverse radices
// 3, then pick_radix<8> over P / 4, then 4; forward radices in reverse order.
//  * First inverse pass (radix 3, stride P): butterfly jj reads positions jj
//    (mode jj), P + jj (inside the zero band) and 2P + jj (conjugate of mode
//    P - jj, zero for jj = 0), and butterfly P - jj needs the same two modes,
//    so one thread loads modes jj and P - jj from global memory and runs both;
//    nothing is placed in LDS beforehand.
//  * Last inverse pass and first forward pass (radix 4): the last inverse
//    butterfly jj leaves theta = jj + q N / 4, exactly the inputs of forward
//    butterfly jj, so one thread runs both with the products in between.
//  * Last forward pass (radix 3, stride P): X[m] for m <= M is output 0 of
//    butterfly m, and X[N - m] output 2 of butterfly P - m; a thread running
//    both butterflies unpacks the two real fields and stores them.
// N_z is transformed as its own (real) sequence.  Five barriers per tile
// instead of eight, and about 40% fewer LDS accesses than the generic plan.
// CFL: also fold the CFL number of u into *ta.cfl (a separate instance, so
// the plain kernel keeps its register budget and occupancy; the monitoring
// instance is held to three waves per SIMD as well where the LDS allows three
// blocks per CU, at the cost of three spilled registers: 172 VGPRs would leave
// it two).
template <int NT, int ZB, bool CFL>
__global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(CFL && ZB <= 4 ? 3 : 1))) void k_theta_p(KP p, int nq, int Q, const double2* __restrict__ zu, int nfu,
                                               double2* __restrict__ tb, TimeArg ta, const BDesc* bd) {
    static_assert(NT % 12 == 0, "N_theta = 3P with P a multiple of 4");
    if (bd) {
        const BDesc& d = bd[blockIdx.z];
        p = d.kp; globalize(p, bd); zu = rebase(bd, d.in[0]); tb = rebase(bd, d.out[0]); ta = d.ta; globalize(ta, bd);
    }
    constexpr int P = NT / 3, MP1 = P;
    constexpr int NIN = 3 * ZB, NOUT = 2 * ZB;
    constexpr int PH = P / 2 + 1;                      // first-pass items per sequence: butterflies jj, P - jj
    constexpr int NST = 3 * PH * ZB;
    constexpr int PST = (NST + TB - 1) / TB;
    constexpr int NBL = NT / 4;
    constexpr int NMID = ZB * NBL;
    constexpr int NEND = NOUT * PH;
    const int nblk = nq * p.nr;
    const int per = (nblk + 7) >> 3;
    const int Lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (Lb >= nblk) return;
    const int j = Lb / nq, zq = Lb - j * nq, nz = p.nz;
    extern __shared__ double2 sh[];
    double2* tw = sh;
    double2* A = sh + NT;
    double2* Bf = A + lp_size(NIN * NT);
    for (int t = threadIdx.x; t < NT; t += TB) tw[t] = p.twt[t];
    double U, Om, cw, sw;
    phase_of(p, ta, cw, sw);
    base_at(p, j, cw, sw, U, Om);
    // CFL monitor: dt / dz, dt / (r dtheta), dt / dr at this radial node (dr:
    // the smaller neighbour gap; the axis gap of the first node is 2 r_0)
    double cmax = 0.0, cz = 0.0, cth = 0.0, cr = 0.0;
    if constexpr (CFL) cfl_scales(p, j, NT, cz, cth, cr);
    const double2* bu = zu + (size_t)j * nfu * MP1 * nz;
    // item e: column zi = e % ZB, butterfly pair jj, field pair pi (u_r u_t,
    // u_z w_r, w_t w_z); modes jj and P - jj of both fields
    double2 a1[PST], b1[PST], a2[PST], b2[PST];
    auto fetch = [&](int z0) {
#pragma unroll
        for (int i = 0; i < PST; ++i) {
            const int e = threadIdx.x + i * TB;
            a1[i] = b1[i] = a2[i] = b2[i] = czero();
            if (e < NST) {
                const int zi = e % ZB, q = e / ZB;
                const int pi = q / PH, jj = q - pi * PH;
                const size_t ra = (size_t)2 * pi * MP1 * nz + z0 + zi, rb = ra + (size_t)MP1 * nz;
                a1[i] = bu[ra + (size_t)jj * nz];
                b1[i] = bu[rb + (size_t)jj * nz];
                if (jj) {
                    a2[i] = bu[ra + (size_t)(P - jj) * nz];
                    b2[i] = bu[rb + (size_t)(P - jj) * nz];
                }
            }
        }
    };
    auto first_pass = [&]() {
#pragma unroll
        for (int i = 0; i < PST; ++i) {
            const int e = threadIdx.x + i * TB;
            if (e >= NST) continue;
            const int zi = e % ZB, q = e / ZB;
            const int pi = q / PH, jj = q - pi * PH;
            theta_first_pair<NT>(A, (pi * ZB + zi) * NT, jj, a1[i], b1[i], a2[i], b2[i]);
        }
    };
    int z0 = zq * ZB;
    fetch(z0);
    for (int tile = 0; tile < Q; ++tile, z0 += nq * ZB) {
        first_pass();
        __syncthreads();
        if (tile + 1 < Q) fetch(z0 + nq * ZB);
        double2* R1 = fft_span<NT, true, 8, 3, NBL>(A, Bf, NIN, tw);
        double2* O = (R1 == A) ? Bf : A;
        for (int t = threadIdx.x; t < NMID; t += TB) {
            const int jj = t % NBL, zi = t / NBL;
            double2 w[4];
#pragma unroll
            for (int q = 1; q < 4; ++q) w[q] = tw[q * jj];
            double2 s0[4], s1[4], s2[4];
            theta_inv_tail<NT>(R1, 0 * ZB + zi, jj, w, s0);
            theta_inv_tail<NT>(R1, 1 * ZB + zi, jj, w, s1);
            theta_inv_tail<NT>(R1, 2 * ZB + zi, jj, w, s2);
            double2 o0[4], o1[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double ur = s0[q].x, ut = s0[q].y, uz = s1[q].x, wr = s1[q].y, wt = s2[q].x, wz = s2[q].y;
                const double uzU = uz + U;
                o0[q] = make_double2(ut * wz - uzU * wt - uz * Om, uzU * wr - ur * wz);
                o1[q] = make_double2(ur * (wt + Om) - ut * wr, 0.0);
                if constexpr (CFL) cmax = fmax(cmax, fabs(uzU) * cz + fabs(ut) * cth + fabs(ur) * cr);
            }
            theta_fwd_head<NT>(O, zi, jj, o0);
            theta_fwd_head<NT>(O, ZB + zi, jj, o1);
        }
        __syncthreads();
        const double2* R2 = fft_span<NT, false, 8, 4, P>(O, R1, NOUT, tw);
        for (int t = threadIdx.x; t < NEND; t += TB) {
            const int s = t % NOUT, jA = t / NOUT;   // columns fastest: contiguous z stores
            const int jB = jA == 0 ? 0 : P - jA;
            double2 yA0, yA2, yB0, yB2;
            theta_last_pair<NT>(R2, tw, s, jA, yA0, yA2);
            if (jB != jA) theta_last_pair<NT>(R2, tw, s, jB, yB0, yB2);
            else { yB0 = yA0; yB2 = yA2; }
            // sequence s < ZB: N_r + i N_t of column s; else N_z of column s - ZB
            const int zc = s < ZB ? s : s - ZB;
            auto emit = [&](int m, double2 a, double2 bm) {
                const double2 b = cconj(bm);      // conj X[N - m]
                const size_t col = (size_t)m * nz + z0 + zc;
                if (s < ZB) {
                    tb[(size_t)(j * 3 + 0) * MP1 * nz + col] = cscale(cadd(a, b), 0.5);
                    tb[(size_t)(j * 3 + 1) * MP1 * nz + col] = cscale(cmuli(csub(b, a)), 0.5);
                } else {
                    tb[(size_t)(j * 3 + 2) * MP1 * nz + col] = cscale(cadd(a, b), 0.5);
                }
            };
            emit(jA, yA0, jA == 0 ? yA0 : yB2);
            if (jB != jA) emit(jB, yB0, yA2);
        }
        __syncthreads();
    }
    if constexpr (CFL) cfl_fold(cmax, ta.cfl);
}

// ================================================ wave-resident azimuthal pass
// Forward azimuthal pass with every sequence in registers.  A column (one
// axial point of one radial node) is spread over L lanes (L = 8 or 16), so a
// wave owns 64/L columns; lane (k1, zi) = k1 + L zi holds the L-strided slice
// k1 + L k2 (k2 = 0..R-1, R = N_theta / L) of the three packed inverse
// sequences of column zi.  Four-step transform of length L R: a length-R DFT
// in registers over k2, the twiddles w^(n2 k1), and a length-L DFT across the
// L lanes of the column as log2(L) radix-2 stages whose partner values come
// from cross-lane moves (DPP quad permutations for lane distances 1 and 2,
// ds_swizzle for 4, a DPP row rotation for 8).  That leaves lane k1 holding
// the points theta = R bitrev(k1) + n2; the products are pointwise, so the
// forward transform takes them in that order and runs the transposed network
// (radix-2 stages across the lanes in reverse order with conjugate twiddles,
// then the twiddles and a length-R DFT) back to the natural slices.  The
// Hermitian unpacking of the two real outputs of a sequence pairs X[m]
// (lane k1) with X[N - m] (lane L - k1), fetched with ds_bpermute.  No LDS pass
// and no barrier besides the twiddle table's.

// Lane-partner moves of one 32-bit value: xor 1, xor 2 (DPP quad_perm), xor 4
// (ds_swizzle, bit mode) and xor 8 (DPP row rotation by 8 within 16 lanes).
template <int D>
__device__ __forceinline__ int xl_i32(int v) {
    if constexpr (D == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
    else if constexpr (D == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
    else if constexpr (D == 4) return __builtin_amdgcn_ds_swizzle(v, (4 << 10) | 0x1F);
    else return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);
}
template <int D>
__device__ __forceinline__ double xl_f64(double v) {
    const int lo = xl_i32<D>(__double2loint(v)), hi = xl_i32<D>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <int D>
__device__ __forceinline__ double2 xl(double2 a) { return make_double2(xl_f64<D>(a.x), xl_f64<D>(a.y)); }
__device__ __forceinline__ double2 bperm(int src_byte, double2 a) {
    auto f = [&](double v) {
        const int lo = __builtin_amdgcn_ds_bpermute(src_byte, __double2loint(v));
        const int hi = __builtin_amdgcn_ds_bpermute(src_byte, __double2hiint(v));
        return __hiloint2double(hi, lo);
    };
    return make_double2(f(a.x), f(a.y));
}
// exp(2 pi i k / (2D)), k = 0..D-1: the inverse twiddle of a radix-2 stage of
// lane distance D (the lane's position k within its half of the sub-DFT)
template <int D>
__device__ __forceinline__ double2 wstage_inv(int k) {
    constexpr double s = 0.70710678118654752440, c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
    if constexpr (D == 1) return make_double2(1.0, 0.0);
    else if constexpr (D == 2) return k ? make_double2(0.0, 1.0) : make_double2(1.0, 0.0);
    else if constexpr (D == 4)
        return k == 0 ? make_double2(1.0, 0.0) : k == 1 ? make_double2(s, s) : k == 2 ? make_double2(0.0, 1.0)
                                                                            : make_double2(-s, s);
    else {
        constexpr double cs[8] = {1.0, c1, s, s1, 0.0, -s1, -s, -c1};
        constexpr double sn[8] = {0.0, s1, s, c1, 1.0, c1, s, s1};
        return make_double2(cs[k & 7], sn[k & 7]);
    }
}

// Inverse length-L DFT across the lanes k1 (decimation in frequency): lane k1
// ends with output bitrev(k1).
// Each stage is branch-free: v <- (s v + q) w' with s = +1, w' = 1 on the
// lanes whose bit D is clear and s = -1, w' = the stage twiddle where it is set.
template <int D, int N>
__device__ __forceinline__ void xlane_inv(double2 (&v)[N], int k1) {
    if constexpr (D >= 1) {
        const bool hi = k1 & D;
        const double sg = hi ? -1.0 : 1.0;
        const double2 w = hi ? wstage_inv<D>(k1 & (D - 1)) : make_double2(1.0, 0.0);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double2 q = xl<D>(v[i]);
            const double2 d = make_double2(fma(sg, v[i].x, q.x), fma(sg, v[i].y, q.y));
            v[i] = D > 1 ? cmul(d, w) : d;
        }
        if constexpr (D > 1) xlane_inv<D / 2>(v, k1);
    }
}
// Its conjugate transpose (decimation in time across the lanes): input in
// bitrev order, lane k1 ends with output k1 of the forward length-L DFT.
template <int D, int DMAX, int N>
__device__ __forceinline__ void xlane_fwd(double2 (&v)[N], int k1) {
    const bool hi = k1 & D;
    const double sg = hi ? -1.0 : 1.0;
    const double2 w = hi ? cconj(wstage_inv<D>(k1 & (D - 1))) : make_double2(1.0, 0.0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double2 t = D > 1 ? cmul(v[i], w) : v[i];
        const double2 q = xl<D>(t);
        v[i] = make_double2(fma(sg, t.x, q.x), fma(sg, t.y, q.y));
    }
    if constexpr (D < DMAX) xlane_fwd<2 * D, DMAX>(v, k1);
}

template <int NT, int L>
__global__ __launch_bounds__(TB) void k_theta_w(KP p, int nzb, const double2* __restrict__ zu, int nfu,
                                               double2* __restrict__ tb, TimeArg ta) {
    constexpr int R = NT / L, P = NT / 3, MP1 = P;
    constexpr int CW = 64 / L;             // columns per wave
    constexpr int KPOS = P / L;            // registers k2 < KPOS hold modes m = k1 + L k2
    constexpr int KNEG = (NT - P) / L;     // registers k2 >= KNEG hold conj of modes NT - k1 - L k2
    static_assert(P % L == 0 && (NT - P) % L == 0, "retained band aligned to the lane slices");
    __shared__ double2 tw[NT];
    const int nblk = nzb * p.nr;
    const int per = (nblk + 7) >> 3;
    const int Lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (Lb >= nblk) return;                                   // whole block
    for (int t = threadIdx.x; t < NT; t += TB) tw[t] = p.twt[t];
    __syncthreads();
    const int j = Lb / nzb, zblk = Lb - j * nzb, nz = p.nz;
    const int zw = zblk * (TB / 64) * CW + (threadIdx.x >> 6) * CW;   // first column of this wave
    if (zw >= nz) return;                                     // whole wave (nz is a multiple of CW)
    const int lane = threadIdx.x & 63, k1 = lane & (L - 1), z = zw + lane / L;
    double U, Om, cw, sw;
    phase_of(p, ta, cw, sw);
    base_at(p, j, cw, sw, U, Om);
    const size_t fs = (size_t)MP1 * nz;
    const double2* bz = zu + (size_t)j * nfu * fs + z;
    // packed inverse sequences (u_r, u_t), (u_z, w_r), (w_t, w_z)
    double2 X0[R], X1[R], X2[R];
    auto load = [&](double2 (&X)[R], int f) {
#pragma unroll
        for (int k2 = 0; k2 < R; ++k2) {
            X[k2] = czero();
            if (k2 < KPOS) {
                const int m = k1 + L * k2;
                const double2 a = bz[(size_t)f * fs + (size_t)m * nz], b = bz[(size_t)(f + 1) * fs + (size_t)m * nz];
                X[k2] = (m == 0) ? make_double2(a.x, b.x) : make_double2(a.x - b.y, a.y + b.x);
            } else if (k2 >= KNEG) {
                const int m = NT - k1 - L * k2;
                if (m < P) {
                    const double2 a = bz[(size_t)f * fs + (size_t)m * nz];
                    const double2 b = bz[(size_t)(f + 1) * fs + (size_t)m * nz];
                    X[k2] = make_double2(a.x + b.y, b.x - a.y);    // conj(a) + i conj(b)
                }
            }
        }
    };
    auto inverse = [&](double2 (&X)[R]) {
        dft<R, true>(X);
#pragma unroll
        for (int n2 = 1; n2 < R; ++n2) X[n2] = tw_mul<true>(X[n2], tw[n2 * k1]);
        xlane_inv<L / 2>(X, k1);
    };
    // one sequence's loads in flight while the previous one is transformed;
    // scheduling barriers keep the compiler from hoisting every load to the
    // top, which would cost the registers of three more waves per SIMD
    load(X0, 0);
    load(X1, 2);
    __builtin_amdgcn_sched_barrier(0);
    inverse(X0);
    __builtin_amdgcn_sched_barrier(0);
    load(X2, 4);
    __builtin_amdgcn_sched_barrier(0);
    inverse(X1);
    __builtin_amdgcn_sched_barrier(0);
    inverse(X2);
    // products at the R points of this lane: N = u x w + U x w + u x Om
#pragma unroll
    for (int n2 = 0; n2 < R; ++n2) {
        const double ur = X0[n2].x, ut = X0[n2].y, uz = X1[n2].x, wr = X1[n2].y, wt = X2[n2].x, wz = X2[n2].y;
        const double uzU = uz + U;
        X0[n2] = make_double2(ut * wz - uzU * wt - uz * Om, uzU * wr - ur * wz);
        X1[n2] = make_double2(ur * (wt + Om) - ut * wr, 0.0);
    }
    auto forward = [&](double2 (&X)[R]) {
        xlane_fwd<1, L / 2>(X, k1);
#pragma unroll
        for (int n2 = 1; n2 < R; ++n2) X[n2] = tw_mul<false>(X[n2], tw[n2 * k1]);
        dft<R, false>(X);
    };
    forward(X0);
    forward(X1);
    // X[N - m] of m = k1 + L k2 sits in lane L - k1, register R - 1 - k2 (k1 > 0),
    // or in this lane, register (R - k2) mod R (k1 = 0)
    const int src = (lane - k1 + ((L - k1) & (L - 1))) * 4;
    const size_t ob = (size_t)j * 3 * fs + z;
#pragma unroll
    for (int k2 = 0; k2 < KPOS; ++k2) {
        const int m = k1 + L * k2;
        const double2 p0 = bperm(src, X0[R - 1 - k2]), p1 = bperm(src, X1[R - 1 - k2]);
        const double2 b0 = cconj(k1 ? p0 : X0[(R - k2) % R]);
        const double2 b1 = cconj(k1 ? p1 : X1[(R - k2) % R]);
        const double2 a0 = X0[k2], a1 = X1[k2];
        tb[ob + (size_t)m * nz] = cscale(cadd(a0, b0), 0.5);
        tb[ob + fs + (size_t)m * nz] = cscale(cmuli(csub(b0, a0)), 0.5);
        tb[ob + 2 * fs + (size_t)m * nz] = cscale(cadd(a1, b1), 0.5);
    }
}

// Adjoint azimuthal pass in the wave-resident form of k_theta_w: inputs the
// state (u_r u_t, u_z w_r, w_t w_z from zu) and the adjoint field (y_r y_t and
// y_z alone from zy), outputs A = (Om + w) x Y and B = Y x (U + u) as the
// sequences (A_r, A_t), (A_z, B_r), (B_t, B_z) of each column.
template <int NT, int L>
__global__ __launch_bounds__(TB) void k_theta_wa(KP p, int nzb, const double2* __restrict__ zu, int nfu,
                                                const double2* __restrict__ zy, int nfy, double2* __restrict__ tb,
                                                TimeArg ta) {
    constexpr int R = NT / L, P = NT / 3, MP1 = P;
    constexpr int CW = 64 / L;
    constexpr int KPOS = P / L, KNEG = (NT - P) / L;
    static_assert(P % L == 0 && (NT - P) % L == 0, "retained band aligned to the lane slices");
    __shared__ double2 tw[NT];
    const int nblk = nzb * p.nr;
    const int per = (nblk + 7) >> 3;
    const int Lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (Lb >= nblk) return;
    for (int t = threadIdx.x; t < NT; t += TB) tw[t] = p.twt[t];
    __syncthreads();
    const int j = Lb / nzb, zblk = Lb - j * nzb, nz = p.nz;
    const int zw = zblk * (TB / 64) * CW + (threadIdx.x >> 6) * CW;
    if (zw >= nz) return;
    const int lane = threadIdx.x & 63, k1 = lane & (L - 1), z = zw + lane / L;
    double U, Om, cw, sw;
    phase_of(p, ta, cw, sw);
    base_at(p, j, cw, sw, U, Om);
    const size_t fs = (size_t)MP1 * nz;
    const double2* bu = zu + (size_t)j * nfu * fs + z;
    const double2* by = zy + (size_t)j * nfy * fs + z;
    // packed sequence of fields fa + i fb of base b (fb < 0: fa alone)
    auto load = [&](double2 (&X)[R], const double2* b, int fa, int fb) {
#pragma unroll
        for (int k2 = 0; k2 < R; ++k2) {
            X[k2] = czero();
            if (k2 < KPOS) {
                const int m = k1 + L * k2;
                const double2 a = b[(size_t)fa * fs + (size_t)m * nz];
                const double2 c = fb >= 0 ? b[(size_t)fb * fs + (size_t)m * nz] : czero();
                X[k2] = (m == 0) ? make_double2(a.x, c.x) : make_double2(a.x - c.y, a.y + c.x);
            } else if (k2 >= KNEG) {
                const int m = NT - k1 - L * k2;
                if (m < P) {
                    const double2 a = b[(size_t)fa * fs + (size_t)m * nz];
                    const double2 c = fb >= 0 ? b[(size_t)fb * fs + (size_t)m * nz] : czero();
                    X[k2] = make_double2(a.x + c.y, c.x - a.y);
                }
            }
        }
    };
    auto inverse = [&](double2 (&X)[R]) {
        dft<R, true>(X);
#pragma unroll
        for (int n2 = 1; n2 < R; ++n2) X[n2] = tw_mul<true>(X[n2], tw[n2 * k1]);
        xlane_inv<L / 2>(X, k1);
    };
    double2 X0[R], X1[R], X2[R], X3[R], X4[R];
    load(X3, by, 0, 1);
    load(X4, by, 2, -1);
    __builtin_amdgcn_sched_barrier(0);
    inverse(X3);
    __builtin_amdgcn_sched_barrier(0);
    load(X0, bu, 0, 1);
    __builtin_amdgcn_sched_barrier(0);
    inverse(X4);
    __builtin_amdgcn_sched_barrier(0);
    load(X1, bu, 2, 3);
    __builtin_amdgcn_sched_barrier(0);
    inverse(X0);
    __builtin_amdgcn_sched_barrier(0);
    load(X2, bu, 4, 5);
    __builtin_amdgcn_sched_barrier(0);
    inverse(X1);
    __builtin_amdgcn_sched_barrier(0);
    inverse(X2);
#pragma unroll
    for (int n2 = 0; n2 < R; ++n2) {
        const double ur = X0[n2].x, ut = X0[n2].y, uz = X1[n2].x, wr = X1[n2].y, wt = X2[n2].x, wz = X2[n2].y;
        const double yr = X3[n2].x, yt = X3[n2].y, yz = X4[n2].x;
        const double wtO = wt + Om, uzU = uz + U;
        X0[n2] = make_double2(wtO * yz - wz * yt, wz * yr - wr * yz);
        X1[n2] = make_double2(wr * yt - wtO * yr, yt * uzU - yz * ut);
        X2[n2] = make_double2(yz * ur - yr * uzU, yr * ut - yt * ur);
    }
    auto forward = [&](double2 (&X)[R]) {
        xlane_fwd<1, L / 2>(X, k1);
#pragma unroll
        for (int n2 = 1; n2 < R; ++n2) X[n2] = tw_mul<false>(X[n2], tw[n2 * k1]);
        dft<R, false>(X);
    };
    forward(X0);
    forward(X1);
    forward(X2);
    const int src = (lane - k1 + ((L - k1) & (L - 1))) * 4;
    const size_t ob = (size_t)j * 6 * fs + z;
    auto emit = [&](const double2 (&X)[R], int f0) {
#pragma unroll
        for (int k2 = 0; k2 < KPOS; ++k2) {
            const int m = k1 + L * k2;
            const double2 pr = bperm(src, X[R - 1 - k2]);
            const double2 b = cconj(k1 ? pr : X[(R - k2) % R]);
            const double2 a = X[k2];
            tb[ob + (size_t)f0 * fs + (size_t)m * nz] = cscale(cadd(a, b), 0.5);
            tb[ob + (size_t)(f0 + 1) * fs + (size_t)m * nz] = cscale(cmuli(csub(b, a)), 0.5);
        }
    };
    emit(X0, 0);
    emit(X1, 2);
    emit(X2, 4);
}

// Adjoint azimuthal pass for N_theta = 3P with the pruned, fused plan of
// k_theta_p: inputs u (u_r u_t, u_z w_r, w_t w_z from zu), y (y_r y_t from zy)
// and y_z of columns zi and zi + H paired; outputs A = (Om + w) x Y and
// B = Y x (U + u) as the three sequences (A_r, A_t), (A_z, B_r), (B_t, B_z)
// of each column.
template <int NT, int ZB>
__global__ __launch_bounds__(TB) void k_theta_pa(KP p, int nq, int Q, const double2* __restrict__ zu, int nfu,
                                                const double2* __restrict__ zy, int nfy, double2* __restrict__ tb,
                                                TimeArg ta, const BDesc* bd) {
    static_assert(NT % 12 == 0, "N_theta = 3P with P a multiple of 4");
    if (bd) {
        const BDesc& d = bd[blockIdx.z];
        p = d.kp; globalize(p, bd); zu = rebase(bd, d.in[0]); zy = rebase(bd, d.in[1]); tb = rebase(bd, d.out[0]); ta = d.ta; globalize(ta, bd);
    }
    constexpr int P = NT / 3, MP1 = P;
    constexpr int H = ZB / 2;
    constexpr int NIN = 4 * ZB + H, NOUT = 3 * ZB;
    constexpr int PH = P / 2 + 1;
    constexpr int NPS = 4 * PH * ZB;                   // first-pass items of the field pairs
    constexpr int NST = NPS + PH * H;                  // + of the paired y_z columns
    constexpr int PST = (NST + TB - 1) / TB;
    constexpr int NBL = NT / 4;
    constexpr int NMID = ZB * NBL;
    constexpr int NEND = NOUT * PH;
    const int nblk = nq * p.nr;
    const int per = (nblk + 7) >> 3;
    const int Lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (Lb >= nblk) return;
    const int j = Lb / nq, zq = Lb - j * nq, nz = p.nz;
    extern __shared__ double2 sh[];
    double2* tw = sh;
    double2* A = sh + NT;
    double2* Bf = A + lp_size(NIN * NT);
    for (int t = threadIdx.x; t < NT; t += TB) tw[t] = p.twt[t];
    double U, Om, cw, sw;
    phase_of(p, ta, cw, sw);
    base_at(p, j, cw, sw, U, Om);
    const double2* bu = zu + (size_t)j * nfu * MP1 * nz;
    const double2* by = zy + (size_t)j * nfy * MP1 * nz;
    double2 a1[PST], b1[PST], a2[PST], b2[PST];
    auto fetch = [&](int z0) {
#pragma unroll
        for (int i = 0; i < PST; ++i) {
            const int e = threadIdx.x + i * TB;
            a1[i] = b1[i] = a2[i] = b2[i] = czero();
            size_t ra = 0, rb = 0;
            const double2* src = nullptr;
            int jj = 0;
            if (e < NPS) {
                const int zi = e % ZB, q = e / ZB;
                const int pi = q / PH;
                jj = q - pi * PH;
                src = pi < 3 ? bu : by;
                ra = (size_t)(pi < 3 ? 2 * pi : 0) * MP1 * nz + z0 + zi;
                rb = ra + (size_t)MP1 * nz;
            } else if (e < NST) {
                const int e2 = e - NPS, zi = e2 % H;
                jj = e2 / H;
                src = by;
                ra = (size_t)2 * MP1 * nz + z0 + zi;
                rb = ra + H;
            }
            if (src) {
                a1[i] = src[ra + (size_t)jj * nz];
                b1[i] = src[rb + (size_t)jj * nz];
                if (jj) {
                    a2[i] = src[ra + (size_t)(P - jj) * nz];
                    b2[i] = src[rb + (size_t)(P - jj) * nz];
                }
            }
        }
    };
    auto first_pass = [&]() {
#pragma unroll
        for (int i = 0; i < PST; ++i) {
            const int e = threadIdx.x + i * TB;
            if (e >= NST) continue;
            int s, jj;
            if (e < NPS) {
                const int zi = e % ZB, q = e / ZB;
                const int pi = q / PH;
                jj = q - pi * PH;
                s = pi * ZB + zi;
            } else {
                const int e2 = e - NPS;
                jj = e2 / H;
                s = 4 * ZB + e2 % H;
            }
            theta_first_pair<NT>(A, s * NT, jj, a1[i], b1[i], a2[i], b2[i]);
        }
    };
    int z0 = zq * ZB;
    fetch(z0);
    for (int tile = 0; tile < Q; ++tile, z0 += nq * ZB) {
        first_pass();
        __syncthreads();
        if (tile + 1 < Q) fetch(z0 + nq * ZB);
        double2* R1 = fft_span<NT, true, 8, 3, NBL>(A, Bf, NIN, tw);
        double2* O = (R1 == A) ? Bf : A;
        for (int t = threadIdx.x; t < NMID; t += TB) {
            const int jj = t % NBL, zi = t / NBL;
            double2 w[4];
#pragma unroll
            for (int q = 1; q < 4; ++q) w[q] = tw[q * jj];
            double2 s0[4], s1[4], s2[4], s3[4], s4[4];
            theta_inv_tail<NT>(R1, 0 * ZB + zi, jj, w, s0);
            theta_inv_tail<NT>(R1, 1 * ZB + zi, jj, w, s1);
            theta_inv_tail<NT>(R1, 2 * ZB + zi, jj, w, s2);
            theta_inv_tail<NT>(R1, 3 * ZB + zi, jj, w, s3);
            theta_inv_tail<NT>(R1, 4 * ZB + (zi < H ? zi : zi - H), jj, w, s4);
            double2 o0[4], o1[4], o2[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double ur = s0[q].x, ut = s0[q].y, uz = s1[q].x, wr = s1[q].y, wt = s2[q].x, wz = s2[q].y;
                const double yr = s3[q].x, yt = s3[q].y, yz = (zi < H) ? s4[q].x : s4[q].y;
                const double wtO = wt + Om, uzU = uz + U;
                o0[q] = make_double2(wtO * yz - wz * yt, wz * yr - wr * yz);
                o1[q] = make_double2(wr * yt - wtO * yr, yt * uzU - yz * ut);
                o2[q] = make_double2(yz * ur - yr * uzU, yr * ut - yt * ur);
            }
            theta_fwd_head<NT>(O, zi, jj, o0);
            theta_fwd_head<NT>(O, ZB + zi, jj, o1);
            theta_fwd_head<NT>(O, 2 * ZB + zi, jj, o2);
        }
        __syncthreads();
        const double2* R2 = fft_span<NT, false, 8, 4, P>(O, R1, NOUT, tw);
        for (int t = threadIdx.x; t < NEND; t += TB) {
            const int s = t % NOUT, jA = t / NOUT;
            const int jB = jA == 0 ? 0 : P - jA;
            double2 yA0, yA2, yB0, yB2;
            theta_last_pair<NT>(R2, tw, s, jA, yA0, yA2);
            if (jB != jA) theta_last_pair<NT>(R2, tw, s, jB, yB0, yB2);
            else { yB0 = yA0; yB2 = yA2; }
            const int f0 = 2 * (s / ZB), zc = s % ZB;
            auto emit = [&](int m, double2 a, double2 bm) {
                const double2 b = cconj(bm);
                const size_t col = (size_t)m * nz + z0 + zc;
                tb[(size_t)(j * 6 + f0) * MP1 * nz + col] = cscale(cadd(a, b), 0.5);
                tb[(size_t)(j * 6 + f0 + 1) * MP1 * nz + col] = cscale(cmuli(csub(b, a)), 0.5);
            };
            emit(jA, yA0, jA == 0 ? yA0 : yB2);
            if (jB != jA) emit(jB, yB0, yA2);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- dispatch
#define NPO_NZ_SIZES(X) X(24) X(48) X(96) X(144) X(192) X(288) X(384) X(576) X(768) X(1024) X(1536)
#define NPO_NT_SIZES(X) X(12) X(24) X(48) X(64) X(96) X(128)

bool fast_nz(int nz) {
    switch (nz) {
#define NPO_CASE(N) case N:
        NPO_NZ_SIZES(NPO_CASE)
#undef NPO_CASE
        return true;
    default:
        return false;
    }
}
bool fast_nt(int nt) {
    switch (nt) {
#define NPO_CASE(N) case N:
        NPO_NT_SIZES(NPO_CASE)
#undef NPO_CASE
        return true;
    default:
        return false;
    }
}

size_t zpass_lds(const npo_plan_s& p, int G) {
    if (fast_nz(p.nz)) return ((size_t)p.nz + 2 * lp_size(p.nz)) * sizeof(double2);   // one field per round
    return (size_t)2 * G * p.nz * sizeof(double2);
}
size_t theta_lds(const npo_plan_s& p, int ZB, int adj) {
    const int H = ZB / 2;
    const int nin = adj ? 4 * ZB + H : 3 * ZB, nout = adj ? 3 * ZB : ZB + H;
    const int nseq = nin > nout ? nin : nout;
    if (fast_nt(p.nt)) return ((size_t)p.nt + 2 * lp_size(nseq * p.nt)) * sizeof(double2);
    return (size_t)2 * nseq * p.nt * sizeof(double2);
}

// m per block of the pruned axial kernels: two when a block would carry only
// three fields (the block start-up, twiddle staging and first load, is then
// paid once per six transforms as in the six-field passes)
template <int NF>
constexpr int zpass_mb() { return NF <= 3 ? 2 : 1; }

// A kernel without a batched form met while recording: the batch falls back
// to launching that instance's step by itself.
static void not_batched() {
    if (Recorder* r = recorder()) r->ok = false;
}

template <int NZ, int F0, int NF>
static void launch_zinv_k(dim3 grid, size_t sh, const npo_plan_s& p, const double2* u, const double2* aux,
                          const double2* y, double2* zb, hipStream_t st) {
    if constexpr (NZ % 12 == 0) {
        constexpr int MB = zpass_mb<NF>();
        const unsigned gx = (p.mp1 + MB - 1) / MB, gy = grid.y;
        BDesc d = desc_of(p);
        d.in[0] = u; d.in[1] = aux; d.in[2] = y; d.out[0] = zb;
        const KP kp = p.kp;
        (void)issue(p, -1, d, st, [=](const BDesc* bd, int nb, hipStream_t s) {
            hipLaunchKernelGGL((k_zinv_p<NZ, F0, NF, MB>), dim3(gx, gy, nb), dim3(TB), sh, s, kp, u, aux, y, zb, bd);
        });
    } else {
        not_batched();
        hipLaunchKernelGGL((k_zinv_t<NZ, F0, NF>), grid, dim3(TB), sh, st, p.kp, u, aux, y, zb);
    }
}

template <int NZ>
static void launch_zinv_n(dim3 grid, size_t sh, const npo_plan_s& p, int nf, const double2* u, const double2* aux,
                          const double2* y, double2* zb, hipStream_t st) {
    if (nf == 9) launch_zinv_k<NZ, 0, 9>(grid, sh, p, u, aux, y, zb, st);
    else if (nf == 3) launch_zinv_k<NZ, 6, 3>(grid, sh, p, u, aux, y, zb, st);
    else launch_zinv_k<NZ, 0, 6>(grid, sh, p, u, aux, y, zb, st);
}

// Inverse axial transforms of fields f0 .. f0+nf-1 (written nf per node).
static void launch_zinv(const npo_plan_s& p, int f0, int nf, const double2* u, const double2* aux, const double2* y,
                        double2* zb, hipStream_t st) {
    const int G = p.zgroup;
    const size_t sh = zpass_lds(p, G);
    const dim3 grid(p.mp1, p.nr);
    switch (p.nz) {
#define NPO_CASE(N)                                                                                         \
    case N:                                                                                                 \
        launch_zinv_n<N>(grid, sh, p, nf, u, aux, y, zb, st);                                               \
        return;
        NPO_NZ_SIZES(NPO_CASE)
#undef NPO_CASE
    default:
        not_batched();
        hipLaunchKernelGGL(k_zinv, grid, dim3(256), sh, st, p.kp, f0, nf, G, u, aux, y, zb);
    }
}

template <int NZ, int NFO>
static void launch_zfwd_k(dim3 grid, size_t sh, const npo_plan_s& p, const double2* tb, double2* out0, double2* out1,
                          double scale, hipStream_t st) {
    if constexpr (NZ % 12 == 0) {
        constexpr int MB = zpass_mb<NFO>();
        const unsigned gx = (p.mp1 + MB - 1) / MB, gy = grid.y;
        BDesc d = desc_of(p);
        d.in[0] = tb; d.out[0] = out0; d.out[1] = out1;
        const KP kp = p.kp;
        (void)issue(p, -1, d, st, [=](const BDesc* bd, int nb, hipStream_t s) {
            hipLaunchKernelGGL((k_zfwd_p<NZ, NFO, MB>), dim3(gx, gy, nb), dim3(TB), sh, s, kp, tb, out0, out1, scale,
                               bd);
        });
    } else {
        not_batched();
        hipLaunchKernelGGL((k_zfwd_t<NZ, NFO>), grid, dim3(TB), sh, st, p.kp, tb, out0, out1, scale);
    }
}

static void launch_zfwd(const npo_plan_s& p, int adj, const double2* tb, double2* out0, double2* out1,
                        double scale, hipStream_t st) {
    const int G = p.zgroup;
    const size_t sh = zpass_lds(p, G);
    const dim3 grid(p.mp1, p.nr);
    switch (p.nz) {
#define NPO_CASE(N)                                                                                      \
    case N:                                                                                              \
        if (adj) launch_zfwd_k<N, 6>(grid, sh, p, tb, out0, out1, scale, st);                                \
        else launch_zfwd_k<N, 3>(grid, sh, p, tb, out0, out1, scale, st);                                    \
        return;
        NPO_NZ_SIZES(NPO_CASE)
#undef NPO_CASE
    default:
        not_batched();
        hipLaunchKernelGGL(k_zfwd, grid, dim3(256), sh, st, p.kp, adj ? 6 : 3, G, tb, out0, out1, scale);
    }
}

// Tiles per azimuthal block: the largest of 4, 2 that divides the tiles of a
// radial node and still leaves at least 2048 blocks (8 per CU), else 1.
static int theta_tiles_per_block(const npo_plan_s& p, int ZB) {
    const int tiles = p.nz / ZB;
    for (int q : {4, 2})
        if (tiles % q == 0 && (long long)(tiles / q) * p.nr >= 2048) return q;
    return 1;
}

template <int NT, int ADJ, int ZB>
static void launch_theta_k(dim3 grid, size_t sh, const npo_plan_s& p, int nq, int Q, const double2* zu, int nfu,
                           const double2* zy, int nfy, double2* tb, const TimeArg& ta, hipStream_t st) {
    if constexpr (NT % 12 == 0) {
        BDesc d = desc_of(p);
        d.in[0] = zu; d.in[1] = zy; d.out[0] = tb; d.ta = ta;
        const KP kp = p.kp;
        const unsigned gx = grid.x;
        (void)issue(p, -1, d, st, [=](const BDesc* bd, int nb, hipStream_t s) {
            if constexpr (!ADJ) {
                if (ta.cfl)
                    hipLaunchKernelGGL((k_theta_p<NT, ZB, true>), dim3(gx, 1, nb), dim3(TB), sh, s, kp, nq, Q, zu, nfu,
                                       tb, ta, bd);
                else
                    hipLaunchKernelGGL((k_theta_p<NT, ZB, false>), dim3(gx, 1, nb), dim3(TB), sh, s, kp, nq, Q, zu,
                                       nfu, tb, ta, bd);
            } else
                hipLaunchKernelGGL((k_theta_pa<NT, ZB>), dim3(gx, 1, nb), dim3(TB), sh, s, kp, nq, Q, zu, nfu, zy, nfy,
                                   tb, ta, bd);
        });
    } else {
        not_batched();
        if (!ADJ && ta.cfl)
            hipLaunchKernelGGL((k_theta_t<NT, 0, ZB, true>), grid, dim3(TB), sh, st, p.kp, nq, Q, zu, nfu, zy, nfy,
                               tb, ta);
        else
            hipLaunchKernelGGL((k_theta_t<NT, ADJ, ZB>), grid, dim3(TB), sh, st, p.kp, nq, Q, zu, nfu, zy, nfy, tb, ta);
    }
}

template <int NT, int ADJ>
static void launch_theta_zb(const npo_plan_s& p, int ZB, dim3 grid, size_t sh, int nq, int Q, const double2* zu,
                            int nfu, const double2* zy, int nfy, double2* tb, const TimeArg& ta, hipStream_t st) {
    if (ZB == 8) launch_theta_k<NT, ADJ, 8>(grid, sh, p, nq, Q, zu, nfu, zy, nfy, tb, ta, st);
    else if (ZB == 4) launch_theta_k<NT, ADJ, 4>(grid, sh, p, nq, Q, zu, nfu, zy, nfy, tb, ta, st);
    else launch_theta_k<NT, ADJ, 2>(grid, sh, p, nq, Q, zu, nfu, zy, nfy, tb, ta, st);
}

// The wave-resident forward kernel with L lanes per column: N_theta in
// {24, 48, 96} for L = 8, {48, 96} for L = 16; N_z a multiple of 64 / L.
bool theta_wave_ok(int nt, int nz, int L) {
    if (L == 8) return (nt == 24 || nt == 48 || nt == 96) && nz % 8 == 0;
    if (L == 16) return (nt == 48 || nt == 96) && nz % 4 == 0;
    return false;
}

template <int L>
static void launch_theta_w(const npo_plan_s& p, int adj, const double2* zu, int nfu, const double2* zy, int nfy,
                           double2* tb, const TimeArg& ta, hipStream_t st) {
    constexpr int cols = (TB / 64) * (64 / L);    // columns per block
    const int nzb = (p.nz + cols - 1) / cols;
    const int nblk = nzb * p.nr;
    const dim3 grid((nblk + 7) / 8 * 8);
#define NPO_W(N)                                                                                              \
    if (adj) hipLaunchKernelGGL((k_theta_wa<N, L>), grid, dim3(TB), 0, st, p.kp, nzb, zu, nfu, zy, nfy, tb, ta); \
    else hipLaunchKernelGGL((k_theta_w<N, L>), grid, dim3(TB), 0, st, p.kp, nzb, zu, nfu, tb, ta);
    if (p.nt == 96) { NPO_W(96) }
    else if (p.nt == 48) { NPO_W(48) }
    else if constexpr (L == 8) { NPO_W(24) }
#undef NPO_W
}

static void launch_theta(const npo_plan_s& p, int adj, const double2* zu, int nfu, const double2* zy, int nfy,
                         double2* tb, const TimeArg& ta, hipStream_t st) {
    const int ZB = adj ? p.zb_theta_adj : p.zb_theta_fwd;
    if (ZB < 0) {                               // tuning value -L: the wave-resident kernels, L lanes per column
        not_batched();
        if (ZB == -8) launch_theta_w<8>(p, adj, zu, nfu, zy, nfy, tb, ta, st);
        else launch_theta_w<16>(p, adj, zu, nfu, zy, nfy, tb, ta, st);
        return;
    }
    const size_t sh = theta_lds(p, ZB, adj);
    if (!fast_nt(p.nt)) {
        not_batched();
        hipLaunchKernelGGL(k_theta, dim3(p.nz / ZB, p.nr), dim3(256), sh, st, p.kp, adj, ZB, zu, nfu, zy, nfy, tb, ta);
        return;
    }
    const int Q = theta_tiles_per_block(p, ZB);
    const int nq = p.nz / ZB / Q;
    const int nblk = nq * p.nr;
    const dim3 grid((nblk + 7) / 8 * 8);
    switch (p.nt) {
#define NPO_CASE(N)                                                                                   \
    case N:                                                                                           \
        if (adj) launch_theta_zb<N, 1>(p, ZB, grid, sh, nq, Q, zu, nfu, zy, nfy, tb, ta, st);         \
        else launch_theta_zb<N, 0>(p, ZB, grid, sh, nq, Q, zu, nfu, zy, nfy, tb, ta, st);             \
        return;
        NPO_NT_SIZES(NPO_CASE)
#undef NPO_CASE
    default:
        return;
    }
}

// ---------------------------------------------------------------- launcher
hipError_t launch_nl(const npo_plan_s& p, int adj, const double2* u, const double2* aux, const double2* y,
                     const TimeArg& ta, double2* out0, double2* out1, void* ws, hipStream_t st, const double2* uw_pre,
                     double2* uw_save) {
    char* base = static_cast<char*>(ws);
    double2* zb = reinterpret_cast<double2*>(base + p.ws.zbuf);
    double2* tb = reinterpret_cast<double2*>(base + p.ws.tbuf);
    const size_t g1 = (size_t)p.mp1 * p.nz;     // one field of one radial node
    if (!adj) {
        double2* zo = uw_save ? uw_save : zb;
        prof_begin(p, KID_ZINV_F, st);
        launch_zinv(p, 0, 6, u, aux, y, zo, st);
        prof_end(p, KID_ZINV_F, st);
        prof_begin(p, KID_THETA_F, st);
        launch_theta(p, 0, zo, 6, nullptr, 0, tb, ta, st);
        prof_end(p, KID_THETA_F, st);
    } else if (uw_pre) {
        // u, w of this state were transformed by an earlier forward evaluation
        prof_begin(p, KID_ZINV_Y, st);
        launch_zinv(p, 6, 3, u, aux, y, zb, st);
        prof_end(p, KID_ZINV_Y, st);
        prof_begin(p, KID_THETA_A, st);
        launch_theta(p, 1, uw_pre, 6, zb, 3, tb, ta, st);
        prof_end(p, KID_THETA_A, st);
    } else {
        prof_begin(p, KID_ZINV_A, st);
        launch_zinv(p, 0, 9, u, aux, y, zb, st);
        prof_end(p, KID_ZINV_A, st);
        prof_begin(p, KID_THETA_A, st);
        launch_theta(p, 1, zb, 9, zb + 6 * g1, 9, tb, ta, st);
        prof_end(p, KID_THETA_A, st);
    }
    const double scale = 1.0 / ((double)p.nt * p.nz);
    prof_begin(p, adj ? KID_ZFWD_A : KID_ZFWD_F, st);
    launch_zfwd(p, adj, tb, out0, out1, scale, st);
    prof_end(p, adj ? KID_ZFWD_A : KID_ZFWD_F, st);
    return hipGetLastError();
}

}  // namespace npo
