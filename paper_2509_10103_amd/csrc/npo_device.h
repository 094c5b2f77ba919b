// Device helpers shared by the kernel sources (complex arithmetic in double2,
// spectral indexing, the base flow).  Not part of the public ABI.
#pragma once
#include "npo_internal.h"

namespace npo {

// ------------------------------------------------------- global pointers
// Pointers read from a work-descriptor table are generic to the compiler,
// which then emits flat loads and stores; flat operations also count against
// the LDS wait counter, so every LDS wait would drain the global prefetches.
// rebase() re-expresses such a pointer as the table's own address (a kernel
// argument, hence known to be global memory) plus a uniform byte offset that
// the optimiser cannot fold away, so the accesses stay global ones.  Null
// stays null.  Every plan table, field and workspace is device global memory.
template <class T>
__device__ __forceinline__ T* rebase(const void* base, T* q) {
    if (!q) return nullptr;
    const long long d = (long long)((const char*)q - (const char*)base);
    unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)d);
    unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(d >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));     // opaque: keeps base + offset from folding back to q
    const long long off = (long long)(((unsigned long long)hi << 32) | lo);
    return (T*)((const char*)base + off);
}
__device__ __forceinline__ void globalize(KP& k, const void* b) {
    k.r = rebase(b, k.r); k.w = rebase(b, k.w); k.D1 = rebase(b, k.D1); k.D2 = rebase(b, k.D2);
    k.B = rebase(b, k.B); k.D1T = rebase(b, k.D1T); k.D1WT = rebase(b, k.D1WT); k.BWT = rebase(b, k.BWT);
    k.col0 = rebase(b, k.col0); k.Ut = rebase(b, k.Ut); k.dUt = rebase(b, k.dUt); k.twz = rebase(b, k.twz);
    k.twt = rebase(b, k.twt); k.HLU = rebase(b, k.HLU); k.PLU = rebase(b, k.PLU); k.HOM = rebase(b, k.HOM);
}
__device__ __forceinline__ void globalize(TimeArg& t, const void* b) {
    t.dstep = rebase(b, t.dstep);
    t.cfl = rebase(b, t.cfl);
}

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

}  // namespace npo
