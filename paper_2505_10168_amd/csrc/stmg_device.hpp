// Device-side building blocks of the STMG kernels: the per-node stencil of the
// BE-FE all-at-once operator (Section 2.2, eq. stencil of J, with the Dirichlet
// treatment of Appendix A) and the damped Jacobi update (Section 3.1).
//
// Every kernel (reference one-thread-per-DOF kernels and fused streaming kernels)
// evaluates J through the same inline functions below, in the same operation
// order, so both kernel families produce bit-identical iterates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stmg {

// Per-node stencil coefficients of one level (arrays of length N+1, node i):
//   lo[i] = A_{i,i-1}, di[i] = A_{i,i}, up[i] = A_{i,i+1}   with A = C/dt + K
//   mlo/mdi/mup[i]       = the same entries of C/dt
//   kl[i] = k_{i-1}/h, kr[i] = k_i/h  (conductances of the elements left/right of node i)
//   wd[i] = omega / A_{i,i}
// Entries that couple to the Dirichlet node 0 (lo[1], mlo[1]) and entries beyond the
// last node (up[N], mup[N], kr[N]) are 0: this removes the eliminated columns of
// Appendix A.  Node 0 itself is a Dirichlet row handled separately (J u = W u there,
// as on time level 0).
template <typename T>
struct LevelView {
    int N;          // elements; nodes 0..N
    int Nt;         // time steps; levels 0..Nt
    int64_t P;      // row pitch (elements of T) of every vector of this level
    const T* lo;
    const T* di;
    const T* up;
    const T* mlo;
    const T* mdi;
    const T* mup;
    const T* wd;
    const T* kl;
    const T* kr;
    T W;            // W_Diri of this level (Appendix A)
    T wW;           // omega / W_Diri
};

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Neighbour exchange across the whole wave with DPP wave shifts (ALU latency, no LDS
// round trip): shfl_up1 gives lane i the value of lane i-1, shfl_dn1 the value of
// lane i+1; the edge lane (0, resp. 63) receives 0.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;

template <int CTRL>
__device__ __forceinline__ int dpp32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)dpp32<CTRL>((int)(unsigned)b);
    const unsigned hi = (unsigned)dpp32<CTRL>((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// value of lane l (wave-uniform l), broadcast to the whole wave
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)bits, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(bits >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double shfl_up1(double v) { return dpp64<kDppWaveShr1>(v); }
__device__ __forceinline__ double shfl_dn1(double v) { return dpp64<kDppWaveShl1>(v); }
__device__ __forceinline__ float shfl_up1(float v) {
    return __int_as_float(dpp32<kDppWaveShr1>(__float_as_int(v)));
}
__device__ __forceinline__ float shfl_dn1(float v) {
    return __int_as_float(dpp32<kDppWaveShl1>(__float_as_int(v)));
}

// (J x) at an interior DOF (i >= 1, n >= 1), evaluated in difference form
//   sum_j (C/dt)_ij (x_{j,n} - x_{j,m}) + k_{i-1}/h (x_i - x_{i-1}) + k_i/h (x_i - x_{i+1})
// which equals sum_j A_ij x_{j,n} - sum_j (C/dt)_ij x_{j,m} but keeps the large,
// cancelling terms out of the rounding.  m = n-1 for J (coupled iff n >= 2) and
// m = n+1 for J^T (coupled iff n < Nt); uncoupled rows use y = 0.
// The left conductance term is formed as fma(nm, xm, x0): nm = -1 gives exactly
// x0 - xm (one rounding of the exact difference), nm = 0 drops the left neighbour,
// which is how i = 1 removes the eliminated column of node 0 (mlo[1] = 0 already
// removes it from the mass term).
template <typename T>
__device__ __forceinline__ T stencil_interior(T mlo, T mdi, T mup, T kl, T kr, T nm,
                                              T xm, T x0, T xp, bool coupled,
                                              T ym, T y0, T yp) {
    const T dm = coupled ? xm - ym : xm;
    const T d0 = coupled ? x0 - y0 : x0;
    const T dp = coupled ? xp - yp : xp;
    T s = mdi * d0;
    s = fmaT(mlo, dm, s);
    s = fmaT(mup, dp, s);
    s = fmaT(kl, fmaT(nm, xm, x0), s);
    s = fmaT(kr, x0 - xp, s);
    return s;
}

// One damped Jacobi update of a single DOF given its residual r = b - (J u):
// u' = u + (omega / D) r.
template <typename T>
__device__ __forceinline__ T jacobi_update(T u, T scale, T r) { return fmaT(scale, r, u); }

}  // namespace stmg
