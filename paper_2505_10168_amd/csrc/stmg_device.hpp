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
//   lo[i] = A_{i,i-1}, di[i] = A_{i,i}, up[i] = A_{i,i+1}  with A = C/dt + K
//   mlo/mdi/mup          = the same entries of C/dt
//   wd[i] = omega / A_{i,i}
// Entries that couple to the Dirichlet node 0 (lo[1], mlo[1]) and entries beyond
// the last node (up[N], mup[N]) are stored as 0, which removes the eliminated
// columns of Appendix A.  Node 0 itself is a Dirichlet row handled separately
// (J u = W u there, as on time level 0).
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
    T W;            // W_Diri of this level (Appendix A)
    T wW;           // omega / W_Diri
};

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// (J x) at an interior DOF (i >= 1, n >= 1):
//   sum_j A_ij x_{j,n} - [coupled] sum_j (C/dt)_ij x_{j,m}
// with m = n-1 for J (coupled iff n >= 2) and m = n+1 for J^T (coupled iff n < Nt).
template <typename T>
__device__ __forceinline__ T stencil_interior(T lo, T di, T up, T mlo, T mdi, T mup,
                                              T xm, T x0, T xp, bool coupled,
                                              T ym, T y0, T yp) {
    T s = di * x0;
    s = fmaT(lo, xm, s);
    s = fmaT(up, xp, s);
    if (coupled) {
        T t = mdi * y0;
        t = fmaT(mlo, ym, t);
        t = fmaT(mup, yp, t);
        s = s - t;
    }
    return s;
}

// One damped Jacobi update of a single DOF given its residual r = b - (J u):
// u' = u + (omega / D) r.
template <typename T>
__device__ __forceinline__ T jacobi_update(T u, T scale, T r) { return fmaT(scale, r, u); }

}  // namespace stmg
