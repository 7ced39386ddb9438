// Setup, reference (one thread per DOF), reduction and sensitivity kernels of libstmg.
//
// Layout: every space-time vector of a level is time-major with a padded row pitch
// P >= N+4 (multiple of 32 elements); entry (n, i) sits at n*P + i.  Padding
// columns are zero and never written.
#include <hip/hip_runtime.h>
#include <math.h>

#include "stmg_launch.hpp"

namespace stmg {

namespace {
constexpr int kBlock = 256;
inline unsigned blocks_for(int64_t n, int b = kBlock) {
    int64_t g = (n + b - 1) / b;
    return (unsigned)(g < 1 ? 1 : (g > 1048576 ? 1048576 : g));
}
inline unsigned rows_grid(int rows) { return (unsigned)(rows < 65535 ? rows : 65535); }
}  // namespace

// =====================================================================================
// Setup
// =====================================================================================

// SIMP interpolation v = v_ins + (v_con - v_ins) rho^p (Section 2.1).
__global__ void k_simp(const double* __restrict__ rho, int n, double vi, double vc, double p,
                       double* __restrict__ out) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = vi + (vc - vi) * pow(rho[e], p);
}

__global__ void k_simp_derivative(const double* __restrict__ rho, int n, double vi, double vc,
                                  double p, double* __restrict__ out) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = (p == 0.0) ? 0.0 : p * (vc - vi) * pow(rho[e], p - 1.0);
}

void launch_simp(const double* rho, int n, double vi, double vc, double p, double* out,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_simp, dim3(blocks_for(n)), dim3(kBlock), 0, s, rho, n, vi, vc, p, out);
}
void launch_simp_derivative(const double* rho, int n, double vi, double vc, double p,
                            double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_simp_derivative, dim3(blocks_for(n)), dim3(kBlock), 0, s, rho, n, vi,
                       vc, p, out);
}

// Coarse element coefficients of an x-coarsening step (Section 5.1): elements 2e and
// 2e+1 of the fine level merge into coarse element e.
//   R: k = 1 / ((1/k_a + 1/k_b) / 2), c = (c_a + c_b) / 2
//   K: k = (k_a + k_b) / 2,            c = (c_a + c_b) / 2
//   D: chi = (chi_a + chi_b) / 2, k = k_SIMP(chi), c = c_SIMP(chi)
// simp = {k_ins, k_con, p_k, c_ins, c_con, p_c} (D only).
__global__ void k_coarsen_x(const double* __restrict__ k, const double* __restrict__ c,
                            const double* __restrict__ chi, int nc, int method,
                            const double* __restrict__ simp, double* __restrict__ kc,
                            double* __restrict__ cc, double* __restrict__ chic) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nc) return;
    double ka = k[2 * e], kb = k[2 * e + 1];
    double ca = c[2 * e], cb = c[2 * e + 1];
    double xa = chi ? chi[2 * e] : 0.0, xb = chi ? chi[2 * e + 1] : 0.0;
    double xm = (xa + xb) / 2.0;
    if (chic) chic[e] = xm;
    if (method == 0) {
        double rho = (1.0 / ka + 1.0 / kb) / 2.0;
        kc[e] = 1.0 / rho;
        cc[e] = (ca + cb) / 2.0;
    } else if (method == 1) {
        kc[e] = (ka + kb) / 2.0;
        cc[e] = (ca + cb) / 2.0;
    } else {
        kc[e] = simp[0] + (simp[1] - simp[0]) * pow(xm, simp[2]);
        cc[e] = simp[3] + (simp[4] - simp[3]) * pow(xm, simp[5]);
    }
}

void launch_coarsen_x(const double* k, const double* c, const double* chi, int nc, int method,
                      const double* simp, double* kc, double* cc, double* chic, hipStream_t s) {
    hipLaunchKernelGGL(k_coarsen_x, dim3(blocks_for(nc)), dim3(kBlock), 0, s, k, c, chi, nc,
                       method, simp, kc, cc, chic);
}

// min / max of the element diffusivity D_e = k_e / c_e (Section 4) and max c, max k
// (Appendix A).  One block; min and max are independent of the reduction order.
__global__ void k_level_stats(const double* __restrict__ k, const double* __restrict__ c, int n,
                              double* __restrict__ out) {
    __shared__ double s[4][1024];
    int t = threadIdx.x;
    double dmin = INFINITY, dmax = -INFINITY, cmax = -INFINITY, kmax = -INFINITY;
    for (int e = t; e < n; e += blockDim.x) {
        double d = k[e] / c[e];
        dmin = fmin(dmin, d);
        dmax = fmax(dmax, d);
        cmax = fmax(cmax, c[e]);
        kmax = fmax(kmax, k[e]);
    }
    s[0][t] = dmin; s[1][t] = dmax; s[2][t] = cmax; s[3][t] = kmax;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w) {
            s[0][t] = fmin(s[0][t], s[0][t + w]);
            s[1][t] = fmax(s[1][t], s[1][t + w]);
            s[2][t] = fmax(s[2][t], s[2][t + w]);
            s[3][t] = fmax(s[3][t], s[3][t + w]);
        }
        __syncthreads();
    }
    if (t < 4) out[t] = s[t][0];
}

void launch_level_stats(const double* k, const double* c, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_level_stats, dim3(1), dim3(1024), 0, s, k, c, n, out);
}

// Per-node stencil coefficients (Section 2.2).  Element e spans nodes e, e+1 and adds
// c_e h/6 [[2,1],[1,2]] to C and k_e/h [[1,-1],[-1,1]] to K.  A = C/dt + K.
// Couplings to the Dirichlet node 0 are removed (Appendix A), so lo[1] = mlo[1] = 0.
__global__ void k_stencil_coef(const double* __restrict__ k, const double* __restrict__ c, int N,
                               double h, double tau, double omega, double W,
                               double* __restrict__ coef, float* __restrict__ coef32) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > N) return;
    const int64_t S = N + 1;
    double lo = 0, di = 0, up = 0, mlo = 0, mdi = 0, mup = 0, wd = 0;
    if (i >= 1) {
        double cl = c[i - 1], kl = k[i - 1];
        double mdiag = 2.0 * cl * h / 6.0, kdiag = kl / h;
        if (i < N) {
            mdiag += 2.0 * c[i] * h / 6.0;
            kdiag += k[i] / h;
            mup = (c[i] * h / 6.0) / tau;
            up = mup - k[i] / h;
        }
        mdi = mdiag / tau;
        di = mdi + kdiag;
        if (i >= 2) {
            mlo = (cl * h / 6.0) / tau;
            lo = mlo - kl / h;
        }
        wd = omega / di;
    }
    // Node 0 is a Dirichlet row, J u = W u: its only non-zero entries are kl = W and
    // wd = omega / W (the fused kernels evaluate it with a zero left neighbour).
    const double kl = (i >= 1) ? k[i - 1] / h : W;
    const double kr = (i >= 1 && i < N) ? k[i] / h : 0.0;
    if (i == 0) wd = omega / W;
    double v[9] = {lo, di, up, mlo, mdi, mup, wd, kl, kr};
    for (int a = 0; a < 9; ++a) {
        coef[a * S + i] = v[a];
        if (coef32) coef32[a * S + i] = (float)v[a];
    }
}

void launch_stencil_coef(const double* k, const double* c, int N, double h, double tau,
                         double omega, double W, double* coef, float* coef32, hipStream_t s) {
    hipLaunchKernelGGL(k_stencil_coef, dim3(blocks_for(N + 1)), dim3(kBlock), 0, s, k, c, N, h,
                       tau, omega, W, coef, coef32);
}

// Thomas factors of the interior tridiagonal A (nodes 1..N); A is time invariant so
// they are computed once per level.  cp[i] = up_i / den_i, inv[i] = 1 / den_i with
// den_1 = di_1, den_i = di_i - lo_i cp_{i-1}.
__global__ void k_thomas_factors(const double* __restrict__ coef, int N, double* __restrict__ cp,
                                 double* __restrict__ inv) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int64_t S = N + 1;
    const double* lo = coef;
    const double* di = coef + S;
    const double* up = coef + 2 * S;
    double prev = 0.0;
    for (int i = 1; i <= N; ++i) {
        double den = (i == 1) ? di[i] : di[i] - lo[i] * prev;
        double iv = 1.0 / den;
        inv[i] = iv;
        prev = up[i] * iv;
        cp[i] = prev;
    }
}

void launch_thomas_factors(const double* coef, int N, double* cp, double* inv, hipStream_t s) {
    hipLaunchKernelGGL(k_thomas_factors, dim3(1), dim3(64), 0, s, coef, N, cp, inv);
}

// Load vector b = B b_Neu (Section 2.2, Appendix A): b_{i,n} = h/2 (q_{i-1,n} + q_{i,n})
// over the elements adjacent to node i, zero at Dirichlet DOFs.  q: [(Nt+1)][N]
// (row n = load at t_n) or NULL for the uniform source q0.
__global__ void k_load_vector(const double* __restrict__ q, double q0, int N, int Nt, double h,
                              double* __restrict__ b, int64_t P) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > N) return;
    for (int n = blockIdx.y; n <= Nt; n += gridDim.y) {
        double v = 0.0;
        if (n >= 1 && i >= 1) {
            double right = 0.0, left;
            if (q) {
                left = q[(int64_t)n * N + (i - 1)];
                if (i < N) right = q[(int64_t)n * N + i];
            } else {
                left = q0;
                if (i < N) right = q0;
            }
            v = right * h / 2.0 + left * h / 2.0;
        }
        b[(int64_t)n * P + i] = v;
    }
}

void launch_load_vector(const double* q, double q0, int N, int Nt, double h, double* b,
                        int64_t P, hipStream_t s) {
    hipLaunchKernelGGL(k_load_vector, dim3(blocks_for(N + 1), rows_grid(Nt + 1)), dim3(kBlock),
                       0, s, q, q0, N, Nt, h, b, P);
}

// =====================================================================================
// Data movement
// =====================================================================================

template <typename T>
__global__ void k_fill(T* __restrict__ x, int64_t n, T v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = v;
}

template <typename T>
void launch_fill(T* x, int64_t n, T v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, x, n, v);
}

template <typename Tin, typename Tout>
__global__ void k_copy2d(const Tin* __restrict__ src, int64_t sp, Tout* __restrict__ dst,
                         int64_t dp, int rows, int cols, double scale) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    for (int r = blockIdx.y; r < rows; r += gridDim.y) {
        double v = (double)src[(int64_t)r * sp + c];
        dst[(int64_t)r * dp + c] = (Tout)(scale == 1.0 ? v : scale * v);
    }
}

template <typename Tin, typename Tout>
void launch_copy2d(const Tin* src, int64_t sp, Tout* dst, int64_t dp, int rows, int cols,
                   double scale, hipStream_t s) {
    hipLaunchKernelGGL((k_copy2d<Tin, Tout>), dim3(blocks_for(cols), rows_grid(rows)),
                       dim3(kBlock), 0, s, src, sp, dst, dp, rows, cols, scale);
}

template <typename T>
__global__ void k_fill2d(T* __restrict__ x, int64_t P, int rows, int cols, T v) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    for (int r = blockIdx.y; r < rows; r += gridDim.y) x[(int64_t)r * P + c] = v;
}

template <typename T>
void launch_fill2d(T* x, int64_t P, int rows, int cols, T v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill2d<T>, dim3(blocks_for(cols), rows_grid(rows)), dim3(kBlock), 0, s,
                       x, P, rows, cols, v);
}

template <typename Tin>
__global__ void k_axpy2d(const Tin* __restrict__ src, int64_t sp, double* __restrict__ dst,
                         int64_t dp, int rows, int cols, double scale) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    for (int r = blockIdx.y; r < rows; r += gridDim.y) {
        int64_t o = (int64_t)r * dp + c;
        dst[o] = __builtin_fma(scale, (double)src[(int64_t)r * sp + c], dst[o]);
    }
}

template <typename Tin>
void launch_axpy2d(const Tin* src, int64_t sp, double* dst, int64_t dp, int rows, int cols,
                   double scale, hipStream_t s) {
    hipLaunchKernelGGL((k_axpy2d<Tin>), dim3(blocks_for(cols), rows_grid(rows)), dim3(kBlock), 0,
                       s, src, sp, dst, dp, rows, cols, scale);
}

// =====================================================================================
// Reference kernels: one thread per DOF
// =====================================================================================

// mode APPLY_J: y = J x; APPLY_RESIDUAL: y = b - J x;
// APPLY_JACOBI: y = x + omega D^-1 (b - J x) (Section 3.1).  zero_in: x == 0, not read.
template <typename T, int TR>
__global__ void k_apply(LevelView<T> L, int mode, const T* __restrict__ x,
                        const T* __restrict__ b, T* __restrict__ y, int zero_in) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > L.N) return;
    const int64_t P = L.P;
    for (int n = blockIdx.y; n <= L.Nt; n += gridDim.y) {
        const int64_t o = (int64_t)n * P + i;
        T x0 = zero_in ? T(0) : x[o];
        T Jx, scale;
        if (n == 0 || i == 0) {
            Jx = L.W * x0;
            scale = L.wW;
        } else {
            T xm = (zero_in || i == 1) ? T(0) : x[o - 1];
            T xp = (zero_in || i == L.N) ? T(0) : x[o + 1];
            bool coupled = TR ? (n < L.Nt) : (n >= 2);
            T ym = 0, y0 = 0, yp = 0;
            if (coupled && !zero_in) {
                const int64_t q = TR ? o + P : o - P;
                ym = (i == 1) ? T(0) : x[q - 1];
                y0 = x[q];
                yp = (i == L.N) ? T(0) : x[q + 1];
            }
            Jx = stencil_interior<T>(L.mlo[i], L.mdi[i], L.mup[i], L.kl[i], L.kr[i], T(-1), xm, x0, xp,
                                     coupled, ym, y0, yp);
            scale = L.wd[i];
        }
        if (mode == APPLY_J) {
            y[o] = Jx;
        } else {
            T r = b[o] - Jx;
            y[o] = (mode == APPLY_RESIDUAL) ? r : jacobi_update<T>(x0, scale, r);
        }
    }
}

template <typename T>
void launch_apply(const LevelView<T>& L, int trans, int mode, const T* x, const T* b, T* y,
                  bool zero_in, hipStream_t s) {
    dim3 g(blocks_for(L.N + 1), rows_grid(L.Nt + 1));
    if (trans)
        hipLaunchKernelGGL((k_apply<T, 1>), g, dim3(kBlock), 0, s, L, mode, x, b, y, (int)zero_in);
    else
        hipLaunchKernelGGL((k_apply<T, 0>), g, dim3(kBlock), 0, s, L, mode, x, b, y, (int)zero_in);
}

// Restriction R = s P^T (Section 3.1).
//   x (s = 1):   bc_{n,I} = r_{n,2I} + 1/2 (r_{n,2I-1} [I>=1] + r_{n,2I+1} [I<Nc])
//   t (s = 1/2): bc_{J,i} = 1/2 (r_{2J,i} + r_{2J+1,i} [2J+1 <= Nt])
template <typename T>
__global__ void k_restrict_x(LevelView<T> F, const T* __restrict__ r, T* __restrict__ bc,
                             int64_t Pc) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int Nc = F.N / 2;
    if (I > Nc) return;
    for (int n = blockIdx.y; n <= F.Nt; n += gridDim.y) {
        const T* row = r + (int64_t)n * F.P;
        T side = T(0);
        if (I >= 1) side += row[2 * I - 1];
        if (I < Nc) side += row[2 * I + 1];
        bc[(int64_t)n * Pc + I] = fmaT(T(0.5), side, row[2 * I]);
    }
}

template <typename T>
__global__ void k_restrict_t(LevelView<T> F, const T* __restrict__ r, T* __restrict__ bc,
                             int64_t Pc) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > F.N) return;
    const int Ntc = F.Nt / 2;
    for (int J = blockIdx.y; J <= Ntc; J += gridDim.y) {
        T v = r[(int64_t)(2 * J) * F.P + i];
        if (2 * J + 1 <= F.Nt) v += r[(int64_t)(2 * J + 1) * F.P + i];
        bc[(int64_t)J * Pc + i] = T(0.5) * v;
    }
}

// Bilinear interpolation in time (B, Section 5.1), s = 1/2:
//   bc_{J,i} = 1/2 (r_{2J,i} + 1/2 (r_{2J-1,i} [J>=1] + r_{2J+1,i} [2J+1 <= Nt]))
template <typename T>
__global__ void k_restrict_tB(LevelView<T> F, const T* __restrict__ r, T* __restrict__ bc,
                              int64_t Pc) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > F.N) return;
    const int Ntc = F.Nt / 2;
    for (int J = blockIdx.y; J <= Ntc; J += gridDim.y) {
        T side = T(0);
        if (J >= 1) side += r[(int64_t)(2 * J - 1) * F.P + i];
        if (2 * J + 1 <= F.Nt) side += r[(int64_t)(2 * J + 1) * F.P + i];
        bc[(int64_t)J * Pc + i] = T(0.5) * fmaT(T(0.5), side, r[(int64_t)(2 * J) * F.P + i]);
    }
}

template <typename T>
void launch_restrict(char dir, const LevelView<T>& F, const T* r, T* bc, int64_t Pc,
                     hipStream_t s, int interp) {
    if (dir == 'x')
        hipLaunchKernelGGL((k_restrict_x<T>), dim3(blocks_for(F.N / 2 + 1), rows_grid(F.Nt + 1)),
                           dim3(kBlock), 0, s, F, r, bc, Pc);
    else if (interp == 1)
        hipLaunchKernelGGL((k_restrict_tB<T>), dim3(blocks_for(F.N + 1), rows_grid(F.Nt / 2 + 1)),
                           dim3(kBlock), 0, s, F, r, bc, Pc);
    else
        hipLaunchKernelGGL((k_restrict_t<T>), dim3(blocks_for(F.N + 1), rows_grid(F.Nt / 2 + 1)),
                           dim3(kBlock), 0, s, F, r, bc, Pc);
}

// Prolongation P (Section 3.1, causal interpolation C):
//   x: u_{n,2I} += z_{n,I},  u_{n,2I+1} += 1/2 (z_{n,I} + z_{n,I+1})
//   t: u_{2J,i} += z_{J,i},  u_{2J+1,i} += z_{J,i}
template <typename T>
__global__ void k_prolong_x(LevelView<T> F, const T* __restrict__ z, int64_t Pc,
                            T* __restrict__ u) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f > F.N) return;
    for (int n = blockIdx.y; n <= F.Nt; n += gridDim.y) {
        const T* zr = z + (int64_t)n * Pc;
        T* uo = u + (int64_t)n * F.P + f;
        if (f & 1)
            *uo = fmaT(T(0.5), zr[f >> 1] + zr[(f >> 1) + 1], *uo);
        else
            *uo += zr[f >> 1];
    }
}

template <typename T>
__global__ void k_prolong_t(LevelView<T> F, const T* __restrict__ z, int64_t Pc,
                            T* __restrict__ u) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > F.N) return;
    for (int n = blockIdx.y; n <= F.Nt; n += gridDim.y)
        u[(int64_t)n * F.P + i] += z[(int64_t)(n >> 1) * Pc + i];
}

// Bilinear in time (B):  u_{2J,i} += z_{J,i},  u_{2J+1,i} += 1/2 (z_{J,i} + z_{J+1,i})
// (a t-coarsened level has an even N_t, so J+1 <= N_t/2 for every odd fine level).
template <typename T>
__global__ void k_prolong_tB(LevelView<T> F, const T* __restrict__ z, int64_t Pc,
                             T* __restrict__ u) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > F.N) return;
    for (int n = blockIdx.y; n <= F.Nt; n += gridDim.y) {
        T* uo = u + (int64_t)n * F.P + i;
        const T* zr = z + (int64_t)(n >> 1) * Pc + i;
        if (n & 1)
            *uo = fmaT(T(0.5), zr[0] + zr[Pc], *uo);
        else
            *uo += zr[0];
    }
}

template <typename T>
void launch_prolong_add(char dir, const LevelView<T>& F, const T* z, int64_t Pc, T* u,
                        hipStream_t s, int interp) {
    dim3 g(blocks_for(F.N + 1), rows_grid(F.Nt + 1));
    if (dir == 'x')
        hipLaunchKernelGGL((k_prolong_x<T>), g, dim3(kBlock), 0, s, F, z, Pc, u);
    else if (interp == 1)
        hipLaunchKernelGGL((k_prolong_tB<T>), g, dim3(kBlock), 0, s, F, z, Pc, u);
    else
        hipLaunchKernelGGL((k_prolong_t<T>), g, dim3(kBlock), 0, s, F, z, Pc, u);
}

// Exact solve on the coarsest level (Algorithm 1, first branch): Dirichlet DOFs take
// z = b / W; the free nodes step through time with A z_n = b_n + (C/dt) z_{n-1}
// (forward) or A z_n = b_n + (C/dt) z_{n+1} (transposed, backwards from Nt).  One
// block: the right-hand side of each step is formed in parallel, the tridiagonal
// solve (precomputed Thomas factors) runs in thread 0.  rhs: N+1 doubles scratch in
// global memory (the level's padding row area is not used).
template <typename TV>
__global__ void k_coarsest(LevelView<double> L, const double* __restrict__ cp,
                           const double* __restrict__ inv, const TV* __restrict__ b,
                           TV* __restrict__ u, int trans, double* __restrict__ rhs) {
    const int t = threadIdx.x;
    const int64_t P = L.P;
    const int N = L.N, Nt = L.Nt;
    for (int i = t; i <= N; i += blockDim.x) u[i] = (TV)((double)b[i] / L.W);
    for (int n = 1 + t; n <= Nt; n += blockDim.x) u[(int64_t)n * P] = (TV)((double)b[(int64_t)n * P] / L.W);
    __syncthreads();
    for (int s = 0; s < Nt; ++s) {
        const int n = trans ? Nt - s : 1 + s;
        const int m = trans ? n + 1 : n - 1;
        const bool coupled = trans ? (n < Nt) : (n >= 2);
        for (int i = 1 + t; i <= N; i += blockDim.x) {
            double v = (double)b[(int64_t)n * P + i];
            if (coupled) {
                const int64_t q = (int64_t)m * P + i;
                double y0 = (double)u[q];
                double ym = (i >= 2) ? (double)u[q - 1] : 0.0;
                double yp = (i < N) ? (double)u[q + 1] : 0.0;
                double w = L.mdi[i] * y0;
                w = __builtin_fma(L.mlo[i], ym, w);
                w = __builtin_fma(L.mup[i], yp, w);
                v = v + w;
            }
            rhs[i] = v;
        }
        __syncthreads();
        if (t == 0) {
            double d = 0.0;
            for (int i = 1; i <= N; ++i) {
                d = (i == 1) ? rhs[1] * inv[1] : (rhs[i] - L.lo[i] * d) * inv[i];
                rhs[i] = d;
            }
            double x = 0.0;
            TV* row = u + (int64_t)n * P;
            for (int i = N; i >= 1; --i) {
                x = (i == N) ? rhs[N] : rhs[i] - cp[i] * x;
                row[i] = (TV)x;
            }
        }
        __syncthreads();
    }
}

template <typename TV>
void launch_coarsest(const LevelView<double>& L, const double* cp, const double* inv,
                     const TV* b, TV* u, int trans, hipStream_t s) {
    // cp and inv hold N+1 entries each, followed by N+1 entries of rhs scratch.
    double* rhs = const_cast<double*>(inv) + (L.N + 1);
    hipLaunchKernelGGL((k_coarsest<TV>), dim3(1), dim3(256), 0, s, L, cp, inv, b, u, trans, rhs);
}

// Columns of A^{-1} for a small coarsest level (N <= 64): thread j solves A x = e_j
// with the Thomas factors.  ainv is row-major N x N (row i = node i+1).
__global__ void k_dense_inverse(const double* __restrict__ coef, int N, const double* __restrict__ cp,
                                const double* __restrict__ inv, double* __restrict__ ainv) {
    const int j = threadIdx.x;
    if (j >= N) return;
    const double* lo = coef;
    double d = 0.0;
    for (int i = 1; i <= N; ++i) {
        const double e = (i - 1 == j) ? 1.0 : 0.0;
        d = (i == 1) ? e * inv[1] : (e - lo[i] * d) * inv[i];
        ainv[(int64_t)(i - 1) * N + j] = d;
    }
    double x = 0.0;
    for (int i = N; i >= 1; --i) {
        x = (i == N) ? ainv[(int64_t)(i - 1) * N + j] : ainv[(int64_t)(i - 1) * N + j] - cp[i] * x;
        ainv[(int64_t)(i - 1) * N + j] = x;
    }
}

void launch_dense_inverse(const double* coef, int N, const double* cp, const double* inv,
                          double* ainv, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_inverse, dim3(1), dim3(64), 0, s, coef, N, cp, inv, ainv);
}

// Exact coarsest solve with a register-resident inverse (one wave, node i+1 in lane
// i): each time step forms b_n + (C/dt) z_{n-1} (z_{n+1} for J^T) in parallel and
// multiplies by A^{-1}, broadcasting the right-hand side lane by lane.  Lanes without a
// node hold a zero right-hand side and zero rows of A^{-1}.
template <typename TV, int NMAX>
__global__ __launch_bounds__(64) void k_coarsest_dense(LevelView<double> L,
                                                       const double* __restrict__ ainv,
                                                       const TV* __restrict__ b,
                                                       TV* __restrict__ u, int trans) {
    const int lane = threadIdx.x;
    const int N = L.N, Nt = L.Nt;
    const int64_t P = L.P;
    for (int i = lane; i <= N; i += 64) u[i] = (TV)((double)b[i] / L.W);
    for (int n = 1 + lane; n <= Nt; n += 64) u[(int64_t)n * P] = (TV)((double)b[(int64_t)n * P] / L.W);
    const int node = lane + 1;
    const bool act = node <= N;
    double a[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) a[j] = (act && j < N) ? ainv[(int64_t)lane * N + j] : 0.0;
    const double mlo = act ? L.mlo[node] : 0.0;
    const double mdi = act ? L.mdi[node] : 0.0;
    const double mup = act ? L.mup[node] : 0.0;
    double zprev = 0.0;
    // the right-hand side of the next step is loaded one step ahead
    auto row = [&](int s) { return trans ? Nt - s : 1 + s; };
    double bn = (act && Nt > 0) ? (double)b[(int64_t)row(0) * P + node] : 0.0;
    for (int s = 0; s < Nt; ++s) {
        const int n = row(s);
        const bool coupled = trans ? (n < Nt) : (n >= 2);
        double rhs = bn;
        if (s + 1 < Nt) bn = act ? (double)b[(int64_t)row(s + 1) * P + node] : 0.0;
        const double zl = shfl_up1(zprev);   // 0 at lane 0 (node 1 has no coupled left node)
        const double zr = shfl_dn1(zprev);
        if (coupled) {
            double w = mdi * zprev;
            w = __builtin_fma(mlo, zl, w);
            w = __builtin_fma(mup, zr, w);
            rhs = rhs + w;
        }
        if (!act) rhs = 0.0;   // also when a neighbour's value is not finite
        // a[j] = 0 for j >= N and rhs = 0 on inactive lanes: the terms beyond N add an
        // exact zero, and the product runs without a branch per term
        double z = 0.0;
#pragma unroll
        for (int j = 0; j < NMAX; ++j) z = __builtin_fma(a[j], readlane_f64(rhs, j), z);
        if (act) u[(int64_t)n * P + node] = (TV)z;
        zprev = act ? z : 0.0;
    }
}

template <typename TV>
void launch_coarsest_dense(const LevelView<double>& L, const double* ainv, const TV* b, TV* u,
                           int trans, hipStream_t s) {
    if (L.N <= 8)
        hipLaunchKernelGGL((k_coarsest_dense<TV, 8>), dim3(1), dim3(64), 0, s, L, ainv, b, u, trans);
    else if (L.N <= 16)
        hipLaunchKernelGGL((k_coarsest_dense<TV, 16>), dim3(1), dim3(64), 0, s, L, ainv, b, u, trans);
    else if (L.N <= 32)
        hipLaunchKernelGGL((k_coarsest_dense<TV, 32>), dim3(1), dim3(64), 0, s, L, ainv, b, u, trans);
    else
        hipLaunchKernelGGL((k_coarsest_dense<TV, 64>), dim3(1), dim3(64), 0, s, L, ainv, b, u, trans);
}

// =====================================================================================
// Deterministic reductions
// =====================================================================================

int reduce_parts(int rows) { return rows < 1024 ? rows : 1024; }

__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    return sh[0];
}

template <typename T>
__global__ void k_sumsq_partial(const T* __restrict__ x, int rows, int cols, int64_t P,
                                double* __restrict__ parts) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int r = blockIdx.x; r < rows; r += gridDim.x)
        for (int c = threadIdx.x; c < cols; c += blockDim.x) {
            double v = (double)x[(int64_t)r * P + c];
            acc = __builtin_fma(v, v, acc);
        }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

template <typename T>
void launch_sumsq_partial(const T* x, int rows, int cols, int64_t P, double* parts,
                          hipStream_t s) {
    hipLaunchKernelGGL((k_sumsq_partial<T>), dim3(reduce_parts(rows)), dim3(kBlock), 0, s, x,
                       rows, cols, P, parts);
}

__global__ void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                              int rows, int cols, int64_t Pa, int64_t Pb,
                              double* __restrict__ parts) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int r = blockIdx.x; r < rows; r += gridDim.x)
        for (int c = threadIdx.x; c < cols; c += blockDim.x)
            acc = __builtin_fma(a[(int64_t)r * Pa + c], b[(int64_t)r * Pb + c], acc);
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

void launch_dot_partial(const double* a, const double* b, int rows, int cols, int64_t Pa,
                        int64_t Pb, double* parts, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_partial, dim3(reduce_parts(rows)), dim3(kBlock), 0, s, a, b, rows,
                       cols, Pa, Pb, parts);
}

__global__ void k_reduce_final(const double* __restrict__ parts, int n, double scale,
                               double* __restrict__ out) {
    __shared__ double sh[1024];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += parts[i];
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[0] = scale * s;
}

void launch_reduce_final(const double* parts, int n, double scale, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, s, parts, n, scale, out);
}

// The same sum, written to pinned host memory: host[0] = scale * sum, then (after a
// system-scope fence) host[1] = tag, so a host that sees the tag sees the value.
__global__ void k_reduce_to_host(const double* __restrict__ parts, int n, double scale,
                                 double* host, double tag) {
    __shared__ double sh[1024];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += parts[i];
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        *reinterpret_cast<volatile double*>(host) = scale * s;
        __threadfence_system();
        *reinterpret_cast<volatile double*>(host + 1) = tag;
    }
}

void launch_reduce_to_host(const double* parts, int n, double scale, double* host, double tag,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_to_host, dim3(1), dim3(1024), 0, s, parts, n, scale, host, tag);
}

template <typename T, int TR>
__global__ void k_residual_sumsq(LevelView<T> L, const T* __restrict__ u, const T* __restrict__ b,
                                 double* __restrict__ parts) {
    __shared__ double sh[kBlock];
    const int64_t P = L.P;
    double acc = 0.0;
    for (int n = blockIdx.x; n <= L.Nt; n += gridDim.x)
        for (int i = threadIdx.x; i <= L.N; i += blockDim.x) {
            const int64_t o = (int64_t)n * P + i;
            T Jx;
            if (n == 0 || i == 0) {
                Jx = L.W * u[o];
            } else {
                bool coupled = TR ? (n < L.Nt) : (n >= 2);
                T ym = 0, y0 = 0, yp = 0;
                if (coupled) {
                    const int64_t q = TR ? o + P : o - P;
                    ym = (i == 1) ? T(0) : u[q - 1];
                    y0 = u[q];
                    yp = (i == L.N) ? T(0) : u[q + 1];
                }
                Jx = stencil_interior<T>(L.mlo[i], L.mdi[i], L.mup[i], L.kl[i], L.kr[i], T(-1),
                                         (i == 1) ? T(0) : u[o - 1], u[o],
                                         (i == L.N) ? T(0) : u[o + 1], coupled, ym, y0, yp);
            }
            double r = (double)(b[o] - Jx);
            acc = __builtin_fma(r, r, acc);
        }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

template <typename T>
void launch_residual_sumsq_partial(const LevelView<T>& L, int trans, const T* u, const T* b,
                                   double* parts, hipStream_t s) {
    dim3 g(reduce_parts(L.Nt + 1));
    if (trans)
        hipLaunchKernelGGL((k_residual_sumsq<T, 1>), g, dim3(kBlock), 0, s, L, u, b, parts);
    else
        hipLaunchKernelGGL((k_residual_sumsq<T, 0>), g, dim3(kBlock), 0, s, L, u, b, parts);
}

// =====================================================================================
// Sensitivities (Section 7.2, discrete adjoint)
// =====================================================================================
// g_e = - sum_{n>=1} [ (k'_e/h) (L_{e+1,n} - L_{e,n})(u_{e+1,n} - u_{e,n})
//                      + (c'_e h / (6 dt)) (L_e, L_{e+1}) [[2,1],[1,2]] (du_e, du_{e+1}) ]
// with du = u_n - u_{n-1} and Dirichlet entries (node 0, level 0) of u and L set to 0.

int gradient_chunks(int Nt) {
    int c = (Nt + 127) / 128;
    return c < 1 ? 1 : (c > 1024 ? 1024 : c);
}

__global__ void k_gradient_partial(const double* __restrict__ u, const double* __restrict__ lam,
                                   int N, int Nt, int64_t Pu, int64_t Pl,
                                   const double* __restrict__ kp, const double* __restrict__ cpd,
                                   double h, double tau, double* __restrict__ parts) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N) return;
    const int chunks = gridDim.y;
    const int per = (Nt + chunks - 1) / chunks;
    const int n0 = 1 + blockIdx.y * per;
    const int n1 = min(Nt, n0 + per - 1);
    double sk = 0.0, sc = 0.0;
    for (int n = n0; n <= n1; ++n) {
        const double* ur = u + (int64_t)n * Pu;
        const double* lr = lam + (int64_t)n * Pl;
        double ua = (e == 0) ? 0.0 : ur[e], ub = ur[e + 1];
        double la = (e == 0) ? 0.0 : lr[e], lb = lr[e + 1];
        sk = __builtin_fma(lb - la, ub - ua, sk);
        double pa = 0.0, pb = 0.0;
        if (n >= 2) {
            const double* up = ur - Pu;
            pa = (e == 0) ? 0.0 : up[e];
            pb = up[e + 1];
        }
        double da = ua - pa, db = ub - pb;
        sc += la * (2.0 * da + db) + lb * (da + 2.0 * db);
    }
    parts[(int64_t)blockIdx.y * N + e] = -(kp[e] / h) * sk - (cpd[e] * h / (6.0 * tau)) * sc;
}

void launch_gradient_partial(const double* u, const double* lam, int N, int Nt, int64_t Pu,
                             int64_t Pl, const double* kp, const double* cpd, double h, double tau,
                             double* parts, hipStream_t s) {
    hipLaunchKernelGGL(k_gradient_partial, dim3(blocks_for(N), gradient_chunks(Nt)), dim3(kBlock),
                       0, s, u, lam, N, Nt, Pu, Pl, kp, cpd, h, tau, parts);
}

__global__ void k_gradient_final(const double* __restrict__ parts, int N, int chunks,
                                 double* __restrict__ g) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N) return;
    double acc = 0.0;
    for (int c = 0; c < chunks; ++c) acc += parts[(int64_t)c * N + e];
    g[e] = acc;
}

void launch_gradient_final(const double* parts, int N, int chunks, double* g, hipStream_t s) {
    hipLaunchKernelGGL(k_gradient_final, dim3(blocks_for(N)), dim3(kBlock), 0, s, parts, N,
                       chunks, g);
}

// =====================================================================================
// Design update (optimisation problem of Section 7.1)
// =====================================================================================

// One workgroup: thread t owns elements t, t + kOcThreads, ...  Every sum and maximum
// goes through the same fixed tree (butterfly inside a wave, then the 16 wave values
// in order), so the bisection takes the same steps on every run.
constexpr int kOcThreads = 1024;
constexpr int kOcWaves = kOcThreads / 64;
constexpr int kOcHalvings = 96;
constexpr double kOcBracket = 1e40;

__device__ __forceinline__ double oc_trial(double chi, double drive, double lam, double eta,
                                           double lo, double hi) {
    return fmin(fmax(chi * pow(drive / lam, eta), lo), hi);
}

// sum (MAX = false) or maximum (MAX = true) over the workgroup, returned to every
// thread; sh[buf * kOcWaves ...] is written, so consecutive calls alternate buf
template <bool MAX>
__device__ __forceinline__ double oc_block_reduce(double v, double* sh, int buf) {
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o);
        v = MAX ? fmax(v, w) : v + w;
    }
    if ((threadIdx.x & 63) == 0) sh[buf * kOcWaves + (threadIdx.x >> 6)] = v;
    __syncthreads();
    double r = sh[buf * kOcWaves];
    for (int i = 1; i < kOcWaves; ++i) {
        const double w = sh[buf * kOcWaves + i];
        r = MAX ? fmax(r, w) : r + w;
    }
    return r;
}

// Optimality-criteria step: D = max(-g, 0), lo = max(chi_min, chi - move),
// hi = min(1, chi + move), chi'(lam) = min(max(chi (D / lam)^eta, lo), hi), with lam
// from kOcHalvings halvings of [maxD / kOcBracket, maxD kOcBracket] in log space,
// stepping up while mean(chi'(lam)) exceeds the volume bound.  chi_new may alias chi:
// a thread writes only its own elements, after its last read of them.
__global__ __launch_bounds__(kOcThreads) void k_oc_update(const double* chi,
                                                          const double* __restrict__ g, int n,
                                                          double volume, double move,
                                                          double eta, double chi_min,
                                                          double* chi_new) {
    __shared__ double sh[2 * kOcWaves];
    const int t = threadIdx.x;
    double dmax = 0.0;
    for (int e = t; e < n; e += kOcThreads) dmax = fmax(dmax, fmax(-g[e], 0.0));
    dmax = oc_block_reduce<true>(dmax, sh, 1);
    const double scale = dmax > 0.0 ? dmax : 1.0;
    double a = scale / kOcBracket, b = scale * kOcBracket;
    for (int it = 0; it < kOcHalvings; ++it) {
        const double mid = sqrt(a) * sqrt(b);
        double s = 0.0;
        for (int e = t; e < n; e += kOcThreads) {
            const double c = chi[e];
            s += oc_trial(c, fmax(-g[e], 0.0), mid, eta, fmax(chi_min, c - move),
                          fmin(1.0, c + move));
        }
        s = oc_block_reduce<false>(s, sh, it & 1);
        if (s / n > volume) a = mid;
        else b = mid;
    }
    const double lam = sqrt(a) * sqrt(b);
    for (int e = t; e < n; e += kOcThreads) {
        const double c = chi[e];
        chi_new[e] = oc_trial(c, fmax(-g[e], 0.0), lam, eta, fmax(chi_min, c - move),
                              fmin(1.0, c + move));
    }
}

void launch_oc_update(const double* chi, const double* g, int n, double volume, double move,
                      double eta, double chi_min, double* chi_new, hipStream_t s) {
    hipLaunchKernelGGL(k_oc_update, dim3(1), dim3(kOcThreads), 0, s, chi, g, n, volume, move,
                       eta, chi_min, chi_new);
}

// ---- explicit instantiations ---------------------------------------------------------
template void launch_fill<double>(double*, int64_t, double, hipStream_t);
template void launch_fill<float>(float*, int64_t, float, hipStream_t);
template void launch_fill2d<double>(double*, int64_t, int, int, double, hipStream_t);
template void launch_fill2d<float>(float*, int64_t, int, int, float, hipStream_t);
template void launch_copy2d<double, double>(const double*, int64_t, double*, int64_t, int, int,
                                            double, hipStream_t);
template void launch_copy2d<double, float>(const double*, int64_t, float*, int64_t, int, int,
                                           double, hipStream_t);
template void launch_copy2d<float, double>(const float*, int64_t, double*, int64_t, int, int,
                                           double, hipStream_t);
template void launch_copy2d<float, float>(const float*, int64_t, float*, int64_t, int, int,
                                          double, hipStream_t);
template void launch_axpy2d<float>(const float*, int64_t, double*, int64_t, int, int, double,
                                   hipStream_t);
template void launch_axpy2d<double>(const double*, int64_t, double*, int64_t, int, int, double,
                                    hipStream_t);
template void launch_apply<double>(const LevelView<double>&, int, int, const double*,
                                   const double*, double*, bool, hipStream_t);
template void launch_apply<float>(const LevelView<float>&, int, int, const float*, const float*,
                                  float*, bool, hipStream_t);
template void launch_restrict<double>(char, const LevelView<double>&, const double*, double*,
                                      int64_t, hipStream_t, int);
template void launch_restrict<float>(char, const LevelView<float>&, const float*, float*,
                                     int64_t, hipStream_t, int);
template void launch_prolong_add<double>(char, const LevelView<double>&, const double*, int64_t,
                                         double*, hipStream_t, int);
template void launch_prolong_add<float>(char, const LevelView<float>&, const float*, int64_t,
                                        float*, hipStream_t, int);
template void launch_coarsest<double>(const LevelView<double>&, const double*, const double*,
                                      const double*, double*, int, hipStream_t);
template void launch_coarsest<float>(const LevelView<double>&, const double*, const double*,
                                     const float*, float*, int, hipStream_t);
template void launch_coarsest_dense<double>(const LevelView<double>&, const double*,
                                            const double*, double*, int, hipStream_t);
template void launch_coarsest_dense<float>(const LevelView<double>&, const double*,
                                           const float*, float*, int, hipStream_t);
template void launch_sumsq_partial<double>(const double*, int, int, int64_t, double*,
                                           hipStream_t);
template void launch_sumsq_partial<float>(const float*, int, int, int64_t, double*, hipStream_t);
template void launch_residual_sumsq_partial<double>(const LevelView<double>&, int, const double*,
                                                    const double*, double*, hipStream_t);
template void launch_residual_sumsq_partial<float>(const LevelView<float>&, int, const float*,
                                                   const float*, double*, hipStream_t);

}  // namespace stmg
