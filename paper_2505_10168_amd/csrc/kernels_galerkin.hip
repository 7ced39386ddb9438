// Galerkin coarse operators (P reassembly, Section 5.1): J^(l+1) = R^(l) J^(l) P^(l).
//
// With the semi-coarsening transfers of Section 3.1 / 5.1 the product of two 3 x 3
// space-time stencils stays 3 x 3, so every Galerkin level is stored as a 9-point
// stencil: 9 arrays of (Nt+1) x P doubles in the level's vector layout, array
// k = 3 (dt + 1) + (dx + 1) holding at (n, i) the coefficient of x(n + dt, i + dx) in
// row (n, i).  Coefficients that would reach outside the grid are zero.  These levels
// are smoothed, applied and restricted one thread per DOF; with the causal transfers
// no row couples to a later time level, so the coarsest level is solved by time
// stepping with one tridiagonal solve per time level.
#include <hip/hip_runtime.h>

#include "stmg_launch.hpp"

namespace stmg {

namespace {
constexpr int kBlock = 256;
inline unsigned blocks_for(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    return (unsigned)(g < 1 ? 1 : g);
}
inline unsigned rows_grid(int rows) { return (unsigned)(rows < 65535 ? rows : 65535); }

// 1-D transfer of Section 3.1 / 5.1 along one axis.  kind: 0 = identity (the axis is
// not coarsened), 1 = linear (x, or bilinear t), 2 = causal t.
struct Tap {
    int idx[3];
    double w[3];
    int n;
};

// fine points that coarse point C prolongs to (column C of P), inside 0..nf
__device__ __forceinline__ Tap children(int kind, int C, int nf) {
    Tap t;
    t.n = 0;
    if (kind == 0) {
        t.idx[0] = C; t.w[0] = 1.0; t.n = 1;
        return t;
    }
    if (kind == 1 && 2 * C - 1 >= 0) { t.idx[t.n] = 2 * C - 1; t.w[t.n] = 0.5; ++t.n; }
    t.idx[t.n] = 2 * C; t.w[t.n] = 1.0; ++t.n;
    if (2 * C + 1 <= nf) { t.idx[t.n] = 2 * C + 1; t.w[t.n] = kind == 1 ? 0.5 : 1.0; ++t.n; }
    return t;
}

// coarse points that fine point f takes its prolonged value from (row f of P)
__device__ __forceinline__ Tap parents(int kind, int f) {
    Tap t;
    if (kind == 0) { t.idx[0] = f; t.w[0] = 1.0; t.n = 1; }
    else if (kind == 2 || (f & 1) == 0) { t.idx[0] = f >> 1; t.w[0] = 1.0; t.n = 1; }
    else { t.idx[0] = (f - 1) >> 1; t.w[0] = 0.5; t.idx[1] = (f + 1) >> 1; t.w[1] = 0.5; t.n = 2; }
    return t;
}

// Entry (dt, dx) of row (n, i) of the Appendix A operator of a rediscretised level:
// Dirichlet rows (n = 0 or i = 0) are W on the diagonal; other rows hold A = C/dt + K
// on time level n and -C/dt on level n - 1 (n >= 2), with the couplings to the
// Dirichlet node 0 removed (lo[1] = mlo[1] = 0 in the coefficient arrays).
__device__ __forceinline__ double rediscretised_entry(const LevelView<double>& V, int n, int i,
                                                      int dt, int dx) {
    if (n == 0 || i == 0) return (dt == 0 && dx == 0) ? V.W : 0.0;
    if (dt == 0) return dx < 0 ? V.lo[i] : (dx == 0 ? V.di[i] : V.up[i]);
    if (dt < 0 && n >= 2) return -(dx < 0 ? V.mlo[i] : (dx == 0 ? V.mdi[i] : V.mup[i]));
    return 0.0;
}
}  // namespace

// Coarse stencil of row (J, I): s sum_a sum_b P_{a,(J,I)} J_{a,b} P_{b,(J',I')}, i.e.
// R = s P^T applied to the fine rows a that (J, I) prolongs to.  The fine operator is
// the rediscretised one (fs == nullptr) or a stored stencil.  All weights are powers
// of two, so each term is exact and only the order of the sum is a choice: fine rows
// in time-major order, then the fine stencil in array order, then the parents.
__global__ void k_galerkin(LevelView<double> F, const double* __restrict__ fs, int kt, int kx,
                           double s, int Nc, int Ntc, int64_t Pc, double* __restrict__ cs) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I > Nc) return;
    const int64_t FE = (int64_t)(F.Nt + 1) * F.P, CE = (int64_t)(Ntc + 1) * Pc;
    for (int J = blockIdx.y; J <= Ntc; J += gridDim.y) {
        double acc[9];
        for (int k = 0; k < 9; ++k) acc[k] = 0.0;
        const Tap ct = children(kt, J, F.Nt), cx = children(kx, I, F.N);
        for (int a = 0; a < ct.n; ++a) {
            const int ft = ct.idx[a];
            for (int c = 0; c < cx.n; ++c) {
                const int fx = cx.idx[c];
                const double wa = s * ct.w[a] * cx.w[c];
                for (int k = 0; k < 9; ++k) {
                    const int dt = k / 3 - 1, dx = k % 3 - 1;
                    const int bt = ft + dt, bx = fx + dx;
                    if (bt < 0 || bt > F.Nt || bx < 0 || bx > F.N) continue;
                    const double v = fs ? fs[k * FE + (int64_t)ft * F.P + fx]
                                        : rediscretised_entry(F, ft, fx, dt, dx);
                    if (v == 0.0) continue;
                    const Tap pt = parents(kt, bt), px = parents(kx, bx);
                    for (int p = 0; p < pt.n; ++p) {
                        const int ot = pt.idx[p] - J;
                        if (ot < -1 || ot > 1) continue;
                        for (int q = 0; q < px.n; ++q) {
                            const int ox = px.idx[q] - I;
                            if (ox < -1 || ox > 1) continue;
                            acc[3 * (ot + 1) + (ox + 1)] += wa * v * pt.w[p] * px.w[q];
                        }
                    }
                }
            }
        }
        for (int k = 0; k < 9; ++k) cs[k * CE + (int64_t)J * Pc + I] = acc[k];
    }
}

void launch_galerkin(const LevelView<double>& F, const double* fs, char dir, int interp,
                     int Nc, int Ntc, int64_t Pc, double* cs, hipStream_t s) {
    const int kt = dir == 't' ? (interp == 1 ? 1 : 2) : 0;
    const int kx = dir == 'x' ? 1 : 0;
    const double sc = dir == 't' ? 0.5 : 1.0;
    dim3 g(blocks_for(Nc + 1), rows_grid(Ntc + 1));
    hipLaunchKernelGGL(k_galerkin, g, dim3(kBlock), 0, s, F, fs, kt, kx, sc, Nc, Ntc, Pc, cs);
}

// y = J x, b - J x or x + omega (b - J x) / J_ii with a stored stencil.  The transpose
// reads row (n + dt, i + dx)'s coefficient of (n, i), i.e. array 8 - k there.
template <int TR>
__global__ void k_apply_stencil(StencilView S, int mode, double omega, const double* __restrict__ x,
                                const double* __restrict__ b, double* __restrict__ y, int zero_in) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > S.N) return;
    const int64_t P = S.P, E = S.E;
    for (int n = blockIdx.y; n <= S.Nt; n += gridDim.y) {
        const int64_t o = (int64_t)n * P + i;
        double Jx = 0.0;
        if (!zero_in) {
            for (int k = 0; k < 9; ++k) {
                const int nn = n + k / 3 - 1, ii = i + k % 3 - 1;
                if (nn < 0 || nn > S.Nt || ii < 0 || ii > S.N) continue;
                const int64_t q = (int64_t)nn * P + ii;
                const double c = TR ? S.s[(8 - k) * E + q] : S.s[k * E + o];
                Jx = __builtin_fma(c, x[q], Jx);
            }
        }
        if (mode == APPLY_J) {
            y[o] = Jx;
        } else {
            const double r = b[o] - Jx;
            if (mode == APPLY_RESIDUAL) y[o] = r;
            else y[o] = (zero_in ? 0.0 : x[o]) + omega * r / S.s[4 * E + o];
        }
    }
}

void launch_apply_stencil(const StencilView& S, int trans, int mode, double omega, const double* x,
                          const double* b, double* y, bool zero_in, hipStream_t s) {
    dim3 g(blocks_for(S.N + 1), rows_grid(S.Nt + 1));
    if (trans)
        hipLaunchKernelGGL(k_apply_stencil<1>, g, dim3(kBlock), 0, s, S, mode, omega, x, b, y,
                           (int)zero_in);
    else
        hipLaunchKernelGGL(k_apply_stencil<0>, g, dim3(kBlock), 0, s, S, mode, omega, x, b, y,
                           (int)zero_in);
}

// Thomas factors of the tridiagonal block of every time level (nodes 0..N), for J
// (lo = array 3, up = array 5 of the row) and for J^T (lo_i = array 5 of row i - 1,
// up_i = array 3 of row i + 1): cp_i = up_i / den_i, inv_i = 1 / den_i with
// den_0 = di_0, den_i = di_i - lo_i cp_{i-1}.  One thread per time level and matrix.
__global__ void k_stencil_thomas(StencilView S, double* __restrict__ f) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n > 2 * S.Nt + 1) return;
    const int tr = n > S.Nt;
    const int m = tr ? n - S.Nt - 1 : n;
    const int64_t E = S.E, row = (int64_t)m * S.P;
    double* cp = f + (tr ? 2 : 0) * E + row;
    double* inv = f + (tr ? 3 : 1) * E + row;
    const double* s3 = S.s + 3 * E + row;
    const double* s4 = S.s + 4 * E + row;
    const double* s5 = S.s + 5 * E + row;
    double c = 0.0;
    for (int i = 0; i <= S.N; ++i) {
        const double lo = i == 0 ? 0.0 : (tr ? s5[i - 1] : s3[i]);
        const double up = i == S.N ? 0.0 : (tr ? s3[i + 1] : s5[i]);
        const double den = s4[i] - lo * c;
        const double r = 1.0 / den;
        c = up * r;
        cp[i] = c;
        inv[i] = r;
    }
}

void launch_stencil_thomas(const StencilView& S, double* factors, hipStream_t s) {
    hipLaunchKernelGGL(k_stencil_thomas, dim3(blocks_for(2 * (int64_t)S.Nt + 2)), dim3(kBlock), 0,
                       s, S, factors);
}

// Exact solve on a stencil level whose rows couple only to their own and the previous
// time level (J; for J^T: the next one, stepping backwards).  One workgroup: the
// right-hand side of a time level is formed in parallel, then thread 0 runs the
// Thomas recurrence from LDS.
constexpr int kStencilSolveThreads = 1024;
__global__ __launch_bounds__(kStencilSolveThreads) void k_stencil_coarsest(
    StencilView S, const double* __restrict__ f, int trans, const double* __restrict__ b,
    double* __restrict__ z) {
    __shared__ double r[kStencilCoarsestMaxNodes];
    __shared__ double lo[kStencilCoarsestMaxNodes];
    __shared__ double cp[kStencilCoarsestMaxNodes];
    __shared__ double inv[kStencilCoarsestMaxNodes];
    const int64_t E = S.E, P = S.P;
    const double* fcp = f + (trans ? 2 : 0) * E;
    const double* finv = f + (trans ? 3 : 1) * E;
    for (int step = 0; step <= S.Nt; ++step) {
        const int n = trans ? S.Nt - step : step;
        const int64_t row = (int64_t)n * P;
        for (int i = threadIdx.x; i <= S.N; i += blockDim.x) {
            double v = b[row + i];
            if (!trans && n >= 1) {
                for (int dx = -1; dx <= 1; ++dx) {
                    const int j = i + dx;
                    if (j >= 0 && j <= S.N) v -= S.s[(dx + 1) * E + row + i] * z[row - P + j];
                }
            } else if (trans && n < S.Nt) {
                for (int dx = -1; dx <= 1; ++dx) {
                    const int j = i + dx;
                    if (j >= 0 && j <= S.N) v -= S.s[(1 - dx) * E + row + P + j] * z[row + P + j];
                }
            }
            r[i] = v;
            lo[i] = i == 0 ? 0.0 : (trans ? S.s[5 * E + row + i - 1] : S.s[3 * E + row + i]);
            cp[i] = fcp[row + i];
            inv[i] = finv[row + i];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double d = 0.0;
            for (int i = 0; i <= S.N; ++i) {
                d = (r[i] - lo[i] * d) * inv[i];
                r[i] = d;
            }
            double x = 0.0;
            for (int i = S.N; i >= 0; --i) {
                x = r[i] - cp[i] * x;
                r[i] = x;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i <= S.N; i += blockDim.x) z[row + i] = r[i];
        __syncthreads();
    }
}

void launch_stencil_coarsest(const StencilView& S, const double* factors, int trans,
                             const double* b, double* z, hipStream_t s) {
    hipLaunchKernelGGL(k_stencil_coarsest, dim3(1), dim3(kStencilSolveThreads), 0, s, S, factors,
                       trans, b, z);
}

}  // namespace stmg
