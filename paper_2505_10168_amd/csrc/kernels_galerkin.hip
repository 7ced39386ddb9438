// Galerkin coarse operators (P reassembly, Section 5.1): J^(l+1) = R^(l) J^(l) P^(l).
//
// With the semi-coarsening transfers of Section 3.1 / 5.1 the product of two 3 x 3
// space-time stencils stays 3 x 3, so every Galerkin level is a 9-point stencil: array
// k = 3 (dt + 1) + (dx + 1) holds at (n, i) the coefficient of x(n + dt, i + dx) in row
// (n, i); coefficients that would reach outside the grid are zero.  The operators do
// not depend on the time level except near the first and last levels, so a level
// stores only its R distinct stencil rows (R is 3 or 4 in practice; array 9 holds the
// Jacobi scale omega / J_ii of each) and a map from time level to stored row; all time
// levels of a row class are built by the same arithmetic from the same inputs and are
// therefore exactly equal.  These levels are smoothed by streaming passes
// (k_stencil_fused, which also forms the residual and its restriction) or one step per
// launch, and applied one thread per DOF.  With the causal transfers no row couples to a
// later time level, so the coarsest level is solved by time stepping, one tridiagonal
// block per time level (k_stencil_coarsest_dense with the blocks' inverses up to 64
// nodes, else k_stencil_coarsest with Thomas factors); with bilinear transfers it is
// factored by a band LU (k_lu_*).  The kernels are instantiated for FP64 vectors and, for
// the FP32 cycles of mixed precision, for FP32 vectors with an FP32 copy of the stencil;
// the coarsest solves keep FP64 arithmetic and factors for both.
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
// the rediscretised one (fs == nullptr) or a stored stencil with row map frow and
// array stride FE.  One stored coarse row r is formed from its representative time
// level J = crep[r].  All weights are powers of two, so each term is exact and only
// the order of the sum is a choice: fine rows in time-major order, then the fine
// stencil in array order, then the parents.
__global__ void k_galerkin(LevelView<double> F, const double* __restrict__ fs,
                           const int* __restrict__ frow, int64_t FE, int kt, int kx, double s,
                           int Nc, int Ntc, int64_t Pc, int Rc, const int* __restrict__ crep,
                           double omega, double* __restrict__ cs) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I > Nc) return;
    const int64_t CE = (int64_t)Rc * Pc;
    for (int r = blockIdx.y; r < Rc; r += gridDim.y) {
        const int J = crep[r];
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
                    const double v = fs ? fs[k * FE + (int64_t)frow[ft] * F.P + fx]
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
        for (int k = 0; k < 9; ++k) cs[k * CE + (int64_t)r * Pc + I] = acc[k];
        cs[9 * CE + (int64_t)r * Pc + I] = omega / acc[4];   // Jacobi scale omega / J_ii
    }
}

void launch_galerkin(const LevelView<double>& F, const StencilView* fsv, char dir, int interp,
                     const StencilView& C, const int* crep, double omega, double* cs,
                     hipStream_t s) {
    const int kt = dir == 't' ? (interp == 1 ? 1 : 2) : 0;
    const int kx = dir == 'x' ? 1 : 0;
    const double sc = dir == 't' ? 0.5 : 1.0;
    dim3 g(blocks_for(C.N + 1), rows_grid(C.R));
    hipLaunchKernelGGL(k_galerkin, g, dim3(kBlock), 0, s, F, fsv ? fsv->s : nullptr,
                       fsv ? fsv->row : nullptr, fsv ? fsv->E : 0, kt, kx, sc, C.N, C.Nt, C.P,
                       C.R, crep, omega, cs);
}

// y = J x, b - J x or x + (omega / J_ii) (b - J x) with a stored stencil (the scale is
// the stencil's array 9).  The transpose
// reads row (n + dt, i + dx)'s coefficient of (n, i), i.e. array 8 - k there.
template <typename T, int TR>
__global__ void k_apply_stencil(StencilViewT<T> S, int mode, const T* __restrict__ x,
                                const T* __restrict__ b, T* __restrict__ y, int zero_in) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > S.N) return;
    const int64_t P = S.P, E = S.E;
    for (int n = blockIdx.y; n <= S.Nt; n += gridDim.y) {
        const int64_t o = (int64_t)n * P + i;
        const int64_t co = (int64_t)S.row[n] * P + i;   // this row's coefficients
        T Jx = T(0);
        if (!zero_in) {
            for (int k = 0; k < 9; ++k) {
                const int nn = n + k / 3 - 1, ii = i + k % 3 - 1;
                if (nn < 0 || nn > S.Nt || ii < 0 || ii > S.N) continue;
                const int64_t q = (int64_t)nn * P + ii;
                const T c = TR ? S.s[(8 - k) * E + (int64_t)S.row[nn] * P + ii] : S.s[k * E + co];
                Jx = fmaT(c, x[q], Jx);
            }
        }
        if (mode == APPLY_J) {
            y[o] = Jx;
        } else {
            const T r = b[o] - Jx;
            if (mode == APPLY_RESIDUAL) y[o] = r;
            else y[o] = fmaT(S.s[9 * E + co], r, zero_in ? T(0) : x[o]);
        }
    }
}

template <typename T>
void launch_apply_stencil(const StencilViewT<T>& S, int trans, int mode, const T* x, const T* b,
                          T* y, bool zero_in, hipStream_t s) {
    dim3 g(blocks_for(S.N + 1), rows_grid(S.Nt + 1));
    if (trans)
        hipLaunchKernelGGL((k_apply_stencil<T, 1>), g, dim3(kBlock), 0, s, S, mode, x, b, y,
                           (int)zero_in);
    else
        hipLaunchKernelGGL((k_apply_stencil<T, 0>), g, dim3(kBlock), 0, s, S, mode, x, b, y,
                           (int)zero_in);
}

// ---- fused Jacobi passes on a stencil level ------------------------------------------
// S damped Jacobi steps in one pass that streams through time (forward for J, backward
// for J^T): step k at time level n needs step k-1 at levels n and n -/+ 1, both already
// in registers.  One wave owns a strip of 64 - 2 S useful columns (one per lane, S halo
// lanes per side: each step spoils one more column from the strip's edge) and a
// segment of time levels, started S levels early (the warm-up rows: a step that lacks
// its earlier-level input is wrong only on the first levels it sees).  Neighbouring
// columns are exchanged between lanes.  The terms of J x are added in the order of
// k_apply_stencil, so this pass and S one-step launches give the same values.
// HEAD 1 / 2 first adds the x / t prolongation of the coarse correction z (the
// expressions of k_prolong_x / k_prolong_t); TAIL 2 / 3 also form the residual
// b - J y_S (one more warm-up row and halo lane: it needs y_S at the neighbours) and
// write its t / x restriction, with the expressions of k_restrict_t / k_restrict_x
// (causal interpolation): t pairs the levels 2J, 2J+1 of one segment (segments start at
// even levels and have even lengths), x takes the neighbour columns' residuals from the
// adjacent lanes (one more halo lane).
#ifndef STMG_STENCIL_TARGET_WAVES_ALU
#define STMG_STENCIL_TARGET_WAVES_ALU 3072
#endif
constexpr int kStencilWave = 64;
constexpr int kStencilWavesPerBlock = 4;

template <typename T, int TR, int S, int HEAD, int TAIL>
__global__ __launch_bounds__(kStencilWave * kStencilWavesPerBlock) void k_stencil_fused(
    StencilViewT<T> V, const T* __restrict__ u, const T* __restrict__ b, T* __restrict__ out,
    int zero_in, const T* __restrict__ z, int64_t Pz, T* __restrict__ bc, int64_t Pbc, int Nc,
    int xw, int seg, int nwaves) {
    // halo lanes per side, warm-up rows
    constexpr int H = S + (TAIL ? 1 : 0) + (TAIL == 3 ? 1 : 0);
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * kStencilWavesPerBlock +
                                                    (int)(threadIdx.x >> 6));
    if (wave >= nwaves) return;
    const int lane = threadIdx.x & (kStencilWave - 1);
    const int U = kStencilWave - 2 * H;
    const int wx = wave % xw, wt = wave / xw;
    const int i = wx * U - H + lane;                  // this lane's column
    const bool valid = i >= 0 && i <= V.N;
    const bool useful = valid && lane >= H && lane < kStencilWave - H;
    const int64_t P = V.P, E = V.E;
    const int n0 = wt * seg, n1 = min(V.Nt + 1, n0 + seg);   // output levels [n0, n1)
    const int first = TR ? min(V.Nt, n1 - 1 + H) : max(0, n0 - H);
    const int count = TR ? first - n0 + 1 : n1 - first;

    T prev[S + 1];
#pragma unroll
    for (int k = 0; k <= S; ++k) prev[k] = T(0);
    T r_pair = T(0);   // TAIL 2: the residual of the level met first in a pair
    // coefficients of the current row class: J: (row n: dt = -1 at dx = -1, 0, 1, then
    // dt = 0); J^T: (row n at columns i-1, i, i+1, then row n+1 at i-1, i, i+1)
    T c[6] = {T(0), T(0), T(0), T(0), T(0), T(0)}, wd = T(0);
    int key = -1;
    // rows are loaded two levels ahead of use: the row classes (wave-uniform), u, b and
    // the coarse values of the head
    constexpr int NZ = HEAD == 1 ? 2 : (HEAD == 2 ? 1 : 0);
    T ru[2] = {T(0), T(0)}, rb[2] = {T(0), T(0)}, rz[2][NZ > 0 ? NZ : 1] = {};
    int rc[2] = {0, 0}, rc1[2] = {-1, -1};
    auto fetch = [&](int it, int slot) {
        ru[slot] = T(0);
        rb[slot] = T(0);
#pragma unroll
        for (int q = 0; q < NZ; ++q) rz[slot][q] = T(0);
        if (it >= count) return;
        const int n = TR ? first - it : first + it;
        rc[slot] = V.row[n];
        rc1[slot] = (TR && n < V.Nt) ? V.row[n + 1] : -1;
        if (!valid) return;
        const int64_t o = (int64_t)n * P + i;
        if (!zero_in) ru[slot] = u[o];
        rb[slot] = b[o];
        if (HEAD == 1) {
            const T* zr = z + (int64_t)n * Pz + (i >> 1);
            rz[slot][0] = zr[0];
            if (i & 1) rz[slot][NZ - 1] = zr[1];
        } else if (HEAD == 2) {
            rz[slot][0] = z[(int64_t)(n >> 1) * Pz + i];
        }
    };
    fetch(0, 0);
    fetch(1, 1);
    for (int it = 0; it < count; ++it) {
        const int n = TR ? first - it : first + it;
        const int slot = it & 1;
        T cur = ru[slot];
        const T bb = rb[slot];
        const int rn = rc[slot];
        const int rk = TR ? rc1[slot] : 0;
        if (HEAD == 1 && valid)   // the expressions of k_prolong_x
            cur = (i & 1) ? fmaT(T(0.5), rz[slot][0] + rz[slot][NZ - 1], cur)
                          : cur + rz[slot][0];
        else if (HEAD == 2 && valid)
            cur = cur + rz[slot][0];
        fetch(it + 2, slot);
        const int nk = rn * 64 + (rk + 1);
        if (nk != key) {   // wave-uniform: the row class changes only near the ends
            key = nk;
            const int64_t cr = (int64_t)rn * P;
            if (TR) {
                const int64_t nr = (int64_t)(rk < 0 ? 0 : rk) * P;
                const bool l = valid && i >= 1, r = valid && i + 1 <= V.N;
                c[0] = l ? V.s[5 * E + cr + i - 1] : T(0);
                c[1] = valid ? V.s[4 * E + cr + i] : T(0);
                c[2] = r ? V.s[3 * E + cr + i + 1] : T(0);
                c[3] = (l && rk >= 0) ? V.s[2 * E + nr + i - 1] : T(0);
                c[4] = (valid && rk >= 0) ? V.s[1 * E + nr + i] : T(0);
                c[5] = (r && rk >= 0) ? V.s[0 * E + nr + i + 1] : T(0);
            } else {
#pragma unroll
                for (int k = 0; k < 6; ++k) c[k] = valid ? V.s[k * E + cr + i] : T(0);
            }
            wd = valid ? V.s[9 * E + cr + i] : T(0);
        }
        const int64_t o = (int64_t)n * P + i;
#pragma unroll
        for (int k = 1; k <= S; ++k) {
            const T xm = shfl_up1(cur), xp = shfl_dn1(cur);
            const T pm = shfl_up1(prev[k - 1]), pp = shfl_dn1(prev[k - 1]);
            T acc = T(0);
            if (TR) {   // level n first, then level n + 1
                acc = fmaT(c[0], xm, acc);
                acc = fmaT(c[1], cur, acc);
                acc = fmaT(c[2], xp, acc);
                acc = fmaT(c[3], pm, acc);
                acc = fmaT(c[4], prev[k - 1], acc);
                acc = fmaT(c[5], pp, acc);
            } else {    // level n - 1 first, then level n
                acc = fmaT(c[0], pm, acc);
                acc = fmaT(c[1], prev[k - 1], acc);
                acc = fmaT(c[2], pp, acc);
                acc = fmaT(c[3], xm, acc);
                acc = fmaT(c[4], cur, acc);
                acc = fmaT(c[5], xp, acc);
            }
            // invalid lanes have wd = 0 and zero data: they stay 0
            const T y = fmaT(wd, bb - acc, cur);
            prev[k - 1] = cur;
            cur = y;
        }
        if (TAIL) {   // residual of y_S at this level, before prev[S] moves on
            const T xm = shfl_up1(cur), xp = shfl_dn1(cur);
            const T pm = shfl_up1(prev[S]), pp = shfl_dn1(prev[S]);
            T acc = T(0);
            if (TR) {
                acc = fmaT(c[0], xm, acc);
                acc = fmaT(c[1], cur, acc);
                acc = fmaT(c[2], xp, acc);
                acc = fmaT(c[3], pm, acc);
                acc = fmaT(c[4], prev[S], acc);
                acc = fmaT(c[5], pp, acc);
            } else {
                acc = fmaT(c[0], pm, acc);
                acc = fmaT(c[1], prev[S], acc);
                acc = fmaT(c[2], pp, acc);
                acc = fmaT(c[3], xm, acc);
                acc = fmaT(c[4], cur, acc);
                acc = fmaT(c[5], xp, acc);
            }
            const T res = bb - acc;
            const bool out_row = n >= n0 && n < n1;   // wave-uniform
            if (TAIL == 2) {
                if (out_row) {
                    // pairs (2J, 2J+1) -> J: 1/2 (r_2J + r_2J+1 [2J+1 <= Nt]); the
                    // transposed stream meets 2J+1 first
                    T* dst = bc + (int64_t)(n >> 1) * Pbc + i;
                    const bool odd = (n & 1) != 0;
                    if (!TR) {
                        if (odd) {
                            if (useful) *dst = T(0.5) * (r_pair + res);
                        } else if (n == V.Nt) {
                            if (useful) *dst = T(0.5) * res;
                        } else {
                            r_pair = res;
                        }
                    } else {
                        if (odd) {
                            r_pair = res;
                        } else if (n == V.Nt) {
                            if (useful) *dst = T(0.5) * res;
                        } else {
                            if (useful) *dst = T(0.5) * (res + r_pair);
                        }
                    }
                }
            } else if (TAIL == 3) {
                // coarse node I = i/2 for even i: r_2I + 1/2 (r_2I-1 [I >= 1] + r_2I+1 [I < Nc])
                const T rl = shfl_up1(res), rr = shfl_dn1(res);
                if (useful && out_row && (i & 1) == 0) {
                    const int I = i >> 1;
                    T side = T(0);
                    if (I >= 1) side += rl;
                    if (I < Nc) side += rr;
                    bc[(int64_t)n * Pbc + I] = fmaT(T(0.5), side, res);
                }
            }
        }
        prev[S] = cur;
        if (useful && n >= n0 && n < n1) out[o] = cur;
    }
}

// Thomas factors of the tridiagonal block of every stored row (nodes 0..N), for J
// (lo = array 3, up = array 5 of the row) and for J^T (lo_i = array 5 of row i - 1,
// up_i = array 3 of row i + 1): cp_i = up_i / den_i, inv_i = 1 / den_i with
// den_0 = di_0, den_i = di_i - lo_i cp_{i-1}.  One thread per stored row and matrix;
// factor arrays have the stencil's layout (row r at r P).
__global__ void k_stencil_thomas(StencilView S, double* __restrict__ f) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= 2 * S.R) return;
    const int tr = n >= S.R;
    const int m = tr ? n - S.R : n;
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

template <typename T, int TR, int S, int HEAD, int TAIL>
void launch_stencil_fused_s(const StencilViewT<T>& V, const StencilPass<T>& p, hipStream_t s) {
    constexpr int H = S + (TAIL ? 1 : 0) + (TAIL == 3 ? 1 : 0);
    const int U = kStencilWave - 2 * H;
    const int xw = (V.N + 1 + U - 1) / U;
    const int64_t rows = V.Nt + 1;
    // Short time segments: a wave's levels are a serial chain, so small levels need
    // many segments even though each recomputes H warm-up levels (the policy of the
    // rediscretised fused passes: fewer, longer segments when S >= 4 makes the pass
    // arithmetic-bound on large levels).
    const int64_t target = S >= 4 ? STMG_STENCIL_TARGET_WAVES_ALU : 16384;
    int64_t seg = (rows * xw + target - 1) / target;
    if (seg < 2) seg = 2;
    if (seg > 1024) seg = 1024;
    if (seg & 1) ++seg;
    const int nw = (int)(xw * ((rows + seg - 1) / seg));
    const int blocks = (nw + kStencilWavesPerBlock - 1) / kStencilWavesPerBlock;
    hipLaunchKernelGGL((k_stencil_fused<T, TR, S, HEAD, TAIL>), dim3(blocks),
                       dim3(kStencilWave * kStencilWavesPerBlock), 0, s, V, p.u, p.b, p.out,
                       (int)p.zero_in, p.z, p.Pz, p.bc, p.Pbc, p.Nc, xw, (int)seg, nw);
}

template <typename T, int TR, int S>
void launch_stencil_fused_ht(const StencilViewT<T>& V, const StencilPass<T>& p, hipStream_t s) {
    if (p.restrict_dir == 't') launch_stencil_fused_s<T, TR, S, 0, 2>(V, p, s);
    else if (p.restrict_dir == 'x') launch_stencil_fused_s<T, TR, S, 0, 3>(V, p, s);
    else if (p.head == 'x') launch_stencil_fused_s<T, TR, S, 1, 0>(V, p, s);
    else if (p.head == 't') launch_stencil_fused_s<T, TR, S, 2, 0>(V, p, s);
    else launch_stencil_fused_s<T, TR, S, 0, 0>(V, p, s);
}

template <typename T, int TR>
void launch_stencil_fused_t(const StencilViewT<T>& V, const StencilPass<T>& p, hipStream_t s) {
    switch (p.sweeps) {
        case 1: launch_stencil_fused_ht<T, TR, 1>(V, p, s); break;
        case 2: launch_stencil_fused_ht<T, TR, 2>(V, p, s); break;
        case 3: launch_stencil_fused_ht<T, TR, 3>(V, p, s); break;
        case 4: launch_stencil_fused_ht<T, TR, 4>(V, p, s); break;
        case 5: launch_stencil_fused_ht<T, TR, 5>(V, p, s); break;
        default: launch_stencil_fused_ht<T, TR, 6>(V, p, s); break;
    }
}

template <typename T>
int launch_stencil_fused(const StencilViewT<T>& V, const StencilPass<T>& p, hipStream_t s) {
    if (p.sweeps < 1 || p.sweeps > kStencilMaxFused || (p.restrict_dir && p.head)) return -1;
    if (p.restrict_dir && p.restrict_dir != 'x' && p.restrict_dir != 't') return -1;
    if (p.trans) launch_stencil_fused_t<T, 1>(V, p, s);
    else launch_stencil_fused_t<T, 0>(V, p, s);
    return 0;
}

void launch_stencil_thomas(const StencilView& S, double* factors, hipStream_t s) {
    hipLaunchKernelGGL(k_stencil_thomas, dim3(blocks_for(2 * (int64_t)S.R)), dim3(kBlock), 0, s,
                       S, factors);
}

// Exact solve on a stencil level whose rows couple only to their own and the previous
// time level (J; for J^T: the next one, stepping backwards).  One workgroup, one node
// per thread: the right-hand side of a time level is formed in parallel from the
// previous level's solution in LDS (the next level's b is already loading), then
// thread 0 runs the Thomas recurrence from LDS.  The arithmetic is FP64 whatever the
// vector type TV of b and z.
constexpr int kStencilSolveThreads = kStencilCoarsestMaxNodes;   // one node per thread
template <typename TV>
__global__ __launch_bounds__(kStencilSolveThreads) void k_stencil_coarsest(
    StencilView S, const double* __restrict__ f, int trans, const TV* __restrict__ b,
    TV* __restrict__ z) {
    // solutions of the current and the previous time level, and the Thomas factors
    // of the current row class
    __shared__ double xs[2][kStencilCoarsestMaxNodes];
    __shared__ double lo[kStencilCoarsestMaxNodes];
    __shared__ double cp[kStencilCoarsestMaxNodes];
    __shared__ double inv[kStencilCoarsestMaxNodes];
    const int i = threadIdx.x;
    const bool act = i <= S.N;
    const int64_t E = S.E, P = S.P;
    const double* fcp = f + (trans ? 2 : 0) * E;
    const double* finv = f + (trans ? 3 : 1) * E;
    // coupling of node i to the previous (J) or next (J^T) level at columns i-1, i, i+1
    double c0 = 0.0, c1 = 0.0, c2 = 0.0;
    int key = -1;
    double bnext = act ? (double)b[(int64_t)(trans ? S.Nt : 0) * P + i] : 0.0;
    // row classes of the next time level, read one step ahead
    auto classes = [&](int step, int& rn, int& rk) {
        const int n = trans ? S.Nt - step : step;
        rn = S.row[n];
        rk = trans ? (n < S.Nt ? S.row[n + 1] : -1) : rn;
    };
    int rn_next, rk_next;
    classes(0, rn_next, rk_next);
    for (int step = 0; step <= S.Nt; ++step) {
        const int n = trans ? S.Nt - step : step;
        const int cur = step & 1, prv = cur ^ 1;
        const int rn = rn_next, rk = rk_next;
        if (step < S.Nt) classes(step + 1, rn_next, rk_next);
        const int nk = rn * 64 + (rk + 1);
        if (nk != key) {   // wave-uniform: the row class changes only near the ends
            key = nk;
            if (act) {
                const int64_t cr = (int64_t)rn * P;
                lo[i] = i == 0 ? 0.0 : (trans ? S.s[5 * E + cr + i - 1] : S.s[3 * E + cr + i]);
                cp[i] = fcp[cr + i];
                inv[i] = finv[cr + i];
                if (trans) {
                    const int64_t nr = (int64_t)(rk < 0 ? 0 : rk) * P;
                    c0 = (rk >= 0 && i >= 1) ? S.s[2 * E + nr + i - 1] : 0.0;
                    c1 = rk >= 0 ? S.s[1 * E + nr + i] : 0.0;
                    c2 = (rk >= 0 && i + 1 <= S.N) ? S.s[0 * E + nr + i + 1] : 0.0;
                } else {
                    c0 = S.s[0 * E + cr + i];
                    c1 = S.s[1 * E + cr + i];
                    c2 = S.s[2 * E + cr + i];
                }
            }
            __syncthreads();
        }
        if (act) {
            double v = bnext;
            if (trans ? n < S.Nt : n >= 1) {   // terms in the order dx = -1, 0, 1
                if (i >= 1) v -= c0 * xs[prv][i - 1];
                v -= c1 * xs[prv][i];
                if (i + 1 <= S.N) v -= c2 * xs[prv][i + 1];
            }
            xs[cur][i] = v;
            if (step < S.Nt) bnext = (double)b[(int64_t)(trans ? n - 1 : n + 1) * P + i];
        }
        __syncthreads();
        if (i == 0) {
            double* x = xs[cur];
            double d = 0.0;
            for (int k = 0; k <= S.N; ++k) {
                d = (x[k] - lo[k] * d) * inv[k];
                x[k] = d;
            }
            double y = 0.0;
            for (int k = S.N; k >= 0; --k) {
                y = x[k] - cp[k] * y;
                x[k] = y;
            }
        }
        __syncthreads();
        if (act) z[(int64_t)n * P + i] = (TV)xs[cur][i];
    }
}

template <typename TV>
void launch_stencil_coarsest(const StencilView& S, const double* factors, int trans, const TV* b,
                             TV* z, hipStream_t s) {
    hipLaunchKernelGGL(k_stencil_coarsest<TV>, dim3(1), dim3(kStencilSolveThreads), 0, s, S, factors,
                       trans, b, z);
}

// Inverse of the tridiagonal block of every stored row (the couplings of a time level to
// itself), one thread per stored row and column j: the Thomas solve of J's block with the
// right-hand side e_j, written as column j of the row-major inverse.
__global__ void k_stencil_block_inverse(StencilView S, const double* __restrict__ f,
                                        double* __restrict__ inv) {
    const int W = S.N + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S.R * W) return;
    const int r = t / W, j = t - r * W;
    const int64_t E = S.E, row = (int64_t)r * S.P;
    const double* cp = f + row;
    const double* iv = f + E + row;
    const double* s3 = S.s + 3 * E + row;
    double* A = inv + (int64_t)r * W * W;
    double d = 0.0;
    for (int k = 0; k <= S.N; ++k) {
        const double lo = k == 0 ? 0.0 : s3[k];
        d = ((k == j ? 1.0 : 0.0) - lo * d) * iv[k];
        A[(int64_t)k * W + j] = d;
    }
    double y = 0.0;
    for (int k = S.N; k >= 0; --k) {
        y = A[(int64_t)k * W + j] - cp[k] * y;
        A[(int64_t)k * W + j] = y;
    }
}

void launch_stencil_block_inverse(const StencilView& S, const double* factors, double* inv,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_stencil_block_inverse, dim3(blocks_for((int64_t)S.R * (S.N + 1))),
                       dim3(kBlock), 0, s, S, factors, inv);
}

// The time-stepping solve of k_stencil_coarsest in one wave, node i in lane i: the
// right-hand side of a time level (the same expression as there, the previous level's
// solution taken from the neighbour lanes) is multiplied by the inverse of the level's
// block (its transpose for J^T), held in registers, with the right-hand side broadcast
// from LDS.  The inverse is zero beyond N and lanes without a node carry a zero
// right-hand side, so the product runs over NMAX terms without a branch per term.
template <typename TV, int NMAX>
__global__ __launch_bounds__(64) void k_stencil_coarsest_dense(StencilView S,
                                                               const double* __restrict__ ainv,
                                                               int trans,
                                                               const TV* __restrict__ b,
                                                               TV* __restrict__ z) {
    __shared__ double rs[2][64];
    __shared__ double bs[64][64];   // [time level within the chunk][lane]
    const int i = threadIdx.x;
    const int W = S.N + 1;
    const bool act = i <= S.N;
    const int64_t E = S.E, P = S.P;
    double a[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) a[j] = 0.0;
    double c0 = 0.0, c1 = 0.0, c2 = 0.0;
    int key = -1;
    double zprev = 0.0;
    // Every 64 time levels, one round trip to memory fetches what the next 64 steps read:
    // each lane's right-hand side column into LDS (only the lane itself reads it back),
    // and the row classes, one per lane, picked with readlane.  No step then waits on
    // memory.  J^T couples level n to n + 1, the previous step's.
    int chunk = 0, rprev = -1;
    for (int step = 0; step <= S.Nt; ++step) {
        const int n = trans ? S.Nt - step : step;
        if ((step & 63) == 0) {
            const int st = step + i;
            chunk = st <= S.Nt ? S.row[trans ? S.Nt - st : st] : 0;
#pragma unroll
            for (int k0 = 0; k0 < 64; k0 += 16) {
                double t[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int sk = step + k0 + k;
                    t[k] = (act && sk <= S.Nt) ? (double)b[(int64_t)(trans ? S.Nt - sk : sk) * P + i]
                                               : 0.0;
                }
#pragma unroll
                for (int k = 0; k < 16; ++k) bs[k0 + k][i] = t[k];
            }
        }
        const int rn = __builtin_amdgcn_readlane(chunk, step & 63);
        const int rk = trans ? rprev : rn;
        rprev = rn;
        const int nk = rn * 64 + (rk + 1);
        if (nk != key) {   // wave-uniform: the row class changes only near the ends
            key = nk;
            const double* A = ainv + (int64_t)rn * W * W;
#pragma unroll
            for (int j = 0; j < NMAX; ++j)
                a[j] = (act && j < W) ? (trans ? A[(int64_t)j * W + i] : A[(int64_t)i * W + j]) : 0.0;
            if (act) {
                const int64_t cr = (int64_t)rn * P;
                if (trans) {
                    const int64_t nr = (int64_t)(rk < 0 ? 0 : rk) * P;
                    c0 = (rk >= 0 && i >= 1) ? S.s[2 * E + nr + i - 1] : 0.0;
                    c1 = rk >= 0 ? S.s[1 * E + nr + i] : 0.0;
                    c2 = (rk >= 0 && i + 1 <= S.N) ? S.s[0 * E + nr + i + 1] : 0.0;
                } else {
                    c0 = S.s[0 * E + cr + i];
                    c1 = S.s[1 * E + cr + i];
                    c2 = S.s[2 * E + cr + i];
                }
            }
        }
        double v = bs[step & 63][i];
        // the previous level's solution at i-1, i+1 (0 beyond the nodes)
        const double zl = shfl_up1(zprev), zr = shfl_dn1(zprev);
        if (trans ? n < S.Nt : n >= 1) {   // terms in the order dx = -1, 0, 1
            v -= c0 * zl;
            v -= c1 * zprev;
            v -= c2 * zr;
        }
        if (!act) v = 0.0;
        // broadcast through LDS (one wave: its LDS accesses complete in order; two buffers
        // keep the next level's writes clear of this level's reads); lane-by-lane reads
        // into scalar registers would need 2 NMAX of them
        double* rv = rs[step & 1];
        rv[i] = v;
        __builtin_amdgcn_wave_barrier();
        double y = 0.0;
#pragma unroll
        for (int j = 0; j < NMAX; ++j) y = __builtin_fma(a[j], rv[j], y);
        __builtin_amdgcn_wave_barrier();
        if (act) z[(int64_t)n * P + i] = (TV)y;
        zprev = act ? y : 0.0;
    }
}

template <typename TV>
void launch_stencil_coarsest_dense(const StencilView& S, const double* inv, int trans,
                                   const TV* b, TV* z, hipStream_t s) {
    const int W = S.N + 1;
    if (W <= 16)
        hipLaunchKernelGGL((k_stencil_coarsest_dense<TV, 16>), dim3(1), dim3(64), 0, s, S, inv,
                           trans, b, z);
    else if (W <= 32)
        hipLaunchKernelGGL((k_stencil_coarsest_dense<TV, 32>), dim3(1), dim3(64), 0, s, S, inv,
                           trans, b, z);
    else if (W <= 48)
        hipLaunchKernelGGL((k_stencil_coarsest_dense<TV, 48>), dim3(1), dim3(64), 0, s, S, inv,
                           trans, b, z);
    else
        hipLaunchKernelGGL((k_stencil_coarsest_dense<TV, 64>), dim3(1), dim3(64), 0, s, S, inv,
                           trans, b, z);
}

// ---- exact solve of a level whose rows also couple to the next time level ------------
// (bilinear interpolation with Galerkin operators).  The operator is assembled as a
// dense n x n matrix, n = (N+1)(Nt+1), DOF (t, i) at index t (N+1) + i, and factored by
// LU with partial pivoting.  Its bandwidth is N + 2 each side, so with row pivoting L
// keeps that band and U at most twice it: the factorization and the solves only touch
// those bands.

// row r of J (trans = 0) or J^T (trans = 1); A zeroed before
__global__ void k_stencil_dense(StencilView S, int trans, double* __restrict__ A) {
    const int W = S.N + 1;
    const int64_t n = (int64_t)W * (S.Nt + 1);
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int t = (int)(r / W), i = (int)(r % W);
    for (int k = 0; k < 9; ++k) {
        const int tt = t + k / 3 - 1, ii = i + k % 3 - 1;
        if (tt < 0 || tt > S.Nt || ii < 0 || ii > S.N) continue;
        const double c = trans ? S.s[(8 - k) * S.E + (int64_t)S.row[tt] * S.P + ii]
                               : S.s[k * S.E + (int64_t)S.row[t] * S.P + i];
        A[r * n + (int64_t)tt * W + ii] = c;
    }
}

constexpr int kLuThreads = 1024;

// column k: pivot row p = argmax_{k <= r <= k + bl} |A[r][k]| (the first on ties), swap
// rows k and p over the columns [k, k + bl + bu], then the multipliers A[r][k] /= A[k][k]
__global__ __launch_bounds__(kLuThreads) void k_lu_pivot(double* __restrict__ A, int n, int k, int bl,
                                                      int bu, int* __restrict__ piv) {
    __shared__ double sv[kLuThreads / 64];
    __shared__ int si[kLuThreads / 64];
    __shared__ int sp;
    const int rend = min(n - 1, k + bl);
    double best = -1.0;
    int bi = k;
    for (int r = k + threadIdx.x; r <= rend; r += kLuThreads) {
        const double v = fabs(A[(int64_t)r * n + k]);
        if (v > best) { best = v; bi = r; }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if ((threadIdx.x & 63) == 0) { sv[threadIdx.x >> 6] = best; si[threadIdx.x >> 6] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = sv[0];
        int p = si[0];
        for (int w = 1; w < kLuThreads / 64; ++w)
            if (sv[w] > b || (sv[w] == b && si[w] < p)) { b = sv[w]; p = si[w]; }
        sp = p;
        piv[k] = p;
    }
    __syncthreads();
    const int p = sp;
    const int cend = min(n - 1, k + bl + bu);
    if (p != k) {
        for (int c = k + threadIdx.x; c <= cend; c += kLuThreads) {
            const double a = A[(int64_t)k * n + c];
            A[(int64_t)k * n + c] = A[(int64_t)p * n + c];
            A[(int64_t)p * n + c] = a;
        }
    }
    __syncthreads();
    const double d = A[(int64_t)k * n + k];
    for (int r = k + 1 + threadIdx.x; r <= rend; r += kLuThreads) A[(int64_t)r * n + k] /= d;
}

// trailing update A[r][c] -= A[r][k] A[k][c], k < r <= k + bl, k < c <= k + bl + bu
__global__ void k_lu_update(double* __restrict__ A, int n, int k, int bl, int bu) {
    const int c = k + 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int r = k + 1 + blockIdx.y;
    if (c > min(n - 1, k + bl + bu) || r > min(n - 1, k + bl)) return;
    A[(int64_t)r * n + c] -= A[(int64_t)r * n + k] * A[(int64_t)k * n + c];
}

void launch_stencil_lu(const StencilView& S, int trans, double* A, int* piv, hipStream_t s) {
    const int W = S.N + 1;
    const int n = W * (S.Nt + 1);
    const int b = S.N + 2;   // bandwidth of the 9-point operator in this ordering
    launch_fill<double>(A, (int64_t)n * n, 0.0, s);
    hipLaunchKernelGGL(k_stencil_dense, dim3(blocks_for(n)), dim3(kBlock), 0, s, S, trans, A);
    for (int k = 0; k < n; ++k) {
        hipLaunchKernelGGL(k_lu_pivot, dim3(1), dim3(kLuThreads), 0, s, A, n, k, b, b, piv);
        const int rows = min(n - 1, k + b) - k, cols = min(n - 1, k + 2 * b) - k;
        if (rows > 0 && cols > 0)
            hipLaunchKernelGGL(k_lu_update, dim3(blocks_for(cols), rows), dim3(kBlock), 0, s, A,
                               n, k, b, b);
    }
}

// z = A^-1 b from the factors: L (unit, band b, with the interchanges) forward and U
// (band 2b) backward, one workgroup; x: n doubles of scratch in global memory.  FP64
// arithmetic whatever the vector type TV of b and z.
template <typename TV>
__global__ __launch_bounds__(kLuThreads) void k_lu_solve(StencilView S, const double* __restrict__ A,
                                                      const int* __restrict__ piv,
                                                      const TV* __restrict__ bv,
                                                      TV* __restrict__ z, double* x) {
    const int W = S.N + 1;
    const int n = W * (S.Nt + 1);
    const int b = S.N + 2;
    for (int r = threadIdx.x; r < n; r += kLuThreads)
        x[r] = (double)bv[(int64_t)(r / W) * S.P + r % W];
    __syncthreads();
    // the factorization swapped rows from the pivot column on only (earlier multipliers
    // stay in place), so each interchange is applied just before its elimination step
    for (int k = 0; k < n; ++k) {
        if (threadIdx.x == 0) {
            const int p = piv[k];
            if (p != k) { const double a = x[k]; x[k] = x[p]; x[p] = a; }
        }
        __syncthreads();
        const double xk = x[k];
        const int rend = min(n - 1, k + b);
        for (int r = k + 1 + threadIdx.x; r <= rend; r += kLuThreads)
            x[r] -= A[(int64_t)r * n + k] * xk;
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        const double xk = x[k] / A[(int64_t)k * n + k];
        const int r0 = max(0, k - 2 * b);
        __syncthreads();
        for (int r = r0 + threadIdx.x; r < k; r += kLuThreads) x[r] -= A[(int64_t)r * n + k] * xk;
        if (threadIdx.x == 0) x[k] = xk;
        __syncthreads();
    }
    for (int r = threadIdx.x; r < n; r += kLuThreads) z[(int64_t)(r / W) * S.P + r % W] = (TV)x[r];
}

template <typename TV>
void launch_stencil_lu_solve(const StencilView& S, const double* A, const int* piv, const TV* b,
                             TV* z, double* scratch, hipStream_t s) {
    hipLaunchKernelGGL(k_lu_solve<TV>, dim3(1), dim3(kLuThreads), 0, s, S, A, piv, b, z, scratch);
}

template void launch_apply_stencil<double>(const StencilViewT<double>&, int, int, const double*,
                                           const double*, double*, bool, hipStream_t);
template void launch_apply_stencil<float>(const StencilViewT<float>&, int, int, const float*,
                                          const float*, float*, bool, hipStream_t);
template int launch_stencil_fused<double>(const StencilViewT<double>&, const StencilPass<double>&,
                                          hipStream_t);
template int launch_stencil_fused<float>(const StencilViewT<float>&, const StencilPass<float>&,
                                         hipStream_t);
template void launch_stencil_coarsest<double>(const StencilView&, const double*, int,
                                              const double*, double*, hipStream_t);
template void launch_stencil_coarsest<float>(const StencilView&, const double*, int, const float*,
                                             float*, hipStream_t);
template void launch_stencil_coarsest_dense<double>(const StencilView&, const double*, int,
                                                    const double*, double*, hipStream_t);
template void launch_stencil_coarsest_dense<float>(const StencilView&, const double*, int,
                                                   const float*, float*, hipStream_t);
template void launch_stencil_lu_solve<double>(const StencilView&, const double*, const int*,
                                              const double*, double*, double*, hipStream_t);
template void launch_stencil_lu_solve<float>(const StencilView&, const double*, const int*,
                                             const float*, float*, double*, hipStream_t);

}  // namespace stmg
