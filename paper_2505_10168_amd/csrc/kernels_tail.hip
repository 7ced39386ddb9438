// Single-workgroup V-cycle over the smallest levels of the hierarchy (gfx950).
//
// On levels of a few thousand DOFs a fused streaming launch is bound by latency
// (dispatch, first loads, the serial chain of rows inside one wave), not by its work:
// every such level costs about the same ~10 us per pass however small it is.  This
// kernel runs the whole lower part of Algorithm 1 from a level l_s down — on every
// level nu damped Jacobi steps from a zero start, the residual and its restriction
// R = s P^T (Section 3.1); the exact solve on the coarsest level; then the
// prolongation P and nu post-smoothing steps on the way back up — in ONE workgroup of
// 1024 threads.  The u and b vectors of all these levels stay in LDS; the steps are
// separated by workgroup barriers.  Only b of level l_s is read from HBM and only its
// u is written back.
//
// Each thread owns a block of consecutive time rows of one node column of the level
// it works on: the stencil coefficients, the owned b and the owned iterate stay in
// registers, and a Jacobi step only reads the two neighbour columns and one coupled
// row from LDS.  It computes the new values of all owned DOFs, then (after a
// barrier) publishes them to LDS for the neighbours.  A level's LDS footprint is its
// u and b.
//
// Every value is formed with the operands and the operation order of the reference
// kernels (k_apply, k_restrict_x/t, k_prolong_x/t, k_coarsest_dense), so this kernel
// gives bit-identical results to a V-cycle built from those.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "stmg_launch.hpp"

namespace stmg {

namespace {

template <typename T>
struct TailArgs {
    LevelView<T> V[kTailMaxLevels];   // levels l_s .. coarsest (index 0 = l_s)
    int off_u[kTailMaxLevels];        // LDS offsets (elements of T), row pitch N+1
    int off_b[kTailMaxLevels];
    int dir[kTailMaxLevels];          // 'x' / 't' towards the next level
    int nlev;
    int nu;
    int lds_elems;
    LevelView<double> Vc;             // coarsest level with its FP64 coefficients
    const double* ainv;               // coarsest A^{-1}, row-major N x N
    const T* b_in;                    // b of level l_s in HBM, pitch P_in
    int64_t P_in;
    T* u_out;                         // u of level l_s in HBM, pitch P_out
    int64_t P_out;
};

// Ownership on a level with W = N+1 node columns and Nt+1 time levels: thread t
// owns column i = t % W and the M consecutive rows n0 = (t / W) M .. n0 + M - 1, where
// R = 1024 / W groups of W threads share the rows and M = ceil((Nt+1) / R) rounded
// up to even (a time pair 2J, 2J+1 of the t restriction stays in one thread).
struct Owner {
    int i, n0, M;
    bool act;
};
// M: rows per thread; even when the level restricts in t, so that a time pair
// (2J, 2J+1) stays with one thread.
__device__ __forceinline__ int rows_per_owner(int W, int Nt, bool even) {
    const int R = kTailThreads / W;
    const int M = (Nt + 1 + R - 1) / R;
    return even ? M + (M & 1) : M;
}
__device__ __forceinline__ Owner owner_of(int W, int Nt, bool even) {
    Owner o;
    o.M = rows_per_owner(W, Nt, even);
    o.i = threadIdx.x % W;
    const int g = threadIdx.x / W;
    o.n0 = g * o.M;
    o.act = g < kTailThreads / W && o.n0 <= Nt;
    return o;
}
// Time level of owned row k.  For J the rows run forward from n0; for J^T backward from
// n0 + M - 1.  Either way the row row k is coupled to is owned row k - 1, and for k = 0
// the row outside the block.
template <int TR>
__device__ __forceinline__ int row_of(const Owner& o, int k) {
    return TR ? o.n0 + o.M - 1 - k : o.n0 + k;
}

template <typename T>
struct ColCoef {
    T mlo, mdi, mup, kl, kr, wd;
    T nm;   // multiplier of the left neighbour: 0 at nodes 0 and 1, -1 elsewhere
};
template <typename T>
__device__ __forceinline__ ColCoef<T> col_coef(const LevelView<T>& V, int i) {
    ColCoef<T> c;
    c.mlo = V.mlo[i];
    c.mdi = V.mdi[i];
    c.mup = V.mup[i];
    c.kl = V.kl[i];
    c.kr = V.kr[i];
    c.wd = V.wd[i];
    c.nm = i <= 1 ? T(0) : T(-1);
    return c;
}

// One damped Jacobi step (JAC) or the residual r = b - J x (!JAC) of the owned DOFs,
// in place in x.  bb: the owned b; u: the level's current iterate in LDS (row pitch
// W), which holds the same values as x for the owned DOFs.  Neighbour columns are
// loaded unconditionally (clamped into range) and need no boundary selects: node 1
// drops its eliminated left neighbour through nm, node N has zero right coefficients,
// and node 0 (Dirichlet) is expressed through its coefficients (kl = W_Diri,
// wd = omega / W_Diri, the rest 0, nm = 0), exactly as the fused kernels do.  An
// uncoupled row forms its differences as fma(0, y, x) = x.  Each rounded operation
// has the operands k_apply gives it.  Rows are visited from k = M-1 down to 0, so the
// coupled row k-1 is still at its old value when read.  Rows beyond Nt produce values
// that are never stored.  MM = o.M, the rows per thread of the level (uniform), as a
// constant: the row loops then run without a test per row.
template <int TR, int MM>
__device__ __forceinline__ int row_m(const Owner& o, int k) {
    return TR ? o.n0 + MM - 1 - k : o.n0 + k;
}
template <typename T, int TR, bool JAC, int MM>
__device__ __forceinline__ void owned_step(const LevelView<T>& V, const ColCoef<T>& c,
                                           const Owner& o, const T* u, T (&x)[kTailMaxRows],
                                           const T (&bb)[kTailMaxRows]) {
    const int N = V.N, Nt = V.Nt, W = N + 1, i = o.i;
    const int im = i > 0 ? i - 1 : 0, ip = i < N ? i + 1 : N;
    T XM[MM], XP[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        const int n = min(row_m<TR, MM>(o, k), Nt);
        XM[k] = u[n * W + im];
        XP[k] = u[n * W + ip];
    }
    const int e = min(max(TR ? o.n0 + MM : o.n0 - 1, 0), Nt);   // coupled row outside the block
    const T EM = u[e * W + im], E0 = u[e * W + i], EP = u[e * W + ip];
#pragma unroll
    for (int kk = 0; kk < MM; ++kk) {
        const int k = MM - 1 - kk;
        {
            const int n = row_m<TR, MM>(o, k);
            const T negc = (TR ? (n < Nt) : (n >= 2)) ? T(-1) : T(0);
            const T cm = k == 0 ? EM : XM[k > 0 ? k - 1 : 0];
            const T c0 = k == 0 ? E0 : x[k > 0 ? k - 1 : 0];
            const T cp = k == 0 ? EP : XP[k > 0 ? k - 1 : 0];
            const T dm = fmaT(negc, cm, XM[k]);
            const T d0 = fmaT(negc, c0, x[k]);
            const T dp = fmaT(negc, cp, XP[k]);
            T s = c.mdi * d0;
            s = fmaT(c.mlo, dm, s);
            s = fmaT(c.mup, dp, s);
            s = fmaT(c.kl, fmaT(c.nm, XM[k], x[k]), s);
            s = fmaT(c.kr, x[k] - XP[k], s);
            const bool dir_row = n == 0;
            const T r = bb[k] - (dir_row ? V.W * x[k] : s);
            x[k] = JAC ? jacobi_update<T>(x[k], dir_row ? V.wW : c.wd, r) : r;
        }
    }
}

// Calls f(std::integral_constant<int, M>) for the uniform rows per thread M, 1 <= M <= MX.
template <int MX, typename F>
__device__ __forceinline__ void with_rows(int M, F&& f) {
    if constexpr (MX <= 1) {
        f(std::integral_constant<int, 1>{});
    } else {
        if (M == MX) f(std::integral_constant<int, MX>{});
        else with_rows<MX - 1>(M, f);
    }
}

// One Jacobi step or the residual, with the level's rows per thread as a constant.
template <typename T, int TR, bool JAC>
__device__ __forceinline__ void owned_step_any(const LevelView<T>& V, const ColCoef<T>& c,
                                               const Owner& o, const T* u,
                                               T (&x)[kTailMaxRows],
                                               const T (&bb)[kTailMaxRows]) {
    with_rows<kTailMaxRows>(o.M, [&](auto mm) {
        owned_step<T, TR, JAC, decltype(mm)::value>(V, c, o, u, x, bb);
    });
}

// nu damped Jacobi steps; x holds the owned values before and after, u (LDS) too.
template <typename T, int TR>
__device__ void tail_smooth(const LevelView<T>& V, const ColCoef<T>& c, const Owner& o, T* u,
                            T (&x)[kTailMaxRows], const T (&bb)[kTailMaxRows], int nu) {
    const int W = V.N + 1;
    with_rows<kTailMaxRows>(o.M, [&](auto mm) {
        constexpr int MM = decltype(mm)::value;
        for (int s = 0; s < nu; ++s) {
            owned_step<T, TR, true, MM>(V, c, o, u, x, bb);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < MM; ++k) {
                const int n = row_m<TR, MM>(o, k);
                if (o.act && n <= V.Nt) u[n * W + o.i] = x[k];
            }
            __syncthreads();
        }
    });
}

// Owned rows of u and b from LDS into registers (zero where not owned).
template <typename T, int TR>
__device__ __forceinline__ void load_owned(const Owner& o, int W, int Nt, const T* v,
                                           T (&x)[kTailMaxRows]) {
#pragma unroll
    for (int k = 0; k < kTailMaxRows; ++k) {
        const int n = row_of<TR>(o, k);
        x[k] = (k < o.M && o.act && n <= Nt) ? v[n * W + o.i] : T(0);
    }
}

// Pre-smoothing from zero, then bc = R (b - J u) into the next level's b (x: s = 1,
// t: s = 1/2).  The x restriction stages the fine residual in the next level's u and
// b area (together at least as large as one fine vector) and clears its u after.
template <typename T, int TR>
__device__ void tail_down(const LevelView<T>& F, T* u, const T* b, int dir, T* uc, T* bc,
                          int nu) {
    const int W = F.N + 1, Nt = F.Nt;
    const Owner o = owner_of(W, Nt, dir == 't');
    ColCoef<T> c{};
    if (o.act) c = col_coef(F, o.i);
    T x[kTailMaxRows], bb[kTailMaxRows];
    load_owned<T, TR>(o, W, Nt, b, bb);
#pragma unroll
    for (int k = 0; k < kTailMaxRows; ++k) x[k] = T(0);
    tail_smooth<T, TR>(F, c, o, u, x, bb, nu);
    T (&r)[kTailMaxRows] = x;
    owned_step_any<T, TR, false>(F, c, o, u, r, bb);
    if (dir == 't') {
        // pairs (2J, 2J+1) of one owner: bc_J = 1/2 (r_2J + r_2J+1 [2J+1 <= Nt]); time
        // level 2J is owned row k = 2m (J) or 2m+1 (J^T), 2J+1 the row next to it
#pragma unroll
        for (int k = TR ? 1 : 0; k < kTailMaxRows; k += 2) {
            const int n = row_of<TR>(o, k);
            const int k1 = TR ? k - 1 : (k + 1 < kTailMaxRows ? k + 1 : k);
            if (k < o.M && o.act && n <= Nt) {
                T v = r[k];
                if (n + 1 <= Nt) v += r[k1];
                bc[(n >> 1) * W + o.i] = T(0.5) * v;
            }
        }
        __syncthreads();
        return;
    }
    // x: stage r (pitch W) over uc/bc, then bc_I = r_2I + 1/2 (r_2I-1 [I>=1] + r_2I+1 [I<Nc])
    T* rs = uc;
#pragma unroll
    for (int k = 0; k < kTailMaxRows; ++k) {
        const int n = row_of<TR>(o, k);
        if (k < o.M && o.act && n <= Nt) rs[n * W + o.i] = r[k];
    }
    __syncthreads();
    const int Nc = F.N / 2, Wc = Nc + 1;
    const Owner q = owner_of(Wc, Nt, false);
    const int I = q.i;
    T v[kTailMaxRows];
#pragma unroll
    for (int k = 0; k < kTailMaxRows; ++k) {
        const int n = q.n0 + k;
        v[k] = T(0);
        if (k < q.M && q.act && n <= Nt) {
            const T* row = rs + n * W;
            T side = T(0);
            if (I >= 1) side += row[2 * I - 1];
            if (I < Nc) side += row[2 * I + 1];
            v[k] = fmaT(T(0.5), side, row[2 * I]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTailMaxRows; ++k) {
        const int n = q.n0 + k;
        if (k < q.M && q.act && n <= Nt) {
            bc[n * Wc + I] = v[k];
            uc[n * Wc + I] = T(0);
        }
    }
    __syncthreads();
}

// u += P z (causal interpolation C of Section 3.1), then nu post-smoothing steps.
template <typename T, int TR>
__device__ void tail_up(const LevelView<T>& F, T* u, const T* b, int dir, const T* z, int nu) {
    const int W = F.N + 1, Nt = F.Nt;
    const Owner o = owner_of(W, Nt, dir == 't');
    ColCoef<T> c{};
    if (o.act) c = col_coef(F, o.i);
    T x[kTailMaxRows], bb[kTailMaxRows];
    load_owned<T, TR>(o, W, Nt, u, x);
    load_owned<T, TR>(o, W, Nt, b, bb);
    const int f = o.i;
#pragma unroll
    for (int k = 0; k < kTailMaxRows; ++k) {
        const int n = row_of<TR>(o, k);
        if (k < o.M && o.act && n <= Nt) {
            if (dir == 'x') {
                const T* zr = z + n * (F.N / 2 + 1);
                if (f & 1)
                    x[k] = fmaT(T(0.5), zr[f >> 1] + zr[(f >> 1) + 1], x[k]);
                else
                    x[k] += zr[f >> 1];
            } else {
                x[k] += z[(n >> 1) * W + f];
            }
            u[n * W + f] = x[k];
        }
    }
    __syncthreads();
    tail_smooth<T, TR>(F, c, o, u, x, bb, nu);
}

// Exact coarsest solve (Algorithm 1, first branch) with the precomputed A^{-1}: the
// Dirichlet DOFs take b / W_Diri, then wave 0 steps through time, lane i holding row
// i+1 of A^{-1} and the right-hand side broadcast lane by lane.
template <typename T, int TR, int NMAX>
__device__ void tail_coarsest(const LevelView<double>& L, const double* ainv, const T* b, T* u) {
    const int N = L.N, Nt = L.Nt, W = N + 1;
    for (int i = threadIdx.x; i <= N; i += kTailThreads) u[i] = (T)((double)b[i] / L.W);
    for (int n = 1 + (int)threadIdx.x; n <= Nt; n += kTailThreads)
        u[n * W] = (T)((double)b[n * W] / L.W);
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int node = lane + 1;
        const bool act = node <= N;
        double a[NMAX];
#pragma unroll
        for (int j = 0; j < NMAX; ++j) a[j] = (act && j < N) ? ainv[(int64_t)lane * N + j] : 0.0;
        const double mlo = act ? L.mlo[node] : 0.0;
        const double mdi = act ? L.mdi[node] : 0.0;
        const double mup = act ? L.mup[node] : 0.0;
        double zprev = 0.0;
        // the right-hand side of the next step is read one step ahead
        double bn = (act && Nt > 0) ? (double)b[(TR ? Nt : 1) * W + node] : 0.0;
        for (int s = 0; s < Nt; ++s) {
            const int n = TR ? Nt - s : 1 + s;
            const bool coupled = TR ? (n < Nt) : (n >= 2);
            double rhs = bn;
            if (s + 1 < Nt) bn = act ? (double)b[(TR ? n - 1 : n + 1) * W + node] : 0.0;
            const double zl = shfl_up1(zprev);   // 0 at lane 0 (node 1 has no coupled left node)
            const double zr = shfl_dn1(zprev);
            if (coupled) {
                double w = mdi * zprev;
                w = __builtin_fma(mlo, zl, w);
                w = __builtin_fma(mup, zr, w);
                rhs = rhs + w;
            }
            if (!act) rhs = 0.0;   // also when a neighbour's value is not finite
            // a[j] = 0 for j >= N and rhs = 0 on lanes without a node: the terms beyond
            // N add an exact zero, and the product runs without a branch per term
            double z = 0.0;
#pragma unroll
            for (int j = 0; j < NMAX; ++j) z = __builtin_fma(a[j], readlane_f64(rhs, j), z);
            if (act) u[n * W + node] = (T)z;
            zprev = act ? z : 0.0;
        }
    }
    __syncthreads();
}

template <typename T, int TR, int NMAX>
__global__ __launch_bounds__(kTailThreads) void k_vcycle_tail(TailArgs<T> a) {
    extern __shared__ __align__(16) unsigned char tail_lds[];
    T* S = reinterpret_cast<T*>(tail_lds);
    // every u starts from zero (Algorithm 1 on the coarse levels); b of level l_s in
    for (int q = threadIdx.x; q < a.lds_elems; q += kTailThreads) S[q] = T(0);
    __syncthreads();
    {
        const LevelView<T>& V = a.V[0];
        const int W = V.N + 1;
        T* b0 = S + a.off_b[0];
        for (int q = threadIdx.x; q < (V.Nt + 1) * W; q += kTailThreads) {
            const int n = q / W, i = q - n * W;
            b0[q] = a.b_in[(int64_t)n * a.P_in + i];
        }
    }
    __syncthreads();
    const int last = a.nlev - 1;
    for (int l = 0; l < last; ++l)
        tail_down<T, TR>(a.V[l], S + a.off_u[l], S + a.off_b[l], a.dir[l], S + a.off_u[l + 1],
                         S + a.off_b[l + 1], a.nu);
    tail_coarsest<T, TR, NMAX>(a.Vc, a.ainv, S + a.off_b[last], S + a.off_u[last]);
    for (int l = last - 1; l >= 0; --l)
        tail_up<T, TR>(a.V[l], S + a.off_u[l], S + a.off_b[l], a.dir[l], S + a.off_u[l + 1], a.nu);
    {
        const LevelView<T>& V = a.V[0];
        const int W = V.N + 1;
        const T* u0 = S + a.off_u[0];
        for (int q = threadIdx.x; q < (V.Nt + 1) * W; q += kTailThreads) {
            const int n = q / W, i = q - n * W;
            a.u_out[(int64_t)n * a.P_out + i] = u0[q];
        }
    }
}

template <typename T, int TR, int NMAX>
void* tail_kernel() {
    return reinterpret_cast<void*>(&k_vcycle_tail<T, TR, NMAX>);
}

template <typename T>
void* tail_kernel_for(int trans, int nmax) {
    if (trans) {
        if (nmax <= 8) return tail_kernel<T, 1, 8>();
        if (nmax <= 16) return tail_kernel<T, 1, 16>();
        return tail_kernel<T, 1, 32>();
    }
    if (nmax <= 8) return tail_kernel<T, 0, 8>();
    if (nmax <= 16) return tail_kernel<T, 0, 16>();
    return tail_kernel<T, 0, 32>();
}

}  // namespace

int tail_rows_per_owner(int N, int Nt, bool even) {
    const int W = N + 1;
    if (W > kTailThreads) return kTailMaxRows + 1;
    const int R = kTailThreads / W;
    const int M = (Nt + 1 + R - 1) / R;
    return even ? M + (M & 1) : M;
}

template <typename T>
int tail_lds_bytes(const int* N, const int* Nt, int nlev) {
    int64_t e = 0;
    for (int l = 0; l < nlev; ++l) e += 2 * (int64_t)(N[l] + 1) * (Nt[l] + 1);
    return (int)(e * (int64_t)sizeof(T));
}

template <typename T>
int tail_prepare(int lds_bytes, int coarsest_n) {
    if (coarsest_n > kTailMaxCoarsestN) return -1;
    for (int trans = 0; trans < 2; ++trans) {
        hipError_t e = hipFuncSetAttribute(tail_kernel_for<T>(trans, coarsest_n),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return -1;
        }
    }
    return 0;
}

template <typename T>
int launch_vcycle_tail(const TailLaunch<T>& t, hipStream_t s) {
    if (t.nlev < 2 || t.nlev > kTailMaxLevels || t.Vc.N > kTailMaxCoarsestN) return -1;
    TailArgs<T> a{};
    int off = 0;
    for (int l = 0; l < t.nlev; ++l) {
        const LevelView<T>& V = t.V[l];
        const int W = V.N + 1;
        // every level but the coarsest (solved by wave 0) is mapped onto the threads
        if (l + 1 < t.nlev && tail_rows_per_owner(V.N, V.Nt, t.dir[l] == 't') > kTailMaxRows) return -1;
        a.V[l] = V;
        a.dir[l] = t.dir[l];
        a.off_u[l] = off;
        off += W * (V.Nt + 1);
        a.off_b[l] = off;
        off += W * (V.Nt + 1);
    }
    if ((int64_t)off * (int64_t)sizeof(T) > t.lds_bytes) return -1;
    a.nlev = t.nlev;
    a.nu = t.nu;
    a.lds_elems = off;
    a.Vc = t.Vc;
    a.ainv = t.ainv;
    a.b_in = t.b_in;
    a.P_in = t.P_in;
    a.u_out = t.u_out;
    a.P_out = t.P_out;
    const size_t lds = (size_t)off * sizeof(T);
    const int n = t.Vc.N;
    if (t.trans) {
        if (n <= 8)
            hipLaunchKernelGGL((k_vcycle_tail<T, 1, 8>), dim3(1), dim3(kTailThreads), lds, s, a);
        else if (n <= 16)
            hipLaunchKernelGGL((k_vcycle_tail<T, 1, 16>), dim3(1), dim3(kTailThreads), lds, s, a);
        else
            hipLaunchKernelGGL((k_vcycle_tail<T, 1, 32>), dim3(1), dim3(kTailThreads), lds, s, a);
    } else {
        if (n <= 8)
            hipLaunchKernelGGL((k_vcycle_tail<T, 0, 8>), dim3(1), dim3(kTailThreads), lds, s, a);
        else if (n <= 16)
            hipLaunchKernelGGL((k_vcycle_tail<T, 0, 16>), dim3(1), dim3(kTailThreads), lds, s, a);
        else
            hipLaunchKernelGGL((k_vcycle_tail<T, 0, 32>), dim3(1), dim3(kTailThreads), lds, s, a);
    }
    return 0;
}

template int tail_lds_bytes<double>(const int*, const int*, int);
template int tail_lds_bytes<float>(const int*, const int*, int);
template int tail_prepare<double>(int, int);
template int tail_prepare<float>(int, int);
template int launch_vcycle_tail<double>(const TailLaunch<double>&, hipStream_t);
template int launch_vcycle_tail<float>(const TailLaunch<float>&, hipStream_t);

}  // namespace stmg
