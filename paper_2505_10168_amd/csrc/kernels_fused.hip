// Fused streaming smoother kernels of libstmg (gfx950, wave64).
//
// The BE-FE operator J (Section 2.2) couples time level n only to level n-1 (J^T:
// only to n+1), so S damped-Jacobi steps (Section 3.1) can be evaluated in ONE pass
// that streams through time: at row n, step k needs step k-1 at rows n and n-1,
// both already available.  Every wavefront owns a strip of 256 contiguous columns
// (4 per lane) and a segment of time levels; the S+1 sweep states of the previous
// row stay in registers, neighbouring columns are exchanged between lanes, so each
// DOF is read and written once per pass instead of once per sweep.
//
// A pass optionally starts with the prolongation u += P z (the post-smoothing side
// of Algorithm 1) and optionally ends with the residual r = b - J u followed by the
// restriction R r (x or t, the pre-smoothing side) or by the squared residual norm
// (termination test of Section 3.1).
//
// Redundant work: 4*HL halo columns per strip side (HL = ceil((S+2)/4) lanes) and
// S(+1) warm-up rows per time segment, both recomputed rather than exchanged.
// The arithmetic of each DOF goes through stencil_interior/jacobi_update in the
// same order as the reference kernels, so both paths give identical bits.
#include <hip/hip_runtime.h>

#include "stmg_launch.hpp"

namespace stmg {

namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kCols = 4;   // contiguous columns per lane

enum Tail { TAIL_NONE = 0, TAIL_RX = 1, TAIL_RT = 2, TAIL_NORM = 3 };

template <typename T>
struct FusedArgs {
    const T* u;
    const T* b;
    T* out;
    const T* z;
    int64_t Pz;
    T* bc;
    int64_t Pbc;
    double* parts;
    int Nc;
    int head;      // 0, 1 = prolong x, 2 = prolong t
    int zero_in;
    int HL;        // halo lanes per side
    int xw;        // strips along x
    int seg;       // time levels per segment
    int nwaves;
};

__device__ __forceinline__ double shfl_up1(double v) { return __shfl_up(v, 1, kWave); }
__device__ __forceinline__ double shfl_dn1(double v) { return __shfl_down(v, 1, kWave); }
__device__ __forceinline__ float shfl_up1(float v) { return __shfl_up(v, 1, kWave); }
__device__ __forceinline__ float shfl_dn1(float v) { return __shfl_down(v, 1, kWave); }

__device__ __forceinline__ void load4(const double* p, double (&v)[4]) {
    const double2* q = reinterpret_cast<const double2*>(p);
    double2 a = q[0], b = q[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void load4(const float* p, float (&v)[4]) {
    float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
__device__ __forceinline__ void store4(double* p, const double (&v)[4]) {
    double2* q = reinterpret_cast<double2*>(p);
    q[0] = make_double2(v[0], v[1]);
    q[1] = make_double2(v[2], v[3]);
}
__device__ __forceinline__ void store4(float* p, const float (&v)[4]) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void load2(const double* p, double& a, double& b) {
    double2 v = *reinterpret_cast<const double2*>(p);
    a = v.x; b = v.y;
}
__device__ __forceinline__ void load2(const float* p, float& a, float& b) {
    float2 v = *reinterpret_cast<const float2*>(p);
    a = v.x; b = v.y;
}
__device__ __forceinline__ void store2(double* p, double a, double b) {
    *reinterpret_cast<double2*>(p) = make_double2(a, b);
}
__device__ __forceinline__ void store2(float* p, float a, float b) {
    *reinterpret_cast<float2*>(p) = make_float2(a, b);
}

// Per-lane stencil coefficients of its 4 columns.
template <typename T>
struct LaneCoef {
    T lo[4], di[4], up[4], mlo[4], mdi[4], mup[4], wd[4];
};

// One Jacobi step (or, with JAC = false, the residual) of the lane's 4 columns at
// row n.  x: current state, xl/xr: left/right neighbour column values; p/pl/pr: the
// same at the coupled row.  Invalid columns produce 0.
template <typename T, bool JAC>
__device__ __forceinline__ void row_step(const LevelView<T>& L, const LaneCoef<T>& C,
                                         const bool (&valid)[4], bool dir_col0, bool dir_row,
                                         bool coupled, const T (&x)[4], T xl, T xr,
                                         const T (&p)[4], T pl, T pr, const T (&bb)[4],
                                         T (&y)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!valid[j]) {
            y[j] = T(0);
            continue;
        }
        T Jx, scale;
        if (dir_row || (j == 0 && dir_col0)) {
            Jx = L.W * x[j];
            scale = L.wW;
        } else {
            const T xm = (j > 0) ? x[j - 1] : xl;
            const T xp = (j < 3) ? x[j + 1] : xr;
            const T pm = (j > 0) ? p[j - 1] : pl;
            const T pp = (j < 3) ? p[j + 1] : pr;
            Jx = stencil_interior<T>(C.lo[j], C.di[j], C.up[j], C.mlo[j], C.mdi[j], C.mup[j], xm,
                                     x[j], xp, coupled, pm, p[j], pp);
            scale = C.wd[j];
        }
        const T r = bb[j] - Jx;
        y[j] = JAC ? jacobi_update<T>(x[j], scale, r) : r;
    }
}

template <typename T, int TR, int S, int TAIL>
__global__ __launch_bounds__(256) void k_fused(LevelView<T> L, FusedArgs<T> a) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (wave >= a.nwaves) return;
    const int HL = a.HL;
    const int U = (kWave - 2 * HL) * kCols;
    const int wx = wave % a.xw;
    const int wt = wave / a.xw;
    const int g = wx * U - kCols * HL + kCols * lane;   // first column of this lane
    const bool useful = (lane >= HL) && (lane < kWave - HL);
    const bool lane_in = (g >= 0) && (g <= L.N);
    const int N = L.N, Nt = L.Nt;
    const int64_t P = L.P;

    bool valid[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) valid[j] = lane_in && (g + j <= N);
    const bool dir_col0 = (g == 0);

    LaneCoef<T> C;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = g + j;
        const bool v = valid[j];
        C.lo[j] = v ? L.lo[c] : T(0);
        C.di[j] = v ? L.di[c] : T(0);
        C.up[j] = v ? L.up[c] : T(0);
        C.mlo[j] = v ? L.mlo[c] : T(0);
        C.mdi[j] = v ? L.mdi[c] : T(0);
        C.mup[j] = v ? L.mup[c] : T(0);
        C.wd[j] = v ? L.wd[c] : T(0);
    }

    // Time segment and warm-up.
    const int rows = Nt + 1;
    const int n0 = wt * a.seg;
    const int n1 = min(rows, n0 + a.seg);   // output rows [n0, n1)
    constexpr int WARM = S + (TAIL != TAIL_NONE ? 1 : 0);
    const int first = TR ? min(Nt, n1 - 1 + WARM) : max(0, n0 - WARM);
    const int count = TR ? (first - n0 + 1) : (n1 - first);

    // Sweep states of the previous streamed row: level k = 0..S.
    T prev[S + 1][4];
    T prevl[S + 1], prevr[S + 1];
#pragma unroll
    for (int k = 0; k <= S; ++k) {
#pragma unroll
        for (int j = 0; j < 4; ++j) prev[k][j] = T(0);
        prevl[k] = T(0);
        prevr[k] = T(0);
    }
    T r_pair[4] = {T(0), T(0), T(0), T(0)};   // t-restriction: residual of the partner row
    double acc = 0.0;                         // norm tail

    for (int it = 0; it < count; ++it) {
        const int n = TR ? first - it : first + it;
        const bool out_row = (n >= n0) && (n < n1);
        const bool dir_row = (n == 0);
        const bool coupled = TR ? (n < Nt) : (n >= 2);
        const int64_t ro = (int64_t)n * P + g;

        T x[4] = {T(0), T(0), T(0), T(0)};
        T bb[4] = {T(0), T(0), T(0), T(0)};
        if (lane_in) {
            if (!a.zero_in) load4(a.u + ro, x);
            if (S > 0 || TAIL != TAIL_NONE) load4(a.b + ro, bb);
        }
        // Prolongation head: x += P z.
        if (a.head == 1) {
            T z0 = T(0), z1 = T(0);
            if (lane_in) load2(a.z + (int64_t)n * a.Pz + (g >> 1), z0, z1);
            const T z2 = shfl_dn1(z0);
            if (valid[0]) x[0] += z0;
            if (valid[1]) x[1] = fmaT(T(0.5), z0 + z1, x[1]);
            if (valid[2]) x[2] += z1;
            if (valid[3]) x[3] = fmaT(T(0.5), z1 + z2, x[3]);
        } else if (a.head == 2) {
            if (lane_in) {
                T zz[4];
                load4(a.z + (int64_t)(n >> 1) * a.Pz + g, zz);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (valid[j]) x[j] += zz[j];
            }
        }
        T xl = shfl_up1(x[3]);
        T xr = shfl_dn1(x[0]);

#pragma unroll
        for (int k = 0; k < S; ++k) {
            T y[4];
            row_step<T, true>(L, C, valid, dir_col0, dir_row, coupled, x, xl, xr, prev[k],
                              prevl[k], prevr[k], bb, y);
#pragma unroll
            for (int j = 0; j < 4; ++j) prev[k][j] = x[j];
            prevl[k] = xl;
            prevr[k] = xr;
#pragma unroll
            for (int j = 0; j < 4; ++j) x[j] = y[j];
            xl = shfl_up1(x[3]);
            xr = shfl_dn1(x[0]);
        }

        if (out_row && useful && lane_in) store4(a.out + ro, x);

        if constexpr (TAIL != TAIL_NONE) {
            T r[4];
            row_step<T, false>(L, C, valid, dir_col0, dir_row, coupled, x, xl, xr, prev[S],
                               prevl[S], prevr[S], bb, r);
#pragma unroll
            for (int j = 0; j < 4; ++j) prev[S][j] = x[j];
            prevl[S] = xl;
            prevr[S] = xr;
            if constexpr (TAIL == TAIL_RX) {
                const T rl = shfl_up1(r[3]);
                if (out_row && useful && lane_in) {
                    const int I0 = g >> 1;
                    const T c0 = fmaT(T(0.5), rl + r[1], r[0]);
                    const T c1 = fmaT(T(0.5), r[1] + r[3], r[2]);
                    T* dst = a.bc + (int64_t)n * a.Pbc + I0;
                    if (I0 + 1 <= a.Nc)
                        store2(dst, c0, c1);
                    else if (I0 <= a.Nc)
                        dst[0] = c0;
                }
            } else if constexpr (TAIL == TAIL_RT) {
                if (out_row && useful && lane_in) {
                    // pairs (2J, 2J+1) -> J; in the transposed stream 2J+1 comes first
                    const bool second = TR ? ((n & 1) == 0) : ((n & 1) == 1);
                    const bool lone = TR ? false : ((n & 1) == 0 && n == Nt);
                    const bool lone_tr = TR ? (n == Nt && (n & 1) == 0) : false;
                    if (second && !lone_tr) {
                        T v[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            v[j] = T(0.5) * (TR ? (r[j] + r_pair[j]) : (r_pair[j] + r[j]));
                        store4(a.bc + (int64_t)(n >> 1) * a.Pbc + g, v);
                    } else if (lone || lone_tr) {
                        T v[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) v[j] = T(0.5) * r[j];
                        store4(a.bc + (int64_t)(n >> 1) * a.Pbc + g, v);
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j) r_pair[j] = r[j];
                    }
                }
            } else if constexpr (TAIL == TAIL_NORM) {
                if (out_row && useful) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const double rv = (double)r[j];
                        acc = __builtin_fma(rv, rv, acc);
                    }
                }
            }
        }
    }

    if constexpr (TAIL == TAIL_NORM) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if (lane == 0) a.parts[wave] = acc;
    }
}

struct Geometry {
    int HL, U, xw, seg, nwaves;
};

Geometry geometry(int N, int Nt, int sweeps) {
    Geometry G;
    G.HL = (sweeps + 2 + kCols - 1) / kCols;
    if (G.HL < 1) G.HL = 1;
    G.U = (kWave - 2 * G.HL) * kCols;
    G.xw = (N + 1 + G.U - 1) / G.U;
    const int rows = Nt + 1;
    const int64_t target = 8192;
    int64_t seg = ((int64_t)rows * G.xw + target - 1) / target;
    const int64_t min_seg = 32;
    if (seg < min_seg) seg = min_seg;
    if (seg > 512) seg = 512;
    if (seg & 1) ++seg;
    G.seg = (int)seg;
    G.nwaves = G.xw * ((rows + G.seg - 1) / G.seg);
    return G;
}

template <typename T, int TR, int S, int TAIL>
void launch_one(const LevelView<T>& L, const FusedArgs<T>& a, hipStream_t s) {
    const int blocks = (a.nwaves + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL((k_fused<T, TR, S, TAIL>), dim3(blocks), dim3(kWave * kWavesPerBlock), 0,
                       s, L, a);
}

template <typename T, int TR, int S>
void dispatch_tail(int tail, const LevelView<T>& L, const FusedArgs<T>& a, hipStream_t s) {
    switch (tail) {
        case TAIL_NONE: launch_one<T, TR, S, TAIL_NONE>(L, a, s); break;
        case TAIL_RX: launch_one<T, TR, S, TAIL_RX>(L, a, s); break;
        case TAIL_RT: launch_one<T, TR, S, TAIL_RT>(L, a, s); break;
        default: launch_one<T, TR, S, TAIL_NORM>(L, a, s); break;
    }
}

template <typename T, int TR>
void dispatch_sweeps(int S, int tail, const LevelView<T>& L, const FusedArgs<T>& a,
                     hipStream_t s) {
    switch (S) {
        case 0: dispatch_tail<T, TR, 0>(tail, L, a, s); break;
        case 1: dispatch_tail<T, TR, 1>(tail, L, a, s); break;
        case 2: dispatch_tail<T, TR, 2>(tail, L, a, s); break;
        case 3: dispatch_tail<T, TR, 3>(tail, L, a, s); break;
        default: dispatch_tail<T, TR, 4>(tail, L, a, s); break;
    }
}

}  // namespace

int fused_parts(int N, int Nt, int sweeps) { return geometry(N, Nt, sweeps).nwaves; }

template <typename T>
int launch_fused(const LevelView<T>& L, const FusedPass& fp, const T* u, const T* b, T* out,
                 hipStream_t s) {
    if (fp.sweeps < 0 || fp.sweeps > 4) return -1;
    Geometry G = geometry(L.N, L.Nt, fp.sweeps);
    FusedArgs<T> a;
    a.u = u;
    a.b = b;
    a.out = out;
    a.z = static_cast<const T*>(fp.z);
    a.Pz = fp.Pz;
    a.bc = static_cast<T*>(fp.bc);
    a.Pbc = fp.Pbc;
    a.parts = fp.parts;
    a.Nc = fp.Nc;
    a.head = fp.prolong == 'x' ? 1 : (fp.prolong == 't' ? 2 : 0);
    a.zero_in = fp.zero_in;
    a.HL = G.HL;
    a.xw = G.xw;
    a.seg = G.seg;
    a.nwaves = G.nwaves;
    const int tail = fp.tail == 'x' ? TAIL_RX : (fp.tail == 't' ? TAIL_RT : (fp.tail == 'n' ? TAIL_NORM : TAIL_NONE));
    if (fp.trans)
        dispatch_sweeps<T, 1>(fp.sweeps, tail, L, a, s);
    else
        dispatch_sweeps<T, 0>(fp.sweeps, tail, L, a, s);
    return G.nwaves;
}

template int launch_fused<double>(const LevelView<double>&, const FusedPass&, const double*,
                                  const double*, double*, hipStream_t);
template int launch_fused<float>(const LevelView<float>&, const FusedPass&, const float*,
                                 const float*, float*, hipStream_t);

}  // namespace stmg
