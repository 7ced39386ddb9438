// Fused streaming smoother kernels of libstmg (gfx950, wave64).
//
// The BE-FE operator J (Section 2.2) couples time level n only to level n-1 (J^T:
// only to n+1), so S damped-Jacobi steps (Section 3.1) can be evaluated in ONE pass
// that streams through time: at row n, step k needs step k-1 at rows n and n-1,
// both already available.  Every wavefront owns a strip of 64*K contiguous columns
// (K = 16 bytes / element size per lane: one dwordx4 access per vector and row) and
// a segment of time levels; the S+1 sweep states of the previous row stay in
// registers, neighbouring columns are exchanged between lanes, and the next row is
// prefetched while the current one is computed.  Each DOF is read and written once
// per pass instead of once per sweep.
//
// A pass optionally starts with the prolongation u += P z (the post-smoothing side
// of Algorithm 1) and optionally ends with the residual r = b - J u followed by the
// restriction R r (x or t, the pre-smoothing side) or by the squared residual norm
// (termination test of Section 3.1).
//
// Redundant work: K*HL halo columns per strip side (HL = ceil((S+2)/K) lanes) and
// S(+1) warm-up rows per time segment, both recomputed rather than exchanged.
// The arithmetic of each DOF goes through stencil_interior/jacobi_update in the
// same order as the reference kernels, so both paths give identical bits.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <type_traits>

#include "stmg_launch.hpp"

namespace stmg {

namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
#ifndef STMG_PREFETCH_ROWS
#define STMG_PREFETCH_ROWS 3
#endif
#ifndef STMG_NT_STORES
#define STMG_NT_STORES 1
#endif
#ifndef STMG_TARGET_WAVES
#define STMG_TARGET_WAVES 16384
#endif
#ifndef STMG_TARGET_WAVES_ALU
#define STMG_TARGET_WAVES_ALU 3072
#endif
#ifndef STMG_TARGET_WAVES_ALU_COARSE
#define STMG_TARGET_WAVES_ALU_COARSE 2048
#endif
#ifndef STMG_ALIGN_HALO
#define STMG_ALIGN_HALO 1
#endif
#ifndef STMG_BIG_LEVEL_BYTES
#define STMG_BIG_LEVEL_BYTES 268435456.0
#endif
#ifndef STMG_ZERO_FIRST
#define STMG_ZERO_FIRST 1   // first step of a zero-start chain as a scaled copy of b
#endif
#ifndef STMG_SPLIT_LOOP
#define STMG_SPLIT_LOOP 1   // 0: one copy of the streaming loop, with the row-0 tests
#endif
#ifndef STMG_MIN_SEGMENT
#define STMG_MIN_SEGMENT 2
#endif
#ifndef STMG_SINGLE_ROW_MAX_WAVES
#define STMG_SINGLE_ROW_MAX_WAVES 640   // 2-row segments giving at most this many waves: 1-row
#endif
constexpr int kPrefetchRows = STMG_PREFETCH_ROWS;   // rows in flight per wave (register ring)
constexpr int kXcds = 8;     // accelerator complex dies of an MI355X
constexpr int kMaxFused = 6; // Jacobi steps one pass can fuse
constexpr int kMaxChain = 6; // Jacobi steps of a chain pass (recompute, cycle)
constexpr int kMaxMixedSweeps = 2;   // steps per smoothing of the fused mixed pass

enum Tail { TAIL_NONE = 0, TAIL_RX = 1, TAIL_RT = 2, TAIL_NORM = 3, TAIL_DEFECT = 4 };

template <typename T>
struct FusedArgs {
    const T* u;
    const T* b;
    T* out;        // the chain's result (not stored when null)
    T* mid;        // MID: the iterate after the S2 steps
    const T* z;
    int64_t Pz;
    T* bc;
    int64_t Pbc;
    double* parts;
    int Nc;
    int head;      // 0, 1 = prolong x, 2 = prolong t, 3 = defect correction u += s e
    int zero_in;
    int b_const;   // b is constant in time: two rows, row 0 (zeros) for n = 0, row 1 after
    const float* e32;    // head 3: FP32 correction, same pitch as u
    double s_old;        // head 3: scale of the correction
    float* f32;          // TAIL_DEFECT: FP32 right-hand side r / s_new
    double inv_s_new;
    int HL;        // halo lanes per side
    int xw;        // strips along x
    int seg;       // time levels per segment
    int nwaves;
};

template <typename T> struct Lanes;
template <> struct Lanes<double> { static constexpr int K = 2; };
template <> struct Lanes<float> { static constexpr int K = 4; };


// 16-byte row accesses of one lane.
__device__ __forceinline__ void ld(const double* p, double (&v)[2]) {
    double2 a = *reinterpret_cast<const double2*>(p);
    v[0] = a.x; v[1] = a.y;
}
__device__ __forceinline__ void ld(const float* p, float (&v)[4]) {
    float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
__device__ __forceinline__ void st(double* p, const double (&v)[2]) {
#if STMG_NT_STORES
    __builtin_nontemporal_store(v[0], p);
    __builtin_nontemporal_store(v[1], p + 1);
#else
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
#endif
}
__device__ __forceinline__ void st(float* p, const float (&v)[4]) {
#if STMG_NT_STORES
    for (int j = 0; j < 4; ++j) __builtin_nontemporal_store(v[j], p + j);
#else
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
#endif
}
// coarse x-prolongation / x-restriction touch K/2 coarse values per lane
__device__ __forceinline__ void ldh(const double* p, double (&v)[1]) { v[0] = p[0]; }
__device__ __forceinline__ void ldh(const float* p, float (&v)[2]) {
    float2 a = *reinterpret_cast<const float2*>(p);
    v[0] = a.x; v[1] = a.y;
}
__device__ __forceinline__ void sth(double* p, const double (&v)[1]) { p[0] = v[0]; }
__device__ __forceinline__ void sth(float* p, const float (&v)[2]) {
    *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
}

template <typename T, int K>
struct LaneCoef {
    T mlo[K], mdi[K], mup[K], kl[K], kr[K], wd[K];
    T me[K];   // multiplier of x_j in e_j = x_j - x_{j+1}: 0 for column 0, else 1
};

// One Jacobi step (JAC) or the residual (!JAC) of the lane's K columns at one row.
// x: state at this row, p: the same sweep state at the coupled row (zero on uncoupled
// rows).  The operands of stencil_interior are shared between neighbouring columns
// instead of being formed per column:
//   d_j = x_j - p_j        (the mass differences dm, d0, dp of columns j+1, j, j-1)
//   e_j = x_j - x_{j+1}    (x0 - xp of column j; x0 - xm of column j+1 is -e_j)
// Each rounded operation has the same operands as in stencil_interior (negation and
// fma(1, a, -b) = a - b are exact), so the result is bit-identical, with 9 instead of
// 12 floating-point operations per DOF.  Column 0 (Dirichlet) is expressed through its
// coefficients (kl = W_Diri, wd = omega / W_Diri, the rest 0) and the zero column to
// its left, which lies in a halo lane; column 1 drops its eliminated left neighbour
// through me (e_0 = -x_1, and mlo[1] = 0); columns beyond the last node have zero
// coefficients and zero data.  Time level 0 is a Dirichlet row for every column: DIR
// selects that form at compile time (the caller branches once per row, on a
// wave-uniform test).
template <typename T, int K, bool JAC, bool DIR>
__device__ __forceinline__ void row_step(const LevelView<T>& L, const LaneCoef<T, K>& C,
                                         const T (&x)[K], const T (&p)[K], const T (&bb)[K],
                                         T (&y)[K]) {
    if constexpr (DIR) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const T r = bb[j] - L.W * x[j];
            y[j] = JAC ? jacobi_update<T>(x[j], L.wW, r) : r;
        }
    } else {
        T d[K], e[K];
#pragma unroll
        for (int j = 0; j < K; ++j) d[j] = x[j] - p[j];
        const T xr = shfl_dn1(x[0]);
#pragma unroll
        for (int j = 0; j < K; ++j) e[j] = fmaT(C.me[j], x[j], -((j < K - 1) ? x[j + 1] : xr));
        const T dl = shfl_up1(d[K - 1]);
        const T dr = shfl_dn1(d[0]);
        const T el = shfl_up1(e[K - 1]);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const T dm = (j > 0) ? d[j - 1] : dl;
            const T dp = (j < K - 1) ? d[j + 1] : dr;
            const T em = (j > 0) ? e[j - 1] : el;
            T s = C.mdi[j] * d[j];
            s = fmaT(C.mlo[j], dm, s);
            s = fmaT(C.mup[j], dp, s);
            s = fmaT(C.kl[j], -em, s);
            s = fmaT(C.kr[j], e[j], s);
            const T r = bb[j] - s;
            y[j] = JAC ? jacobi_update<T>(x[j], C.wd[j], r) : r;
        }
    }
}

// Wave index of a multi-workgroup launch.  Workgroups are dealt to the 8 XCDs round
// robin; renumber them so that each XCD gets a contiguous range of strips and time
// segments, whose shared halo columns and warm-up rows then hit the same L2.
// Wave-uniform by construction; readfirstlane lets the compiler know it, so that the
// per-row tests of the pass are scalar branches.
__device__ __forceinline__ int grid_wave() {
    const int nb = gridDim.x, q = nb / kXcds, r = nb % kXcds;
    const int xcd = blockIdx.x % kXcds, idx = blockIdx.x / kXcds;
    const int lb = (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
    return __builtin_amdgcn_readfirstlane(lb * kWavesPerBlock + (threadIdx.x >> 6));
}

// One fused pass as executed by wave `wave` of the a.nwaves waves of the pass: a chain
// of stages applied to every row as it streams past,
//   S1 Jacobi steps -> HEAD -> S2 steps -> [MID] -> S3 steps -> store -> [TAIL]
// HEAD: 0 none, 1 x prolongation, 2 t prolongation, 3 defect correction u += s e.
// MID: the iterate after S2 steps is stored to a.mid (unless null) and its residual
// norm summed (the end of one V-cycle, whose S3 steps then pre-smooth the next cycle).
// The store of the chain's result is skipped when a.out is null.
// PF: rows in flight per wave (register prefetch ring).
template <typename T, int TR, int S1, int HEAD, int S2, int MID, int S3, int TAIL,
          int PF = kPrefetchRows>
__device__ __forceinline__ void fused_body(const LevelView<T>& L, const FusedArgs<T>& a,
                                           const int wave) {
    constexpr int K = Lanes<T>::K;
    constexpr int KH = K / 2;
    constexpr int S = S1 + S2 + S3;            // Jacobi steps of the chain
    constexpr int IM = S;                      // state slot of the MID residual
    constexpr int IT = S + (MID ? 1 : 0);      // state slot of the TAIL residual
    const int lane = threadIdx.x & (kWave - 1);
    if (wave >= a.nwaves) return;
    const int HL = a.HL;
    const int U = (kWave - 2 * HL) * K;
    const int wx = wave % a.xw;
    const int wt = wave / a.xw;
    const int g = wx * U - K * HL + K * lane;   // first column of this lane
    const bool useful = (lane >= HL) && (lane < kWave - HL);
    const bool lane_in = (g >= 0) && (g <= L.N);
    const int N = L.N, Nt = L.Nt;
    const int64_t P = L.P;
    const bool store_out = a.out != nullptr;

    bool valid[K];
#pragma unroll
    for (int j = 0; j < K; ++j) valid[j] = lane_in && (g + j <= N);

    LaneCoef<T, K> C;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int c = g + j;
        const bool v = valid[j];
        C.mlo[j] = v ? L.mlo[c] : T(0);
        C.mdi[j] = v ? L.mdi[c] : T(0);
        C.mup[j] = v ? L.mup[c] : T(0);
        C.kl[j] = v ? L.kl[c] : T(0);
        C.kr[j] = v ? L.kr[c] : T(0);
        C.wd[j] = v ? L.wd[c] : T(0);
        C.me[j] = (c == 0) ? T(0) : T(1);
    }

    // Time segment and warm-up: every coupled stage on the way to an output needs the
    // previous row of its input, so a segment starts that many rows early.
    const int rows = Nt + 1;
    const int n0 = wt * a.seg;
    const int n1 = min(rows, n0 + a.seg);   // output rows [n0, n1)
    // A chain with S1 > 0 starts from u = 0 (it redoes a smoothing from zero): its first
    // step is y = (omega / J_ii) b, since with a zero iterate and a zero coupled row every
    // stencil term is +0; the same value, no stencil work, and no previous row needed, so
    // the segment starts one row later.
    constexpr bool ZF = STMG_ZERO_FIRST && S1 > 0;
    constexpr int WCHAIN = S + (TAIL != TAIL_NONE ? 1 : 0) - (ZF ? 1 : 0);
    constexpr int WMID = MID ? S1 + S2 + 1 : 0;
    constexpr int WARM = WCHAIN > WMID ? WCHAIN : WMID;
    const int first = TR ? min(Nt, n1 - 1 + WARM) : max(0, n0 - WARM);
    const int count = TR ? (first - n0 + 1) : (n1 - first);
    constexpr bool need_b = (S > 0 || TAIL != TAIL_NONE || MID);

    // Stage states of the previous streamed row: the inputs of the S Jacobi steps and
    // of the MID and TAIL residuals.  Their neighbour columns are fetched again by DPP
    // when needed rather than kept in registers.
    constexpr int NST = S + (MID ? 1 : 0) + (TAIL != TAIL_NONE ? 1 : 0);
    T prev[NST > 0 ? NST : 1][K];
#pragma unroll
    for (int k = 0; k < NST; ++k)
#pragma unroll
        for (int j = 0; j < K; ++j) prev[k][j] = T(0);
    T r_pair[K];
#pragma unroll
    for (int j = 0; j < K; ++j) r_pair[j] = T(0);
    double acc = 0.0;

    // Row buffers: rows are fetched PF steps ahead of use (a register ring that the
    // unrolled inner loop indexes statically).
    constexpr bool HASZ = HEAD != 0;
    // coarse values per lane and row: K/2 for the x prolongation, K otherwise
    constexpr int KZ = HEAD == 1 ? KH : (HASZ ? K : 1);
    T ru[PF][K], rb[PF][K], rz[PF][KZ];
    auto fetch = [&](int n, T (&fu)[K], T (&fb)[K], T (&fz)[KZ]) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            fu[j] = T(0);
            fb[j] = T(0);
        }
#pragma unroll
        for (int j = 0; j < KZ; ++j) fz[j] = T(0);
        if (!lane_in) return;
        const int64_t ro = (int64_t)n * P + g;
        if (!a.zero_in) ld(a.u + ro, fu);
        if (need_b) ld(a.b + (a.b_const ? (n > 0 ? P : 0) : (int64_t)n * P) + g, fb);
        if constexpr (HEAD == 1) {
            ldh(a.z + (int64_t)n * a.Pz + (g >> 1), fz);
        } else if constexpr (HEAD == 2) {
            ld(a.z + (int64_t)(n >> 1) * a.Pz + g, fz);
        } else if constexpr (HEAD == 3 && std::is_same<T, double>::value) {
            const float2 e = *reinterpret_cast<const float2*>(a.e32 + ro);
            fz[0] = (T)e.x;
            fz[1] = (T)e.y;
        }
    };
    auto row_of = [&](int it) { return TR ? first - it : first + it; };
#pragma unroll
    for (int d = 0; d < PF; ++d)
        if (d < count) fetch(row_of(d), ru[d], rb[d], rz[d]);

    // Waves whose rows include the Dirichlet row 0 or a row without time coupling run
    // the loop with those tests; every other wave runs a copy without them, whose rows
    // then need no join of the two compiled chains (a join costs register moves).
    auto stream = [&](auto special_tag) {
        constexpr bool SPECIAL = decltype(special_tag)::value;
        for (int it0 = 0; it0 < count; it0 += PF) {
#pragma unroll
        for (int d = 0; d < PF; ++d) {
            const int it = it0 + d;
            if (it >= count) break;
            const int n = row_of(it);
            T x[K], bb[K], zz[KZ];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                x[j] = ru[d][j];
                bb[j] = rb[d][j];
            }
#pragma unroll
            for (int j = 0; j < KZ; ++j) zz[j] = rz[d][j];
            if (it + PF < count) fetch(row_of(it + PF), ru[d], rb[d], rz[d]);
            const bool out_row = (n >= n0) && (n < n1);
            const bool dir_row = SPECIAL && (n == 0);
            const bool coupled = !SPECIAL || (TR ? (n < Nt) : (n >= 2));
            if (SPECIAL && !coupled) {
                // first levels of J (last of J^T): no coupling, i.e. a zero coupled row
#pragma unroll
                for (int k = 0; k < NST; ++k)
#pragma unroll
                    for (int j = 0; j < K; ++j) prev[k][j] = T(0);
            }

            // The chain, compiled twice: for the Dirichlet row 0 and for every other row.
            T r[K], rm[K];
            auto chain = [&](auto dir_tag) {
                constexpr bool DIR = decltype(dir_tag)::value;
                auto steps = [&](auto k0_tag, auto k1_tag) {
                    constexpr int k0 = decltype(k0_tag)::value, k1 = decltype(k1_tag)::value;
#pragma unroll
                    for (int k = k0; k < k1; ++k) {
                        T y[K];
                        if (ZF && k == 0) {
#pragma unroll
                            for (int j = 0; j < K; ++j)
                                y[j] = jacobi_update<T>(T(0), DIR ? L.wW : C.wd[j], bb[j]);
                        } else {
                            row_step<T, K, true, DIR>(L, C, x, prev[k], bb, y);
                        }
#pragma unroll
                        for (int j = 0; j < K; ++j) {
                            prev[k][j] = x[j];
                            x[j] = y[j];
                        }
                    }
                };
                steps(std::integral_constant<int, 0>{}, std::integral_constant<int, S1>{});
                // Prolongation head: x += P z.
                if constexpr (HEAD == 1) {
                    const T znext = shfl_dn1(zz[0]);   // first coarse value of the next lane
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        const T za = zz[j >> 1];
                        if ((j & 1) == 0) {
                            x[j] += za;
                        } else {
                            const T zb = ((j >> 1) + 1 < KH) ? zz[((j >> 1) + 1) % KZ] : znext;
                            x[j] = fmaT(T(0.5), za + zb, x[j]);
                        }
                    }
                } else if constexpr (HEAD == 2) {
#pragma unroll
                    for (int j = 0; j < K; ++j) x[j] += zz[j];
                } else if constexpr (HEAD == 3) {
#pragma unroll
                    for (int j = 0; j < K; ++j) x[j] = fmaT((T)a.s_old, zz[j], x[j]);
                }
                if constexpr (HASZ) {
                    // the interpolation reaches past the last node and into the lane left of
                    // column 0; those columns must stay zero (padding, eliminated neighbour)
#pragma unroll
                    for (int j = 0; j < K; ++j) x[j] = valid[j] ? x[j] : T(0);
                }
                steps(std::integral_constant<int, S1>{}, std::integral_constant<int, S1 + S2>{});
                if constexpr (MID) {
                    if (a.mid != nullptr && out_row && useful && lane_in) st(a.mid + (int64_t)n * P + g, x);
                    row_step<T, K, false, DIR>(L, C, x, prev[IM], bb, rm);
#pragma unroll
                    for (int j = 0; j < K; ++j) prev[IM][j] = x[j];
                }
                steps(std::integral_constant<int, S1 + S2>{}, std::integral_constant<int, S>{});
                if constexpr (TAIL != TAIL_NONE) {
                    row_step<T, K, false, DIR>(L, C, x, prev[IT], bb, r);
#pragma unroll
                    for (int j = 0; j < K; ++j) prev[IT][j] = x[j];
                }
            };
            if constexpr (SPECIAL) {
                if (dir_row)
                    chain(std::true_type{});
                else
                    chain(std::false_type{});
            } else {
                chain(std::false_type{});
            }

            if (store_out && out_row && useful && lane_in) st(a.out + (int64_t)n * P + g, x);

            if constexpr (MID) {
                if (out_row && useful) {
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        const double rv = (double)rm[j];
                        acc = __builtin_fma(rv, rv, acc);
                    }
                }
            }
            if constexpr (TAIL != TAIL_NONE) {
                if constexpr (TAIL == TAIL_RX) {
                    // coarse node I = (g + j)/2 for even j: r_{2I} + 1/2 (r_{2I-1} + r_{2I+1})
                    const T rl = shfl_up1(r[K - 1]);
                    if (out_row && useful && lane_in) {
                        const int I0 = g >> 1;
                        T c[KH];
#pragma unroll
                        for (int q = 0; q < KH; ++q) {
                            const T left = (q == 0) ? rl : r[2 * q - 1];
                            c[q] = fmaT(T(0.5), left + r[2 * q + 1], r[2 * q]);
                        }
                        T* dst = a.bc + (int64_t)n * a.Pbc + I0;
                        if (I0 + KH - 1 <= a.Nc) {
                            sth(dst, c);
                        } else {
#pragma unroll
                            for (int q = 0; q < KH; ++q)
                                if (I0 + q <= a.Nc) dst[q] = c[q];
                        }
                    }
                } else if constexpr (TAIL == TAIL_RT) {
                    if (out_row && useful && lane_in) {
                        // pairs (2J, 2J+1) -> J; the transposed stream meets 2J+1 first
                        const bool odd = (n & 1) != 0;
                        T v[K];
                        T* dst = a.bc + (int64_t)(n >> 1) * a.Pbc + g;
                        if (!TR) {
                            if (odd) {
#pragma unroll
                                for (int j = 0; j < K; ++j) v[j] = T(0.5) * (r_pair[j] + r[j]);
                                st(dst, v);
                            } else if (n == Nt) {
#pragma unroll
                                for (int j = 0; j < K; ++j) v[j] = T(0.5) * r[j];
                                st(dst, v);
                            } else {
#pragma unroll
                                for (int j = 0; j < K; ++j) r_pair[j] = r[j];
                            }
                        } else {
                            if (odd) {
#pragma unroll
                                for (int j = 0; j < K; ++j) r_pair[j] = r[j];
                            } else if (n == Nt) {
#pragma unroll
                                for (int j = 0; j < K; ++j) v[j] = T(0.5) * r[j];
                                st(dst, v);
                            } else {
#pragma unroll
                                for (int j = 0; j < K; ++j) v[j] = T(0.5) * (r[j] + r_pair[j]);
                                st(dst, v);
                            }
                        }
                    }
                } else if constexpr (TAIL == TAIL_NORM || TAIL == TAIL_DEFECT) {
                    if (out_row && useful) {
#pragma unroll
                        for (int j = 0; j < K; ++j) {
                            const double rv = (double)r[j];
                            acc = __builtin_fma(rv, rv, acc);
                        }
                    }
                    if constexpr (TAIL == TAIL_DEFECT && std::is_same<T, double>::value) {
                        if (out_row && useful && lane_in) {
                            const float2 f = make_float2((float)(r[0] * a.inv_s_new),
                                                         (float)(r[1] * a.inv_s_new));
                            *reinterpret_cast<float2*>(a.f32 + (int64_t)n * P + g) = f;
                        }
                    }
                }
            }
        }
        }
    };
    const bool special = TR ? (first == Nt || n0 == 0) : (first <= 1);
    if (!STMG_SPLIT_LOOP || special)
        stream(std::true_type{});
    else
        stream(std::false_type{});

    if constexpr (MID || TAIL == TAIL_NORM || TAIL == TAIL_DEFECT) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if (lane == 0) a.parts[wave] = acc;
    }
}

// Two entry points with the same body: the finest level gets its own symbol so that
// profiles attribute the dominant passes separately from the coarse levels.
template <typename T, int TR, int S1, int HEAD, int S2, int MID, int S3, int TAIL>
__global__ __launch_bounds__(256) void k_fused(LevelView<T> L, FusedArgs<T> a) {
    fused_body<T, TR, S1, HEAD, S2, MID, S3, TAIL>(L, a, grid_wave());
}
template <typename T, int TR, int S1, int HEAD, int S2, int MID, int S3, int TAIL>
__global__ __launch_bounds__(256) void k_fused_fine(LevelView<T> L, FusedArgs<T> a) {
    fused_body<T, TR, S1, HEAD, S2, MID, S3, TAIL>(L, a, grid_wave());
}

// ---------------------------------------------------------------------------------
// Mixed precision: the end of one FP32 inner cycle, the FP64 defect correction and the
// start of the next inner cycle in one streaming pass on the finest level.  Per row:
//   FP32  e = S steps from zero on f, + P z, S steps          (post-smoothing, with
//         the pre-smoothing recomputed: the inner cycle starts from e = 0)
//   FP64  u' = u + s_e e,  r = b - J u',  f' = r / s (FP32),  ||r||^2 partials
//   FP32  (PRE) S steps from zero on f', residual, restriction into bc
// Reads f, z (FP32), u, b (FP64); writes u', f' and bc: the FP32 correction e is never
// stored.  Lanes hold K = 2 columns (the FP64 layout; FP32 values as pairs).  Every
// value is computed by the operations of the separate passes, so the bits are those of
// the unfused mixed cycle.
struct MixedArgs {
    const float* e;      // FROM_E: the pre-smoothed FP32 iterate of the inner cycle that ends
    const float* f;      // FP32 right-hand side of the inner cycle that ends here
    const float* z;      // FP32 coarse correction, pitch Pz
    int64_t Pz;
    const double* u;     // FP64 iterate
    const double* b;     // FP64 right-hand side (b_const: two rows)
    int b_const;
    double* u_out;
    float* f_out;        // FP32 right-hand side of the next inner cycle
    float* bc;           // its restricted residual (PRE), pitch Pbc
    int64_t Pbc;
    int Nc;
    double s_e;          // scale of f (and so of e)
    double inv_s;        // 1 / scale of f'
    double* parts;
    int HL, xw, seg, nwaves;
};

template <int TR, int S, int HEAD, int PRE, int TAIL, int FROM_E, int PF = 2>
__device__ __forceinline__ void mixed_body(const LevelView<float>& L32, const LevelView<double>& L64,
                                           const MixedArgs& a, const int wave) {
    constexpr int K = 2;
    const int lane = threadIdx.x & (kWave - 1);
    if (wave >= a.nwaves) return;
    const int HL = a.HL;
    const int U = (kWave - 2 * HL) * K;
    const int wx = wave % a.xw;
    const int wt = wave / a.xw;
    const int g = wx * U - K * HL + K * lane;
    const bool useful = (lane >= HL) && (lane < kWave - HL);
    const bool lane_in = (g >= 0) && (g <= L64.N);
    const int N = L64.N, Nt = L64.Nt;
    const int64_t P = L64.P;

    bool valid[K];
#pragma unroll
    for (int j = 0; j < K; ++j) valid[j] = lane_in && (g + j <= N);
    LaneCoef<float, K> C32;
    LaneCoef<double, K> C64;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int c = g + j;
        const bool v = valid[j];
        C32.mlo[j] = v ? L32.mlo[c] : 0.0f;
        C32.mdi[j] = v ? L32.mdi[c] : 0.0f;
        C32.mup[j] = v ? L32.mup[c] : 0.0f;
        C32.kl[j] = v ? L32.kl[c] : 0.0f;
        C32.kr[j] = v ? L32.kr[c] : 0.0f;
        C32.wd[j] = v ? L32.wd[c] : 0.0f;
        C32.me[j] = (c == 0) ? 0.0f : 1.0f;
        C64.mlo[j] = v ? L64.mlo[c] : 0.0;
        C64.mdi[j] = v ? L64.mdi[c] : 0.0;
        C64.mup[j] = v ? L64.mup[c] : 0.0;
        C64.kl[j] = v ? L64.kl[c] : 0.0;
        C64.kr[j] = v ? L64.kr[c] : 0.0;
        C64.wd[j] = 0.0;
        C64.me[j] = (c == 0) ? 0.0 : 1.0;
    }

    const int rows = Nt + 1;
    const int n0 = wt * a.seg;
    const int n1 = min(rows, n0 + a.seg);
    constexpr int NA = FROM_E ? S : 2 * S;       // FP32 steps of the ending inner cycle
    constexpr int KH0 = FROM_E ? 0 : S;          // steps before its prolongation
    constexpr int NC = PRE ? S : 0;              // FP32 steps of the next one
    constexpr int WARM = NA + 1 + (PRE ? NC + 1 : 0);
    const int first = TR ? min(Nt, n1 - 1 + WARM) : max(0, n0 - WARM);
    const int count = TR ? (first - n0 + 1) : (n1 - first);

    constexpr int NS32 = NA + NC + (PRE ? 1 : 0);   // FP32 stage states
    float pa[NS32][K];
    double p64[K];
#pragma unroll
    for (int k = 0; k < NS32; ++k)
#pragma unroll
        for (int j = 0; j < K; ++j) pa[k][j] = 0.0f;
#pragma unroll
    for (int j = 0; j < K; ++j) p64[j] = 0.0;
    float r_pair[K] = {0.0f, 0.0f};
    double acc = 0.0;

    constexpr int KZ = HEAD == 1 ? 1 : K;
    constexpr int KE = FROM_E ? K : 1;
    float rf[PF][K], rz[PF][KZ], re[PF][KE];
    double ru[PF][K], rb[PF][K];
    auto fetch = [&](int n, float (&ff)[K], float (&fz)[KZ], float (&fe)[KE], double (&fu)[K],
                     double (&fb)[K]) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            ff[j] = 0.0f;
            fu[j] = 0.0;
            fb[j] = 0.0;
        }
#pragma unroll
        for (int j = 0; j < KE; ++j) fe[j] = 0.0f;
#pragma unroll
        for (int j = 0; j < KZ; ++j) fz[j] = 0.0f;
        if (!lane_in) return;
        const int64_t ro = (int64_t)n * P + g;
        const float2 fv = *reinterpret_cast<const float2*>(a.f + ro);
        ff[0] = fv.x;
        ff[1] = fv.y;
        if constexpr (FROM_E) {
            const float2 ev = *reinterpret_cast<const float2*>(a.e + ro);
            fe[0] = ev.x;
            fe[1] = ev.y;
        }
        if constexpr (HEAD == 1) {
            fz[0] = a.z[(int64_t)n * a.Pz + (g >> 1)];
        } else {
            const float2 zv = *reinterpret_cast<const float2*>(a.z + (int64_t)(n >> 1) * a.Pz + g);
            fz[0] = zv.x;
            fz[1] = zv.y;
        }
        ld(a.u + ro, fu);
        ld(a.b + (a.b_const ? (n > 0 ? P : 0) : (int64_t)n * P) + g, fb);
    };
    auto row_of = [&](int it) { return TR ? first - it : first + it; };
#pragma unroll
    for (int d = 0; d < PF; ++d)
        if (d < count) fetch(row_of(d), rf[d], rz[d], re[d], ru[d], rb[d]);

    // the loop in two copies, as in fused_body: with and without the tests for the
    // Dirichlet row and the rows without time coupling
    auto stream = [&](auto special_tag) {
        constexpr bool SPECIAL = decltype(special_tag)::value;
        for (int it0 = 0; it0 < count; it0 += PF) {
#pragma unroll
        for (int d = 0; d < PF; ++d) {
            const int it = it0 + d;
            if (it >= count) break;
            const int n = row_of(it);
            float fr[K], zz[KZ], ee[KE];
            double uu[K], bb[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                fr[j] = rf[d][j];
                uu[j] = ru[d][j];
                bb[j] = rb[d][j];
            }
#pragma unroll
            for (int j = 0; j < KZ; ++j) zz[j] = rz[d][j];
#pragma unroll
            for (int j = 0; j < KE; ++j) ee[j] = re[d][j];
            if (it + PF < count) fetch(row_of(it + PF), rf[d], rz[d], re[d], ru[d], rb[d]);
            const bool out_row = (n >= n0) && (n < n1);
            const bool dir_row = SPECIAL && (n == 0);
            const bool coupled = !SPECIAL || (TR ? (n < Nt) : (n >= 2));
            if (SPECIAL && !coupled) {
#pragma unroll
                for (int k = 0; k < NS32; ++k)
#pragma unroll
                    for (int j = 0; j < K; ++j) pa[k][j] = 0.0f;
#pragma unroll
                for (int j = 0; j < K; ++j) p64[j] = 0.0;
            }
            double r64[K];
            float rc[K], fn[K];
            auto chain = [&](auto dir_tag) {
                constexpr bool DIR = decltype(dir_tag)::value;
                // ending inner cycle: S steps from zero (or its stored pre-smoothed iterate),
                // prolongation, S steps
                float x[K] = {0.0f, 0.0f};
                if constexpr (FROM_E) {
#pragma unroll
                    for (int j = 0; j < K; ++j) x[j] = ee[j];
                }
#pragma unroll
                for (int k = 0; k <= NA; ++k) {
                    if (k == KH0) {
                        if constexpr (HEAD == 1) {
                            const float znext = shfl_dn1(zz[0]);
                            x[0] += zz[0];
                            x[1] = fmaT(0.5f, zz[0] + znext, x[1]);
                        } else {
                            x[0] += zz[0];
                            x[1] += zz[1];
                        }
#pragma unroll
                        for (int j = 0; j < K; ++j) x[j] = valid[j] ? x[j] : 0.0f;
                    }
                    if (k == NA) break;
                    float y[K];
                    row_step<float, K, true, DIR>(L32, C32, x, pa[k], fr, y);
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        pa[k][j] = x[j];
                        x[j] = y[j];
                    }
                }
                // FP64 defect correction
                double xu[K];
#pragma unroll
                for (int j = 0; j < K; ++j) xu[j] = valid[j] ? fmaT(a.s_e, (double)x[j], uu[j]) : 0.0;
                if (out_row && useful && lane_in) st(a.u_out + (int64_t)n * P + g, xu);
                row_step<double, K, false, DIR>(L64, C64, xu, p64, bb, r64);
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    p64[j] = xu[j];
                    fn[j] = (float)(r64[j] * a.inv_s);
                }
                if constexpr (PRE) {
                    // next inner cycle: S steps from zero on f', residual
                    float w[K] = {0.0f, 0.0f};
#pragma unroll
                    for (int k = NA; k < NA + NC; ++k) {
                        float y[K];
                        row_step<float, K, true, DIR>(L32, C32, w, pa[k], fn, y);
#pragma unroll
                        for (int j = 0; j < K; ++j) {
                            pa[k][j] = w[j];
                            w[j] = y[j];
                        }
                    }
                    row_step<float, K, false, DIR>(L32, C32, w, pa[NA + NC], fn, rc);
#pragma unroll
                    for (int j = 0; j < K; ++j) pa[NA + NC][j] = w[j];
                }
            };
            if constexpr (SPECIAL) {
                if (dir_row)
                    chain(std::true_type{});
                else
                    chain(std::false_type{});
            } else {
                chain(std::false_type{});
            }
            if (out_row && useful) {
#pragma unroll
                for (int j = 0; j < K; ++j) acc = __builtin_fma(r64[j], r64[j], acc);
            }
            if (out_row && useful && lane_in)
                *reinterpret_cast<float2*>(a.f_out + (int64_t)n * P + g) = make_float2(fn[0], fn[1]);
            if constexpr (PRE && TAIL == TAIL_RX) {
                // coarse node g/2: r_{2I} + 1/2 (r_{2I-1} + r_{2I+1})
                const float rl = shfl_up1(rc[K - 1]);
                if (out_row && useful && lane_in) {
                    const int I0 = g >> 1;
                    if (I0 <= a.Nc) a.bc[(int64_t)n * a.Pbc + I0] = fmaT(0.5f, rl + rc[1], rc[0]);
                }
            } else if constexpr (PRE && TAIL == TAIL_RT) {
                if (out_row && useful && lane_in) {
                    const bool odd = (n & 1) != 0;
                    float* dst = a.bc + (int64_t)(n >> 1) * a.Pbc + g;
                    float v[K];
                    bool put = true;
                    if (!TR) {
                        if (odd) {
                            for (int j = 0; j < K; ++j) v[j] = 0.5f * (r_pair[j] + rc[j]);
                        } else if (n == Nt) {
                            for (int j = 0; j < K; ++j) v[j] = 0.5f * rc[j];
                        } else {
                            for (int j = 0; j < K; ++j) r_pair[j] = rc[j];
                            put = false;
                        }
                    } else {
                        if (odd) {
                            for (int j = 0; j < K; ++j) r_pair[j] = rc[j];
                            put = false;
                        } else if (n == Nt) {
                            for (int j = 0; j < K; ++j) v[j] = 0.5f * rc[j];
                        } else {
                            for (int j = 0; j < K; ++j) v[j] = 0.5f * (rc[j] + r_pair[j]);
                        }
                    }
                    if (put) *reinterpret_cast<float2*>(dst) = make_float2(v[0], v[1]);
                }
            }
        }
        }
    };
    const bool special = TR ? (first == Nt || n0 == 0) : (first <= 1);
    if (!STMG_SPLIT_LOOP || special)
        stream(std::true_type{});
    else
        stream(std::false_type{});
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if (lane == 0) a.parts[wave] = acc;
}

template <int TR, int S, int HEAD, int PRE, int TAIL, int FROM_E>
__global__ __launch_bounds__(256) void k_mixed_fine(LevelView<float> L32, LevelView<double> L64,
                                                    MixedArgs a) {
    mixed_body<TR, S, HEAD, PRE, TAIL, FROM_E>(L32, L64, a, grid_wave());
}

struct Geometry {
    int HL, U, xw, seg, nwaves;
};

// even_seg: segments of an even number of time levels (a t restriction pairs the levels
// 2J, 2J+1 inside one wave's segment).  Other passes on levels small enough that even
// the shortest even segments leave SIMDs idle take single-level segments: each wave then
// walks one row fewer of its serial chain, which is what bounds those launches.
template <typename T>
Geometry geometry(int N, int Nt, int sweeps, bool fine, bool even_seg = true) {
    constexpr int K = Lanes<T>::K;
    Geometry G;
    // Halo lanes: ceil((S+2)/K), rounded up so that the useful strip of every wave is
    // a whole number of 128-byte lines; then no two waves write the same line.
    constexpr int lanes_per_line = 128 / (K * (int)sizeof(T));
    const int align = lanes_per_line / 2 > 0 ? lanes_per_line / 2 : 1;
    G.HL = (sweeps + 2 + K - 1) / K;
    if (STMG_ALIGN_HALO) G.HL = (G.HL + align - 1) / align * align;
    G.U = (kWave - 2 * G.HL) * K;
    G.xw = (N + 1 + G.U - 1) / G.U;
    const int64_t rows = Nt + 1;
    // Enough waves to keep every SIMD busy several times over.  Passes of four or
    // more sweeps on levels that the 256 MB Infinity Cache holds are bound by their
    // arithmetic, not by memory latency: they get fewer, longer time segments, which
    // cuts the recomputed warm-up rows; fewer still on the coarse levels, whose passes
    // share the GPU with the other levels' latency-bound launches (measured: 2048 waves
    // there against 3072 on the finest level).  Levels whose vectors exceed the cache
    // stream from HBM whatever the chain, and keep the many-wave target.
    const bool hbm = (double)rows * (N + 1) * sizeof(T) > STMG_BIG_LEVEL_BYTES;
    const int64_t target = (sweeps < 4 || hbm) ? STMG_TARGET_WAVES
                           : (fine ? STMG_TARGET_WAVES_ALU : STMG_TARGET_WAVES_ALU_COARSE);
    int64_t seg = (rows * G.xw + target - 1) / target;
    const int64_t min_seg = STMG_MIN_SEGMENT;
    if (seg < min_seg) seg = min_seg;
    if (seg > 1024) seg = 1024;
    if (seg & 1) ++seg;
    if (!even_seg && seg == 2 && G.xw * ((rows + 1) / 2) <= STMG_SINGLE_ROW_MAX_WAVES) seg = 1;
    G.seg = (int)seg;
    G.nwaves = (int)(G.xw * ((rows + G.seg - 1) / G.seg));
    return G;
}

// Launch options: the finest level has kernels of its own; non-null events are recorded
// at the kernel's own start and end (the dispatch timestamps a profiler reads), so a
// timing excludes the wait for compute units held by other streams' kernels.
struct LaunchCfg {
    bool fine;
    hipEvent_t start;
    hipEvent_t stop;
};

template <typename T, int TR, int S1, int HEAD, int S2, int MID, int S3, int TAIL>
void launch_one(const LevelView<T>& L, const FusedArgs<T>& a, const LaunchCfg& lc, hipStream_t s) {
    const int blocks = (a.nwaves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (lc.fine && lc.start)
        hipExtLaunchKernelGGL((k_fused_fine<T, TR, S1, HEAD, S2, MID, S3, TAIL>), dim3(blocks),
                              dim3(kWave * kWavesPerBlock), 0, s, lc.start, lc.stop, 0, L, a);
    else if (lc.fine)
        hipLaunchKernelGGL((k_fused_fine<T, TR, S1, HEAD, S2, MID, S3, TAIL>), dim3(blocks),
                           dim3(kWave * kWavesPerBlock), 0, s, L, a);
    else
        hipLaunchKernelGGL((k_fused<T, TR, S1, HEAD, S2, MID, S3, TAIL>), dim3(blocks),
                           dim3(kWave * kWavesPerBlock), 0, s, L, a);
}

// Plain passes: S steps, then a restriction, norm or no tail (pre-smoothing), or a
// prolongation head, then S steps and a norm or no tail (post-smoothing).
template <typename T, int TR, int S>
void dispatch_plain(int tail, const LevelView<T>& L, const FusedArgs<T>& a, const LaunchCfg& lc,
                    hipStream_t s) {
    if (a.head == 1) {
        if (tail == TAIL_NORM)
            launch_one<T, TR, 0, 1, S, 0, 0, TAIL_NORM>(L, a, lc, s);
        else
            launch_one<T, TR, 0, 1, S, 0, 0, TAIL_NONE>(L, a, lc, s);
        return;
    }
    if (a.head == 2) {
        if (tail == TAIL_NORM)
            launch_one<T, TR, 0, 2, S, 0, 0, TAIL_NORM>(L, a, lc, s);
        else
            launch_one<T, TR, 0, 2, S, 0, 0, TAIL_NONE>(L, a, lc, s);
        return;
    }
    switch (tail) {
        case TAIL_NONE: launch_one<T, TR, 0, 0, S, 0, 0, TAIL_NONE>(L, a, lc, s); break;
        case TAIL_RX: launch_one<T, TR, 0, 0, S, 0, 0, TAIL_RX>(L, a, lc, s); break;
        case TAIL_RT: launch_one<T, TR, 0, 0, S, 0, 0, TAIL_RT>(L, a, lc, s); break;
        default: launch_one<T, TR, 0, 0, S, 0, 0, TAIL_NORM>(L, a, lc, s); break;
    }
}

template <typename T, int TR>
void dispatch_sweeps(int S, int tail, const LevelView<T>& L, const FusedArgs<T>& a,
                     const LaunchCfg& lc, hipStream_t s) {
    switch (S) {
        case 0: dispatch_plain<T, TR, 0>(tail, L, a, lc, s); break;
        case 1: dispatch_plain<T, TR, 1>(tail, L, a, lc, s); break;
        case 2: dispatch_plain<T, TR, 2>(tail, L, a, lc, s); break;
        case 3: dispatch_plain<T, TR, 3>(tail, L, a, lc, s); break;
        case 4: dispatch_plain<T, TR, 4>(tail, L, a, lc, s); break;
        case 5: dispatch_plain<T, TR, 5>(tail, L, a, lc, s); break;
        default: dispatch_plain<T, TR, 6>(tail, L, a, lc, s); break;
    }
}

// Pre-smoothing of a coarse level from a zero start, its residual and restriction: the S
// steps run as a chain from zero (S1 = S), whose first step needs no stencil and no
// previous row.  Coarse levels only (k_fused).
template <typename T, int TR, int S>
void launch_zero_pre(int tail, const LevelView<T>& L, const FusedArgs<T>& a, hipStream_t s) {
    const dim3 grid((a.nwaves + kWavesPerBlock - 1) / kWavesPerBlock), block(kWave * kWavesPerBlock);
    if (tail == TAIL_RX)
        hipLaunchKernelGGL((k_fused<T, TR, S, 0, 0, 0, 0, TAIL_RX>), grid, block, 0, s, L, a);
    else
        hipLaunchKernelGGL((k_fused<T, TR, S, 0, 0, 0, 0, TAIL_RT>), grid, block, 0, s, L, a);
}

template <typename T, int TR>
void dispatch_zero_pre(int S, int tail, const LevelView<T>& L, const FusedArgs<T>& a, hipStream_t s) {
    switch (S) {
        case 1: launch_zero_pre<T, TR, 1>(tail, L, a, s); break;
        case 2: launch_zero_pre<T, TR, 2>(tail, L, a, s); break;
        case 3: launch_zero_pre<T, TR, 3>(tail, L, a, s); break;
        case 4: launch_zero_pre<T, TR, 4>(tail, L, a, s); break;
        case 5: launch_zero_pre<T, TR, 5>(tail, L, a, s); break;
        default: launch_zero_pre<T, TR, 6>(tail, L, a, s); break;
    }
}

// Post-smoothing from a zero start that first redoes the S pre-smoothing steps (from
// zero, on the level's own b) instead of reading their stored result.
template <typename T, int TR>
void dispatch_recompute(int S, const LevelView<T>& L, const FusedArgs<T>& a, const LaunchCfg& lc,
                        hipStream_t s) {
#define STMG_RECOMPUTE(SS)                                                             \
    if (a.head == 1) launch_one<T, TR, SS, 1, SS, 0, 0, TAIL_NONE>(L, a, lc, s);     \
    else launch_one<T, TR, SS, 2, SS, 0, 0, TAIL_NONE>(L, a, lc, s);
    switch (S) {
        case 1: STMG_RECOMPUTE(1) break;
        case 2: STMG_RECOMPUTE(2) break;
        default: STMG_RECOMPUTE(3) break;
    }
#undef STMG_RECOMPUTE
}

// The end of one V-cycle and the start of the next in one pass on the finest level:
// prolongation of the coarse correction, S post-smoothing steps (MID: the cycle's
// iterate stored, its residual norm summed), S pre-smoothing steps of the next cycle,
// their residual restricted.
template <int TR>
void dispatch_cycle(int S, int tail, const LevelView<double>& L, const FusedArgs<double>& a,
                    const LaunchCfg& lc, hipStream_t s) {
#define STMG_CYCLE(SS)                                                                          \
    if (a.head == 1) {                                                                          \
        if (tail == TAIL_RX) launch_one<double, TR, 0, 1, SS, 1, SS, TAIL_RX>(L, a, lc, s);     \
        else launch_one<double, TR, 0, 1, SS, 1, SS, TAIL_RT>(L, a, lc, s);                     \
    } else {                                                                                    \
        if (tail == TAIL_RX) launch_one<double, TR, 0, 2, SS, 1, SS, TAIL_RX>(L, a, lc, s);     \
        else launch_one<double, TR, 0, 2, SS, 1, SS, TAIL_RT>(L, a, lc, s);                     \
    }
    switch (S) {
        case 1: STMG_CYCLE(1) break;
        case 2: STMG_CYCLE(2) break;
        default: STMG_CYCLE(3) break;
    }
#undef STMG_CYCLE
}

// Two V-cycles meet on a level that starts from zero: the post-smoothing of the first
// (its pre-smoothing recomputed, the prolongation between), then the pre-smoothing of
// the second from that iterate, which is stored, and its restricted residual.
template <typename T, int TR>
void dispatch_cycle_zero(int S, int tail, const LevelView<T>& L, const FusedArgs<T>& a,
                         const LaunchCfg& lc, hipStream_t s) {
#define STMG_CYCLE0(SS)                                                                        \
    if (a.head == 1) {                                                                         \
        if (tail == TAIL_RX) launch_one<T, TR, SS, 1, SS, 0, SS, TAIL_RX>(L, a, lc, s);        \
        else launch_one<T, TR, SS, 1, SS, 0, SS, TAIL_RT>(L, a, lc, s);                        \
    } else {                                                                                   \
        if (tail == TAIL_RX) launch_one<T, TR, SS, 2, SS, 0, SS, TAIL_RX>(L, a, lc, s);        \
        else launch_one<T, TR, SS, 2, SS, 0, SS, TAIL_RT>(L, a, lc, s);                        \
    }
    if (S == 1) {
        STMG_CYCLE0(1)
    } else {
        STMG_CYCLE0(2)
    }
#undef STMG_CYCLE0
}

// Two FP32 inner cycles meet on the finest level of a mixed-precision solve, the first
// from a stored pre-smoothed iterate: its prolongation and S post-smoothing steps, then
// the S pre-smoothing steps of the next inner cycle, which are stored, and their
// restricted residual.
template <int TR>
void dispatch_join(int S, int tail, const LevelView<float>& L, const FusedArgs<float>& a,
                   const LaunchCfg& lc, hipStream_t s) {
#define STMG_JOIN(SS)                                                                          \
    if (a.head == 1) {                                                                         \
        if (tail == TAIL_RX) launch_one<float, TR, 0, 1, SS, 0, SS, TAIL_RX>(L, a, lc, s);     \
        else launch_one<float, TR, 0, 1, SS, 0, SS, TAIL_RT>(L, a, lc, s);                     \
    } else {                                                                                   \
        if (tail == TAIL_RX) launch_one<float, TR, 0, 2, SS, 0, SS, TAIL_RX>(L, a, lc, s);     \
        else launch_one<float, TR, 0, 2, SS, 0, SS, TAIL_RT>(L, a, lc, s);                     \
    }
    if (S == 1) {
        STMG_JOIN(1)
    } else {
        STMG_JOIN(2)
    }
#undef STMG_JOIN
}

}  // namespace

int fused_max_sweeps() { return kMaxFused; }
int fused_max_chain_sweeps() { return kMaxChain; }

int fused_geometry(int N, int Nt, int sweeps, bool fp32, bool fine, int* strip_cols, int* strips,
                   int* seg_rows, int* waves) {
    if (sweeps < 0 || sweeps > kMaxFused) return -1;
    const Geometry G = fp32 ? geometry<float>(N, Nt, sweeps, fine) : geometry<double>(N, Nt, sweeps, fine);
    *strip_cols = G.U;
    *strips = G.xw;
    *seg_rows = G.seg;
    *waves = G.nwaves;
    return 0;
}

int fused_parts(int N, int Nt, int sweeps) {
    // the FP32 geometry (wider lanes) never needs more waves than the FP64 one, and
    // odd segments never fewer
    return geometry<double>(N, Nt, sweeps, true, false).nwaves;
}

template <typename T>
int launch_fused(const LevelView<T>& L, const FusedPass& fp, const T* u, const T* b, T* out,
                 hipStream_t s) {
    const int S1 = fp.pre_sweeps, S2 = fp.sweeps, S3 = fp.next_sweeps;
    if (S1 < 0 || S2 < 0 || S3 < 0 || S2 > kMaxFused) return -1;
    const int chain = S1 + S2 + S3;
    const bool cyc = fp.mid_norm != 0;
    const bool cyc0 = S1 > 0 && S3 > 0;    // two zero-start cycles meet (no MID)
    const bool recompute = S1 > 0 && S3 == 0;
    const bool join = S1 == 0 && S3 > 0 && !cyc;   // two FP32 inner cycles meet
    if (join) {
        if (!std::is_same<T, float>::value || S2 != S3 || S2 > kMaxMixedSweeps || fp.zero_in ||
            (fp.prolong != 'x' && fp.prolong != 't') || (fp.tail != 'x' && fp.tail != 't'))
            return -1;
    } else if (cyc || recompute || cyc0) {
        // the chain passes: S1 = S2 (recompute), S2 = S3 with MID (cycle) or
        // S1 = S2 = S3 (cycle from zero); x / t head
        if (chain > kMaxChain || (fp.prolong != 'x' && fp.prolong != 't')) return -1;
        if (recompute && (cyc || S2 != S1 || fp.tail != 0 || !fp.zero_in)) return -1;
        if (cyc && (S1 != 0 || S2 != S3 || S2 < 1 || (fp.tail != 'x' && fp.tail != 't') ||
                    !std::is_same<T, double>::value))
            return -1;
        if (cyc0 && (cyc || S2 != S1 || S3 != S1 || S1 > 2 || !fp.zero_in ||
                     (fp.tail != 'x' && fp.tail != 't')))
            return -1;
    } else if (S3 != 0) {
        return -1;
    }
    Geometry G = geometry<T>(L.N, L.Nt, chain, fp.fine != 0, fp.tail == 't');
    FusedArgs<T> a;
    a.u = u;
    a.b = b;
    a.out = out;
    a.mid = static_cast<T*>(fp.mid);
    a.z = static_cast<const T*>(fp.z);
    a.Pz = fp.Pz;
    a.bc = static_cast<T*>(fp.bc);
    a.Pbc = fp.Pbc;
    a.parts = fp.parts;
    a.Nc = fp.Nc;
    a.head = fp.prolong == 'x' ? 1 : (fp.prolong == 't' ? 2 : (fp.prolong == 'c' ? 3 : 0));
    a.zero_in = fp.zero_in;
    a.b_const = fp.b_const;
    a.e32 = fp.e32;
    a.s_old = fp.s_old;
    a.f32 = fp.f32;
    a.inv_s_new = fp.inv_s_new;
    a.HL = G.HL;
    a.xw = G.xw;
    a.seg = G.seg;
    a.nwaves = G.nwaves;
    const LaunchCfg lc{fp.fine != 0, fp.ev_start, fp.ev_stop};
    const int tail = fp.tail == 'x' ? TAIL_RX
                     : (fp.tail == 't' ? TAIL_RT : (fp.tail == 'n' ? TAIL_NORM : TAIL_NONE));
    if (recompute) {
        if (fp.trans) dispatch_recompute<T, 1>(S1, L, a, lc, s);
        else dispatch_recompute<T, 0>(S1, L, a, lc, s);
        return G.nwaves;
    }
    if (cyc0) {
        if (fp.trans) dispatch_cycle_zero<T, 1>(S1, tail, L, a, lc, s);
        else dispatch_cycle_zero<T, 0>(S1, tail, L, a, lc, s);
        return G.nwaves;
    }
    if (join) {
        if constexpr (std::is_same<T, float>::value) {
            if (fp.trans) dispatch_join<1>(S2, tail, L, a, lc, s);
            else dispatch_join<0>(S2, tail, L, a, lc, s);
        }
        return G.nwaves;
    }
    if (cyc) {
        if constexpr (std::is_same<T, double>::value) {
            if (fp.trans) dispatch_cycle<1>(S2, tail, L, a, lc, s);
            else dispatch_cycle<0>(S2, tail, L, a, lc, s);
        }
        return G.nwaves;
    }
    if (fp.tail == 'c' || fp.prolong == 'c') {
        // defect correction (FP64 only): u += s_old e; r = b - J u; f = r / s_new; norm.
        // Without the head ('c' tail alone) u is taken as it is: the first step of a
        // solve, which must not read a correction left by an earlier solve.
        if constexpr (std::is_same<T, double>::value) {
            if (S2 != 0 || fp.tail != 'c' || (fp.prolong != 'c' && fp.prolong != 0)) return -1;
            if (fp.prolong == 'c') {
                if (fp.trans)
                    launch_one<T, 1, 0, 3, 0, 0, 0, TAIL_DEFECT>(L, a, lc, s);
                else
                    launch_one<T, 0, 0, 3, 0, 0, 0, TAIL_DEFECT>(L, a, lc, s);
            } else {
                if (fp.trans)
                    launch_one<T, 1, 0, 0, 0, 0, 0, TAIL_DEFECT>(L, a, lc, s);
                else
                    launch_one<T, 0, 0, 0, 0, 0, 0, TAIL_DEFECT>(L, a, lc, s);
            }
            return G.nwaves;
        } else {
            return -1;
        }
    }
    if (STMG_ZERO_FIRST && fp.zero_in && a.head == 0 && S2 > 0 && !fp.fine &&
        (tail == TAIL_RX || tail == TAIL_RT)) {
        if (fp.trans) dispatch_zero_pre<T, 1>(S2, tail, L, a, s);
        else dispatch_zero_pre<T, 0>(S2, tail, L, a, s);
        return G.nwaves;
    }
    if (fp.trans)
        dispatch_sweeps<T, 1>(S2, tail, L, a, lc, s);
    else
        dispatch_sweeps<T, 0>(S2, tail, L, a, lc, s);
    return G.nwaves;
}

int mixed_chain_sweeps(int S, bool from_e) { return (from_e ? 2 : 3) * S + 2; }
int mixed_max_sweeps() { return kMaxMixedSweeps; }

int launch_mixed(const LevelView<float>& L32, const LevelView<double>& L64, const MixedPass& mp,
                 hipStream_t s) {
    const int S = mp.sweeps;
    if (S < 1 || S > kMaxMixedSweeps || (mp.prolong != 'x' && mp.prolong != 't')) return -1;
    if (mp.pre && mp.tail != 'x' && mp.tail != 't') return -1;
    const bool from_e = mp.e != nullptr;
    const Geometry G = geometry<double>(L64.N, L64.Nt, mixed_chain_sweeps(S, from_e), true);
    MixedArgs a;
    a.e = mp.e;
    a.f = mp.f;
    a.z = mp.z;
    a.Pz = mp.Pz;
    a.u = mp.u;
    a.b = mp.b;
    a.b_const = mp.b_const;
    a.u_out = mp.u_out;
    a.f_out = mp.f_out;
    a.bc = mp.bc;
    a.Pbc = mp.Pbc;
    a.Nc = mp.Nc;
    a.s_e = mp.s_e;
    a.inv_s = mp.inv_s;
    a.parts = mp.parts;
    a.HL = G.HL;
    a.xw = G.xw;
    a.seg = G.seg;
    a.nwaves = G.nwaves;
    const int blocks = (a.nwaves + kWavesPerBlock - 1) / kWavesPerBlock;
    const dim3 grid(blocks), block(kWave * kWavesPerBlock);
    const int head = mp.prolong == 'x' ? 1 : 2;
    const int tail = mp.tail == 'x' ? TAIL_RX : TAIL_RT;
#define STMG_MIXED_LAUNCH1(TR_, S_, H_, P_, T_, E_)                                             \
    do {                                                                                       \
        if (mp.ev_start)                                                                       \
            hipExtLaunchKernelGGL((k_mixed_fine<TR_, S_, H_, P_, T_, E_>), grid, block, 0, s,  \
                                  mp.ev_start, mp.ev_stop, 0, L32, L64, a);                     \
        else                                                                                   \
            hipLaunchKernelGGL((k_mixed_fine<TR_, S_, H_, P_, T_, E_>), grid, block, 0, s,     \
                               L32, L64, a);                                                   \
    } while (0)
#define STMG_MIXED_LAUNCH(TR_, S_, H_, P_, T_)                                                  \
    do {                                                                                       \
        if (from_e) STMG_MIXED_LAUNCH1(TR_, S_, H_, P_, T_, 1);                                 \
        else STMG_MIXED_LAUNCH1(TR_, S_, H_, P_, T_, 0);                                        \
    } while (0)
#define STMG_MIXED_TAIL(TR_, S_, H_)                                                            \
    do {                                                                                       \
        if (!mp.pre) STMG_MIXED_LAUNCH(TR_, S_, H_, 0, TAIL_NONE);                             \
        else if (tail == TAIL_RX) STMG_MIXED_LAUNCH(TR_, S_, H_, 1, TAIL_RX);                  \
        else STMG_MIXED_LAUNCH(TR_, S_, H_, 1, TAIL_RT);                                        \
    } while (0)
#define STMG_MIXED_HEAD(TR_, S_)                                                                \
    do {                                                                                       \
        if (head == 1) STMG_MIXED_TAIL(TR_, S_, 1);                                            \
        else STMG_MIXED_TAIL(TR_, S_, 2);                                                      \
    } while (0)
    if (mp.trans) {
        if (S == 1) STMG_MIXED_HEAD(1, 1);
        else STMG_MIXED_HEAD(1, 2);
    } else {
        if (S == 1) STMG_MIXED_HEAD(0, 1);
        else STMG_MIXED_HEAD(0, 2);
    }
#undef STMG_MIXED_HEAD
#undef STMG_MIXED_TAIL
#undef STMG_MIXED_LAUNCH
#undef STMG_MIXED_LAUNCH1
    return G.nwaves;
}

template int launch_fused<double>(const LevelView<double>&, const FusedPass&, const double*,
                                  const double*, double*, hipStream_t);
template int launch_fused<float>(const LevelView<float>&, const FusedPass&, const float*,
                                 const float*, float*, hipStream_t);

}  // namespace stmg
