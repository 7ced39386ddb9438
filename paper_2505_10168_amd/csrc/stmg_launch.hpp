// Host-side launch wrappers of the STMG kernels (internal to libstmg).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stmg_device.hpp"

namespace stmg {

// Operator modes of the one-thread-per-DOF kernel.
enum ApplyMode { APPLY_J = 0, APPLY_RESIDUAL = 1, APPLY_JACOBI = 2 };

// ---- setup (Section 2.1, Section 5.1, Appendix A) ---------------------------------
void launch_simp(const double* rho, int n, double v_ins, double v_con, double p, double* out,
                 hipStream_t s);
void launch_simp_derivative(const double* rho, int n, double v_ins, double v_con, double p,
                            double* out, hipStream_t s);
// method: 0 = R (resistivity), 1 = K (conductivity), 2 = D (design field + SIMP)
void launch_coarsen_x(const double* k, const double* c, const double* chi, int n_coarse,
                      int method, const double* simp_params, double* kc, double* cc,
                      double* chic, hipStream_t s);
// out[0] = min_e k_e/c_e, out[1] = max_e k_e/c_e, out[2] = max_e c_e, out[3] = max_e k_e
void launch_level_stats(const double* k, const double* c, int n, double* out, hipStream_t s);
// coef: 9 arrays of N+1 doubles (lo, di, up, mlo, mdi, mup, wd, kl, kr); coef32: FP32 copy
void launch_stencil_coef(const double* k, const double* c, int N, double h, double tau,
                         double omega, double W, double* coef, float* coef32, hipStream_t s);
void launch_thomas_factors(const double* coef, int N, double* cp, double* inv, hipStream_t s);
void launch_load_vector(const double* q, double q0, int N, int Nt, double h, double* b,
                        int64_t P, hipStream_t s);

// ---- data movement ------------------------------------------------------------------
template <typename T>
void launch_fill(T* x, int64_t n, T v, hipStream_t s);
// x[r*P + c] = v for r < rows, c < cols (columns beyond cols, the padding, untouched)
template <typename T>
void launch_fill2d(T* x, int64_t P, int rows, int cols, T v, hipStream_t s);
// dst[r*dp + c] = (Tout)(scale * src[r*sp + c]) for r < rows, c < cols
template <typename Tin, typename Tout>
void launch_copy2d(const Tin* src, int64_t sp, Tout* dst, int64_t dp, int rows, int cols,
                   double scale, hipStream_t s);
// dst += scale * src (2-D, FP64 destination)
template <typename Tin>
void launch_axpy2d(const Tin* src, int64_t sp, double* dst, int64_t dp, int rows, int cols,
                   double scale, hipStream_t s);

// ---- reference (one thread per DOF) kernels -----------------------------------------
template <typename T>
void launch_apply(const LevelView<T>& L, int trans, int mode, const T* x, const T* b, T* y,
                  bool zero_in, hipStream_t s);
// interp: 0 = causal (C), 1 = bilinear in time (B); only t transfers differ
template <typename T>
void launch_restrict(char dir, const LevelView<T>& F, const T* r, T* bc, int64_t Pc,
                     hipStream_t s, int interp);
template <typename T>
void launch_prolong_add(char dir, const LevelView<T>& F, const T* z, int64_t Pc, T* u,
                        hipStream_t s, int interp);
// Exact coarsest solve (time stepping + Thomas) in FP64 on vectors of type TV.
template <typename TV>
void launch_coarsest(const LevelView<double>& L, const double* cp, const double* inv,
                     const TV* b, TV* u, int trans, hipStream_t s);

// Coarsest levels with N <= kDenseCoarsestMax: A^{-1} built once, applied per step.
constexpr int kDenseCoarsestMax = 64;
void launch_dense_inverse(const double* coef, int N, const double* cp, const double* inv,
                          double* ainv, hipStream_t s);
template <typename TV>
void launch_coarsest_dense(const LevelView<double>& L, const double* ainv, const TV* b, TV* u,
                           int trans, hipStream_t s);

// ---- reductions (deterministic: fixed partition, fixed tree) ------------------------
int reduce_parts(int rows);
template <typename T>
void launch_sumsq_partial(const T* x, int rows, int cols, int64_t P, double* parts,
                          hipStream_t s);
void launch_dot_partial(const double* a, const double* b, int rows, int cols, int64_t Pa,
                        int64_t Pb, double* parts, hipStream_t s);
// out[0] = scale * sum(parts[0..n))
void launch_reduce_final(const double* parts, int n, double scale, double* out, hipStream_t s);
// host[0] = scale * sum(parts[0..n)), then host[1] = tag; host is pinned host memory
void launch_reduce_to_host(const double* parts, int n, double scale, double* host, double tag,
                           hipStream_t s);
// residual norm^2 of the fine level, one-thread-per-DOF: parts from b - J u
template <typename T>
void launch_residual_sumsq_partial(const LevelView<T>& L, int trans, const T* u, const T* b,
                                   double* parts, hipStream_t s);

// ---- sensitivities (Section 7) -------------------------------------------------------
int gradient_chunks(int Nt);
void launch_gradient_partial(const double* u, const double* lam, int N, int Nt, int64_t Pu,
                             int64_t Pl, const double* kp, const double* cp, double h,
                             double tau, double* parts, hipStream_t s);
void launch_gradient_final(const double* parts, int N, int chunks, double* grad,
                           hipStream_t s);
// optimality-criteria design update (one workgroup); chi_new may alias chi
void launch_oc_update(const double* chi, const double* grad, int n, double volume, double move,
                      double eta, double chi_min, double* chi_new, hipStream_t s);

// ---- Galerkin levels (P reassembly): stored 9-point stencils ---------------------------
// 10 arrays of E = R P doubles (R stored rows of P); array 3 (dt+1) + (dx+1) holds at
// (row[n], i) the coefficient of x(n+dt, i+dx) in row (n, i), array 9 the Jacobi scale
// omega / J_ii
template <typename C>
struct StencilViewT {
    int N;
    int Nt;
    int64_t P;
    int R;           // stored rows
    int64_t E;       // R P
    const int* row;  // Nt+1 entries: time level -> stored row
    const C* s;      // coefficients (FP64, or their FP32 copy for the FP32 inner cycles)
};
using StencilView = StencilViewT<double>;
// widest coarsest stencil level the time-stepping solve takes (nodes per time level)
constexpr int kStencilCoarsestMaxNodes = 1024;
// cs = stored rows of R J P for the level below F (shape C, representative time level
// crep[r] for stored row r): from F's rediscretised operator when fsv is null, else from
// F's stored stencil
void launch_galerkin(const LevelView<double>& F, const StencilView* fsv, char dir, int interp,
                     const StencilView& C, const int* crep, double omega, double* cs,
                     hipStream_t s);
template <typename T>
void launch_apply_stencil(const StencilViewT<T>& S, int trans, int mode, const T* x, const T* b,
                          T* y, bool zero_in, hipStream_t s);
// `sweeps` (1..kStencilMaxFused) damped Jacobi steps in one streaming pass, u -> out
// (distinct buffers); the same values as the prolongation, `sweeps` launches of
// launch_apply_stencil, the residual and the restriction launched one after the other
constexpr int kStencilMaxFused = 6;
template <typename T>
struct StencilPass {
    int trans;
    int sweeps;
    const T* u;
    const T* b;
    T* out;
    int zero_in;
    char head;          // 0, 'x' or 't': add P z (coarse pitch Pz) to u first
    const T* z;
    int64_t Pz;
    char restrict_dir;  // 'x' / 't': also write R (b - J out) (causal interpolation) to
    T* bc;              // this coarse vector (Nc elements, pitch Pbc); not with a head
    int64_t Pbc;
    int Nc;
};
// -1 (nothing launched) for sweeps outside 1..kStencilMaxFused, another restriction
// direction or a head with a restriction
template <typename T>
int launch_stencil_fused(const StencilViewT<T>& V, const StencilPass<T>& p, hipStream_t s);
// exact solve of a stencil level with couplings to the next time level (bilinear
// interpolation): band LU with partial pivoting of the dense n x n operator,
// n = (N+1)(Nt+1) <= kStencilLuMax; A: n*n doubles, piv: n ints, scratch: n doubles
constexpr int kStencilLuMax = 16384;
void launch_stencil_lu(const StencilView& S, int trans, double* A, int* piv, hipStream_t s);
// FP64 arithmetic; vectors of type TV
template <typename TV>
void launch_stencil_lu_solve(const StencilView& S, const double* A, const int* piv, const TV* b,
                             TV* z, double* scratch, hipStream_t s);
// factors: 4 arrays of E doubles (cp, inv of J's blocks, then of J^T's), per stored row
void launch_stencil_thomas(const StencilView& S, double* factors, hipStream_t s);
// FP64 arithmetic; vectors of type TV
template <typename TV>
void launch_stencil_coarsest(const StencilView& S, const double* factors, int trans, const TV* b,
                             TV* z, hipStream_t s);
// coarsest stencil levels of at most kStencilDenseMaxNodes nodes per time level: inv gets
// the inverse of every stored row's tridiagonal block (R arrays of (N+1)^2 doubles,
// row-major), formed column by column from the Thomas factors of J
constexpr int kStencilDenseMaxNodes = 64;
void launch_stencil_block_inverse(const StencilView& S, const double* factors, double* inv,
                                  hipStream_t s);
// the same exact solve as launch_stencil_coarsest with those inverses, in one wave;
// FP64 arithmetic, vectors of type TV
template <typename TV>
void launch_stencil_coarsest_dense(const StencilView& S, const double* inv, int trans,
                                   const TV* b, TV* z, hipStream_t s);

// ---- fused streaming kernels ----------------------------------------------------------
// Pass descriptor of one fused streaming launch on a level.
// One streaming pass: pre_sweeps Jacobi steps, the prolongation head, `sweeps` steps,
// optionally the MID stage (iterate stored to `mid`, its residual norm into parts),
// next_sweeps steps, the result stored to `out` (unless null), the tail.  Besides the
// plain passes (pre_sweeps = next_sweeps = 0, no MID) two chains are instantiated, for
// 1..3 steps: recompute (zero_in, pre_sweeps = sweeps, x/t head, no tail) and cycle
// (FP64, mid_norm, sweeps = next_sweeps, x/t head, x/t tail).
struct FusedPass {
    int trans;          // 0: J, 1: J^T (streams backwards in time)
    int sweeps;         // Jacobi steps after the head (0..fused_max_sweeps())
    int pre_sweeps;     // steps before the head
    int next_sweeps;    // steps after the MID stage
    int mid_norm;       // MID stage: residual norm of the iterate after `sweeps` steps
    void* mid;          // and that iterate stored here (type T, level pitch) unless null
    int zero_in;        // input u is identically zero (not read)
    int b_const;        // b holds two rows: zeros (time level 0) and every later level
    char prolong;       // 0, 'x' or 't': add P z to the input first; 'c': u += s_old e32
    const void* z;      // coarse correction (type T), pitch Pz
    int64_t Pz;
    int Nc;             // coarse elements (prolong/restrict)
    int Ntc;            // coarse steps
    char tail;          // 0: none, 'x'/'t': residual + restriction, 'n': residual norm,
                        // 'c': residual norm and f32 = r * inv_s_new (with prolong 'c')
    void* bc;           // restricted residual output (type T), pitch Pbc
    int64_t Pbc;
    double* parts;      // norm partials ('n')
    int fine;           // finest level: launched under its own kernel symbol
    const float* e32;   // 'c': FP32 correction
    double s_old;       // 'c': its scale
    float* f32;         // 'c': FP32 scaled residual output
    double inv_s_new;
    hipEvent_t ev_start;  // finest level, non-null: recorded at the kernel's own start and end
    hipEvent_t ev_stop;
};
template <typename T>
int launch_fused(const LevelView<T>& L, const FusedPass& fp, const T* u, const T* b, T* out,
                 hipStream_t s);
// The fused mixed-precision pass of the finest level: the FP32 post-smoothing of the
// inner cycle that ends (its pre-smoothing recomputed from zero), the FP64 defect
// correction u' = u + s_e e, r = b - J u', f' = r inv_s (FP32) with the norm partials,
// and (pre) the FP32 pre-smoothing of the next inner cycle with its restricted residual.
struct MixedPass {
    int trans;
    int sweeps;           // steps per smoothing (1..mixed_max_sweeps())
    char prolong;         // 'x' / 't': direction of the finest coarsening
    const float* e;       // non-null: the ending inner cycle's stored pre-smoothed iterate
                          // (it started from a previous one); null: from zero, recomputed
    const float* f;
    const float* z;
    int64_t Pz;
    const double* u;
    const double* b;
    int b_const;
    double* u_out;
    float* f_out;
    int pre;              // also pre-smooth the next inner cycle and restrict
    char tail;            // its restriction direction ('x' / 't')
    float* bc;
    int64_t Pbc;
    int Nc;
    double s_e;
    double inv_s;
    double* parts;
    hipEvent_t ev_start;  // non-null: recorded at the kernel's own start and end
    hipEvent_t ev_stop;
};
int launch_mixed(const LevelView<float>& L32, const LevelView<double>& L64, const MixedPass& mp,
                 hipStream_t s);
int mixed_chain_sweeps(int S, bool from_e);   // chain length the pass's geometry is sized for
int mixed_max_sweeps();
// y = a (b null) or y = a + s b over n FP64 values (n even), 16-byte accesses;
// -1 for an odd or too large n
int launch_stream(const double* a, const double* b, double s, double* y, int64_t n, bool nt,
                  hipStream_t st);
// launch geometry of a fused pass: columns per strip, strips, time levels per
// segment, wavefronts (-1 for an unsupported sweep count)
int fused_geometry(int N, int Nt, int sweeps, bool fp32, bool fine, int* strip_cols, int* strips,
                   int* seg_rows, int* waves);
int fused_parts(int N, int Nt, int sweeps);
int fused_max_sweeps();
int fused_max_chain_sweeps();

// ---- single-workgroup V-cycle tail (the smallest levels, resident in LDS) -----------
constexpr int kTailThreads = 1024;     // one workgroup
constexpr int kTailMaxLevels = 8;      // levels l_s .. coarsest
#ifndef STMG_TAIL_MAX_ROWS
#define STMG_TAIL_MAX_ROWS 4
#endif
constexpr int kTailMaxRows = STMG_TAIL_MAX_ROWS;   // time rows per thread and level
constexpr int kTailMaxCoarsestN = 32;  // A^{-1} rows held in registers
template <typename T>
struct TailLaunch {
    LevelView<T> V[kTailMaxLevels];    // index 0 = l_s, last = coarsest
    int dir[kTailMaxLevels];           // 'x' / 't' towards the next level
    int nlev;
    int nu;
    int trans;
    int lds_bytes;                     // dynamic LDS made available by tail_prepare
    LevelView<double> Vc;              // coarsest level, FP64 coefficients
    const double* ainv;
    const T* b_in;                     // restricted right-hand side of level l_s
    int64_t P_in;
    T* u_out;                          // its coarse-grid correction
    int64_t P_out;
};
// time rows per thread on a level (it must not exceed kTailMaxRows); even when the
// level restricts in t
int tail_rows_per_owner(int N, int Nt, bool even);
// LDS bytes of u and b of the given levels
template <typename T>
int tail_lds_bytes(const int* N, const int* Nt, int nlev);
// allows lds_bytes of dynamic LDS for the kernels of a coarsest level with N nodes;
// -1 when the device or the coarsest level does not allow it
template <typename T>
int tail_prepare(int lds_bytes, int coarsest_n);
// -1 (nothing launched) when the levels do not fit the kernel's limits
template <typename T>
int launch_vcycle_tail(const TailLaunch<T>& t, hipStream_t s);

}  // namespace stmg
