// Host side of libstmg: level hierarchy (Algorithms 3/4, Section 5.1), V-cycle
// driver (Algorithm 1), FP64 and mixed-precision solve loops with the termination
// rule of Section 3.1, objective and gradient (Section 7), and the C ABI of stmg.h.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <type_traits>
#include <utility>
#include <array>
#include <atomic>
#include <mutex>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "stmg.h"
#include "stmg_launch.hpp"

using namespace stmg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                       \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess)                                                           \
            return fail(STMG_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));     \
    } while (0)

#define CHK(x)                     \
    do {                           \
        int rc_ = (x);             \
        if (rc_ < 0) return rc_;   \
    } while (0)

constexpr int kCoefArrays = 9;   // lo, di, up, mlo, mdi, mup, wd, kl, kr
constexpr int kStencilRowsBound = 8;   // footprint bound of stored Galerkin stencil rows

int64_t pitch_for(int N) { return ((int64_t)N + 4 + 31) / 32 * 32; }
int64_t dofs_of(int N, int Nt) { return (int64_t)(N + 1) * (Nt + 1); }

struct Level {
    int N = 0, Nt = 0;
    int64_t P = 0;
    double h = 0, tau = 0, W = 0;
    char dir = 0;            // direction that builds the next level ('x' / 't'); 0 = coarsest
    double lambda = 0;
    double* k = nullptr;
    double* c = nullptr;
    double* chi = nullptr;
    double* coef = nullptr;  // kCoefArrays (N+1)
    float* coef32 = nullptr;
    double* thomas = nullptr;  // coarsest: cp, inv, rhs scratch (3 (N+1))
    double* ainv = nullptr;    // coarsest with N <= kDenseCoarsestMax: A^{-1}, N x N
    double* sten = nullptr;    // Galerkin levels: 9-point stencil and Jacobi scale, 10 arrays of R rows of P
    float* sten32 = nullptr;   // and its FP32 copy for the FP32 inner cycles
    double* sfac = nullptr;    // coarsest Galerkin level: Thomas factors, 4 arrays of R P
    double* sinv = nullptr;    // and, up to kStencilDenseMaxNodes nodes, its blocks' inverses (R (N+1)^2)
    double* lu = nullptr;      // coarsest bilinear Galerkin level: LU factors of J, J^T (2 n^2)
    int* piv = nullptr;        // and their interchanges (2 n)
    double* lux = nullptr;     // and the FP64 work vector of their solves (n)
    int R = 0;                 // stored stencil rows
    int* srow = nullptr;       // device: time level -> stored row (Nt+1)
    int* srep = nullptr;       // device: stored row -> its representative time level (R)
    std::vector<int> hrow, hrep;   // host copies
    double* u = nullptr;
    double* b = nullptr;
    double* t = nullptr;
    double* w = nullptr;     // fine level, pipelined solves: keeps the previous iterate
    double* v = nullptr;     // fine level, chained solves: fourth vector of the rotation
    float* u32 = nullptr;
    float* b32 = nullptr;
    float* t32 = nullptr;
    int64_t elems() const { return (int64_t)(Nt + 1) * P; }
    int64_t dofs() const { return dofs_of(N, Nt); }
};

StencilView stencil_view(const Level& l) {
    return StencilView{l.N, l.Nt, l.P, l.R, (int64_t)l.R * l.P, l.srow, l.sten};
}
// the stored stencil in the vector type of a cycle
template <typename T>
StencilViewT<T> sview(const Level& l) {
    if constexpr (std::is_same<T, double>::value) return stencil_view(l);
    else return StencilViewT<float>{l.N, l.Nt, l.P, l.R, (int64_t)l.R * l.P, l.srow, l.sten32};
}

// Stored-row classes of a Galerkin level.  A coarse row's stencil is fixed by the
// stored rows of the fine rows it is formed from and by which of its neighbours fall
// outside the grid; time levels with the same such signature get exactly equal
// stencils and share one stored row.  The rediscretised fine level has three classes:
// time level 0 (Dirichlet), 1 (no coupling to level 0) and the rest.
void stencil_rows(const std::vector<int>& frow, int Nt, char dir, int interp, std::vector<int>& row,
                  std::vector<int>& rep) {
    const int Ntc = dir == 't' ? Nt / 2 : Nt;
    std::vector<std::array<int, 6>> sigs;
    row.assign(Ntc + 1, 0);
    rep.clear();
    for (int J = 0; J <= Ntc; ++J) {
        std::array<int, 6> sig;
        if (dir == 't' && interp == STMG_INTERP_B)   // fine rows 2J-1, 2J, 2J+1
            sig = {J >= 1 ? frow[2 * J - 1] : -1, frow[2 * J], 2 * J + 1 <= Nt ? frow[2 * J + 1] : -1,
                   J == 0, 2 * J + 1 > Nt, 2 * J + 2 > Nt};
        else if (dir == 't')                         // fine rows 2J, 2J+1
            sig = {frow[2 * J], 2 * J + 1 <= Nt ? frow[2 * J + 1] : -1, -1, J == 0, 2 * J + 2 > Nt, 0};
        else
            sig = {frow[J], -1, -1, J == 0, J == Ntc, 0};
        size_t r = 0;
        while (r < sigs.size() && sigs[r] != sig) ++r;
        if (r == sigs.size()) {
            sigs.push_back(sig);
            rep.push_back(J);
        }
        row[J] = (int)r;
    }
}

template <typename T> T*& U(Level& l);
template <typename T> T*& B(Level& l);
template <typename T> T*& Tt(Level& l);
template <> double*& U<double>(Level& l) { return l.u; }
template <> double*& B<double>(Level& l) { return l.b; }
template <> double*& Tt<double>(Level& l) { return l.t; }
template <> float*& U<float>(Level& l) { return l.u32; }
template <> float*& B<float>(Level& l) { return l.b32; }
template <> float*& Tt<float>(Level& l) { return l.t32; }

template <typename T>
LevelView<T> view(const Level& l, double omega);

template <>
LevelView<double> view<double>(const Level& l, double omega) {
    LevelView<double> v;
    const int64_t S = l.N + 1;
    v.N = l.N; v.Nt = l.Nt; v.P = l.P;
    v.lo = l.coef; v.di = l.coef + S; v.up = l.coef + 2 * S;
    v.mlo = l.coef + 3 * S; v.mdi = l.coef + 4 * S; v.mup = l.coef + 5 * S;
    v.wd = l.coef + 6 * S;
    v.kl = l.coef + 7 * S; v.kr = l.coef + 8 * S;
    v.W = l.W;
    v.wW = omega / l.W;
    return v;
}

template <>
LevelView<float> view<float>(const Level& l, double omega) {
    LevelView<float> v;
    const int64_t S = l.N + 1;
    v.N = l.N; v.Nt = l.Nt; v.P = l.P;
    v.lo = l.coef32; v.di = l.coef32 + S; v.up = l.coef32 + 2 * S;
    v.mlo = l.coef32 + 3 * S; v.mdi = l.coef32 + 4 * S; v.mup = l.coef32 + 5 * S;
    v.wd = l.coef32 + 6 * S;
    v.kl = l.coef32 + 7 * S; v.kr = l.coef32 + 8 * S;
    v.W = (float)l.W;
    v.wW = (float)(omega / l.W);
    return v;
}

// Bytes of the fine-level fused passes that the event timer records (algorithmic:
// every vector read or written once per pass).
struct KernelTimer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<double> bytes;
    size_t used = 0;
};

// Level-by-level device time of the sampled cycles: an event is recorded on the stream
// at every level boundary, tagged with the level whose work follows it (-1: none, the
// end of a cycle); the interval up to the next event belongs to that level.
struct LevelTimer {
    std::vector<hipEvent_t> ev;
    std::vector<int> tag;
    size_t used = 0;
    bool on = false;       // the current cycle is sampled
    int64_t seen = 0;      // cycles started in this solve
    int cycles = 0;        // of them sampled
};

// roctx range names, one pair per level ("stmg L3 pre", "stmg L3 post")
const char* level_range(int l, bool post) {
    static const auto names = [] {
        std::vector<std::string> v;
        for (int i = 0; i < 64; ++i) {
            v.push_back("stmg L" + std::to_string(i) + " pre");
            v.push_back("stmg L" + std::to_string(i) + " post");
        }
        return v;
    }();
    if (l < 0 || l >= 64) return "stmg level";
    return names[2 * l + (post ? 1 : 0)].c_str();
}

// a roctx range over a scope (a no-op unless a profiler collects markers)
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

}  // namespace

struct stmg_ctx {
    stmg_problem p{};
    stmg_options o{};
    hipStream_t s = nullptr;
    std::vector<Level> L;
    double* bload = nullptr;     // fine load vector b (Section 2.2)
    double* brow = nullptr;      // uniform load: its rows 0 (zeros) and 1, the same for n >= 1
    double* brow_adj = nullptr;  // the same scaled by dt / Theta_ref (adjoint right-hand side)
    const double* bfine = nullptr;   // during a solve: the two rows the fine passes read
    bool b_const = false;        // during a solve: the fine right-hand side is bfine
    double* rho = nullptr;       // current densities
    double* kp = nullptr;        // dk/drho
    double* cpd = nullptr;       // dc/drho
    double* simp = nullptr;      // device {k_ins, k_con, p_k, c_ins, c_con, p_c}
    double* stats = nullptr;     // device scratch for level stats (4 doubles)
    double* dscal = nullptr;     // device scalars
    double* hscal = nullptr;     // host scalars: pinned when possible, else pageable
    bool hscal_pinned = false;
    double* parts = nullptr;
    int64_t nparts = 0;
    std::vector<void*> allocs;
    size_t bytes = 0;
    KernelTimer timer;
    LevelTimer lt;
    int tail_start = -1;         // first level of the single-workgroup tail (-1: none)
    bool rotate_in = false;      // the next fine pass keeps its input in L[0].w
    uint64_t vcycles = 0;        // fine-level V-cycles started (sampled kernel timing)
    int tail_lds = 0;            // its dynamic LDS bytes (FP64 vectors: an upper bound)
    int norm_parts = 0;          // partial count written by the last fused norm
    double setup_ms = 0;         // wall time of the last build or re-assembly
    double bload_norm = -1;      // ||assembled load||, computed on first use
    int64_t fine_passes = 0;     // finest-level fused passes of the current solve

    ~stmg_ctx() {
        for (void* q : allocs) (void)hipFree(q);
        if (hscal && hscal_pinned) (void)hipHostFree(hscal);
        else delete[] hscal;
        for (auto& e : timer.ev) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        for (hipEvent_t e : lt.ev) (void)hipEventDestroy(e);
    }

    template <typename T>
    int alloc(T** out, int64_t n) {
        if (n <= 0) n = 1;
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, (size_t)n * sizeof(T));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(STMG_ENOMEM, "hipMalloc of " + std::to_string((size_t)n * sizeof(T)) +
                                         " bytes failed");
        }
        allocs.push_back(q);
        bytes += (size_t)n * sizeof(T);
        e = hipMemsetAsync(q, 0, (size_t)n * sizeof(T), s);
        if (e != hipSuccess) return fail(STMG_EHIP, "hipMemsetAsync failed");
        *out = static_cast<T*>(q);
        return 0;
    }
};

namespace {

// ------------------------------------------------------------------------------------
// Validation and footprint
// ------------------------------------------------------------------------------------

int validate(const stmg_problem* p, const stmg_options* o) {
    if (!p || !o) return fail(STMG_EINVAL, "null problem or options");
    if (p->n_el < 1 || p->n_t < 1) return fail(STMG_EINVAL, "n_el and n_t must be >= 1");
    if ((int64_t)p->n_el > (1 << 24) || (int64_t)p->n_t > (1 << 26))
        return fail(STMG_EINVAL, "grid too large");
    if (!(p->length > 0) || !(p->t_final > 0)) return fail(STMG_EINVAL, "length and t_final must be > 0");
    if (!(p->k_ins > 0) || !(p->k_con > 0) || !(p->c_ins > 0) || !(p->c_con > 0))
        return fail(STMG_EINVAL, "material constants must be > 0");
    if (!(p->theta_ref > 0)) return fail(STMG_EINVAL, "theta_ref must be > 0");
    if (p->field_kind != STMG_FIELD_DENSITY && p->field_kind != STMG_FIELD_CONDUCTIVITY)
        return fail(STMG_EINVAL, "unknown field_kind");
    if (!std::isfinite(p->q_uniform)) return fail(STMG_EINVAL, "q_uniform must be finite");
    if (o->nu < 0 || o->nu > 64) return fail(STMG_EINVAL, "nu must be in [0, 64]");
    if (!(o->omega > 0)) return fail(STMG_EINVAL, "omega must be > 0");
    if (o->max_levels < 0 || o->max_levels > 64) return fail(STMG_EINVAL, "max_levels must be in [0, 64]");
    if (o->min_coarse_dofs < 1) return fail(STMG_EINVAL, "min_coarse_dofs must be >= 1");
    if (o->max_cycles < 1 || o->max_cycles > STMG_MAX_HISTORY)
        return fail(STMG_EINVAL, "max_cycles must be in [1, STMG_MAX_HISTORY]");
    if (o->reassembly < 0 || o->reassembly > 3) return fail(STMG_EINVAL, "unknown reassembly method");
    if (o->deff_mode < 0 || o->deff_mode > 1) return fail(STMG_EINVAL, "unknown deff_mode");
    if (o->precision != STMG_FP64 && o->precision != STMG_MIXED)
        return fail(STMG_EINVAL, "unknown precision");
    if (o->fused < 0 || o->fused > 2) return fail(STMG_EINVAL, "fused must be 0, 1 or 2");
    if (o->time_kernels < 0) return fail(STMG_EINVAL, "time_kernels must be >= 0");
    if (o->interp != STMG_INTERP_C && o->interp != STMG_INTERP_B)
        return fail(STMG_EINVAL, "unknown interpolation");
    if (!(o->tol > 0) || !(o->diverge > 0)) return fail(STMG_EINVAL, "tol and diverge must be > 0");
    if (o->debug_poison != 0 && o->debug_poison != 1) return fail(STMG_EINVAL, "debug_poison must be 0 or 1");
    if (o->precision == STMG_MIXED && (o->inner_cycles < 1 || o->inner_cycles > 8))
        return fail(STMG_EINVAL, "inner_cycles must be in [1, 8]");
    if (o->time_levels < 0) return fail(STMG_EINVAL, "time_levels must be >= 0");
    if (p->field_kind == STMG_FIELD_CONDUCTIVITY &&
        (o->reassembly == STMG_REASSEMBLE_D || o->deff_mode == 1))
        return fail(STMG_EINVAL, "a conductivity field has no design densities: reassembly D and "
                                 "deff_mode 1 need field_kind = STMG_FIELD_DENSITY");
    return 0;
}

bool can_x(int N) { return N % 2 == 0 && N >= 2; }
bool can_t(int Nt) { return Nt % 2 == 0 && Nt >= 2; }

// Bytes a level of (N, Nt) holds for the given precision and position.
// pipelined: the fine level of an FP64 handle with streaming kernels keeps a third
// vector, so that one V-cycle can run while the previous one's residual is checked
bool pipelined_options(const stmg_options* o) { return o->precision == STMG_FP64 && o->fused != 0; }

size_t level_bytes(int N, int Nt, int precision, bool fine, bool coarsest, bool pipelined,
                   bool galerkin, bool bilinear = false) {
    const int64_t P = pitch_for(N), E = (int64_t)(Nt + 1) * P;
    size_t b = 3 * (size_t)N * 8 + kCoefArrays * (size_t)(N + 1) * 8;
    // stored stencil rows: at most kStencilRowsBound (3 or 4 in practice)
    if (galerkin && !fine) {
        const size_t rows = (size_t)std::min(Nt + 1, kStencilRowsBound) * P;
        b += (10 + (coarsest ? 4 : 0)) * rows * 8 + (size_t)(Nt + 1 + kStencilRowsBound) * 4;
        if (precision == STMG_MIXED) b += 10 * rows * 4;   // FP32 copy of the stencil
    }
    if (galerkin && !bilinear && coarsest && !fine && N + 1 <= kStencilDenseMaxNodes)
        b += (size_t)kStencilRowsBound * (N + 1) * (N + 1) * 8;   // block inverses
    if (galerkin && bilinear && coarsest && !fine) {
        const size_t n = (size_t)(N + 1) * (Nt + 1);
        if (n <= (size_t)kStencilLuMax) b += 2 * n * n * 8 + 2 * n * 4 + n * 8;
    }
    if (precision == STMG_MIXED) b += kCoefArrays * (size_t)(N + 1) * 4;
    if (coarsest) b += 3 * (size_t)(N + 1) * 8 + (N <= kDenseCoarsestMax ? (size_t)N * N * 8 : 0);
    if (precision == STMG_FP64 || fine) b += 3 * (size_t)E * 8;
    if (precision == STMG_MIXED) b += 3 * (size_t)E * 4;
    if (fine && pipelined) b += 2 * (size_t)E * 8;
    return b;
}

// Footprint of a handle.  Directions are not known without the field (deff_mode 0),
// so for every level count the largest grid any x/t sequence can produce is used.
size_t footprint_of(const stmg_problem* p, const stmg_options* o) {
    const int N0 = p->n_el, T0 = p->n_t;
    size_t total = 0;
    const int fine_parts = 1 << 20;
    total += (size_t)(T0 + 1) * pitch_for(N0) * 8;   // bload
    total += 4 * (size_t)pitch_for(N0) * 8;            // its two rows, forward and adjoint
    total += (size_t)N0 * 8 * 4 + 64 + 4096;          // rho, kp, cpd, scalars
    total += (size_t)fine_parts * 8;
    if (o->deff_mode == 1) {
        const double deff = std::sqrt((p->k_ins / p->c_ins) * (p->k_con / p->c_con));
        int N = N0, Nt = T0, lev = 1;
        double h = p->length / N0, tau = p->t_final / T0;
        while (true) {
            bool last;
            char want = 0;
            if (o->max_levels) last = (lev == o->max_levels);
            else last = dofs_of(N, Nt) <= o->min_coarse_dofs;
            if (!last) {
                double lam = deff * tau / (h * h);
                want = lam < o->lambda_crit ? 't' : 'x';
                if (o->M_min_elems && N / 2.0 < o->M_min_elems) want = 't';
                if (want == 'x' && !can_x(N)) want = can_t(Nt) ? 't' : 0;
                else if (want == 't' && !can_t(Nt)) want = can_x(N) ? 'x' : 0;
                if (!want) last = true;
            }
            total += level_bytes(N, Nt, o->precision, lev == 1, last, pipelined_options(o),
                                 o->reassembly == STMG_REASSEMBLE_P, o->interp == STMG_INTERP_B);
            if (last) break;
            if (want == 'x') { N /= 2; h *= 2; } else { Nt /= 2; tau *= 2; }
            ++lev;
        }
        return total;
    }
    // field-dependent path: bound each level by the largest (N, Nt) of any path
    struct S { int N, Nt; };
    std::vector<S> frontier{{N0, T0}};
    int lev = 1;
    while (!frontier.empty() && lev <= 64) {
        size_t worst = 0;
        std::vector<S> next;
        bool any_continue = false;
        for (auto& f : frontier) {
            bool last = o->max_levels ? (lev == o->max_levels) : (dofs_of(f.N, f.Nt) <= o->min_coarse_dofs);
            if (!last && !can_x(f.N) && !can_t(f.Nt)) last = true;
            worst = std::max(worst, level_bytes(f.N, f.Nt, o->precision, lev == 1, true,
                                                pipelined_options(o),
                                                o->reassembly == STMG_REASSEMBLE_P,
                                                o->interp == STMG_INTERP_B));
            if (!last) {
                any_continue = true;
                if (can_x(f.N)) next.push_back({f.N / 2, f.Nt});
                if (can_t(f.Nt)) next.push_back({f.N, f.Nt / 2});
            }
        }
        total += worst;
        if (!any_continue) break;
        // keep the frontier small: distinct (N, Nt) pairs only
        std::vector<S> uniq;
        for (auto& q : next) {
            bool seen = false;
            for (auto& w : uniq) seen |= (w.N == q.N && w.Nt == q.Nt);
            if (!seen) uniq.push_back(q);
        }
        frontier.swap(uniq);
        ++lev;
    }
    return total;
}

// ------------------------------------------------------------------------------------
// Setup
// ------------------------------------------------------------------------------------

int fetch_stats(stmg_ctx* h, const Level& l, double out[4]) {
    launch_level_stats(l.k, l.c, l.N, h->stats, h->s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h->hscal, h->stats, 4 * sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    for (int i = 0; i < 4; ++i) out[i] = h->hscal[i];
    return 0;
}

// The fine level's element statistics must describe a positive, finite material.
int check_material(const double st[4]) {
    if (!(st[0] > 0) || !std::isfinite(st[1]) || !std::isfinite(st[3]) || !(st[2] > 0))
        return fail(STMG_EINVAL, "conductivities and heat capacities must be positive and finite");
    return 0;
}

double level_w(const stmg_options& o, const Level& l, const double st[4]) {
    if (o.w_diri_override > 0) return o.w_diri_override;
    // W_Diri = max_e c_e dx/dt + max_e k_e / dx  (Appendix A)
    return st[2] * l.h / l.tau + st[3] / l.h;
}

// Fills k, c, chi of level 0 and the field derivatives of k and c from the field:
// densities through SIMP (Section 2.1), or conductivities with c = c_con (then
// dk/dfield = 1 and dc/dfield = 0).
int level0_material(stmg_ctx* h) {
    Level& f = h->L[0];
    const stmg_problem& p = h->p;
    HIPCHK(hipMemcpyAsync(f.chi, h->rho, (size_t)f.N * 8, hipMemcpyDeviceToDevice, h->s));
    if (p.field_kind == STMG_FIELD_CONDUCTIVITY) {
        HIPCHK(hipMemcpyAsync(f.k, h->rho, (size_t)f.N * 8, hipMemcpyDeviceToDevice, h->s));
        launch_fill<double>(f.c, f.N, p.c_con, h->s);
        launch_fill<double>(h->kp, f.N, 1.0, h->s);
        launch_fill<double>(h->cpd, f.N, 0.0, h->s);
        HIPCHK(hipGetLastError());
        return 0;
    }
    launch_simp(h->rho, f.N, p.k_ins, p.k_con, p.p_k, f.k, h->s);
    launch_simp(h->rho, f.N, p.c_ins, p.c_con, p.p_c, f.c, h->s);
    launch_simp_derivative(h->rho, f.N, p.k_ins, p.k_con, p.p_k, h->kp, h->s);
    launch_simp_derivative(h->rho, f.N, p.c_ins, p.c_con, p.p_c, h->cpd, h->s);
    HIPCHK(hipGetLastError());
    return 0;
}

// Direction leaving level `cur` (Algorithm 3; Algorithm 4 guard; Section 7.2 D_eff).
char choose_direction(const stmg_ctx* h, const Level& cur, const double st[4], double* lam_out) {
    const stmg_options& o = h->o;
    const stmg_problem& p = h->p;
    double lam;
    if (o.deff_mode == 1) {
        const double deff = std::sqrt((p.k_ins / p.c_ins) * (p.k_con / p.c_con));
        lam = deff * cur.tau / (cur.h * cur.h);
    } else {
        lam = std::sqrt(st[0] * st[1]) * cur.tau / (cur.h * cur.h);
    }
    *lam_out = lam;
    char want = lam < o.lambda_crit ? 't' : 'x';
    if (o.M_min_elems && cur.N / 2.0 < o.M_min_elems) want = 't';
    if (want == 'x' && !can_x(cur.N)) want = can_t(cur.Nt) ? 't' : 0;
    else if (want == 't' && !can_t(cur.Nt)) want = can_x(cur.N) ? 'x' : 0;
    return want;
}

bool is_last(const stmg_ctx* h, size_t nlev, const Level& cur) {
    if (h->o.max_levels) return (int)nlev == h->o.max_levels;
    return cur.dofs() <= h->o.min_coarse_dofs;
}

int coarse_coefficients(stmg_ctx* h, const Level& f, char dir, Level& c) {
    if (dir == 't') {
        HIPCHK(hipMemcpyAsync(c.k, f.k, (size_t)f.N * 8, hipMemcpyDeviceToDevice, h->s));
        HIPCHK(hipMemcpyAsync(c.c, f.c, (size_t)f.N * 8, hipMemcpyDeviceToDevice, h->s));
        HIPCHK(hipMemcpyAsync(c.chi, f.chi, (size_t)f.N * 8, hipMemcpyDeviceToDevice, h->s));
        return 0;
    }
    // P keeps K-averaged k and c as the proxy that steers the coarsening decision
    const int method = h->o.reassembly == STMG_REASSEMBLE_R ? 0 : (h->o.reassembly == STMG_REASSEMBLE_D ? 2 : 1);
    launch_coarsen_x(f.k, f.c, f.chi, c.N, method, h->simp, c.k, c.c, c.chi, h->s);
    HIPCHK(hipGetLastError());
    return 0;
}

int finish_level(stmg_ctx* h, Level& l, bool coarsest) {
    launch_stencil_coef(l.k, l.c, l.N, l.h, l.tau, h->o.omega, l.W, l.coef, l.coef32, h->s);
    if (coarsest) {
        launch_thomas_factors(l.coef, l.N, l.thomas, l.thomas + (l.N + 1), h->s);
        if (l.ainv)
            launch_dense_inverse(l.coef, l.N, l.thomas, l.thomas + (l.N + 1), l.ainv, h->s);
    }
    HIPCHK(hipGetLastError());
    return 0;
}

// The lowest levels that one workgroup solves with u and b in LDS: the longest chain
// l_s .. coarsest (l_s >= 1) whose FP64 vectors fit the device's LDS per workgroup and
// whose levels fit the kernel's thread mapping.  Sets tail_start = -1 when no chain
// of at least two levels qualifies.
void plan_tail(stmg_ctx* h) {
    h->tail_start = -1;
    if (h->o.interp != STMG_INTERP_C) return;   // the tail kernel transfers causally
    if (h->o.reassembly == STMG_REASSEMBLE_P) return;   // it rediscretises every level
    const int nl = (int)h->L.size();
    const Level& c = h->L[nl - 1];
    if (nl < 3 || !c.ainv || c.N > kTailMaxCoarsestN) return;
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    int best = -1, best_bytes = 0;
    for (int s0 = nl - 2; s0 >= 1 && nl - s0 <= kTailMaxLevels; --s0) {
        const Level& l = h->L[s0];
        if (tail_rows_per_owner(l.N, l.Nt, l.dir == 't') > kTailMaxRows) break;
        int N[kTailMaxLevels], Nt[kTailMaxLevels];
        for (int j = s0; j < nl; ++j) {
            N[j - s0] = h->L[j].N;
            Nt[j - s0] = h->L[j].Nt;
        }
        const int bytes = tail_lds_bytes<double>(N, Nt, nl - s0);
        if (bytes > lds_max) break;
        best = s0;
        best_bytes = bytes;
    }
    if (best < 0) return;
    if (tail_prepare<double>(best_bytes, c.N) != 0 || tail_prepare<float>(best_bytes, c.N) != 0) return;
    h->tail_start = best;
    h->tail_lds = best_bytes;
}

// Galerkin operators of levels 1 .. coarsest (Section 5.1, P method), each from the
// level above, and the time-stepping factors of the coarsest one.
int galerkin_levels(stmg_ctx* h) {
    const size_t nl = h->L.size();
    for (size_t i = 0; i + 1 < nl; ++i) {
        const Level& f = h->L[i];
        Level& c = h->L[i + 1];
        const StencilView fs = stencil_view(f);
        launch_galerkin(view<double>(f, h->o.omega), i == 0 ? nullptr : &fs, f.dir, h->o.interp,
                        stencil_view(c), c.srep, h->o.omega, c.sten, h->s);
        if (c.sten32)
            launch_copy2d<double, float>(c.sten, c.P, c.sten32, c.P, 10 * c.R, c.N + 1, 1.0, h->s);
    }
    if (nl > 1) {
        Level& c = h->L[nl - 1];
        if (c.lu) {
            const int64_t n = c.dofs();
            launch_stencil_lu(stencil_view(c), 0, c.lu, c.piv, h->s);
            launch_stencil_lu(stencil_view(c), 1, c.lu + n * n, c.piv + n, h->s);
        } else {
            launch_stencil_thomas(stencil_view(c), c.sfac, h->s);
            if (c.sinv) launch_stencil_block_inverse(stencil_view(c), c.sfac, c.sinv, h->s);
        }
    }
    HIPCHK(hipGetLastError());
    return 0;
}

int build(stmg_ctx* h, const double* d_q) {
    const stmg_problem& p = h->p;
    Level f;
    f.N = p.n_el;
    f.Nt = p.n_t;
    f.P = pitch_for(f.N);
    f.h = p.length / p.n_el;
    f.tau = p.t_final / p.n_t;
    h->L.push_back(f);
    // directions first (needs only k, c); vectors are allocated once the path is known
    CHK(h->alloc(&h->L[0].k, f.N));
    CHK(h->alloc(&h->L[0].c, f.N));
    CHK(h->alloc(&h->L[0].chi, f.N));
    CHK(level0_material(h));
    while (true) {
        Level& cur = h->L.back();
        double st[4];
        CHK(fetch_stats(h, cur, st));
        if (h->L.size() == 1) CHK(check_material(st));
        cur.W = level_w(h->o, cur, st);
        if (is_last(h, h->L.size(), cur)) break;
        double lam;
        char d = choose_direction(h, cur, st, &lam);
        if (!d) break;
        cur.dir = d;
        cur.lambda = lam;
        Level c;
        c.N = d == 'x' ? cur.N / 2 : cur.N;
        c.Nt = d == 't' ? cur.Nt / 2 : cur.Nt;
        c.P = pitch_for(c.N);
        c.h = d == 'x' ? 2.0 * cur.h : cur.h;
        c.tau = d == 't' ? 2.0 * cur.tau : cur.tau;
        CHK(h->alloc(&c.k, c.N));
        CHK(h->alloc(&c.c, c.N));
        CHK(h->alloc(&c.chi, c.N));
        CHK(coarse_coefficients(h, cur, d, c));
        h->L.push_back(c);
        if (h->L.size() >= 64) break;
    }
    const size_t nl = h->L.size();
    for (size_t i = 0; i < nl; ++i) {
        Level& l = h->L[i];
        // k, c, chi already allocated: allocate the rest
        const bool fine = i == 0, last = i + 1 == nl;
        CHK(h->alloc(&l.coef, kCoefArrays * (int64_t)(l.N + 1)));
        if (h->o.precision == STMG_MIXED) CHK(h->alloc(&l.coef32, kCoefArrays * (int64_t)(l.N + 1)));
        if (last) CHK(h->alloc(&l.thomas, 3 * (int64_t)(l.N + 1)));
        if (last && l.N <= kDenseCoarsestMax) CHK(h->alloc(&l.ainv, (int64_t)l.N * l.N));
        if (h->o.reassembly == STMG_REASSEMBLE_P && fine) {
            l.hrow.assign(l.Nt + 1, 2);
            l.hrow[0] = 0;
            if (l.Nt >= 1) l.hrow[1] = 1;
        }
        if (h->o.reassembly == STMG_REASSEMBLE_P && !fine) {
            if (last && l.N + 1 > kStencilCoarsestMaxNodes)
                return fail(STMG_EUNSUPPORTED, "Galerkin coarsest level wider than " +
                                                   std::to_string(kStencilCoarsestMaxNodes) +
                                                   " nodes (allow more levels)");
            const Level& f = h->L[i - 1];
            stencil_rows(f.hrow, f.Nt, f.dir, h->o.interp, l.hrow, l.hrep);
            l.R = (int)l.hrep.size();
            CHK(h->alloc(&l.sten, 10 * (int64_t)l.R * l.P));
            if (h->o.precision == STMG_MIXED) CHK(h->alloc(&l.sten32, 10 * (int64_t)l.R * l.P));
            if (last && h->o.interp == STMG_INTERP_B) {
                const int64_t n = l.dofs();
                if (n > kStencilLuMax)
                    return fail(STMG_EUNSUPPORTED, "bilinear Galerkin coarsest level above " +
                                                       std::to_string(kStencilLuMax) +
                                                       " DOFs (allow more levels)");
                CHK(h->alloc(&l.lu, 2 * n * n));
                CHK(h->alloc(&l.piv, 2 * n));
                CHK(h->alloc(&l.lux, n));
            } else if (last) {
                CHK(h->alloc(&l.sfac, 4 * (int64_t)l.R * l.P));
                if (l.N + 1 <= kStencilDenseMaxNodes)
                    CHK(h->alloc(&l.sinv, (int64_t)l.R * (l.N + 1) * (l.N + 1)));
            }
            CHK(h->alloc(&l.srow, (int64_t)l.Nt + 1));
            CHK(h->alloc(&l.srep, (int64_t)l.R));
            HIPCHK(hipMemcpyAsync(l.srow, l.hrow.data(), l.hrow.size() * sizeof(int),
                                  hipMemcpyHostToDevice, h->s));
            HIPCHK(hipMemcpyAsync(l.srep, l.hrep.data(), l.hrep.size() * sizeof(int),
                                  hipMemcpyHostToDevice, h->s));
        }
        if (h->o.precision == STMG_FP64 || fine) {
            CHK(h->alloc(&l.u, l.elems()));
            CHK(h->alloc(&l.b, l.elems()));
            CHK(h->alloc(&l.t, l.elems()));
        }
        if (fine && pipelined_options(&h->o)) {
            CHK(h->alloc(&l.w, l.elems()));
            CHK(h->alloc(&l.v, l.elems()));
        }
        if (h->o.precision == STMG_MIXED) {
            CHK(h->alloc(&l.u32, l.elems()));
            CHK(h->alloc(&l.b32, l.elems()));
            CHK(h->alloc(&l.t32, l.elems()));
        }
        CHK(finish_level(h, l, last));
    }
    if (h->o.reassembly == STMG_REASSEMBLE_P) CHK(galerkin_levels(h));
    Level& fl = h->L[0];
    CHK(h->alloc(&h->bload, fl.elems()));
    launch_load_vector(d_q, p.q_uniform, fl.N, fl.Nt, fl.h, h->bload, fl.P, h->s);
    if (!d_q) {
        // a uniform source gives the same load on every time level n >= 1 (and zeros on
        // level 0): two rows stand for the whole vector in the fine passes
        CHK(h->alloc(&h->brow, 2 * fl.P));
        CHK(h->alloc(&h->brow_adj, 2 * fl.P));
        launch_copy2d<double, double>(h->bload, fl.P, h->brow, fl.P, std::min(2, fl.Nt + 1), fl.N + 1, 1.0, h->s);
        launch_copy2d<double, double>(h->bload, fl.P, h->brow_adj, fl.P, std::min(2, fl.Nt + 1), fl.N + 1,
                                      fl.tau / p.theta_ref, h->s);
    }
    HIPCHK(hipGetLastError());
    // partial-sum buffer: largest fused pass on the fine level, reductions, gradient
    int64_t need = 1024;
    for (int S = 0; S <= fused_max_sweeps(); ++S) need = std::max<int64_t>(need, fused_parts(fl.N, fl.Nt, S));
    for (int S = 1; S <= mixed_max_sweeps(); ++S)
        for (bool e : {false, true})
            need = std::max<int64_t>(need, fused_parts(fl.N, fl.Nt, mixed_chain_sweeps(S, e)));
    need = std::max<int64_t>(need, (int64_t)gradient_chunks(fl.Nt) * fl.N);
    CHK(h->alloc(&h->parts, need));
    h->nparts = need;
    plan_tail(h);
    HIPCHK(hipStreamSynchronize(h->s));
    return 0;
}

// ------------------------------------------------------------------------------------
// V-cycle (Algorithm 1)
// ------------------------------------------------------------------------------------

// The next fine pass records its start and end in a fresh event pair (events recorded by
// the kernel launch itself: see FusedPass::ev_start).
void timer_begin(stmg_ctx* h, bool on, FusedPass& fp) {
    if (fp.fine) ++h->fine_passes;
    if (!on) return;
    KernelTimer& T = h->timer;
    if (T.used == T.ev.size()) {
        hipEvent_t a, b;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        T.ev.push_back({a, b});
        T.bytes.push_back(0);
    }
    fp.ev_start = T.ev[T.used].first;
    fp.ev_stop = T.ev[T.used].second;
}

void timer_end(stmg_ctx* h, bool on, double bytes) {
    if (!on) return;
    KernelTimer& T = h->timer;
    T.bytes[T.used] = bytes;
    ++T.used;
}

// The work enqueued from here to the next mark belongs to level l (-1: to no level).
void level_mark(stmg_ctx* h, int l) {
    LevelTimer& T = h->lt;
    if (!T.on) return;
    if (T.used == T.ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            T.on = false;   // no timing rather than a failed solve
            return;
        }
        T.ev.push_back(e);
        T.tag.push_back(0);
    }
    if (hipEventRecord(T.ev[T.used], h->s) != hipSuccess) {
        (void)hipGetLastError();
        T.on = false;
        return;
    }
    T.tag[T.used++] = l;
}

// One cycle of a solve loop (a V-cycle, or an outer correction of the mixed form):
// a roctx range, and the level marks when the cycle is sampled.
void cycle_begin(stmg_ctx* h) {
    roctxRangePushA("stmg cycle");
    LevelTimer& T = h->lt;
    T.on = h->o.time_levels > 0 && T.seen++ % h->o.time_levels == 0;
    if (T.on) ++T.cycles;
}

void cycle_end(stmg_ctx* h) {
    level_mark(h, -1);
    h->lt.on = false;
    roctxRangePop();
}

struct CycleScope {
    stmg_ctx* h;
    explicit CycleScope(stmg_ctx* c) : h(c) { cycle_begin(h); }
    ~CycleScope() { cycle_end(h); }
    CycleScope(const CycleScope&) = delete;
    CycleScope& operator=(const CycleScope&) = delete;
};

// After the stream has drained: the marked intervals summed per level, as the mean
// per sampled cycle.
void collect_levels(stmg_ctx* h, stmg_stats* st) {
    LevelTimer& T = h->lt;
    if (st && T.cycles > 0) {
        double acc[64] = {0};
        for (size_t i = 0; i + 1 < T.used; ++i) {
            if (T.tag[i] < 0 || T.tag[i] >= 64) continue;
            float ms = 0;
            if (hipEventElapsedTime(&ms, T.ev[i], T.ev[i + 1]) == hipSuccess) acc[T.tag[i]] += ms;
            else (void)hipGetLastError();
        }
        st->level_cycles = T.cycles;
        for (int l = 0; l < 64; ++l) st->level_ms[l] = acc[l] / T.cycles;
    }
    T.used = 0;
    T.on = false;
    T.seen = 0;
    T.cycles = 0;
}

// Sweep chunk sizes for nu steps: the fewest fused passes, of near-equal size.
std::vector<int> chunks_of(int nu) {
    const int m = fused_max_sweeps();
    const int n = nu <= m ? 1 : (nu + m - 1) / m;
    std::vector<int> c;
    for (int k = 0; k < n; ++k) c.push_back(nu / n + (k < nu % n ? 1 : 0));
    return c;
}

// Galerkin levels run the streaming passes with the fused kernels and causal
// interpolation; bilinear Galerkin levels couple to the next time level as well.
bool stencil_streams(const stmg_ctx* h) { return h->o.fused && h->o.interp == STMG_INTERP_C; }

// nu damped Jacobi steps on a Galerkin level (stored stencil), in place: streaming
// passes of up to kStencilMaxFused steps with the fused kernels and causal
// interpolation (the stencil then couples to earlier time levels only), else one
// launch per step.  head ('x' / 't'): the first pass adds the prolongation of z (pitch
// Pz) first; rdir ('x' / 't'): the last pass also restricts its residual into bc (pitch
// Pbc, Nc coarse elements).  Both only with the fused kernels, which the caller checks.
template <typename T>
int stencil_smooth(stmg_ctx* h, Level& lv, int trans, bool zero_start, int nu, char head = 0,
                   const T* z = nullptr, int64_t Pz = 0, char rdir = 0, T* bc = nullptr,
                   int64_t Pbc = 0, int Nc = 0) {
    const StencilViewT<T> S = sview<T>(lv);
    T*& u = U<T>(lv);
    T* b = B<T>(lv);
    T*& t = Tt<T>(lv);
    bool zero = zero_start;
    int left = nu;
    const bool stream = stencil_streams(h);
    while (left > 0) {
        const int passes = (left + kStencilMaxFused - 1) / kStencilMaxFused;
        const int k = stream ? (left + passes - 1) / passes : 1;
        if (stream) {
            const bool lastp = left == k;
            StencilPass<T> p{trans, k, u, b, t, zero, head, z, Pz, lastp ? rdir : (char)0,
                             bc, Pbc, Nc};
            if (launch_stencil_fused<T>(S, p, h->s) != 0) return fail(STMG_EINVAL, "bad stencil pass");
            head = 0;
        } else {
            launch_apply_stencil<T>(S, trans, APPLY_JACOBI, u, b, t, zero, h->s);
        }
        std::swap(u, t);
        zero = false;
        left -= k;
    }
    if (nu == 0 && zero_start) launch_fill<T>(u, lv.elems(), T(0), h->s);
    return 0;
}

// Right-hand side a pass on level l reads: during a solve with a uniform load the
// finest FP64 passes read its two rows (time level 0 and every later level) instead of
// a full vector.
template <typename T>
const T* level_b(const stmg_ctx* h, Level& lv, int l, int* b_const) {
    if constexpr (std::is_same<T, double>::value) {
        if (l == 0 && h->b_const) {
            *b_const = 1;
            return h->bfine;
        }
    }
    *b_const = 0;
    return B<T>(lv);
}

// Levels that start from zero (every coarse level, and the finest level of an FP32
// inner cycle) can skip storing their pre-smoothed iterate: the post-smoothing pass
// recomputes it from b in registers (the same steps, so the same bits), which saves
// writing and reading one vector of the level per cycle.  Taken when the whole
// recomputed chain fits one pass.
#ifndef STMG_RECOMPUTE
#define STMG_RECOMPUTE 1
#endif
template <typename T>
bool recompute_pre(const stmg_ctx* h, int l, bool zero_start, int nu) {
    const Level& lv = h->L[l];
    return STMG_RECOMPUTE && h->o.fused && zero_start && !lv.sten && nu >= 1 &&
           2 * nu <= fused_max_chain_sweeps() && !(lv.dir == 't' && h->o.interp == STMG_INTERP_B);
}

template <typename T>
int pre_smooth_restrict(stmg_ctx* h, int l, int trans, bool zero_start, int nu,
                        bool no_store = false) {
    Level& lv = h->L[l];
    Level& cl = h->L[l + 1];
    const auto V = view<T>(lv, h->o.omega);
    if (lv.sten) {
        if (stencil_streams(h) && nu > 0) {
            // the last smoothing pass restricts its residual into the coarse b
            CHK(stencil_smooth<T>(h, lv, trans, zero_start, nu, 0, nullptr, 0, lv.dir, B<T>(cl),
                                  cl.P, cl.N));
        } else {
            CHK(stencil_smooth<T>(h, lv, trans, zero_start, nu));
            launch_apply_stencil<T>(sview<T>(lv), trans, APPLY_RESIDUAL, U<T>(lv), B<T>(lv),
                                    Tt<T>(lv), false, h->s);
            launch_restrict<T>(lv.dir, V, Tt<T>(lv), B<T>(cl), cl.P, h->s, h->o.interp);
        }
        HIPCHK(hipGetLastError());
        return 0;
    }
    T*& u = U<T>(lv);
    int bconst = 0;
    const T* b = level_b<T>(h, lv, l, &bconst);
    T*& t = Tt<T>(lv);
    const bool timed = l == 0 && h->o.time_kernels > 0 && h->vcycles % h->o.time_kernels == 0;
    // bilinear t transfers run as their own kernels after the fused passes
    const bool split = lv.dir == 't' && h->o.interp == STMG_INTERP_B;
    if (h->o.fused) {
        std::vector<int> ch = chunks_of(nu);
        bool zero = zero_start;
        for (size_t k = 0; k < ch.size(); ++k) {
            FusedPass fp{};
            fp.trans = trans;
            fp.b_const = bconst;
            fp.sweeps = ch[k];
            fp.zero_in = zero;
            const bool lastc = k + 1 == ch.size();
            fp.tail = (lastc && !split) ? lv.dir : 0;
            fp.bc = B<T>(cl);
            fp.Pbc = cl.P;
            fp.Nc = cl.N;
            fp.Ntc = cl.Nt;
            fp.fine = l == 0;
            timer_begin(h, timed, fp);
            const bool skip = no_store && lastc;
            launch_fused<T>(V, fp, u, b, skip ? nullptr : t, h->s);
            timer_end(h, timed, (double)lv.dofs() * sizeof(T) *
                                    ((zero ? 0 : 1) + (bconst ? 0 : 1) + (skip ? 0 : 1)) +
                                    (lastc ? (double)cl.dofs() * sizeof(T) : 0.0));
            if (skip) break;
            if constexpr (std::is_same<T, double>::value) {
                if (l == 0 && k == 0 && h->rotate_in) {
                    // keep this cycle's input: (u, t, w) <- (t, w, u)
                    T* in = u;
                    u = t;
                    t = lv.w;
                    lv.w = in;
                    zero = false;
                    continue;
                }
            }
            std::swap(u, t);
            zero = false;
        }
        if (split) {
            launch_apply<T>(V, trans, APPLY_RESIDUAL, u, b, t, false, h->s);
            launch_restrict<T>(lv.dir, V, t, B<T>(cl), cl.P, h->s, h->o.interp);
        }
    } else {
        for (int k = 0; k < nu; ++k) {
            launch_apply<T>(V, trans, APPLY_JACOBI, u, b, t, zero_start && k == 0, h->s);
            std::swap(u, t);
        }
        if (nu == 0 && zero_start) launch_fill<T>(u, lv.elems(), T(0), h->s);
        launch_apply<T>(V, trans, APPLY_RESIDUAL, u, b, t, false, h->s);
        launch_restrict<T>(lv.dir, V, t, B<T>(cl), cl.P, h->s, h->o.interp);
    }
    HIPCHK(hipGetLastError());
    return 0;
}

template <typename T>
int prolong_post_smooth(stmg_ctx* h, int l, int trans, int nu, bool norm, bool recompute = false) {
    Level& lv = h->L[l];
    Level& cl = h->L[l + 1];
    const auto V = view<T>(lv, h->o.omega);
    T*& u = U<T>(lv);
    int bconst = 0;
    const T* b = level_b<T>(h, lv, l, &bconst);
    T*& t = Tt<T>(lv);
    const T* z = U<T>(cl);
    const bool timed = l == 0 && h->o.time_kernels > 0 && h->vcycles % h->o.time_kernels == 0;
    const bool split = lv.dir == 't' && h->o.interp == STMG_INTERP_B;
    if (lv.sten) {
        // norms are taken on the finest level only, which is never a stencil level
        if (stencil_streams(h) && nu > 0) {
            CHK(stencil_smooth<T>(h, lv, trans, false, nu, lv.dir, z, cl.P));
        } else {
            launch_prolong_add<T>(lv.dir, V, z, cl.P, u, h->s, h->o.interp);
            CHK(stencil_smooth<T>(h, lv, trans, false, nu));
        }
        HIPCHK(hipGetLastError());
        return 0;
    }
    if (recompute) {
        // the pre-smoothing steps again from zero, the prolongation, the post-smoothing
        FusedPass fp{};
        fp.trans = trans;
        fp.b_const = bconst;
        fp.pre_sweeps = nu;
        fp.sweeps = nu;
        fp.zero_in = 1;
        fp.prolong = lv.dir;
        fp.z = z;
        fp.Pz = cl.P;
        fp.Nc = cl.N;
        fp.Ntc = cl.Nt;
        fp.fine = l == 0;
        timer_begin(h, timed, fp);
        if (launch_fused<T>(V, fp, nullptr, b, t, h->s) < 0) return fail(STMG_EINVAL, "recompute pass rejected");
        timer_end(h, timed, (double)lv.dofs() * sizeof(T) * 2 + (double)cl.dofs() * sizeof(T));
        std::swap(u, t);
        HIPCHK(hipGetLastError());
        return 0;
    }
    if (h->o.fused) {
        if (split) launch_prolong_add<T>(lv.dir, V, z, cl.P, u, h->s, h->o.interp);
        std::vector<int> ch = chunks_of(nu);
        for (size_t k = 0; k < ch.size(); ++k) {
            FusedPass fp{};
            fp.trans = trans;
            fp.b_const = bconst;
            fp.sweeps = ch[k];
            fp.prolong = (k == 0 && !split) ? lv.dir : 0;
            fp.z = z;
            fp.Pz = cl.P;
            fp.Nc = cl.N;
            fp.Ntc = cl.Nt;
            const bool lastc = k + 1 == ch.size();
            fp.tail = (lastc && norm) ? 'n' : 0;
            fp.parts = h->parts;
            fp.fine = l == 0;
            timer_begin(h, timed, fp);
            int nw = launch_fused<T>(V, fp, u, b, t, h->s);
            timer_end(h, timed, (double)lv.dofs() * sizeof(T) * (bconst ? 2 : 3) +
                                    (k == 0 ? (double)cl.dofs() * sizeof(T) : 0.0));
            if (lastc && norm) h->norm_parts = nw;
            std::swap(u, t);
        }
    } else {
        launch_prolong_add<T>(lv.dir, V, z, cl.P, u, h->s, h->o.interp);
        for (int k = 0; k < nu; ++k) {
            launch_apply<T>(V, trans, APPLY_JACOBI, u, b, t, false, h->s);
            std::swap(u, t);
        }
        if (norm) {
            launch_residual_sumsq_partial<T>(V, trans, u, b, h->parts, h->s);
            h->norm_parts = reduce_parts(lv.Nt + 1);
        }
    }
    HIPCHK(hipGetLastError());
    return 0;
}

template <typename T>
int coarsest_solve(stmg_ctx* h, int l, int trans) {
    Level& lv = h->L[l];
    const auto V = view<double>(lv, h->o.omega);
    // FP64 arithmetic on the vectors of the cycle
    if (lv.sten && lv.lu) {
        const int64_t n = lv.dofs();
        launch_stencil_lu_solve<T>(stencil_view(lv), lv.lu + trans * n * n, lv.piv + trans * n,
                                   B<T>(lv), U<T>(lv), lv.lux, h->s);
        HIPCHK(hipGetLastError());
        return 0;
    }
    if (lv.sten && lv.sinv) {
        launch_stencil_coarsest_dense<T>(stencil_view(lv), lv.sinv, trans, B<T>(lv), U<T>(lv), h->s);
        HIPCHK(hipGetLastError());
        return 0;
    }
    if (lv.sten) {
        launch_stencil_coarsest<T>(stencil_view(lv), lv.sfac, trans, B<T>(lv), U<T>(lv), h->s);
        HIPCHK(hipGetLastError());
        return 0;
    }
    if (lv.ainv)
        launch_coarsest_dense<T>(V, lv.ainv, B<T>(lv), U<T>(lv), trans, h->s);
    else
        launch_coarsest<T>(V, lv.thomas, lv.thomas + (lv.N + 1), B<T>(lv), U<T>(lv), trans, h->s);
    HIPCHK(hipGetLastError());
    return 0;
}

// Levels l .. coarsest in one launch of the single-workgroup kernel (zero start).
template <typename T>
int tail_vcycle(stmg_ctx* h, int l, int trans) {
    const int last = (int)h->L.size() - 1;
    TailLaunch<T> t{};
    t.nlev = last - l + 1;
    for (int j = l; j <= last; ++j) {
        t.V[j - l] = view<T>(h->L[j], h->o.omega);
        t.dir[j - l] = h->L[j].dir;
    }
    t.nu = h->o.nu;
    t.trans = trans;
    t.lds_bytes = h->tail_lds;
    t.Vc = view<double>(h->L[last], h->o.omega);
    t.ainv = h->L[last].ainv;
    t.b_in = B<T>(h->L[l]);
    t.P_in = h->L[l].P;
    t.u_out = U<T>(h->L[l]);
    t.P_out = h->L[l].P;
    if (launch_vcycle_tail<T>(t, h->s) != 0) return fail(STMG_EHIP, "V-cycle tail does not fit its kernel");
    HIPCHK(hipGetLastError());
    return 0;
}

template <typename T>
int vcycle(stmg_ctx* h, int l, int trans, bool zero_start, bool norm) {
    const int last = (int)h->L.size() - 1;
    level_mark(h, l);
    if (l == last) {
        Range r(level_range(l, false));
        return coarsest_solve<T>(h, l, trans);
    }
    if (h->o.fused == 1 && l == h->tail_start && zero_start && !norm) {
        Range r(level_range(l, false));
        return tail_vcycle<T>(h, l, trans);
    }
    const bool rec = recompute_pre<T>(h, l, zero_start, h->o.nu) && !norm;
    {
        Range r(level_range(l, false));
        CHK(pre_smooth_restrict<T>(h, l, trans, zero_start, h->o.nu, rec));
    }
    CHK(vcycle<T>(h, l + 1, trans, true, false));
    level_mark(h, l);
    {
        Range r(level_range(l, true));
        CHK(prolong_post_smooth<T>(h, l, trans, h->o.nu, norm, rec));
    }
    if (l == 0) ++h->vcycles;
    return 0;
}

// sqrt(sum of the norm partials) -> host
int finish_norm(stmg_ctx* h, int nparts, double* out) {
    launch_reduce_final(h->parts, nparts, 1.0, h->dscal, h->s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h->hscal, h->dscal, sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    *out = std::sqrt(h->hscal[0]);
    return 0;
}

int residual_norm64(stmg_ctx* h, int trans, double* out) {
    Level& f = h->L[0];
    launch_residual_sumsq_partial<double>(view<double>(f, h->o.omega), trans, f.u, f.b, h->parts, h->s);
    HIPCHK(hipGetLastError());
    return finish_norm(h, reduce_parts(f.Nt + 1), out);
}

int norm64(stmg_ctx* h, const double* x, const Level& l, double* out) {
    launch_sumsq_partial<double>(x, l.Nt + 1, l.N + 1, l.P, h->parts, h->s);
    HIPCHK(hipGetLastError());
    return finish_norm(h, reduce_parts(l.Nt + 1), out);
}

double cycle_dof_updates(const stmg_ctx* h) {
    double s = 0;
    for (size_t i = 0; i + 1 < h->L.size(); ++i) s += 2.0 * h->o.nu * (double)h->L[i].dofs();
    return s;
}

void collect_timer(stmg_ctx* h, stmg_stats* st) {
    KernelTimer& T = h->timer;
    if (st) {
        for (size_t i = 0; i < T.used; ++i) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, T.ev[i].first, T.ev[i].second) == hipSuccess) {
                st->fine_kernel_ms += ms;
                st->fine_kernel_bytes += T.bytes[i];
                st->fine_kernel_launches += 1;
            }
        }
    }
    T.used = 0;
}

// ------------------------------------------------------------------------------------
// Solve loops
// ------------------------------------------------------------------------------------

int set_rhs(stmg_ctx* h, int trans, const double* d_rhs) {
    Level& f = h->L[0];
    if (d_rhs) {
        launch_copy2d<double, double>(d_rhs, f.N + 1, f.b, f.P, f.Nt + 1, f.N + 1, 1.0, h->s);
    } else {
        const double scale = trans ? f.tau / h->p.theta_ref : 1.0;
        launch_copy2d<double, double>(h->bload, f.P, f.b, f.P, f.Nt + 1, f.N + 1, scale, h->s);
    }
    HIPCHK(hipGetLastError());
    return 0;
}

int set_u0(stmg_ctx* h, const double* d_u0) {
    Level& f = h->L[0];
    if (d_u0)
        launch_copy2d<double, double>(d_u0, f.N + 1, f.u, f.P, f.Nt + 1, f.N + 1, 1.0, h->s);
    else
        launch_fill<double>(f.u, f.elems(), 0.0, h->s);
    HIPCHK(hipGetLastError());
    return 0;
}

int classify(const stmg_options& o, double r, bool* stop) {
    if (!std::isfinite(r) || r > o.diverge) { *stop = true; return STMG_DIVERGED; }
    if (r < o.tol) { *stop = true; return STMG_OK; }
    *stop = false;
    return STMG_NOT_CONVERGED;
}

// Residual norm^2 of the cycle just enqueued, reduced straight into slot `slot` of the
// pinned host scalars (value at hscal[8 + 2 slot], then the tag at hscal[9 + 2 slot]);
// nothing waits.  Tags come from one process-wide counter: pinned blocks are recycled
// between handles with their old contents, so a per-handle count could find a stale
// slot already carrying the tag it waits for.
std::atomic<uint64_t> g_norm_tag{0};

int post_norm_async(stmg_ctx* h, int slot, double* tag) {
    *tag = (double)++g_norm_tag;
    launch_reduce_to_host(h->parts, h->norm_parts, 1.0, h->hscal + 8 + 2 * slot, *tag, h->s);
    HIPCHK(hipGetLastError());
    return 0;
}

// Wait (spinning) until slot `slot` carries `tag`, then read its value.  Gives up with
// an error when the stream fails, or finishes without having written the tag.
int wait_norm(stmg_ctx* h, int slot, double tag, double* out) {
    volatile double* v = h->hscal + 8 + 2 * slot;
    for (unsigned long spins = 1; v[1] != tag; ++spins) {
        __builtin_ia32_pause();
        if ((spins & 4095) != 0) continue;
        const hipError_t e = hipStreamQuery(h->s);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(STMG_EHIP, "V-cycle stream failed while waiting for its residual");
        }
        if (v[1] != tag) return fail(STMG_EHIP, "V-cycle residual was not delivered");
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    *out = v[0];
    return 0;
}

// FP64 V-cycles with the termination test one cycle behind: cycle k+1 is enqueued
// before the residual of cycle k is read, so the device never waits for the host.
// Every cycle's first fine pass keeps its input (the previous result) in L[0].w; when
// cycle k stops the iteration, the speculative cycle k+1 is discarded and u_k is
// taken from w.  Iterates, residual history and cycle count are those of the plain
// loop.
int vcycles_pipelined(stmg_ctx* h, int trans, double nb, stmg_stats* st, int* cycles,
                      double* r_out, int* code) {
    Level& f = h->L[0];
    const int maxc = h->o.max_cycles;
    double tags[2] = {0, 0};
    auto enqueue = [&](int k) -> int {
        {
            CycleScope cs(h);
            CHK(vcycle<double>(h, 0, trans, false, true));
        }
        return post_norm_async(h, k & 1, &tags[k & 1]);
    };
    h->rotate_in = true;
    int rc = enqueue(1);
    int cyc = 1;
    bool ahead = false, stop = false;
    double r = 0;
    while (rc == 0) {
        ahead = cyc < maxc;
        if (ahead && (rc = enqueue(cyc + 1)) != 0) break;
        double ss = 0;
        if ((rc = wait_norm(h, cyc & 1, tags[cyc & 1], &ss)) != 0) break;
        r = std::sqrt(ss) / nb;
        if (st) st->history[cyc] = r;
        *code = classify(h->o, r, &stop);
        if (stop || cyc == maxc) break;
        ++cyc;
    }
    h->rotate_in = false;
    if (hipStreamSynchronize(h->s) != hipSuccess && rc == 0) rc = fail(STMG_EHIP, "stream synchronisation failed");
    if (rc != 0) return rc;
    if (ahead) std::swap(f.u, f.w);   // the discarded cycle's input is the result
    *cycles = cyc;
    *r_out = r;
    return 0;
}

// FP64 V-cycles with the finest level's post-smoothing of cycle k, the residual norm
// of its iterate u_k and the pre-smoothing (with its restricted residual) of cycle
// k + 1 in ONE streaming pass (a chain of 2 nu steps), so the finest level is read
// and written once per cycle instead of twice.  The termination test stays one cycle
// behind (cycle k + 1 runs while the host tests r_k).  u_k itself is not stored: when
// r_k stops the iteration, one post-smoothing pass recomputes it from the pass's input
// and the coarse correction z_k, which are still intact (the inputs rotate over three
// vectors, and the level below keeps its last two corrections in its two vectors).
// Where z_k would not survive the speculative cycle (the level below is the coarsest
// level, the single-workgroup tail or a Galerkin level) the pass stores u_k instead,
// over four rotating vectors.  Iterates are those of the plain loop, bit for bit; the
// norm partials are summed in another order.
#ifndef STMG_CHAINED
#define STMG_CHAINED 1
#endif
bool chained_options(const stmg_ctx* h) {
    const Level& f = h->L[0];
    return STMG_CHAINED && h->o.fused && h->L.size() >= 2 && f.v && h->hscal_pinned && !f.sten &&
           h->o.nu >= 1 && 2 * h->o.nu <= fused_max_chain_sweeps() &&
           !(f.dir == 't' && h->o.interp == STMG_INTERP_B);
}

int vcycles_chained(stmg_ctx* h, int trans, bool zero_u0, double nb, stmg_stats* st, int* cycles,
                    double* r_out, int* code) {
    Level& f = h->L[0];
    Level& c = h->L[1];
    const int nu = h->o.nu, maxc = h->o.max_cycles;
    const auto V = view<double>(f, h->o.omega);
    // the coarse correction of cycle k survives cycle k + 1 when the level below is
    // smoothed by one recomputing pass per cycle (it then alternates its two vectors)
    const bool z_survives = h->L.size() > 2 && !c.sten && !(h->o.fused == 1 && h->tail_start == 1) &&
                            recompute_pre<double>(h, 1, true, nu);
    double* buf[4] = {f.u, f.t, f.w, f.v};
    int bconst = 0;
    const double* bb = level_b<double>(h, f, 0, &bconst);
    auto timed_now = [&]() { return h->o.time_kernels > 0 && h->vcycles % h->o.time_kernels == 0; };
    // input of pass k (pre-smoothed iterate of cycle k) and its stored u_k; u0 is in
    // buf[0] and the first pre-smoothing writes in_1:
    //   recompute mode: in_k = buf[k % 3]; the pass writes buf[(k + 1) % 3]
    //   store mode:     odd k: in buf[3], u_k -> buf[1], out buf[2];
    //                   even k: in buf[2], u_k -> buf[0], out buf[3]
    auto in_of = [&](int k) { return z_survives ? buf[k % 3] : buf[(k & 1) ? 3 : 2]; };
    auto out_of = [&](int k) { return z_survives ? buf[(k + 1) % 3] : buf[(k & 1) ? 2 : 3]; };
    auto mid_of = [&](int k) { return z_survives ? nullptr : buf[(k & 1) ? 1 : 0]; };
    // first pre-smoothing and restriction (from zero: u0 is not read)
    {
        FusedPass fp{};
        fp.trans = trans;
        fp.b_const = bconst;
        fp.sweeps = nu;
        fp.zero_in = zero_u0;
        fp.tail = f.dir;
        fp.bc = c.b;
        fp.Pbc = c.P;
        fp.Nc = c.N;
        fp.Ntc = c.Nt;
        fp.fine = 1;
        // the event timer samples the cross-cycle passes only (one kernel, one byte count)
        timer_begin(h, false, fp);
        if (launch_fused<double>(V, fp, buf[0], bb, in_of(1), h->s) < 0)
            return fail(STMG_EINVAL, "pre-smoothing pass rejected");
        HIPCHK(hipGetLastError());
    }
    double tags[2] = {0, 0};
    double* zs[2] = {nullptr, nullptr};   // coarse corrections of the last two cycles
    auto enqueue = [&](int k) -> int {
        CycleScope cs(h);
        CHK(vcycle<double>(h, 1, trans, true, false));
        zs[k & 1] = c.u;
        level_mark(h, 0);
        Range r0(level_range(0, true));
        FusedPass fp{};
        fp.trans = trans;
        fp.b_const = bconst;
        fp.prolong = f.dir;
        fp.z = c.u;
        fp.Pz = c.P;
        fp.Nc = c.N;
        fp.Ntc = c.Nt;
        fp.sweeps = nu;
        fp.mid = mid_of(k);
        fp.mid_norm = 1;
        fp.next_sweeps = nu;
        fp.tail = f.dir;
        fp.bc = c.b;
        fp.Pbc = c.P;
        fp.parts = h->parts;
        fp.fine = 1;
        const bool timed = timed_now();
        timer_begin(h, timed, fp);
        const int nparts = launch_fused<double>(V, fp, in_of(k), bb, out_of(k), h->s);
        if (nparts < 0) return fail(STMG_EINVAL, "cycle pass rejected");
        // read: input, b (unless constant in time), coarse correction; written: (u_k),
        // the next input, coarse b
        timer_end(h, timed, (double)f.dofs() * 8 * (2 + (bconst ? 0 : 1) + (z_survives ? 0 : 1)) +
                                2.0 * (double)c.dofs() * 8);
        HIPCHK(hipGetLastError());
        ++h->vcycles;
        h->norm_parts = nparts;
        level_mark(h, -1);   // the norm's copy to the host counts on no level
        return post_norm_async(h, k & 1, &tags[k & 1]);
    };
    int rc = enqueue(1);
    int cyc = 1;
    bool stop = false;
    double r = 0;
    while (rc == 0) {
        if (cyc < maxc && (rc = enqueue(cyc + 1)) != 0) break;
        double ss = 0;
        if ((rc = wait_norm(h, cyc & 1, tags[cyc & 1], &ss)) != 0) break;
        r = std::sqrt(ss) / nb;
        if (st) st->history[cyc] = r;
        *code = classify(h->o, r, &stop);
        if (stop || cyc == maxc) break;
        ++cyc;
    }
    if (rc == 0 && z_survives) {
        // u_cyc: the post-smoothing of pass cyc again, from its input and z_cyc, into the
        // vector the speculative pass cyc + 1 wrote
        FusedPass fp{};
        fp.trans = trans;
        fp.b_const = bconst;
        fp.prolong = f.dir;
        fp.z = zs[cyc & 1];
        fp.Pz = c.P;
        fp.Nc = c.N;
        fp.Ntc = c.Nt;
        fp.sweeps = nu;
        fp.fine = 1;
        if (launch_fused<double>(V, fp, in_of(cyc), bb, out_of(cyc + 1), h->s) < 0)
            rc = fail(STMG_EINVAL, "final post-smoothing pass rejected");
        else if (hipGetLastError() != hipSuccess)
            rc = fail(STMG_EHIP, "final post-smoothing launch failed");
    }
    if (hipStreamSynchronize(h->s) != hipSuccess && rc == 0) rc = fail(STMG_EHIP, "stream synchronisation failed");
    if (rc != 0) return rc;
    // keep the four vectors, with f.u on the result
    double* res = z_survives ? out_of(cyc + 1) : mid_of(cyc);
    double* others[3];
    int k = 0;
    for (double* q : buf)
        if (q != res) others[k++] = q;
    f.u = res;
    f.t = others[0];
    f.w = others[1];
    f.v = others[2];
    *cycles = cyc;
    *r_out = r;
    return 0;
}

int solve_fp64(stmg_ctx* h, int trans, bool zero_u0, double nb, stmg_stats* st, int* status) {
    Level& f = h->L[0];
    double r = 1.0;   // ||b - J 0|| / ||b||
    if (!zero_u0) {
        CHK(residual_norm64(h, trans, &r));
        r /= nb;
    }
    if (st) st->history[0] = r;
    const double r0 = r;
    int cyc = 0, code = STMG_NOT_CONVERGED;
    bool stop = false;
    const bool timed = h->o.time_kernels != 0;
    const bool single = h->L.size() == 1;
    if (chained_options(h)) {
        CHK(vcycles_chained(h, trans, zero_u0, nb, st, &cyc, &r, &code));
        if (timed) collect_timer(h, st);
    } else if (!single && f.w && h->hscal_pinned) {
        if (zero_u0) CHK(set_u0(h, nullptr));
        CHK(vcycles_pipelined(h, trans, nb, st, &cyc, &r, &code));
        if (timed) collect_timer(h, st);
    } else {
        if (zero_u0) CHK(set_u0(h, nullptr));
        for (cyc = 1; cyc <= h->o.max_cycles; ++cyc) {
            {
                CycleScope cs(h);
                CHK(vcycle<double>(h, 0, trans, false, true));
            }
            double ss;
            if (single)
                CHK(residual_norm64(h, trans, &ss));
            else
                CHK(finish_norm(h, h->norm_parts, &ss));
            r = ss / nb;
            if (timed) collect_timer(h, st);
            if (st) st->history[cyc] = r;
            code = classify(h->o, r, &stop);
            if (stop) break;
        }
        if (cyc > h->o.max_cycles) cyc = h->o.max_cycles;
    }
    if (st) {
        st->cycles = cyc;
        st->rel_residual = r;
        st->conv_factor = (r0 > 0 && cyc > 0) ? std::pow(r / r0, 1.0 / cyc) : NAN;
        st->dof_updates = cyc * cycle_dof_updates(h);
    }
    *status = code;
    return 0;
}

// Mixed precision: FP64 defect correction around FP32 V-cycles.  Each outer step
// applies u += s_e e (FP64), forms r = b - J u in FP64, writes the FP32 right-hand
// side f = r / s_f of the next inner cycle (s_f = RMS of the previous residual, so
// f stays O(1) in FP32 range) and runs one FP32 V-cycle J e = f from e = 0 (FP32
// smoothers and transfers, FP64 coarsest solve).  Fused path: the update, the
// residual, the FP32 rounding and the norm partials are one streaming pass.
int defect_step(stmg_ctx* h, int trans, double s_e, double s_f, double* norm) {
    Level& f = h->L[0];
    const auto V64 = view<double>(f, h->o.omega);
    const double inv = 1.0 / s_f;
    if (h->o.fused) {
        int bconst = 0;
        const double* bb = level_b<double>(h, f, 0, &bconst);
        FusedPass fp{};
        fp.trans = trans;
        fp.b_const = bconst;
        fp.sweeps = 0;
        fp.prolong = s_e != 0.0 ? 'c' : 0;   // the first step has no correction to add
        fp.tail = 'c';
        fp.e32 = f.u32;
        fp.s_old = s_e;
        fp.f32 = f.b32;
        fp.inv_s_new = inv;
        fp.parts = h->parts;
        fp.fine = 1;
        const bool timed = h->o.time_kernels > 0 && h->vcycles % h->o.time_kernels == 0;
        timer_begin(h, timed, fp);
        const int nw = launch_fused<double>(V64, fp, f.u, bb, f.t, h->s);
        // u, (e), b read; u, f written
        timer_end(h, timed, (double)f.dofs() * (8 + (s_e != 0.0 ? 4 : 0) + (bconst ? 0 : 8) + 8 + 4));
        if (nw < 0) return fail(STMG_EINVAL, "defect-correction pass rejected");
        std::swap(f.u, f.t);
        HIPCHK(hipGetLastError());
        return finish_norm(h, nw, norm);
    }
    if (s_e != 0.0) launch_axpy2d<float>(f.u32, f.P, f.u, f.P, f.Nt + 1, f.N + 1, s_e, h->s);
    launch_apply<double>(V64, trans, APPLY_RESIDUAL, f.u, f.b, f.t, false, h->s);
    launch_copy2d<double, float>(f.t, f.P, f.b32, f.P, f.Nt + 1, f.N + 1, inv, h->s);
    HIPCHK(hipGetLastError());
    return norm64(h, f.t, f, norm);
}

// Mixed precision: FP64 defect correction around FP32 V-cycles.  Each outer step
// applies u += s_e e (FP64), forms r = b - J u in FP64, writes the FP32 right-hand
// side f = r / s_f of the next inner solve (s_f = RMS of the previous residual, so f
// stays O(1) in FP32 range) and solves J e = f approximately by `inner_cycles` FP32
// V-cycles from e = 0 (FP32 smoothers and transfers, FP64 coarsest solve).
//
// On the finest level with the fused kernels, one pass (launch_mixed) does the FP32
// post-smoothing of the last inner cycle, the FP64 defect correction and the FP32
// pre-smoothing of the next outer step's first inner cycle, so the FP32 correction is
// stored only between inner cycles.  Between two inner cycles one FP32 pass joins the
// post-smoothing of the first and the pre-smoothing of the second: after the first
// inner cycle its pre-smoothing is recomputed from zero, after a later one it is read
// back (the pre-smoothed iterate alternates between two FP32 vectors).  Same bits as
// the unfused loop.
#ifndef STMG_MIXED_FUSED
#define STMG_MIXED_FUSED 1
#endif
bool mixed_fused_options(const stmg_ctx* h) {
    const Level& f = h->L[0];
    return STMG_MIXED_FUSED && h->o.fused && h->L.size() >= 2 && !f.sten && h->o.nu >= 1 &&
           h->o.nu <= mixed_max_sweeps() && !(f.dir == 't' && h->o.interp == STMG_INTERP_B);
}

int solve_mixed(stmg_ctx* h, int trans, double nb, stmg_stats* st, int* status) {
    Level& f = h->L[0];
    const int m = h->o.inner_cycles, nu = h->o.nu;
    const double sq = std::sqrt((double)f.dofs());
    double s_f = nb / sq;   // scale of the right-hand side the next step writes
    double rn;
    CHK(defect_step(h, trans, 0.0, s_f, &rn));
    double r = rn / nb;
    if (st) st->history[0] = r;
    const double r0 = r;
    const bool timed = h->o.time_kernels != 0;
    const bool fusedm = mixed_fused_options(h);
    int cyc = 0, code = STMG_NOT_CONVERGED;
    bool stop = false;
    auto timed_now = [&]() { return h->o.time_kernels > 0 && h->vcycles % h->o.time_kernels == 0; };
    if (fusedm) CHK(pre_smooth_restrict<float>(h, 0, trans, true, nu, true));
    for (cyc = 1; cyc <= h->o.max_cycles; ++cyc) {
        const double s_e = s_f;
        s_f = rn > 0 ? rn / sq : 1.0;
        CycleScope cs(h);
        if (fusedm) {
            Level& c = h->L[1];
            // the pre-smoothed iterate of the current inner cycle (none: the first,
            // which starts from zero and is recomputed)
            float* e_in = nullptr;
            for (int i = 1; i < m; ++i) {
                // inner cycle i ends, inner cycle i + 1 starts from its iterate
                CHK(vcycle<float>(h, 1, trans, true, false));
                level_mark(h, 0);
                Range r0(level_range(0, true));
                FusedPass fp{};
                fp.trans = trans;
                fp.pre_sweeps = e_in ? 0 : nu;
                fp.sweeps = nu;
                fp.next_sweeps = nu;
                fp.zero_in = e_in ? 0 : 1;
                fp.prolong = f.dir;
                fp.z = c.u32;
                fp.Pz = c.P;
                fp.Nc = c.N;
                fp.Ntc = c.Nt;
                fp.tail = f.dir;
                fp.bc = c.b32;
                fp.Pbc = c.P;
                fp.fine = 1;
                float* dst = e_in == f.u32 ? f.t32 : f.u32;
                const bool tk = timed_now();
                timer_begin(h, tk, fp);
                if (launch_fused<float>(view<float>(f, h->o.omega), fp, e_in, f.b32, dst, h->s) < 0)
                    return fail(STMG_EINVAL, "inner cycle pass rejected");
                // read (e), f, z; written e', coarse b
                timer_end(h, tk, (double)f.dofs() * (e_in ? 12 : 8) + 2.0 * (double)c.dofs() * 4);
                HIPCHK(hipGetLastError());
                ++h->vcycles;
                e_in = dst;
            }
            CHK(vcycle<float>(h, 1, trans, true, false));
            level_mark(h, 0);
            Range r0(level_range(0, true));
            int bconst = 0;
            MixedPass mp{};
            mp.trans = trans;
            mp.sweeps = nu;
            mp.prolong = f.dir;
            mp.e = e_in;
            mp.f = f.b32;
            mp.z = c.u32;
            mp.Pz = c.P;
            mp.u = f.u;
            mp.b = level_b<double>(h, f, 0, &bconst);
            mp.b_const = bconst;
            mp.u_out = f.t;
            // the next right-hand side goes to the FP32 vector that holds neither e nor f
            mp.f_out = e_in == f.t32 ? f.u32 : f.t32;
            mp.pre = 1;
            mp.tail = f.dir;
            mp.bc = c.b32;
            mp.Pbc = c.P;
            mp.Nc = c.N;
            mp.s_e = s_e;
            mp.inv_s = 1.0 / s_f;
            mp.parts = h->parts;
            const bool tk = timed_now();
            FusedPass ev{};
            ev.fine = 1;
            timer_begin(h, tk, ev);
            mp.ev_start = ev.ev_start;
            mp.ev_stop = ev.ev_stop;
            const int nw = launch_mixed(view<float>(f, h->o.omega), view<double>(f, h->o.omega), mp, h->s);
            if (nw < 0) return fail(STMG_EINVAL, "mixed pass rejected");
            // read (e), f, z, u, b; written u, f', bc
            timer_end(h, tk, (double)f.dofs() * ((e_in ? 4 : 0) + 4 + 8 + (bconst ? 0 : 8) + 8 + 4) +
                                 2.0 * (double)c.dofs() * 4);
            HIPCHK(hipGetLastError());
            ++h->vcycles;
            std::swap(f.u, f.t);
            float* old_f = f.b32;
            f.b32 = mp.f_out;
            if (mp.f_out == f.t32) f.t32 = old_f;
            else f.u32 = old_f;
            level_mark(h, -1);
            CHK(finish_norm(h, nw, &rn));
        } else {
            for (int i = 0; i < m; ++i) CHK(vcycle<float>(h, 0, trans, i == 0, false));
            level_mark(h, 0);
            CHK(defect_step(h, trans, s_e, s_f, &rn));
        }
        r = rn / nb;
        if (timed) collect_timer(h, st);
        if (st) st->history[cyc] = r;
        code = classify(h->o, r, &stop);
        if (stop) break;
    }
    if (cyc > h->o.max_cycles) cyc = h->o.max_cycles;
    if (st) {
        st->cycles = cyc;
        st->rel_residual = r;
        st->conv_factor = (r0 > 0 && cyc > 0) ? std::pow(r / r0, 1.0 / cyc) : NAN;
        st->dof_updates = (double)cyc * m * cycle_dof_updates(h);
    }
    *status = code;
    return 0;
}

int solve(stmg_ctx* h, int trans, const double* d_rhs, const double* d_u0, double* d_u,
          stmg_stats* st) {
    if (!h) return fail(STMG_EINVAL, "null handle");
    if (!d_u) return fail(STMG_EINVAL, "null output");
    auto t0 = std::chrono::steady_clock::now();
    Range range(trans ? "stmg_solve adjoint" : "stmg_solve forward");
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->n_levels = (int)h->L.size();
        st->setup_ms = h->setup_ms;
        for (size_t i = 0; i + 1 < h->L.size() && i + 1 < sizeof(st->path); ++i) st->path[i] = h->L[i].dir;
    }
    h->timer.used = 0;
    h->lt.used = 0;
    h->lt.seen = 0;
    h->lt.cycles = 0;
    h->lt.on = false;
    h->fine_passes = 0;
    const bool zero_u0 = d_u0 == nullptr;
    Level& fl = h->L[0];
    // the fused passes of the finest level read the uniform load's two rows instead of
    // a full right-hand side; paths that read the full vector get it copied as before
    const bool split0 = fl.dir == 't' && h->o.interp == STMG_INTERP_B;
    h->b_const = !d_rhs && h->brow && h->o.fused && h->L.size() >= 2 && !split0 && zero_u0;
    h->bfine = trans ? h->brow_adj : h->brow;
    struct ResetB {
        stmg_ctx* c;
        ~ResetB() { c->b_const = false; }
    } reset_b{h};
    if (!h->b_const) CHK(set_rhs(h, trans, d_rhs));
    if (!zero_u0) CHK(set_u0(h, d_u0));
    Level& f0 = h->L[0];
    double nb;
    if (d_rhs) {
        CHK(norm64(h, f0.b, f0, &nb));
    } else {
        // the assembled load is fixed for the handle: its norm is taken once
        if (h->bload_norm < 0) CHK(norm64(h, h->bload, f0, &h->bload_norm));
        nb = h->bload_norm * (trans ? f0.tau / h->p.theta_ref : 1.0);
    }
    if (!(nb > 0) || !std::isfinite(nb)) return fail(STMG_EINVAL, "right-hand side is zero or not finite");
    int status = STMG_NOT_CONVERGED;
    if (h->o.precision == STMG_FP64) {
        CHK(solve_fp64(h, trans, zero_u0, nb, st, &status));
    } else {
        if (zero_u0) CHK(set_u0(h, nullptr));
        CHK(solve_mixed(h, trans, nb, st, &status));
    }
    Level& f = h->L[0];
    launch_copy2d<double, double>(f.u, f.P, d_u, f.N + 1, f.Nt + 1, f.N + 1, 1.0, h->s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->s));
    collect_levels(h, st);
    if (st) {
        st->fine_passes = h->fine_passes;
        st->status = status;
        st->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    g_err.clear();
    return status;
}

int check_level(stmg_ctx* h, int level) {
    if (!h) return fail(STMG_EINVAL, "null handle");
    if (level < 0 || level >= (int)h->L.size()) return fail(STMG_EINVAL, "level out of range");
    return 0;
}

// FP64 interface vectors (compact) <-> level vectors of the cycle's precision (pitched)
template <typename T>
int copy_in(stmg_ctx* h, const Level& l, const double* src, T* dst) {
    launch_copy2d<double, T>(src, l.N + 1, dst, l.P, l.Nt + 1, l.N + 1, 1.0, h->s);
    HIPCHK(hipGetLastError());
    return 0;
}
template <typename T>
int copy_out(stmg_ctx* h, const Level& l, const T* src, double* dst) {
    launch_copy2d<T, double>(src, l.P, dst, l.N + 1, l.Nt + 1, l.N + 1, 1.0, h->s);
    HIPCHK(hipGetLastError());
    return 0;
}

// debug_poison: NaN in the nodes of a level vector a per-level call is about to compute
// (the padding columns keep their zeros, which the streaming kernels read)
template <typename T>
void poison(stmg_ctx* h, const Level& l, T* x) {
    if (h->o.debug_poison) launch_fill2d<T>(x, l.P, l.Nt + 1, l.N + 1, std::numeric_limits<T>::quiet_NaN(), h->s);
}

template <typename T>
int level_apply(stmg_ctx* h, int level, int transpose, const double* d_x, double* d_y) {
    Level& l = h->L[level];
    CHK(copy_in<T>(h, l, d_x, U<T>(l)));
    poison<T>(h, l, Tt<T>(l));
    if (l.sten)
        launch_apply_stencil<T>(sview<T>(l), transpose, APPLY_J, U<T>(l), B<T>(l), Tt<T>(l), false, h->s);
    else
        launch_apply<T>(view<T>(l, h->o.omega), transpose, APPLY_J, U<T>(l), B<T>(l), Tt<T>(l), false, h->s);
    CHK(copy_out<T>(h, l, Tt<T>(l), d_y));
    HIPCHK(hipStreamSynchronize(h->s));
    return 0;
}

template <typename T>
int level_smooth(stmg_ctx* h, int level, int transpose, int nu, const double* d_b, double* d_u) {
    Level& l = h->L[level];
    CHK(copy_in<T>(h, l, d_b, B<T>(l)));
    CHK(copy_in<T>(h, l, d_u, U<T>(l)));
    poison<T>(h, l, Tt<T>(l));
    const auto V = view<T>(l, h->o.omega);
    T*& u = U<T>(l);
    T*& t = Tt<T>(l);
    if (l.sten) {
        CHK(stencil_smooth<T>(h, l, transpose, false, nu));
    } else if (h->o.fused) {
        for (int S : chunks_of(nu)) {
            FusedPass fp{};
            fp.trans = transpose;
            fp.sweeps = S;
            launch_fused<T>(V, fp, u, B<T>(l), t, h->s);
            std::swap(u, t);
        }
    } else {
        for (int k = 0; k < nu; ++k) {
            launch_apply<T>(V, transpose, APPLY_JACOBI, u, B<T>(l), t, false, h->s);
            std::swap(u, t);
        }
    }
    CHK(copy_out<T>(h, l, u, d_u));
    HIPCHK(hipStreamSynchronize(h->s));
    return 0;
}

template <typename T>
int level_presmooth_restrict(stmg_ctx* h, int level, int transpose, int nu, const double* d_b,
                             double* d_u, double* d_bc) {
    Level& l = h->L[level];
    Level& c = h->L[level + 1];
    CHK(copy_in<T>(h, l, d_b, B<T>(l)));
    CHK(copy_in<T>(h, l, d_u, U<T>(l)));
    poison<T>(h, l, Tt<T>(l));
    poison<T>(h, c, B<T>(c));
    CHK(pre_smooth_restrict<T>(h, level, transpose, false, nu));
    CHK(copy_out<T>(h, l, U<T>(l), d_u));
    CHK(copy_out<T>(h, c, B<T>(c), d_bc));
    HIPCHK(hipStreamSynchronize(h->s));
    return 0;
}

template <typename T>
int level_prolong_postsmooth(stmg_ctx* h, int level, int transpose, int nu, const double* d_b,
                             const double* d_z, double* d_u) {
    Level& l = h->L[level];
    Level& c = h->L[level + 1];
    CHK(copy_in<T>(h, l, d_b, B<T>(l)));
    CHK(copy_in<T>(h, l, d_u, U<T>(l)));
    CHK(copy_in<T>(h, c, d_z, U<T>(c)));
    poison<T>(h, l, Tt<T>(l));
    CHK(prolong_post_smooth<T>(h, level, transpose, nu, false));
    CHK(copy_out<T>(h, l, U<T>(l), d_u));
    HIPCHK(hipStreamSynchronize(h->s));
    return 0;
}

template <typename T>
int level_coarsest_solve(stmg_ctx* h, int transpose, const double* d_b, double* d_z) {
    const int last = (int)h->L.size() - 1;
    Level& l = h->L[last];
    CHK(copy_in<T>(h, l, d_b, B<T>(l)));
    poison<T>(h, l, U<T>(l));
    CHK(coarsest_solve<T>(h, last, transpose));
    CHK(copy_out<T>(h, l, U<T>(l), d_z));
    HIPCHK(hipStreamSynchronize(h->s));
    return 0;
}

int reassemble(stmg_ctx* h, bool check_path) {
    CHK(level0_material(h));
    for (size_t i = 0; i < h->L.size(); ++i) {
        Level& l = h->L[i];
        double st[4];
        CHK(fetch_stats(h, l, st));
        if (i == 0) CHK(check_material(st));
        if (i + 1 < h->L.size()) {
            double lam;
            char d = choose_direction(h, l, st, &lam);
            if (check_path && d != l.dir) return fail(STMG_EUNSUPPORTED, "coarsening path changed with the new design");
            l.lambda = lam;
            CHK(coarse_coefficients(h, l, l.dir, h->L[i + 1]));
        }
        l.W = level_w(h->o, l, st);
        CHK(finish_level(h, l, i + 1 == h->L.size()));
    }
    if (h->o.reassembly == STMG_REASSEMBLE_P) CHK(galerkin_levels(h));
    HIPCHK(hipStreamSynchronize(h->s));
    return 0;
}

// ------------------------------------------------------------------------------------
// Device scratch of the allocation-free gradient (stmg_gradient_noalloc)
// ------------------------------------------------------------------------------------

// Every device the library runs on holds one copy of this array from the load of the
// code object until the process ends.  In host code its name is only a stand-in for the
// symbol: the device address of each device's copy comes from hipGetSymbolAddress, once
// per device, and only that address is handed to kernels.
constexpr size_t kScratchDoubles = size_t(8) << 20;   // 64 MiB
constexpr int kScratchDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kScratchDevices] = {};

// Device address of the current device's scratch, resolved on the first call per device.
int scratch_address(double** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) return fail(STMG_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(STMG_EHIP, std::string("hipGetSymbolAddress of the scratch array: ") +
                                       hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

}  // namespace

// ======================================================================================
// C ABI
// ======================================================================================

extern "C" {

int stmg_default_options(stmg_options* o) {
    if (!o) return fail(STMG_EINVAL, "null options");
    std::memset(o, 0, sizeof(*o));
    o->nu = 2;
    o->omega = 0.5;
    o->lambda_crit = 0.25;
    o->max_levels = 0;
    o->min_coarse_dofs = 1024;
    o->M_min_elems = 0;
    o->reassembly = STMG_REASSEMBLE_R;
    o->deff_mode = 0;
    o->tol = 1e-10;
    o->diverge = 1e9;
    o->max_cycles = 100;
    o->precision = STMG_FP64;
    o->w_diri_override = 0.0;
    o->fused = 1;
    o->time_kernels = 0;
    o->interp = STMG_INTERP_C;
    o->debug_poison = 0;
    o->inner_cycles = 4;
    o->time_levels = 0;
    return 0;
}

int stmg_footprint(const stmg_problem* p, const stmg_options* o, int with_adjoint, size_t* bytes) {
    CHK(validate(p, o));
    if (!bytes) return fail(STMG_EINVAL, "null output");
    // the request's compact outputs: u, and with the adjoint Lambda and the gradient
    const size_t vec = (size_t)dofs_of(p->n_el, p->n_t) * 8;
    *bytes = footprint_of(p, o) + vec + (with_adjoint ? vec + (size_t)p->n_el * 8 : 0);
    return 0;
}

int stmg_create(stmg_t* handle, const stmg_problem* p, const stmg_options* o,
                const double* d_rho, const double* d_q, void* stream) {
    if (!handle) return fail(STMG_EINVAL, "null handle pointer");
    *handle = nullptr;
    CHK(validate(p, o));
    if (!d_rho) return fail(STMG_EINVAL, "null density");
    const auto t0 = std::chrono::steady_clock::now();
    Range range("stmg_create");
    auto* h = new stmg_ctx();
    h->p = *p;
    h->o = *o;
    h->s = static_cast<hipStream_t>(stream);
    int rc = 0;
    do {
        // Pinned scalars make the per-cycle 8-byte read-back cheaper; where pinning is
        // not available a pageable buffer works the same through the stream-ordered copy.
        if (hipHostMalloc(&h->hscal, 64 * sizeof(double)) == hipSuccess) {
            h->hscal_pinned = true;
        } else {
            (void)hipGetLastError();
            h->hscal = new double[64];
            h->hscal_pinned = false;
        }
        std::memset(h->hscal, 0, 64 * sizeof(double));   // no tag is 0
        if ((rc = h->alloc(&h->rho, p->n_el)) < 0) break;
        if ((rc = h->alloc(&h->kp, p->n_el)) < 0) break;
        if ((rc = h->alloc(&h->cpd, p->n_el)) < 0) break;
        if ((rc = h->alloc(&h->simp, 8)) < 0) break;
        if ((rc = h->alloc(&h->stats, 8)) < 0) break;
        if ((rc = h->alloc(&h->dscal, 8)) < 0) break;
        double sp[6] = {p->k_ins, p->k_con, p->p_k, p->c_ins, p->c_con, p->p_c};
        if (hipMemcpyAsync(h->simp, sp, sizeof(sp), hipMemcpyHostToDevice, h->s) != hipSuccess ||
            hipMemcpyAsync(h->rho, d_rho, (size_t)p->n_el * 8, hipMemcpyDeviceToDevice, h->s) != hipSuccess) {
            rc = fail(STMG_EHIP, "copy of the design failed");
            break;
        }
        rc = build(h, d_q);
    } while (0);
    if (rc < 0) {
        (void)hipStreamSynchronize(h->s);
        delete h;
        return rc;
    }
    h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *handle = h;
    g_err.clear();
    return 0;
}

int stmg_set_field(stmg_t h, const double* d_field) {
    if (!h || !d_field) return fail(STMG_EINVAL, "null argument");
    const auto t0 = std::chrono::steady_clock::now();
    Range range("stmg_set_field");
    // keep the old field to restore the handle if the new one is rejected
    std::vector<double> old((size_t)h->p.n_el);
    HIPCHK(hipMemcpyAsync(old.data(), h->rho, old.size() * 8, hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipMemcpyAsync(h->rho, d_field, old.size() * 8, hipMemcpyDeviceToDevice, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    int rc = reassemble(h, h->o.deff_mode == 0);
    if (rc == STMG_EUNSUPPORTED || rc == STMG_EINVAL) {
        std::string msg = g_err;
        HIPCHK(hipMemcpyAsync(h->rho, old.data(), old.size() * 8, hipMemcpyHostToDevice, h->s));
        HIPCHK(hipStreamSynchronize(h->s));
        CHK(reassemble(h, false));
        return fail(rc, msg);
    }
    if (rc == 0)
        h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

int stmg_set_design(stmg_t h, const double* d_rho) { return stmg_set_field(h, d_rho); }

int stmg_solve_forward(stmg_t h, const double* d_rhs, const double* d_u0, double* d_u,
                       stmg_stats* st) {
    return solve(h, 0, d_rhs, d_u0, d_u, st);
}

int stmg_solve_adjoint(stmg_t h, const double* d_rhs, const double* d_l0, double* d_lambda,
                       stmg_stats* st) {
    return solve(h, 1, d_rhs, d_l0, d_lambda, st);
}

int stmg_objective(stmg_t h, const double* d_u, double* theta) {
    if (!h || !d_u || !theta) return fail(STMG_EINVAL, "null argument");
    Level& f = h->L[0];
    launch_dot_partial(h->bload, d_u, f.Nt + 1, f.N + 1, f.P, f.N + 1, h->parts, h->s);
    // Theta = b^T u dt / Theta_ref  (Section 7.1)
    launch_reduce_final(h->parts, reduce_parts(f.Nt + 1), f.tau / h->p.theta_ref, h->dscal, h->s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h->hscal, h->dscal, sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    *theta = h->hscal[0];
    return 0;
}

int stmg_gradient(stmg_t h, const double* d_u, const double* d_lambda, double* d_grad) {
    if (!h || !d_u || !d_lambda || !d_grad) return fail(STMG_EINVAL, "null argument");
    Level& f = h->L[0];
    const int chunks = gradient_chunks(f.Nt);
    launch_gradient_partial(d_u, d_lambda, f.N, f.Nt, f.N + 1, f.N + 1, h->kp, h->cpd, f.h, f.tau,
                            h->parts, h->s);
    launch_gradient_final(h->parts, f.N, chunks, d_grad, h->s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->s));
    return 0;
}

int stmg_gradient_noalloc(const stmg_problem* p, const double* d_rho, const double* d_u,
                          const double* d_lambda, double* d_grad, void* stream) {
    if (!p || !d_rho || !d_u || !d_lambda || !d_grad) return fail(STMG_EINVAL, "null argument");
    if (p->n_el < 1 || p->n_t < 1 || (int64_t)p->n_el > (1 << 24) || (int64_t)p->n_t > (1 << 26))
        return fail(STMG_EINVAL, "n_el and n_t must be in [1, 2^24] and [1, 2^26]");
    if (!(p->length > 0) || !(p->t_final > 0)) return fail(STMG_EINVAL, "length and t_final must be > 0");
    if (p->field_kind != STMG_FIELD_DENSITY && p->field_kind != STMG_FIELD_CONDUCTIVITY)
        return fail(STMG_EINVAL, "unknown field_kind");
    const int N = p->n_el, Nt = p->n_t;
    const int chunks = gradient_chunks(Nt);
    const size_t need = (size_t)N * (size_t)(chunks + 2);
    if (need > kScratchDoubles)
        return fail(STMG_EINVAL, "n_el * (" + std::to_string(chunks) + " time chunks + 2) = " +
                                     std::to_string(need) + " doubles exceeds the " +
                                     std::to_string(kScratchDoubles) + "-double scratch");
    double* sp = nullptr;
    CHK(scratch_address(&sp));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // scratch: dk/drho (N), dc/drho (N), per-chunk partial sums (chunks N); every entry
    // is written before it is read, so nothing needs clearing between calls
    double* kp = sp;
    double* cpd = sp + N;
    double* parts = sp + 2 * (size_t)N;
    if (p->field_kind == STMG_FIELD_CONDUCTIVITY) {
        launch_fill<double>(kp, N, 1.0, s);
        launch_fill<double>(cpd, N, 0.0, s);
    } else {
        launch_simp_derivative(d_rho, N, p->k_ins, p->k_con, p->p_k, kp, s);
        launch_simp_derivative(d_rho, N, p->c_ins, p->c_con, p->p_c, cpd, s);
    }
    const double hx = p->length / p->n_el, tau = p->t_final / p->n_t;
    launch_gradient_partial(d_u, d_lambda, N, Nt, N + 1, N + 1, kp, cpd, hx, tau, parts, s);
    launch_gradient_final(parts, N, chunks, d_grad, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    g_err.clear();
    return 0;
}

int stmg_oc_update(stmg_t h, const double* d_rho, const double* d_grad, double volume,
                   double move, double eta, double rho_min, double* d_rho_new) {
    if (!h || !d_rho || !d_grad || !d_rho_new) return fail(STMG_EINVAL, "null argument");
    if (!(volume > 0.0 && volume <= 1.0) || !(move > 0.0) || !(eta > 0.0 && eta <= 1.0) ||
        !(rho_min >= 0.0 && rho_min < 1.0))
        return fail(STMG_EINVAL, "design update needs 0 < volume <= 1, move > 0, "
                                 "0 < eta <= 1 and 0 <= rho_min < 1");
    launch_oc_update(d_rho, d_grad, h->p.n_el, volume, move, eta, rho_min, d_rho_new, h->s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->s));
    return 0;
}

int stmg_get_info(stmg_t h, stmg_info* info) {
    if (!h || !info) return fail(STMG_EINVAL, "null argument");
    std::memset(info, 0, sizeof(*info));
    info->n_levels = (int)h->L.size();
    for (size_t i = 0; i < h->L.size() && i < 64; ++i) {
        const Level& l = h->L[i];
        info->n_el[i] = l.N;
        info->n_t[i] = l.Nt;
        info->h[i] = l.h;
        info->tau[i] = l.tau;
        info->w_diri[i] = l.W;
        info->lambda_eff[i] = l.lambda;
        if (i + 1 < h->L.size() && i < 63) info->path[i] = l.dir;
    }
    info->device_bytes = h->bytes;
    info->tail_level = h->o.fused == 1 ? h->tail_start : -1;
    return 0;
}

int stmg_destroy(stmg_t h) {
    if (!h) return 0;
    (void)hipStreamSynchronize(h->s);
    delete h;
    return 0;
}

#define STMG_BY_PRECISION(h, call) \
    ((h)->o.precision == STMG_MIXED ? call<float> : call<double>)

int stmg_level_apply(stmg_t h, int level, int transpose, const double* d_x, double* d_y) {
    CHK(check_level(h, level));
    if (!d_x || !d_y) return fail(STMG_EINVAL, "null vector");
    return STMG_BY_PRECISION(h, level_apply)(h, level, transpose, d_x, d_y);
}

int stmg_level_smooth(stmg_t h, int level, int transpose, int nu, const double* d_b, double* d_u) {
    CHK(check_level(h, level));
    if (!d_b || !d_u || nu < 0) return fail(STMG_EINVAL, "bad argument");
    return STMG_BY_PRECISION(h, level_smooth)(h, level, transpose, nu, d_b, d_u);
}

int stmg_level_presmooth_restrict(stmg_t h, int level, int transpose, int nu, const double* d_b,
                                  double* d_u, double* d_bc) {
    CHK(check_level(h, level));
    if (level + 1 >= (int)h->L.size()) return fail(STMG_EINVAL, "coarsest level has no restriction");
    if (!d_b || !d_u || !d_bc || nu < 0) return fail(STMG_EINVAL, "bad argument");
    return STMG_BY_PRECISION(h, level_presmooth_restrict)(h, level, transpose, nu, d_b, d_u, d_bc);
}

int stmg_level_prolong_postsmooth(stmg_t h, int level, int transpose, int nu, const double* d_b,
                                  const double* d_z, double* d_u) {
    CHK(check_level(h, level));
    if (level + 1 >= (int)h->L.size()) return fail(STMG_EINVAL, "coarsest level has no prolongation");
    if (!d_b || !d_u || !d_z || nu < 0) return fail(STMG_EINVAL, "bad argument");
    return STMG_BY_PRECISION(h, level_prolong_postsmooth)(h, level, transpose, nu, d_b, d_z, d_u);
}

int stmg_level_coarsest_solve(stmg_t h, int transpose, const double* d_b, double* d_z) {
    if (!h) return fail(STMG_EINVAL, "null handle");
    CHK(check_level(h, (int)h->L.size() - 1));
    if (!d_b || !d_z) return fail(STMG_EINVAL, "null vector");
    return STMG_BY_PRECISION(h, level_coarsest_solve)(h, transpose, d_b, d_z);
}

int stmg_vcycle(stmg_t h, int transpose, const double* d_b, double* d_u, double* rel_res) {
    CHK(check_level(h, 0));
    if (h->o.precision != STMG_FP64) return fail(STMG_EUNSUPPORTED, "stmg_vcycle needs an FP64 handle");
    if (!d_b || !d_u) return fail(STMG_EINVAL, "null vector");
    Level& f = h->L[0];
    CHK(copy_in<double>(h, f, d_b, f.b));
    CHK(copy_in<double>(h, f, d_u, f.u));
    if (h->o.debug_poison) {
        poison<double>(h, f, f.t);
        for (size_t i = 1; i < h->L.size(); ++i) {
            poison<double>(h, h->L[i], h->L[i].u);
            poison<double>(h, h->L[i], h->L[i].b);
            poison<double>(h, h->L[i], h->L[i].t);
        }
    }
    CHK(vcycle<double>(h, 0, transpose, false, false));
    if (rel_res) {
        double nb, r;
        CHK(norm64(h, f.b, f, &nb));
        CHK(residual_norm64(h, transpose, &r));
        *rel_res = r / nb;
    }
    CHK(copy_out<double>(h, f, f.u, d_u));
    HIPCHK(hipStreamSynchronize(h->s));
    return 0;
}

int stmg_stream_calibrate(const double* d_a, const double* d_b, double s, double* d_y, int64_t n,
                          int nontemporal, void* stream) {
    if (!d_a || !d_y || n < 0 || (n & 1)) return fail(STMG_EINVAL, "bad argument");
    if ((reinterpret_cast<uintptr_t>(d_a) | reinterpret_cast<uintptr_t>(d_b) |
         reinterpret_cast<uintptr_t>(d_y)) & 15)
        return fail(STMG_EINVAL, "vectors must be 16-byte aligned");
    if (launch_stream(d_a, d_b, s, d_y, n, nontemporal != 0, static_cast<hipStream_t>(stream)) != 0)
        return fail(STMG_EINVAL, "vector too long");
    HIPCHK(hipGetLastError());
    return 0;
}

int stmg_pass_geometry(int n_el, int n_t, int sweeps, int fp32, int fine, int* strip_cols,
                       int* strips, int* seg_rows, int* waves) {
    if (n_el < 1 || n_t < 1 || !strip_cols || !strips || !seg_rows || !waves)
        return fail(STMG_EINVAL, "bad argument");
    if (fused_geometry(n_el, n_t, sweeps, fp32 != 0, fine != 0, strip_cols, strips, seg_rows, waves) != 0)
        return fail(STMG_EINVAL, "sweeps must be in [0, " + std::to_string(fused_max_sweeps()) + "]");
    return 0;
}

const char* stmg_status_string(int status) {
    switch (status) {
        case STMG_OK: return "ok";
        case STMG_NOT_CONVERGED: return "not converged (cycle cap reached)";
        case STMG_DIVERGED: return "diverged";
        case STMG_EINVAL: return "invalid argument";
        case STMG_ENOMEM: return "out of device memory";
        case STMG_EHIP: return "HIP runtime error";
        case STMG_EUNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

const char* stmg_last_error(void) { return g_err.c_str(); }

}  // extern "C"
