"""HIP path against the FP64 oracle, element by element (tolerances: 1e-14 for a single
operator application, 1e-13 for a few sweeps, 1e-12 per V-cycle iterate)."""
from __future__ import annotations

import numpy as np
import pytest

from tests.helpers import I, O, oracle_setup, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

# (name, rho, n_t, kappa_min, c_ins, solver options)
CASES = {
    # configuration 1 exactly: 64 x 64, kappa = 1, V(2,2)
    "uniform_64x64": (np.ones(64), 64, 1.0, 1.0, {}),
    # high contrast, several strips and segments, ragged in x and t, t cannot halve below 75
    "block_256x600": (I.block_density(256, 16, seed=7), 600, 1e-3, 1.0, {"nu": 3}),
    # varying heat capacity too, x stops at 75 elements (odd)
    "ramp_300x256": (I.ramp_design(300, 1.0, 10.0, 0.5), 256, 1e-4, 1e-2, {"nu": 2}),
}


def make_pair(name, cuda, fused=1, **extra):
    from paper_2505_10168_amd import binding as B
    rho, n_t, kmin, c_ins, opts = CASES[name]
    opts = dict(opts, **extra)
    prob = B.Problem(len(rho), n_t, k_ins=kmin, c_ins=c_ins)
    # debug_poison: the per-level calls fill their internal outputs with NaN first
    opts.setdefault("debug_poison", 1)
    solver = B.Solver(prob, to_dev(rho, cuda), fused=fused, **opts)
    oopts = {k: v for k, v in opts.items()
             if k in ("nu", "max_levels", "min_coarse_dofs", "max_cycles")}
    mat, lv, h = oracle_setup(rho, n_t, kmin, c_ins=c_ins, **oopts)
    return solver, mat, lv, h


@pytest.mark.parametrize("name", list(CASES))
def test_hierarchy_matches_oracle(name, cuda):
    s, _, _, h = make_pair(name, cuda)
    info = s.info()
    assert info["path"] == h.path
    assert info["n_el"] == [l.n_el for l in h.levels]
    assert info["n_t"] == [l.n_t for l in h.levels]
    for a, l in zip(info["w_diri"], h.levels):
        assert a == pytest.approx(l.W, rel=1e-15)
    for a, b in zip(info["lambda_eff"], h.lambdas):
        assert a == pytest.approx(b, rel=1e-14)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("transpose", [0, 1])
def test_apply_every_level(name, transpose, cuda):
    from paper_2505_10168_amd import binding as B
    s, _, _, h = make_pair(name, cuda)
    for l, lev in enumerate(h.levels):
        x = np.random.default_rng(10 + l).standard_normal(lev.shape)
        y = to_dev(np.full(lev.shape, np.nan), cuda)   # every entry must be written
        B.stmg_level_apply(s.handle, l, transpose, to_dev(x, cuda), y)
        ref = O.apply_J(lev, x, bool(transpose))
        assert rel(to_np(y), ref) <= 1e-14, (l, rel(to_np(y), ref))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("transpose", [0, 1])
@pytest.mark.parametrize("fused", [1, 0])
@pytest.mark.parametrize("nu", [1, 2, 5, 10, 20])
def test_smooth(name, transpose, fused, nu, cuda):
    from paper_2505_10168_amd import binding as B
    s, _, _, h = make_pair(name, cuda, fused=fused)
    for l in (0, len(h.levels) - 1):
        lev = h.levels[l]
        rng = np.random.default_rng(100 + l)
        u = rng.standard_normal(lev.shape)
        b = rng.standard_normal(lev.shape)
        ud = to_dev(u, cuda)
        B.stmg_level_smooth(s.handle, l, transpose, nu, to_dev(b, cuda), ud)
        ref = O.jacobi(h, l, u, b, nu, bool(transpose))
        assert rel(to_np(ud), ref) <= 1e-13


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("transpose", [0, 1])
@pytest.mark.parametrize("fused", [1, 0])
def test_presmooth_restrict_and_prolong_postsmooth(name, transpose, fused, cuda):
    from paper_2505_10168_amd import binding as B
    s, _, _, h = make_pair(name, cuda, fused=fused)
    nu = h.opts.nu
    for l in range(len(h.levels) - 1):
        lev, cl, d = h.levels[l], h.levels[l + 1], h.directions[l]
        rng = np.random.default_rng(200 + l)
        u = rng.standard_normal(lev.shape)
        b = rng.standard_normal(lev.shape)
        z = rng.standard_normal(cl.shape)
        # pre-smoothing and restriction (Algorithm 1)
        ud = to_dev(u, cuda)
        bc = to_dev(np.full(cl.shape, np.nan), cuda)
        B.stmg_level_presmooth_restrict(s.handle, l, transpose, nu, to_dev(b, cuda), ud, bc)
        u_ref = O.jacobi(h, l, u, b, nu, bool(transpose))
        bc_ref = O.restrict(lev, d, b - O.apply_J(lev, u_ref, bool(transpose)))
        assert rel(to_np(ud), u_ref) <= 1e-13
        assert rel(to_np(bc), bc_ref) <= 1e-13
        # prolongation and post-smoothing
        ud = to_dev(u, cuda)
        B.stmg_level_prolong_postsmooth(s.handle, l, transpose, nu, to_dev(b, cuda),
                                        to_dev(z, cuda), ud)
        ref = O.jacobi(h, l, u + O.prolong(lev, d, z), b, nu, bool(transpose))
        assert rel(to_np(ud), ref) <= 1e-13


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("transpose", [0, 1])
def test_coarsest_solve(name, transpose, cuda):
    from paper_2505_10168_amd import binding as B
    s, _, _, h = make_pair(name, cuda)
    lev = h.levels[-1]
    b = np.random.default_rng(3).standard_normal(lev.shape)
    z = to_dev(np.full(lev.shape, np.nan), cuda)
    B.stmg_level_coarsest_solve(s.handle, transpose, to_dev(b, cuda), z)
    ref = O.direct_solve(lev, b, bool(transpose))
    assert rel(to_np(z), ref) <= 1e-13


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("transpose", [0, 1])
@pytest.mark.parametrize("fused", [1, 2, 0])
def test_vcycle_iterates(name, transpose, fused, cuda):
    from paper_2505_10168_amd import binding as B
    s, _, lv, h = make_pair(name, cuda, fused=fused)
    b = O.load_vector(lv, 1.0)
    if transpose:
        b = O.adjoint_rhs(lv, b)
    u = np.zeros(lv.shape)
    ud = to_dev(u, cuda)
    bd = to_dev(b, cuda)
    nb = np.linalg.norm(b)
    for it in range(6):
        r_gpu = B.stmg_vcycle(s.handle, transpose, bd, ud)
        u = O.vcycle(h, 0, u, b, bool(transpose))
        assert rel(to_np(ud), u) <= 1e-12, (it, rel(to_np(ud), u))
        r_ref = np.linalg.norm(O.apply_J(lv, u, bool(transpose)) - b) / nb
        assert r_gpu == pytest.approx(r_ref, rel=1e-9, abs=1e-15)


# first level of the single-workgroup tail with fused = 1 (the coarsest level of
# ramp_300x256 has 75 elements, beyond the tail kernel's dense solve)
TAIL_LEVEL = {"uniform_64x64": 1, "block_256x600": 6, "ramp_300x256": -1}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("transpose", [0, 1])
def test_fused_and_reference_paths_identical(name, transpose, cuda):
    """Streaming kernels with the LDS tail (1), streaming kernels on every level (2)
    and one kernel per step (0) give the same bits."""
    from paper_2505_10168_amd import binding as B
    outs = []
    for fused in (1, 2, 0):
        s, _, lv, h = make_pair(name, cuda, fused=fused)
        assert s.info()["tail_level"] == (TAIL_LEVEL[name] if fused == 1 else -1)
        b = O.load_vector(lv, 1.0)
        if transpose:
            b = O.adjoint_rhs(lv, b)
        bd = to_dev(b, cuda)
        ud = to_dev(np.zeros(lv.shape), cuda)
        for _ in range(3):
            B.stmg_vcycle(s.handle, transpose, bd, ud)
        outs.append(to_np(ud))
    assert np.array_equal(outs[0], outs[2])
    assert np.array_equal(outs[1], outs[2])


def test_solve_uniform_64x64_matches_oracle(cuda):
    s, _, lv, h = make_pair("uniform_64x64", cuda)
    u, st = s.solve_forward()
    b = O.load_vector(lv, 1.0)
    ref = O.stmg_solve(h, b)
    assert st.status == 0 and ref.status == "converged"
    assert st.cycles == ref.cycles
    assert rel(to_np(u), ref.u) <= 1e-12
    np.testing.assert_allclose(st.history, ref.history, rtol=1e-8, atol=1e-15)
    assert st.rel_residual < 1e-10
    # converged answer against the exact discrete solution
    assert rel(to_np(u), O.direct_solve(lv, b)) <= 1e-9


@pytest.mark.parametrize("name", ["block_256x600", "ramp_300x256"])
@pytest.mark.parametrize("transpose", [0, 1])
def test_solve_matches_oracle(name, transpose, cuda):
    s, _, lv, h = make_pair(name, cuda, max_cycles=25)
    b = O.load_vector(lv, 1.0)
    if transpose:
        lam, st = s.solve_adjoint()
        ref = O.stmg_solve(h, O.adjoint_rhs(lv, b), transpose=True)
    else:
        lam, st = s.solve_forward()
        ref = O.stmg_solve(h, b)
    assert st.cycles == ref.cycles
    assert {0: "converged", 1: "max_cycles", 2: "diverged"}[st.status] == ref.status
    assert rel(to_np(lam), ref.u) <= 1e-12


@pytest.mark.parametrize("name,max_cycles", [("block_256x600", 3), ("block_256x600", 400),
                                             ("uniform_64x64", 3), ("uniform_64x64", 100)])
@pytest.mark.parametrize("transpose", [0, 1])
def test_pipelined_solve_returns_its_last_iterate(name, max_cycles, transpose, cuda):
    """The FP64 solve enqueues V-cycle k+1 before it tests cycle k.  It must return the
    k-th iterate exactly, both when the cycle cap ends it (no cycle runs ahead) and when
    the tolerance does (the cycle that ran ahead is discarded), with the residual history
    of those iterates.  On uniform_64x64 the finest pass stores u_k (the level below is
    the single-workgroup tail); on block_256x600 u_k is recomputed from the pass's input
    and the kept coarse correction when the iteration stops.  The assembled load (two
    rows in the finest passes) gives the iterates of the oracle's load vector passed in."""
    from paper_2505_10168_amd import binding as B
    s, _, lv, h = make_pair(name, cuda, max_cycles=max_cycles)
    b = O.load_vector(lv, 1.0)
    if transpose:
        b = O.adjoint_rhs(lv, b)
    bd = to_dev(b, cuda)
    solve = s.solve_adjoint if transpose else s.solve_forward
    u, st = solve(rhs=bd)
    if max_cycles == 3:
        assert st.status == B.STMG_NOT_CONVERGED and st.cycles == 3
    else:
        assert st.status == B.STMG_OK and st.cycles < max_cycles
    ref = to_dev(np.zeros(lv.shape), cuda)
    for k in range(st.cycles):
        r = B.stmg_vcycle(s.handle, transpose, bd, ref)
        assert st.history[k + 1] == pytest.approx(r, rel=1e-9)
    assert np.array_equal(to_np(u), to_np(ref))
    # the library's own load (read as two rows) instead of the oracle's vector: the same
    # values up to the rounding of their assembly
    u2, st2 = solve()
    assert st2.cycles == st.cycles and rel(to_np(u2), to_np(u)) <= 1e-14
    np.testing.assert_allclose(st2.history, st.history, rtol=1e-12)


# Coarsening and re-assembly variants (Section 5.1 K and D methods, the Algorithm 4
# small-feature guard, a fixed level count, the Section 7.2 field-independent D_eff):
# (name, case, libstmg options, oracle options)
VARIANTS = [
    ("K", "block_256x600", {"reassembly": 1}, {"reassembly": "K"}),
    ("D", "ramp_300x256", {"reassembly": 2}, {"reassembly": "D"}),
    ("M_guard", "block_256x600", {"M_min_elems": 100}, {"M_min_elems": 100}),   # xtttxxxx
    ("max_levels", "block_256x600", {"max_levels": 4}, {"max_levels": 4}),
    ("deff_simp", "ramp_300x256", {"deff_mode": 1}, {"deff_mode": "simp"}),
    ("B_block", "block_256x600", {"interp": 1}, {"interp": "B"}),
    ("B_ramp", "ramp_300x256", {"interp": 1}, {"interp": "B"}),
    ("P_block", "block_256x600", {"reassembly": 3}, {"reassembly": "P"}),
    ("P_ramp", "ramp_300x256", {"reassembly": 3}, {"reassembly": "P"}),
    ("BP_block", "block_256x600", {"reassembly": 3, "interp": 1}, {"reassembly": "P", "interp": "B"}),
    ("BP_ramp", "ramp_300x256", {"reassembly": 3, "interp": 1}, {"reassembly": "P", "interp": "B"}),
]


@pytest.mark.parametrize("variant", VARIANTS, ids=[v[0] for v in VARIANTS])
@pytest.mark.parametrize("transpose", [0, 1])
def test_variants_match_oracle(variant, transpose, cuda):
    from paper_2505_10168_amd import binding as B
    _, name, gpu_opts, oracle_opts = variant
    rho, n_t, kmin, c_ins, opts = CASES[name]
    prob = B.Problem(len(rho), n_t, k_ins=kmin, c_ins=c_ins)
    s = B.Solver(prob, to_dev(rho, cuda), **dict(opts, **gpu_opts))
    mat, lv, h = oracle_setup(rho, n_t, kmin, c_ins=c_ins, nu=opts.get("nu", 2), **oracle_opts)
    info = s.info()
    print(f"{variant[0]}: path {info['path']} (oracle {h.path})")
    assert info["path"] == h.path
    for a, l in zip(info["w_diri"], h.levels):
        assert a == pytest.approx(l.W, rel=1e-15)
    for a, b in zip(info["lambda_eff"], h.lambdas):
        assert a == pytest.approx(b, rel=1e-14)
    b = O.load_vector(lv, 1.0)
    if transpose:
        b = O.adjoint_rhs(lv, b)
    u = np.zeros(lv.shape)
    ud, bd = to_dev(u, cuda), to_dev(b, cuda)
    for it in range(3):
        B.stmg_vcycle(s.handle, transpose, bd, ud)
        u = O.vcycle(h, 0, u, b, bool(transpose))
        assert rel(to_np(ud), u) <= 1e-12, (it, rel(to_np(ud), u))


@pytest.mark.parametrize("transpose", [0, 1])
def test_bilinear_fused_and_reference_identical(transpose, cuda):
    """Bilinear time interpolation: fused smoothing passes with separate t transfers
    (fused = 1) and one kernel per step (fused = 0) give the same bits."""
    from paper_2505_10168_amd import binding as B
    outs = []
    for fused in (1, 0):
        s, _, lv, h = make_pair("block_256x600", cuda, fused=fused, interp=B.STMG_INTERP_B)
        assert s.info()["tail_level"] == -1
        b = O.load_vector(lv, 1.0)
        if transpose:
            b = O.adjoint_rhs(lv, b)
        bd, ud = to_dev(b, cuda), to_dev(np.zeros(lv.shape), cuda)
        for _ in range(3):
            B.stmg_vcycle(s.handle, transpose, bd, ud)
        outs.append(to_np(ud))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("name", ["block_256x600", "ramp_300x256"])
@pytest.mark.parametrize("transpose", [0, 1])
@pytest.mark.parametrize("interp", ["C", "B"])
def test_galerkin_levels_match_oracle(name, transpose, interp, cuda):
    """P reassembly: every coarse operator R J P (stored stencil) applied, and the
    coarsest level solved exactly (time stepping for C, band LU for B), against the
    oracle's sparse products."""
    import scipy.sparse.linalg as spla

    from paper_2505_10168_amd import binding as B
    s, _, lv, h = make_pair(name, cuda, reassembly=B.STMG_REASSEMBLE_P,
                            interp=B.STMG_INTERP_B if interp == "B" else B.STMG_INTERP_C)
    h = O.build_hierarchy(lv, O.Options(material=h.opts.material, nu=h.opts.nu, reassembly="P",
                                        interp=interp))
    info = s.info()
    assert info["path"] == h.path and info["tail_level"] == -1
    rng = np.random.default_rng(4)
    for l in range(1, info["n_levels"]):
        G = h.galerkin[l].T if transpose else h.galerkin[l]
        shape = h.levels[l].shape
        x = rng.standard_normal(shape)
        y = to_dev(np.full(shape, np.nan), cuda)
        B.stmg_level_apply(s.handle, l, transpose, to_dev(x, cuda), y)
        ref = (G @ x.ravel()).reshape(shape)
        print(f"level {l} {shape}: apply rel {rel(to_np(y), ref):.1e}")
        assert rel(to_np(y), ref) <= 1e-13
    last = info["n_levels"] - 1
    G = (h.galerkin[last].T if transpose else h.galerkin[last]).tocsc()
    b = rng.standard_normal(h.levels[last].shape)
    z = to_dev(np.full(b.shape, np.nan), cuda)
    B.stmg_level_coarsest_solve(s.handle, transpose, to_dev(b, cuda), z)
    ref = spla.spsolve(G, b.ravel()).reshape(b.shape)
    print(f"coarsest {b.shape}: rel {rel(to_np(z), ref):.1e}")
    assert rel(to_np(z), ref) <= 1e-12


@pytest.mark.parametrize("transpose", [0, 1])
def test_galerkin_fused_and_reference_identical_and_solve(transpose, cuda):
    """P reassembly: the fine level's fused passes and its one-kernel-per-step path give
    the same iterates; the solve reaches the direct solution."""
    from paper_2505_10168_amd import binding as B
    outs = []
    for fused in (1, 0):
        s, _, lv, h = make_pair("block_256x600", cuda, fused=fused, reassembly=B.STMG_REASSEMBLE_P)
        b = O.load_vector(lv, 1.0)
        if transpose:
            b = O.adjoint_rhs(lv, b)
        bd, ud = to_dev(b, cuda), to_dev(np.zeros(lv.shape), cuda)
        for _ in range(3):
            B.stmg_vcycle(s.handle, transpose, bd, ud)
        outs.append(to_np(ud))
    assert np.array_equal(outs[0], outs[1])
    s, _, lv, h = make_pair("block_256x600", cuda, reassembly=B.STMG_REASSEMBLE_P, max_cycles=300)
    b = O.load_vector(lv, 1.0)
    if transpose:
        b = O.adjoint_rhs(lv, b)
    u, st = (s.solve_adjoint if transpose else s.solve_forward)(to_dev(b, cuda))
    ref = O.direct_solve(lv, b, transpose=bool(transpose))
    print(f"P solve: {st.cycles} cycles, residual {st.rel_residual:.2e}, "
          f"factor {st.conv_factor:.3f}, rel err {rel(to_np(u), ref):.1e}")
    assert st.status == 0 and st.rel_residual < 1e-10
    assert rel(to_np(u), ref) <= 1e-8


GALERKIN_EDGE = [
    # (id, rho, n_t, kappa_min, extra options)
    ("odd_x_75x64", I.block_density(75, 5, seed=3), 64, 1e-2, {}),
    ("one_level", I.block_density(64, 8, seed=5), 64, 1e-3, {"max_levels": 1}),
    ("two_grid", I.block_density(64, 8, seed=5), 64, 1e-3, {"max_levels": 2}),
    ("tiny_2x2", np.array([0.3, 0.9]), 2, 1e-2, {"max_levels": 2}),
    ("single_element_1x8", np.array([0.7]), 8, 1e-2, {"max_levels": 3}),
]


@pytest.mark.parametrize("case", GALERKIN_EDGE, ids=[c[0] for c in GALERKIN_EDGE])
@pytest.mark.parametrize("transpose", [0, 1])
def test_galerkin_edge_cases(case, transpose, cuda):
    """P reassembly on grids that cannot halve, with one or two levels, and on the
    smallest grids: path and V-cycle iterates against the oracle."""
    from paper_2505_10168_amd import binding as B
    _, rho, n_t, kmin, extra = case
    prob = B.Problem(len(rho), n_t, k_ins=kmin)
    s = B.Solver(prob, to_dev(rho, cuda), nu=2, reassembly=B.STMG_REASSEMBLE_P, **extra)
    mat, lv, h = oracle_setup(rho, n_t, kmin, nu=2, reassembly="P", **extra)
    assert s.info()["path"] == h.path
    b = O.load_vector(lv, 1.0)
    if transpose:
        b = O.adjoint_rhs(lv, b)
    u = np.zeros(lv.shape)
    ud, bd = to_dev(u, cuda), to_dev(b, cuda)
    for it in range(3):
        B.stmg_vcycle(s.handle, transpose, bd, ud)
        u = O.vcycle(h, 0, u, b, bool(transpose))
        assert rel(to_np(ud), u) <= 1e-12, (it, rel(to_np(ud), u))
    s.close()


@pytest.mark.parametrize("case", GALERKIN_EDGE, ids=[c[0] for c in GALERKIN_EDGE])
@pytest.mark.parametrize("interp", [0, 1], ids=["C", "B"])
@pytest.mark.parametrize("transpose", [0, 1])
def test_galerkin_edge_cases_mixed_precision(case, interp, transpose, cuda):
    """P reassembly with FP32 inner cycles (FP32 copies of the stored stencils, FP64
    coarsest solves) on the same grids: the FP64 residual reaches 1e-10 and the solution
    the direct one.  On 75 x 64 (path ttt) BP diverges, as the FP64 oracle's cycles do
    (Section 5.2): the solve must say so."""
    from paper_2505_10168_amd import binding as B
    name, rho, n_t, kmin, extra = case
    prob = B.Problem(len(rho), n_t, k_ins=kmin)
    # P converges slowly on 75 x 64 (about 0.93 per cycle in the oracle)
    s = B.Solver(prob, to_dev(rho, cuda), nu=2, reassembly=B.STMG_REASSEMBLE_P,
                 precision=B.STMG_MIXED, interp=interp, max_cycles=1000, **extra)
    mat, lv, h = oracle_setup(rho, n_t, kmin, nu=2, reassembly="P",
                              interp="B" if interp else "C", **extra)
    assert s.info()["path"] == h.path
    b = O.load_vector(lv, 1.0)
    if transpose:
        b = O.adjoint_rhs(lv, b)
    x, st = (s.solve_adjoint if transpose else s.solve_forward)(to_dev(b, cuda))
    print(name, interp, transpose, st.status, st.cycles, f"{st.rel_residual:.2e}")
    if name == "odd_x_75x64" and interp == 1:
        assert st.status == B.STMG_DIVERGED
        s.close()
        return
    ref = O.direct_solve(lv, b, transpose=bool(transpose))
    assert st.status == 0 and st.rel_residual < 1e-10
    assert rel(to_np(x), ref) <= 1e-8
    s.close()


def test_galerkin_one_level_equals_rediscretised(cuda):
    """With a single level there is no coarse operator: P and R solve the same way."""
    from paper_2505_10168_amd import binding as B
    rho = I.block_density(64, 8, seed=5)
    prob = B.Problem(64, 64, k_ins=1e-3)
    outs = []
    for method in (B.STMG_REASSEMBLE_R, B.STMG_REASSEMBLE_P):
        s = B.Solver(prob, to_dev(rho, cuda), max_levels=1, reassembly=method)
        u, st = s.solve_forward()
        outs.append(to_np(u))
        s.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("nu", [7, 10, 20])
@pytest.mark.parametrize("transpose", [0, 1])
def test_multi_pass_smoothing_identical_to_reference(nu, transpose, cuda):
    """nu > 6: the fused path smooths in several passes per side (at most 6 steps each);
    its V-cycle iterates equal those of the one-kernel-per-step path bit for bit."""
    from paper_2505_10168_amd import binding as B
    outs = []
    for fused in (1, 0):
        s, _, lv, h = make_pair("block_256x600", cuda, fused=fused, nu=nu)
        b = O.load_vector(lv, 1.0)
        if transpose:
            b = O.adjoint_rhs(lv, b)
        bd, ud = to_dev(b, cuda), to_dev(np.zeros(lv.shape), cuda)
        for _ in range(2):
            B.stmg_vcycle(s.handle, transpose, bd, ud)
        outs.append(to_np(ud))
        s.close()
    assert np.array_equal(outs[0], outs[1])
