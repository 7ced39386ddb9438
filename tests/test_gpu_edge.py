"""Degenerate and ragged grids on the main (rediscretised) path: a single level, one
element, one time step, sizes that cannot halve, hierarchies forced onto tiny levels.
Path, V-cycle iterates and the converged solve against the oracle, for the streaming,
streaming-without-tail and reference kernels."""
from __future__ import annotations

import numpy as np
import pytest

from tests.helpers import I, O, oracle_setup, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

EDGE = [
    # (id, rho, n_t, kappa_min, options)
    ("1x1", np.array([0.6]), 1, 1e-2, {}),
    ("1x2_two_levels", np.array([0.6]), 2, 1e-2, {"max_levels": 2}),
    ("2x1_two_levels", np.array([0.2, 0.9]), 1, 1e-2, {"max_levels": 2}),
    ("2x2_three_levels", np.array([0.2, 0.9]), 2, 1e-2, {"max_levels": 3}),
    ("1x8_four_levels", np.array([0.7]), 8, 1e-2, {"max_levels": 4}),
    ("8x1_four_levels", I.block_density(8, 2, seed=9), 1, 1e-3, {"max_levels": 4}),
    ("3x5_cannot_halve", I.block_density(3, 1, seed=4), 5, 1e-2, {"max_levels": 3}),
    ("7x128_x_cannot_halve", I.block_density(7, 1, seed=6), 128, 1e-3, {}),
    ("128x7_t_cannot_halve", I.block_density(128, 8, seed=8), 7, 1e-3, {}),
    ("62x66_ragged", I.block_density(62, 2, seed=10), 66, 1e-3, {"max_levels": 5}),
]


@pytest.mark.parametrize("case", EDGE, ids=[c[0] for c in EDGE])
@pytest.mark.parametrize("fused", [1, 2, 0])
@pytest.mark.parametrize("transpose", [0, 1])
def test_edge_grids_match_oracle(case, fused, transpose, cuda):
    from paper_2505_10168_amd import binding as B
    _, rho, n_t, kmin, extra = case
    prob = B.Problem(len(rho), n_t, k_ins=kmin)
    s = B.Solver(prob, to_dev(rho, cuda), nu=2, fused=fused, max_cycles=400, **extra)
    oextra = {k: v for k, v in extra.items() if k != "max_cycles"}
    mat, lv, h = oracle_setup(rho, n_t, kmin, nu=2, **oextra)
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
    x, st = (s.solve_adjoint if transpose else s.solve_forward)(bd)
    ref = O.direct_solve(lv, b, transpose=bool(transpose))
    assert st.status == 0 and st.rel_residual < 1e-10
    assert rel(to_np(x), ref) <= 1e-8
    s.close()


@pytest.mark.parametrize("case", EDGE, ids=[c[0] for c in EDGE])
@pytest.mark.parametrize("transpose", [0, 1])
@pytest.mark.parametrize("inner", [1, 4, 8])
def test_edge_grids_mixed_precision(case, transpose, inner, cuda):
    """FP32 inner V-cycles in FP64 defect correction reach the same 1e-10 residual and
    the direct solution on the same grids, with 1, 4 (the default) or 8 inner cycles per
    correction (the fused finest-level passes: nu = 2)."""
    from paper_2505_10168_amd import binding as B
    _, rho, n_t, kmin, extra = case
    prob = B.Problem(len(rho), n_t, k_ins=kmin)
    s = B.Solver(prob, to_dev(rho, cuda), nu=2, precision=B.STMG_MIXED, max_cycles=400,
                 inner_cycles=inner, **extra)
    mat, lv, h = oracle_setup(rho, n_t, kmin, nu=2, **extra)
    b = O.load_vector(lv, 1.0)
    if transpose:
        b = O.adjoint_rhs(lv, b)
    x, st = (s.solve_adjoint if transpose else s.solve_forward)(to_dev(b, cuda))
    ref = O.direct_solve(lv, b, transpose=bool(transpose))
    assert st.status == 0 and st.rel_residual < 1e-10
    assert rel(to_np(x), ref) <= 1e-8
    s.close()


@pytest.mark.parametrize("extra", [{"interp": 1}, {"reassembly": 1}, {"reassembly": 2},
                                   {"M_min_elems": 100}, {"reassembly": 3},
                                   {"reassembly": 3, "fused": 0}],
                         ids=["B", "K", "D", "M_guard", "P", "P_one_step"])
@pytest.mark.parametrize("transpose", [0, 1])
def test_variants_in_mixed_precision(extra, transpose, cuda):
    """The method variants with FP32 inner cycles reach the FP64 residual 1e-10 and the
    direct solution."""
    from paper_2505_10168_amd import binding as B
    rho, n_t, kmin = I.block_density(256, 16, seed=7), 600, 1e-3
    prob = B.Problem(len(rho), n_t, k_ins=kmin)
    s = B.Solver(prob, to_dev(rho, cuda), nu=5, precision=B.STMG_MIXED, max_cycles=400, **extra)
    mat, lv, h = oracle_setup(rho, n_t, kmin, nu=5)
    b = O.load_vector(lv, 1.0)
    if transpose:
        b = O.adjoint_rhs(lv, b)
    x, st = (s.solve_adjoint if transpose else s.solve_forward)(to_dev(b, cuda))
    ref = O.direct_solve(lv, b, transpose=bool(transpose))
    print(extra, st.cycles, f"{st.rel_residual:.2e}", f"{rel(to_np(x), ref):.1e}")
    assert st.status == 0 and st.rel_residual < 1e-10
    assert rel(to_np(x), ref) <= 1e-8
    s.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_bp_diverges_on_the_variant_case(precision, cuda):
    """BP on the same case (path xttxtxxx) is unstable (Section 5.2): the oracle's FP64
    cycles grow the error by about 1e28 per cycle, and both precisions stop with
    'diverged'.  BP in mixed precision where it converges is covered on small grids."""
    from paper_2505_10168_amd import binding as B
    rho, n_t, kmin = I.block_density(256, 16, seed=7), 600, 1e-3
    prob = B.Problem(len(rho), n_t, k_ins=kmin)
    s = B.Solver(prob, to_dev(rho, cuda), nu=5, precision=precision, max_cycles=400,
                 reassembly=B.STMG_REASSEMBLE_P, interp=B.STMG_INTERP_B)
    assert s.info()["path"] == "xttxtxxx"
    _, st = s.solve_forward()
    assert st.status == B.STMG_DIVERGED and st.cycles <= 3
    s.close()
