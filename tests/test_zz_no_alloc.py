"""GPU test of the allocation-free gradient entry point: stmg_gradient_noalloc must give
the bits of stmg_gradient (a handle built from the same problem and design) on two
calls in a row, the second on a smaller problem, so that the shared device scratch
is reused with stale contents from the first call; sizes beyond the scratch are
rejected before any device work."""
from __future__ import annotations

import numpy as np
import pytest

from tests.helpers import I, to_dev

pytestmark = pytest.mark.gpu


def _pair(B, n_el, n_t, seed, kappa_min, cuda, p_c):
    import torch
    prob = B.Problem(n_el, n_t, k_ins=kappa_min, c_ins=0.5, p_c=p_c)
    rho = to_dev(np.clip(I.block_density(n_el, 16, seed=seed) + 0.25 *
                         np.random.default_rng(seed).random(n_el), 0.0, 1.0), cuda)
    s = B.Solver(prob, rho, nu=5)
    u, st = s.solve_forward()
    lam, sta = s.solve_adjoint()
    assert st.status == 0 and sta.status == 0
    ref = s.gradient(u, lam)
    out = torch.full_like(ref, float("nan"))
    B.stmg_gradient_noalloc(prob.c_struct(), rho, u, lam, out)
    torch.cuda.synchronize()
    s.close()
    return ref, out


def test_gradient_noalloc_matches_handle_gradient(cuda):
    import torch

    from paper_2505_10168_amd import binding as B
    # the second call is smaller in both directions; capacity term on (p_c = 2) and off
    for n_el, n_t, seed, kmin, p_c in [(512, 1536, 4, 1e-3, 2.0), (96, 160, 7, 1e-2, 0.0)]:
        ref, out = _pair(B, n_el, n_t, seed, kmin, cuda, p_c)
        print(f"noalloc gradient {n_el}x{n_t}: max|g| = {ref.abs().max().item():.3e}, "
              f"bitwise equal = {torch.equal(ref, out)}", flush=True)
        assert torch.isfinite(out).all()
        assert torch.equal(ref, out)


def test_gradient_noalloc_rejects_sizes_beyond_the_scratch(cuda):
    import torch

    from paper_2505_10168_amd import binding as B
    # 2^20 elements x 2^17 steps needs 2^20 * (1024 + 2) doubles; the tensors passed are
    # small, which is safe because the size check comes before any device work
    prob = B.Problem(1 << 20, 1 << 17)
    x = torch.zeros(4, dtype=torch.float64, device=cuda)
    with pytest.raises(B.StmgError) as e:
        B.stmg_gradient_noalloc(prob.c_struct(), x, x, x, x)
    assert e.value.code == B.STMG_EINVAL
    assert "scratch" in str(e.value)
