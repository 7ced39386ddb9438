"""Shared test helpers: oracle hierarchies mirroring a libstmg handle, tensor moves."""
from __future__ import annotations

import numpy as np

import oracle as O
from paper_2505_10168_amd import inputs as I


def material(kappa_min: float, c_ins: float = 1.0, c_con: float = 1.0, k_con: float = 1.0,
             p_k: float = 3.0, p_c: float = 2.0) -> O.Material:
    return O.Material(kappa_min, k_con, c_ins, c_con, p_k, p_c)


def oracle_setup(rho, n_t, kappa_min, length=1.0, t_final=0.1, c_ins=1.0, c_con=1.0,
                 w_override=None, **opt):
    mat = material(kappa_min, c_ins=c_ins, c_con=c_con)
    lv = O.make_fine_level(rho, mat, n_t, length, t_final, w_override=w_override)
    opts = O.Options(material=mat, **opt)
    h = O.build_hierarchy(lv, opts)
    if w_override is not None:
        for l in h.levels:
            l.w_override = w_override
    return mat, lv, h


def to_np(t):
    return t.detach().cpu().numpy()


def to_dev(a, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)


def rel(a, b) -> float:
    a, b = np.asarray(a), np.asarray(b)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def random_level_vec(level, seed):
    return np.random.default_rng(seed).standard_normal(level.shape)


__all__ = ["material", "oracle_setup", "to_np", "to_dev", "rel", "random_level_vec", "I", "O"]
