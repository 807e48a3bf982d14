"""FP64 singular values of the correlation blocks and their effective rank (test infrastructure
only; the HIP library never imports this module).

App. A.6: for each degree l the block A_l = [sigma_lmm'] (here C^l, assembled by the oracle's
definition of eq. sigmalmm with shells for the radial index) has rank at most the number of radial
indices, and rotating h multiplies it by a unitary matrix, so its singular values do not change.
App. B.1: the effective rank is r_eff(l) = min{k : s_{k+1}(A_l) / s_k(A_l) < rho}, with
s_1 >= s_2 >= ... the singular values (the paper uses rho = 0.2).  Readings where the paper is
silent: k runs over the min(2l+1, R) values of the block; when no ratio is below rho, r_eff is that
count; a zero block has r_eff = 0.  Library primitive used as a step: numpy's SVD.
"""
from __future__ import annotations

import numpy as np

from . import blk, coeff_assemble


def block_singular_values(Lp: int, Rp: int, f, Lf: int, h, Lh: int, w):
    """[Lp + 1] arrays: the descending singular values of C^l, min(2l+1, Rp) of them per degree."""
    C = coeff_assemble(Lp, Rp, f, Lf, h, Lh, w)
    out = []
    for l in range(Lp + 1):
        A = C[blk(l):blk(l + 1)].reshape(2 * l + 1, 2 * l + 1)
        s = np.linalg.svd(A, compute_uv=False)
        out.append(s[: min(2 * l + 1, Rp)])
    return out


def effective_rank(s, rho: float = 0.2) -> int:
    """min{k >= 1 : s_{k+1} / s_k < rho} over the given descending values (see the module note)."""
    s = np.asarray(s, dtype=np.float64)
    if s.size == 0 or not s[0] > 0.0:
        return 0
    for k in range(1, s.size):
        if s[k] < rho * s[k - 1]:
            return k
    return int(s.size)
