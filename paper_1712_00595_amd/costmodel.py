"""Iteration bounds of an update from the size of its seed (Theorem 2 and
the effects of Delta G, Section 3.3).

Every iteration multiplies the L1 norm of the propagated vector by at most
(1-c) (B~^T is column stochastic), so an update whose seed has norm q stops
(first i >= 1 with ||x^(i)||_1 <= eps) after at most
ceil(log(eps / q) / log(1 - c)) iterations, and at least one.  Before any
propagation, q <= (1-c) ||D r_old||_1 bounds the seed from the batch and the
old scores alone; the library reports ||D r_old||_1 as ``dr_l1``.
"""

from __future__ import annotations

import math


def iterations_bound(q_l1: float, eps: float, c: float) -> int:
    """Largest number of iterations an update with seed norm q_l1 can take."""
    if q_l1 <= eps:
        return 1
    return max(1, math.ceil(math.log(eps / q_l1) / math.log(1.0 - c) - 1e-12))


def seed_bound(dr_l1: float, c: float) -> float:
    """Upper bound of ||q_offset||_1 from ||D r_old||_1."""
    return (1.0 - c) * dr_l1


def iterations_bound_before(dr_l1: float, eps: float, c: float) -> int:
    """Iteration bound known before propagation (from ||D r_old||_1)."""
    return iterations_bound(seed_bound(dr_l1, c), eps, c)
