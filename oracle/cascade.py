"""Bound-then-exact cascade and the benefit inequality (test infrastructure).

Sec. 1 and Sec. 6: a conservative bound sits in front of the exact (costly)
test; only queries the bound calls positive reach the exact test.  The final
answer is g where the bound says 1 and 0 elsewhere, so it equals g for every
query iff the bound has no false negative.

Sec. 6 ("Tightness", Eq. Benefit): with bound times t_a, t_b, false-positive
rates p_a, p_b and exact-test time t, method a wins iff
t_a + p_a t < t_b + p_b t, i.e. t < (t_b - t_a)/(p_a - p_b) when p_a > p_b
and t > (t_b - t_a)/(p_a - p_b) when p_a < p_b.
"""

from __future__ import annotations

import numpy as np


def cascade(h, g) -> np.ndarray:
    """answer_i = g_i if h_i else 0."""
    return (np.asarray(h).astype(bool) & np.asarray(g).astype(bool)).astype(np.uint8)


def break_even(t_a: float, t_b: float, p_a: float, p_b: float) -> float:
    """t* = (t_b - t_a) / (p_a - p_b), the exact-test cost where a and b tie."""
    return (t_b - t_a) / (p_a - p_b)


def a_wins(t_a: float, t_b: float, p_a: float, p_b: float, t: float) -> bool:
    """Total time per query n t_i + n p_i t, compared directly."""
    return t_a + p_a * t < t_b + p_b * t


def cascade_time(t_bound: float, p_pos: float, t_exact: float) -> float:
    """Time per query of bound + exact on the positives."""
    return t_bound + p_pos * t_exact
