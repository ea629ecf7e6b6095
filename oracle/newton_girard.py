"""The paper's closed forms for DMAS-n, in plain Python (test infrastructure only).

These are independent evaluations used to pin the FP64 oracle:

* ``dmas_bruteforce``   -- eq. (5): sum over all n-subsets of microphones of the
  product of their signed n-th roots (eq. (4)). O(M^n); tiny inputs only.
* ``dmas2_pairwise``    -- eq. (3): the classic second-order DMAS double loop.
* ``das``               -- eq. (2): delay-and-sum.
* ``power_sums``        -- eq. (7): P_k = sum_i s_i^k.
* ``ng_partitions``     -- eq. (8): E_n as a signed sum over the integer
  partitions of n (k_1 + 2 k_2 + ... + n k_n = n) of
  prod_i P_i^{k_i} / (k_i! i^{k_i}), sign (-1)^{n - sum k_i}.
* ``ng_explicit``       -- eqs. (9)-(12): the expansions for n = 2..5.
* ``newton_recurrence`` -- the recursive form of the same identities:
  k e_k = sum_{i=1..k} (-1)^{i-1} e_{k-i} P_i.
* ``coherence_factor``  -- eq. (13).

Values may be Python floats or ``fractions.Fraction`` (exact arithmetic).
"""

from __future__ import annotations

import itertools
import math
from fractions import Fraction
from typing import Dict, Iterator, List, Sequence, Tuple


def signed_root(x, n: int):
    """Eq. (4): sgn(x) |x|^(1/n); sgn(0) = 0."""
    if n == 1:
        return x
    if x == 0:
        return 0.0
    r = abs(float(x)) ** (1.0 / n)
    return r if x > 0 else -r


def das(xs: Sequence) -> float:
    """Eq. (2)."""
    return sum(xs)


def dmas2_pairwise(xs: Sequence[float]) -> float:
    """Eq. (3): sum_{i<j} sgn(x_i x_j) sqrt(|x_i x_j|)."""
    total = 0.0
    n = len(xs)
    for i in range(n - 1):
        for j in range(i + 1, n):
            p = float(xs[i]) * float(xs[j])
            sg = (1 if p > 0 else 0) - (1 if p < 0 else 0)
            total += sg * math.sqrt(abs(p))
    return total


def elementary_bruteforce(s: Sequence, n: int):
    """Sum over all n-subsets of the product of their members (eq. (5) on given s)."""
    total = 0
    for comb in itertools.combinations(range(len(s)), n):
        p = 1
        for i in comb:
            p = p * s[i]
        total = total + p
    return total


def dmas_bruteforce(xs: Sequence[float], n: int) -> float:
    """Eq. (5) with eq. (4): O(M^n) evaluation from the combinatorial definition."""
    s = [signed_root(x, n) for x in xs]
    return float(elementary_bruteforce(s, n))


def power_sums(s: Sequence, n: int) -> List:
    """Eq. (7): [P_1, ..., P_n]."""
    return [sum(v ** k for v in s) for k in range(1, n + 1)]


def partitions(n: int) -> Iterator[Dict[int, int]]:
    """All multiplicity vectors {i: k_i} with sum_i i k_i = n."""
    def rec(remaining: int, largest: int):
        if remaining == 0:
            yield {}
            return
        for part in range(min(remaining, largest), 0, -1):
            for rest in rec(remaining - part, part):
                d = dict(rest)
                d[part] = d.get(part, 0) + 1
                yield d
    yield from rec(n, n)


def ng_partitions(P: Sequence, n: int):
    """Eq. (8): E_n from power sums P[0] = P_1, ..., P[n-1] = P_n."""
    exact = isinstance(P[0], Fraction)
    total = Fraction(0) if exact else 0.0
    for k in partitions(n):
        sign = -1 if (n - sum(k.values())) % 2 else 1
        term = Fraction(1) if exact else 1.0
        for i, ki in k.items():
            denom = math.factorial(ki) * i ** ki
            term = term * P[i - 1] ** ki / (Fraction(denom) if exact else float(denom))
        total = total + sign * term
    return total


def ng_explicit(P: Sequence, n: int):
    """Eqs. (9)-(12): the printed expansions for orders 2 to 5."""
    P1 = P[0]
    if n == 1:
        return P1
    P2 = P[1]
    if n == 2:
        return (P1 ** 2 - P2) / 2
    P3 = P[2]
    if n == 3:
        return (P1 ** 3 + 2 * P3 - 3 * P1 * P2) / 6
    P4 = P[3]
    if n == 4:
        return (P1 ** 4 - 6 * P4 + 3 * P2 ** 2 - 6 * P2 * P1 ** 2 + 8 * P3 * P1) / 24
    P5 = P[4]
    if n == 5:
        return (P1 ** 5 - 10 * P2 * P1 ** 3 + 15 * P2 ** 2 * P1 + 20 * P3 * P1 ** 2
                - 20 * P3 * P2 - 30 * P1 * P4 + 24 * P5) / 120
    raise ValueError("explicit expansions are printed for n = 2..5 only")


def newton_recurrence(P: Sequence, n: int):
    """k e_k = sum_{i=1..k} (-1)^(i-1) e_{k-i} P_i, e_0 = 1; returns e_n."""
    exact = isinstance(P[0], Fraction)
    e = [Fraction(1) if exact else 1.0]
    for k in range(1, n + 1):
        acc = Fraction(0) if exact else 0.0
        for i in range(1, k + 1):
            term = e[k - i] * P[i - 1]
            acc = acc + term if i % 2 == 1 else acc - term
        e.append(acc / k)
    return e[n]


def complete_homogeneous(a: Sequence, n: int):
    """h_n(a): sum over multisets of size n (brute force over combinations with repetition)."""
    total = 0
    for comb in itertools.combinations_with_replacement(range(len(a)), n):
        p = 1
        for i in comb:
            p = p * a[i]
        total = total + p
    return total


def coherence_factor(xs: Sequence[float], eps: float = 0.0) -> float:
    """Eq. (13): (sum x)^2 / (M sum x^2 + eps)."""
    a = sum(xs)
    b = sum(v * v for v in xs)
    return a * a / (len(xs) * b + eps)


def pixel(xs: Sequence[float], n: int, use_cf: bool, eps: float = 1e-20) -> Tuple[float, float]:
    """(E_n by brute force, y = E_n * CF) for one pixel's delayed samples."""
    e = dmas_bruteforce(xs, n)
    cf = coherence_factor(xs, eps) if use_cf else 1.0
    return e, e * cf
