"""Memory-optimised Runge-Kutta coefficients of App. A, in exact rationals
(oracle; test infrastructure).

App. A, eqs. (A1)-(A4): with y^(1) = y_0 and the vectors
Y = (y^(1), ..., y^(n)), K = (y_0, k_1, ..., k_{n-1}), the relation
y^(i) = y_0 + dt sum_{j<i} a_ij k_j is Y = M K with M lower triangular
(first column ones, entries dt a_ij below the diagonal).  Inverting M
expresses each dt k_j through y^(1..j+1).  Substituting into
y^(i+1) = y_0 + dt sum_{j<=i} a_{i+1,j} k_j while keeping the newest k_i
explicit gives eq. (A6): y^(i+1) = sum_j a*_ij y^(j) + dt a_{i+1,i} k_i;
the same substitution in the update gives eq. (A7):
y_1 = sum_j b*_j y^(j) + dt b_n k_n.

dt is absorbed by working with dt*k_j as the unknowns, so the coefficients
are pure rationals.  Standard tableaux used: Heun's third-order method,
the classic RK4, and the fifth-order weights of Cash and Karp.
"""
from __future__ import annotations

from fractions import Fraction as F


def _inverse_lower(M):
    n = len(M)
    inv = [[F(0)] * n for _ in range(n)]
    for col in range(n):
        e = [F(int(r == col)) for r in range(n)]
        x = [F(0)] * n
        for r in range(n):
            s = e[r] - sum(M[r][c] * x[c] for c in range(r))
            x[r] = s / M[r][r]
        for r in range(n):
            inv[r][col] = x[r]
    return inv


def modified_tableau(A, b):
    """A: strictly lower-triangular Butcher matrix (n x n, Fractions), b: weights.
    Returns (a_star, b_star): a_star[i-1] holds the coefficients of y^(1..i)
    in y^(i+1) for i = 1..n-1, b_star the coefficients of y^(1..n) in y_1."""
    n = len(b)
    # Y = M K' with K' = (y0, dt k_1, ..., dt k_{n-1})
    M = [[F(0)] * n for _ in range(n)]
    for r in range(n):
        M[r][0] = F(1)
        for c in range(1, r + 1):
            M[r][c] = F(A[r][c - 1])
    Minv = _inverse_lower(M)      # K' = Minv Y

    def combine(weights_on_k, upto):
        # y0 + sum_{j=1}^{upto} w_j (dt k_j), each dt k_j expressed via Y
        coef = [F(0)] * n
        coef[0] += 1
        for j in range(1, upto + 1):
            w = F(weights_on_k[j - 1])
            for m in range(n):
                coef[m] += w * Minv[j][m]
        return coef

    a_star = []
    for i in range(1, n):
        coef = combine([A[i][j] for j in range(i - 1)], i - 1)
        a_star.append(coef[:i])
    b_star = combine(list(b[:n - 1]), n - 1)
    return a_star, b_star


def heun3():
    A = [[0, 0, 0], [F(1, 3), 0, 0], [0, F(2, 3), 0]]
    return [[F(v) for v in r] for r in A], [F(1, 4), F(0), F(3, 4)]


def rk4():
    A = [[0, 0, 0, 0], [F(1, 2), 0, 0, 0], [0, F(1, 2), 0, 0], [0, 0, F(1), 0]]
    return [[F(v) for v in r] for r in A], [F(1, 6), F(1, 3), F(1, 3), F(1, 6)]


def cash_karp5():
    A = [[0, 0, 0, 0, 0, 0],
         [F(1, 5), 0, 0, 0, 0, 0],
         [F(3, 40), F(9, 40), 0, 0, 0, 0],
         [F(3, 10), F(-9, 10), F(6, 5), 0, 0, 0],
         [F(-11, 54), F(5, 2), F(-70, 27), F(35, 27), 0, 0],
         [F(1631, 55296), F(175, 512), F(575, 13824), F(44275, 110592), F(253, 4096), 0]]
    b = [F(37, 378), F(0), F(250, 621), F(125, 594), F(0), F(512, 1771)]
    return [[F(v) for v in r] for r in A], b
