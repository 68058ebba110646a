"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

None of these checks re-types the oracle's own formulas: they use closed-form
counts, hand-written tables, exact rational arithmetic (``fractions``),
independent LAPACK solvers (NumPy), planted functions evaluated from their
exponent tuples, hand-worked template examples and the paper's printed
Table 3.  Each is chosen so that a plausible slip in the oracle (a dropped
term, a wrong sign or index, a transposed operand) fails one of them.
"""
import csv
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_1906_00142_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def planted_vector(orc, pl):
    """Planted coefficients in the oracle's order, matched by exponent tuple."""
    num, den = pl.coef_by_tuple()
    En = orc.monomials(pl.nvars, pl.deg_num)
    Ed = orc.monomials(pl.nvars, pl.deg_den)
    return np.array([num[tuple(int(t) for t in e)] for e in En]
                    + [den[tuple(int(t) for t in e)] for e in Ed[1:]])


# --------------------------------------------------------------------------
# monomial tables (Section 4.2 display; total-degree reading)
# --------------------------------------------------------------------------

def test_monomial_counts_closed_form(orc):
    for v in range(1, 6):
        for d in range(0, 7):
            assert len(orc.monomials(v, d)) == math.comb(v + d, d)


def test_monomial_tables_hand_listed(orc):
    # graded; within a degree, larger exponent of x1 first, then x2, ...
    assert orc.monomials(2, 2).tolist() == [
        [0, 0], [1, 0], [0, 1], [2, 0], [1, 1], [0, 2]]
    assert orc.monomials(3, 2).tolist() == [
        [0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1],
        [2, 0, 0], [1, 1, 0], [1, 0, 1], [0, 2, 0], [0, 1, 1], [0, 0, 2]]
    assert orc.monomials(1, 4).tolist() == [[0], [1], [2], [3], [4]]
    e33 = orc.monomials(3, 3).tolist()
    assert e33[10:] == [[3, 0, 0], [2, 1, 0], [2, 0, 1], [1, 2, 0], [1, 1, 1],
                        [1, 0, 2], [0, 3, 0], [0, 2, 1], [0, 1, 2], [0, 0, 3]]


def test_monomial_prefix_property(orc):
    # graded order: the degree-d' table is a prefix of the degree-d table
    for v in (2, 3, 4):
        full = orc.monomials(v, 4).tolist()
        for d in range(0, 4):
            assert full[:math.comb(v + d, d)] == orc.monomials(v, d).tolist()


def test_monomial_box_counts_and_hand_listed(orc):
    # the per-variable degree box of the Section 4.2 display: prod (u_k + 1)
    # exponents, graded order
    for box in ([0], [3], [2, 1], [1, 2], [3, 3], [2, 0, 1], [1, 1, 1, 1], [4, 2, 3, 1]):
        assert len(orc.monomials_box(box)) == math.prod(u + 1 for u in box)
    assert orc.monomials_box([2, 1]).tolist() == [[0, 0], [1, 0], [0, 1], [2, 0], [1, 1], [2, 1]]
    assert orc.monomials_box([1, 1, 1]).tolist() == [
        [0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, 0, 1], [0, 1, 1], [1, 1, 1]]


def test_monomial_box_restricted_to_total_degree_is_the_total_degree_set(orc):
    # the box [d]^v cut at total degree d is the total-degree set, in order
    for v, d in ((1, 4), (2, 3), (3, 2), (4, 2)):
        B = orc.monomials_box([d] * v)
        cut = B[B.astype(int).sum(axis=1) <= d]
        assert np.array_equal(cut, orc.monomials(v, d))


def test_unequal_degrees_recover_planted(orc):
    # numerator and denominator of different degrees (the display bounds p and
    # q separately): exact recovery from noise-free samples
    rng = np.random.default_rng(31)
    for v, dn, dq in ((1, 3, 1), (2, 1, 2), (2, 3, 2), (3, 2, 1)):
        pl = W.plant(rng, v, dn, dq)
        u = rng.uniform(0, 1, size=(v, 300))
        y = pl.value(u)
        c, st, rk, rs = orc.fit(u, y, dn, dq)
        want = planted_vector(orc, pl)
        assert st == 0 and len(c) == orc.num_coefs(v, dn, dq)
        np.testing.assert_allclose(c, want, rtol=1e-8, atol=1e-10)


def test_unknown_counts_of_the_workloads(orc):
    assert orc.num_coefs(2, 2, 2) == 6 + 5
    assert orc.num_coefs(3, 3, 3) == 20 + 19
    assert orc.num_coefs(4, 4, 4) == 70 + 69


# --------------------------------------------------------------------------
# candidate set F (Section 3.3 assumptions, Section 4)
# --------------------------------------------------------------------------

def _num_divisors(p):
    return sum(1 for k in range(1, p + 1) if p % k == 0)


def test_candidates_count_by_divisors(orc):
    c = orc.candidates_2d(1024, 64)
    # every product 64k <= 1024 contributes one pair per divisor of it
    assert len(c) == sum(_num_divisors(64 * k) for k in range(1, 17)) == 230
    assert len(orc.candidates_2d(1024, 32)) == sum(_num_divisors(32 * k) for k in range(1, 33))


def test_candidates_order_and_membership(orc):
    c = orc.candidates_2d(1024, 64)
    prods = c[:, 0].astype(int) * c[:, 1].astype(int)
    assert np.all(prods <= 1024) and np.all(prods % 64 == 0) and np.all(c >= 1)
    keys = [tuple(r) for r in c.tolist()]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    pow2 = [k for k in keys if (k[0] & (k[0] - 1)) == 0 and (k[1] & (k[1] - 1)) == 0]
    assert len(pow2) == 45
    assert keys[0] == (1, 64) and keys[-1] == (1024, 1)


# --------------------------------------------------------------------------
# linearised least squares (Section 4.2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nv,d", [(2, 2), (3, 3), (2, 1), (1, 3)])
def test_exact_recovery_of_planted(orc, nv, d):
    b = W.uniform_batch(3, 400, nv, d, 0.0, seed=11)
    for f in range(b.num_fits):
        u, y = b.fit_samples(f)
        c, st, rk, rs = orc.fit(u, y, d, d)
        want = planted_vector(orc, b.planted[f])
        A, _ = orc.design(u, y, d, d)
        kappa = np.linalg.cond(A)
        assert st == 0 and rk == len(want)
        assert np.max(np.abs(c - want)) / np.max(np.abs(want)) <= 50 * kappa * 2.0 ** -53
        assert rs <= 1e-12 * np.linalg.norm(y)


def test_exact_interpolation_square_system(orc):
    b = W.interpolation_batch(4, 2, 2, seed=5)
    for f in range(b.num_fits):
        u, y = b.fit_samples(f)
        c, st, rk, rs = orc.fit(u, y, 2, 2)
        A, _ = orc.design(u, y, 2, 2)
        assert A.shape[0] == A.shape[1] == 11
        kappa = np.linalg.cond(A)
        assert st == 0
        assert rs <= 100 * kappa * 2.0 ** -53 * np.linalg.norm(y)
        want = planted_vector(orc, b.planted[f])
        assert np.max(np.abs(c - want)) / np.max(np.abs(want)) <= 100 * kappa * 2.0 ** -53


def test_design_rows_from_tuples(orc):
    rng = np.random.default_rng(3)
    u = rng.uniform(0, 1, size=(3, 7))
    y = rng.normal(size=7)
    A, rhs = orc.design(u, y, 2, 1)
    En = orc.monomials(3, 2)
    Ed = orc.monomials(3, 1)[1:]
    for i in range(7):
        mono = lambda e: np.prod([u[k, i] ** int(e[k]) for k in range(3)])
        row = [mono(e) for e in En] + [-y[i] * mono(e) for e in Ed]
        np.testing.assert_allclose(A[i], row, rtol=1e-15, atol=0)
    np.testing.assert_array_equal(rhs, y)


def test_matches_lapack_on_noisy_fits(orc):
    b = W.uniform_batch(4, 512, 3, 3, 0.005, seed=21)
    for f in range(b.num_fits):
        u, y = b.fit_samples(f)
        c, st, rk, rs = orc.fit(u, y, 3, 3)
        A, rhs = orc.design(u, y, 3, 3)
        ref = np.linalg.lstsq(A, rhs, rcond=None)[0]
        kappa = np.linalg.cond(A)
        # noisy degree-3/3 fits often place a root of Q inside the sample box
        # (status 4); the least-squares solution is the same either way
        assert st in (0, 4)
        assert np.max(np.abs(c - ref)) / np.max(np.abs(ref)) <= 20 * kappa * 2.0 ** -53 * kappa
        np.testing.assert_allclose(rs, np.linalg.norm(rhs - A @ ref), rtol=1e-9)


def _exact_normal_solution(A, b):
    """Solve (A^T A) x = A^T b in exact rational arithmetic."""
    A = [[Fraction(v) for v in row] for row in A]
    b = [Fraction(v) for v in b]
    n = len(A[0])
    G = [[sum(A[i][r] * A[i][c] for i in range(len(A))) for c in range(n)] for r in range(n)]
    g = [sum(A[i][r] * b[i] for i in range(len(A))) for r in range(n)]
    M = [G[r] + [g[r]] for r in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                fac = M[r][col] / M[col][col]
                M[r] = [M[r][k] - fac * M[col][k] for k in range(n + 1)]
    return [M[r][n] / M[r][r] for r in range(n)]


def test_exact_rational_least_squares_on_dyadic_data(orc):
    rng = np.random.default_rng(7)
    u = rng.integers(0, 9, size=(2, 14)) / 8.0
    y = rng.integers(-16, 17, size=14) / 16.0
    A, rhs = orc.design(u, y, 1, 1)   # exact: dyadic products
    x_exact = _exact_normal_solution(A, rhs)
    c, st, rk, rs = orc.fit(u, y, 1, 1)
    kappa = np.linalg.cond(A)
    xe = np.array([float(v) for v in x_exact])
    assert st in (0, 4) and rk == 5
    assert np.max(np.abs(c - xe)) / np.max(np.abs(xe)) <= 100 * kappa * 2.0 ** -53


def test_min_norm_on_rank_deficient_design(orc):
    # collinear samples (u1 == u2) make the x1- and x2-columns identical
    rng = np.random.default_rng(9)
    t = rng.uniform(0, 1, size=60)
    u = np.stack([t, t])
    y = 1.0 + 0.5 * t + 0.01 * rng.normal(size=60)
    c, st, rk, rs = orc.fit(u, y, 1, 1)
    A, rhs = orc.design(u, y, 1, 1)
    ref = np.linalg.lstsq(A, rhs, rcond=None)[0]        # LAPACK gelsd: minimum norm
    assert st == 1 and rk == 3
    np.testing.assert_allclose(c, ref, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(c[1], c[2], rtol=1e-8)   # mass split evenly
    np.testing.assert_allclose(c[3], c[4], rtol=1e-8)


def test_underdetermined_gives_min_norm(orc):
    rng = np.random.default_rng(4)
    u = rng.uniform(0, 1, size=(3, 25))
    y = rng.uniform(0.5, 1.5, size=25)
    c, st, rk, rs = orc.fit(u, y, 3, 3)     # 39 unknowns, 25 samples
    A, rhs = orc.design(u, y, 3, 3)
    assert st == 2 and rk == 25
    np.testing.assert_allclose(c, np.linalg.pinv(A) @ rhs, rtol=1e-7, atol=1e-9)
    assert rs <= 1e-9 * np.linalg.norm(y)


def _orthonormal(rng, m, k):
    q, _ = np.linalg.qr(rng.normal(size=(m, k)))
    return q


@pytest.mark.parametrize("factor,kept", [(1.02, True), (0.98, False)])
def test_rank_rule_threshold_on_column_distance(orc, factor, kept):
    # columns 0..4 independent; column 5 = 3 * column 1 plus delta times a
    # unit vector orthogonal to every other column, so its distance from the
    # span of the columns before it is delta and its norm sqrt(9 |a_1|^2 +
    # delta^2): the rule keeps it exactly when delta / norm > TAU_COL
    rng = np.random.default_rng(11)
    Q = _orthonormal(rng, 40, 7)
    A = Q[:, :5] * np.array([1.0, 2.0, 0.5, 4.0, 1.5])
    rho = factor * orc.TAU_COL
    c = 3.0 * 2.0
    delta = rho * c / np.sqrt(1.0 - rho * rho)
    A = np.column_stack([A, c * Q[:, 1] + delta * Q[:, 6]])
    b = rng.normal(size=40)
    x, r = orc.lstsq_fit(A, b)
    if kept:
        assert r == 6
        np.testing.assert_allclose(x, np.linalg.lstsq(A, b, rcond=None)[0], rtol=1e-9, atol=0)
    else:
        # the dependent column is replaced by its projection (3 * column 1),
        # and the minimum-norm minimiser of that problem is returned
        At = A.copy()
        At[:, 5] = c * Q[:, 1]
        assert r == 5
        np.testing.assert_allclose(x, np.linalg.lstsq(At, b, rcond=None)[0], rtol=1e-9, atol=1e-12)


def test_rank_rule_drops_the_later_column(orc):
    # natural order: of two equal columns the later one is dependent; with a
    # third column in between the rule still looks only at kept predecessors
    rng = np.random.default_rng(12)
    Q = _orthonormal(rng, 30, 3)
    A = np.column_stack([Q[:, 0], Q[:, 1], Q[:, 0] * 2.0, Q[:, 2]])
    b = rng.normal(size=30)
    x, r = orc.lstsq_fit(A, b)
    assert r == 3
    # minimum norm: b's component along Q0 is split as x0 + 2 x2 with x2 = 2 x0
    t0 = Q[:, 0] @ b
    np.testing.assert_allclose([x[0], x[2]], [t0 / 5.0, 2.0 * t0 / 5.0], rtol=1e-12)
    np.testing.assert_allclose([x[1], x[3]], [Q[:, 1] @ b, Q[:, 2] @ b], rtol=1e-12)


def test_rank_rule_is_decided_in_natural_order(orc):
    # a1 = a0 + delta Q1 with delta / |a1| = TAU_COL / 2, then a2 = Q2.  In the
    # natural order a1 is dependent on a0 and is replaced by its projection
    # onto the kept columns span(Q0, Q2), which is Q0: the answer is the
    # minimum-norm solution of [Q0, Q0, Q2], x0 = x1 = (Q0.b)/2, x2 = Q2.b.
    # (Taking the largest column first would keep a1 and replace a0 by its
    # projection onto span(a1, Q2), which fits b's Q1 component by delta;
    # a rank rule at rounding level would keep all three, x1 ~ (Q1.b)/delta.)
    rng = np.random.default_rng(15)
    Q = _orthonormal(rng, 25, 3)
    rho = 0.5 * orc.TAU_COL
    delta = rho / np.sqrt(1.0 - rho * rho)
    A = np.column_stack([Q[:, 0], Q[:, 0] + delta * Q[:, 1], Q[:, 2]])
    b = rng.normal(size=25)
    x, r = orc.lstsq_fit(A, b)
    assert r == 2
    t0, t2 = Q[:, 0] @ b, Q[:, 2] @ b
    np.testing.assert_allclose(x, [t0 / 2.0, t0 / 2.0, t2], rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("factor", [1.05, 0.95])
def test_rank_rule_on_samples_when_underdetermined(orc, factor):
    # 6 samples, 10 unknowns.  Row 5 = row 0 plus a perturbation orthogonal
    # to every other row, its distance ratio factor * TAU_ROW.  Above the
    # threshold the answer is the unique minimum-norm interpolant; below it
    # the sample is dependent and the column rule decides, whose answer for
    # a perturbation this small differs from the interpolant.
    rng = np.random.default_rng(13)
    Q = _orthonormal(rng, 10, 7)
    R = (Q[:, :5] * np.array([1.0, 2.0, 3.0, 0.5, 1.5])).T      # 5 x 10 rows
    rho = factor * orc.TAU_ROW
    nr0 = np.linalg.norm(R[0])
    delta = rho * nr0 / np.sqrt(1.0 - rho * rho)
    A = np.vstack([R, R[0] + delta * Q[:, 6]])
    b = rng.normal(size=6)
    x, r = orc.lstsq_fit(A, b)
    if factor > 1:
        assert r == 6
        np.testing.assert_allclose(A @ x, b, rtol=0, atol=1e-8 * np.abs(b).max() / orc.TAU_ROW)
        np.testing.assert_allclose(x, np.linalg.pinv(A, rcond=1e-12) @ b, rtol=1e-6)
    else:
        assert r < 6
        # the column rule's answer: rank 5, a least-squares minimiser of the
        # problem in which the sixth row's perturbation is dropped column by
        # column -- it cannot interpolate b exactly
        assert np.linalg.norm(A @ x - b) > 1e-3 * np.linalg.norm(b)


def test_rank_rule_exact_dependencies_match_lapack_min_norm(orc):
    # exactly repeated samples (m < n) and exactly equal columns (m > n):
    # whatever the rule keeps, the truncated problem is the original one, so
    # the answer is LAPACK's minimum-norm solution
    rng = np.random.default_rng(14)
    A = rng.normal(size=(6, 10))
    A[5] = A[2]
    b = rng.normal(size=6)
    b[5] = b[2]
    x, r = orc.lstsq_fit(A, b)
    assert r == 5
    np.testing.assert_allclose(x, np.linalg.lstsq(A, b, rcond=None)[0], rtol=1e-9, atol=1e-12)
    B = rng.normal(size=(30, 6))
    B[:, 4] = B[:, 1] - 0.5 * B[:, 0]
    c = rng.normal(size=30)
    x, r = orc.lstsq_fit(B, c)
    assert r == 5
    np.testing.assert_allclose(x, np.linalg.lstsq(B, c, rcond=None)[0], rtol=1e-9, atol=1e-12)


def test_status_nonfinite_and_q_nonpositive(orc):
    rng = np.random.default_rng(1)
    u = rng.uniform(0, 1, size=(1, 50))
    y = 1.0 / (1.0 - 2.0 * u[0])            # Q = 1 - 2 u has a root inside
    c, st, rk, rs = orc.fit(u, y, 1, 1)
    assert st == 4
    np.testing.assert_allclose(c, [1.0, 0.0, -2.0], atol=1e-9)
    y2 = y.copy()
    y2[3] = np.nan
    c2, st2, _, _ = orc.fit(u, y2, 1, 1)
    assert st2 == 3 and np.all(np.isnan(c2))


def test_power_of_two_rescaling(orc):
    b = W.uniform_batch(1, 300, 2, 2, 0.01, seed=31)
    u, y = b.fit_samples(0)
    c, *_ = orc.fit(u, y, 2, 2)
    us = u.copy()
    us[1] *= 2.0 ** -3                      # x2 -> x2 / 8
    cs, *_ = orc.fit(us, y, 2, 2)
    E = orc.monomials(2, 2)
    scale = np.array([2.0 ** (3 * int(e[1])) for e in E] + [2.0 ** (3 * int(e[1])) for e in E[1:]])
    np.testing.assert_allclose(cs, c * scale, rtol=1e-9)


# --------------------------------------------------------------------------
# evaluation (Section 2, Definition 1)
# --------------------------------------------------------------------------

def test_evaluation_exact_on_dyadic_inputs(orc):
    rng = np.random.default_rng(12)
    pl = W.plant(rng, 2, 2, 2)
    pl.num_coef = rng.integers(-16, 17, size=len(pl.num_coef)) / 16.0
    pl.den_coef = rng.integers(0, 5, size=len(pl.den_coef)) / 16.0
    coef = planted_vector(orc, pl)
    u = rng.integers(0, 9, size=(2, 40)) / 8.0
    got = orc.eval_rational(2, 2, 2, coef, u)
    num, den = pl.coef_by_tuple()
    for i in range(40):
        mono = lambda e: Fraction(u[0, i]) ** e[0] * Fraction(u[1, i]) ** e[1]
        N = sum(Fraction(c) * mono(e) for e, c in num.items())
        Q = 1 + sum(Fraction(c) * mono(e) for e, c in den.items())
        assert got[i] == float(N / Q)


# --------------------------------------------------------------------------
# argmin (Section 3.3, steps 4-5)
# --------------------------------------------------------------------------

def _single_program(orc, nvars, dn, dq, coef, scale):
    return orc.Program(orc.TEMPLATE_SINGLE, nvars, [dn], [dq], coef, [0], scale=scale)


def test_argmin_planted_unique_minimiser(orc):
    # g = (u_b - 0.5 u_n - 0.25)^2 + 0.1 on u = (n / 2^14, b / 1024)
    terms = {(0, 0): 0.0625 + 0.1, (1, 0): 0.25, (0, 1): -0.5,
             (2, 0): 0.25, (1, 1): -1.0, (0, 2): 1.0}
    E = orc.monomials(2, 2)
    coef = np.array([terms[tuple(int(t) for t in e)] for e in E] + [0.0] * 5)
    prog = _single_program(orc, 2, 2, 2, coef, [2.0 ** 14, 1024.0])
    ks = np.arange(8, 25)                    # target b = 32 k
    n_grid = (ks / 32.0 - 0.25) * 2.0 * 2.0 ** 14
    cand = (32 * np.arange(1, 33)).astype(np.int32)
    am, best, second = orc.argmin(prog, n_grid, cand)
    np.testing.assert_array_equal(am[0], ks - 1)
    np.testing.assert_allclose(best[0], 0.1, rtol=1e-14)
    assert np.all(second[0] > best[0])


def test_argmin_brute_force_against_tuple_evaluation(orc):
    b = W.tiny_fit()
    pl = b.planted[0]
    coef = planted_vector(orc, pl)
    prog = _single_program(orc, 2, 2, 2, coef, [2.0 ** 14, 1024.0])
    n_grid = W.tiny_grid(64)
    cand = (32 * np.arange(1, 33)).astype(np.int32)
    am, best, second = orc.argmin(prog, n_grid, cand)
    for j, n in enumerate(n_grid):
        u = np.stack([np.full(32, n / 2.0 ** 14), cand / 1024.0])
        vals = pl.value(u)
        num = pl.num_coef @ np.prod(u[None] ** pl.num_exps[:, :, None], axis=1)
        den = 1.0 + pl.den_coef @ np.prod(u[None] ** pl.den_exps[:, :, None], axis=1)
        vals = np.where(den > 0, vals, np.inf)
        k = int(np.argmin(vals))
        if am[0, j] != k:   # rounding may reorder exact near-ties only
            assert abs(vals[am[0, j]] - vals[k]) <= 1e-13 * abs(vals[k])
        np.testing.assert_allclose(best[0, j], vals[k], rtol=1e-13)
        np.testing.assert_allclose(second[0, j], np.sort(vals)[1], rtol=1e-13)


def test_argmin_ties_and_invalid(orc):
    E = orc.monomials(2, 1)
    const = np.array([1.0, 0.0, 0.0, 0.0, 0.0])
    prog = _single_program(orc, 2, 1, 1, const, [1.0, 1024.0])
    cand = (32 * np.arange(1, 33)).astype(np.int32)
    am, best, second = orc.argmin(prog, [1.0, 2.0], cand)
    assert am.tolist() == [[0, 0]] and np.all(best == 1.0) and np.all(second == 1.0)
    # Q = 1 - 2 u_b <= 0 for every b >= 512: no valid candidate
    bad = np.array([1.0, 0.0, 0.0, 0.0, -2.0])
    assert E.tolist() == [[0, 0], [1, 0], [0, 1]]
    prog = _single_program(orc, 2, 1, 1, bad, [1.0, 1024.0])
    am, best, second = orc.argmin(prog, [1.0], (32 * np.arange(16, 33)).astype(np.int32))
    assert am.tolist() == [[-1]] and np.isinf(best[0, 0])


# --------------------------------------------------------------------------
# MWP-CWP-style template: hand-worked examples (values derived by hand)
# --------------------------------------------------------------------------

HW_SMALL = dict(wave_size=64, num_cu=4, simd_per_cu=4, max_threads_per_block=1024,
                max_blocks_per_cu=8, max_waves_per_cu=16, regs_per_cu=65536,
                lds_bytes_per_cu=65536, mem_latency=400, l2_latency=100,
                departure_del_coal=4, departure_del_uncoal=40, issue_cycles=4,
                sfu_issue_cycles=8, lds_issue_cycles=2, clock_ghz=1.0,
                mem_bandwidth_gbs=1000)


def _hw(**over):
    d = dict(HW_SMALL)
    d.update(over)
    return np.array([d[k] for k in W.HW_NAMES], dtype=np.float64)


def _g(**vals):
    base = dict(comp_insts=100, coal_mem_insts=10, uncoal_mem_insts=0, synch_insts=0,
                coal_per_mw=1, uncoal_per_mw=1, load_bytes_per_warp=0, regs_per_thread=32,
                lds_bytes_per_block=0, total_blocks=64, sfu_insts=0, lds_insts=0,
                lds_conflict_rate=0, branch_insts=0, l2_hit_rate=0, divergence_rate=0)
    base.update(vals)
    return np.array([base[k] for k in W.METRIC_NAMES], dtype=np.float64)


def test_template_case3_compute_bound_tail(orc):
    # B_active = min(8, 16/2, 65536/(32*64*2), 8) = 8, N = 16, Rep = ceil(64/32) = 2
    # Mem_L = 400, delay 4 -> MWP = 16 = N; Comp = 4*110 = 440, Mem = 4000,
    # CWP = 4440/440 < MWP and Comp < Mem -> (400 + 440*16) * 2 = 14880
    e, parts = orc.mwpcwp(_g(), _hw(), 128, 1)
    assert parts.tolist() == [8, 16, 16, parts[3], 2, 440, 4000, 3]
    assert e == 14880.0


def test_template_case2_memory_parallelism_limited(orc):
    # uncoalesced: Mem_L = 400 + 7*40 = 680, delay = 40*8 = 320, MWP = 2.125;
    # CWP = min(7240/440, 16) = 16 >= MWP -> (6800*16/2.125 + 44*1.125) * 2 = 102499
    g = _g(coal_mem_insts=0, uncoal_mem_insts=10, uncoal_per_mw=8)
    e, parts = orc.mwpcwp(g, _hw(), 128, 1)
    assert parts[2] == 2.125 and parts[3] == 16 and parts[7] == 2
    assert e == 102499.0
    # synchronisation: + 320 * 1.125 * 3 * 8 * 2 = 17280
    e2, _ = orc.mwpcwp(_g(coal_mem_insts=0, uncoal_mem_insts=10, uncoal_per_mw=8,
                          synch_insts=3), _hw(), 128, 1)
    assert e2 == 102499.0 + 17280.0


def test_template_case1_single_resident_wave(orc):
    # LDS use 65536 B -> one block per CU, N = 1 = MWP = CWP; Rep = 64/4 = 16
    # (4000 + 440) * 16 = 71040; MWP - 1 = 0 removes the synchronisation term
    e, parts = orc.mwpcwp(_g(lds_bytes_per_block=65536, synch_insts=2), _hw(), 64, 1)
    assert parts[7] == 1 and parts[1] == 1 and parts[4] == 16
    assert e == 71040.0


def test_template_case2_compute_heavier_than_memory(orc):
    # comp 1000, one coalesced load: Comp = 4004 > Mem = 400; MWP = 16
    # (400*16/16 + 4004/1*15) * 2 = 120920
    e, parts = orc.mwpcwp(_g(comp_insts=1000, coal_mem_insts=1), _hw(), 128, 1)
    assert parts[7] == 2 and e == 120920.0


def test_template_bandwidth_limit(orc):
    # 128 B per warp at 1 GHz over Mem_L 400: 0.32 GB/s per warp; 10 GB/s over 4 CUs
    # -> MWP = 7.8125; CWP 10.09 >= MWP: (4000*16/7.8125 + 44*6.8125) * 2 = 16983.5
    e, parts = orc.mwpcwp(_g(load_bytes_per_warp=128), _hw(mem_bandwidth_gbs=10), 128, 1)
    assert parts[2] == 7.8125 and e == 16983.5


def test_template_extra_issue_terms_and_cache(orc):
    # Comp = 4*(100+10+5*2) + 8*10 + 2*20*1.5 = 620; hit 0.5 -> latency 250
    # Mem = 2500, MWP = 16 = N, CWP < MWP, Comp < Mem -> (250 + 620*16) * 2 = 20340
    g = _g(sfu_insts=10, lds_insts=20, lds_conflict_rate=0.5, branch_insts=5,
           divergence_rate=2.0, l2_hit_rate=0.5)
    e, parts = orc.mwpcwp(g, _hw(), 128, 1)
    assert parts[5] == 620 and parts[6] == 2500 and e == 20340.0


def test_template_occupancy_equation_and_infeasible(orc):
    # equation (occupancy) with 32-wide warps: T = 96 -> 3 warps per block,
    # B_active = min(8, floor(16/3), floor(65536/(32*32*3)), 8) = 5,
    # W_active = min(floor(5*96/32), 16) = 15
    _, parts = orc.mwpcwp(_g(), _hw(wave_size=32), 96, 1)
    assert parts[0] == 5 and parts[1] == 15
    assert math.isinf(orc.mwpcwp(_g(), _hw(), 2048, 1)[0])          # T > T_max
    assert math.isinf(orc.mwpcwp(_g(regs_per_thread=1024), _hw(), 128, 1)[0])


# --------------------------------------------------------------------------
# occupancy program and selection with a second metric (Section 2 Example 1,
# equation (occupancy); Section 3.3 step 5)
# --------------------------------------------------------------------------

# 32-wide warps, 1024 threads, 32 blocks and 64 warps per unit, 64 Ki
# registers, 96 KiB of LDS per unit
HW_W32 = dict(HW_SMALL, wave_size=32, max_blocks_per_cu=32, max_waves_per_cu=64,
              regs_per_cu=65536, lds_bytes_per_cu=98304)
# 64-wide waves, 32 waves and 32 blocks per unit, 4 x 512 x 64 registers,
# 160 KiB of LDS
HW_W64 = dict(HW_SMALL, wave_size=64, max_blocks_per_cu=32, max_waves_per_cu=32,
              regs_per_cu=131072, lds_bytes_per_cu=163840)


def _hwd(d):
    return np.array([d[k] for k in W.HW_NAMES], dtype=np.float64)


@pytest.mark.parametrize("hw,regs,lds,bx,by,want", [
    # 256 threads = 8 warps: 8 blocks by warps, 65536/(32*32*8) = 8 by registers -> 64 warps
    (HW_W32, 32, 0, 16, 16, 1.0),
    # 64 registers: 65536/(64*32*8) = 4 blocks -> 32 of 64 warps
    (HW_W32, 64, 0, 16, 16, 0.5),
    # 48 KiB of LDS per block: 98304/49152 = 2 blocks -> 16 warps
    (HW_W32, 32, 49152, 16, 16, 0.25),
    # 48 threads = 2 warps (one partial): 32 blocks (the block limit), floor(32*48/32) = 48 warps
    (HW_W32, 32, 0, 1, 48, 0.75),
    # 128 registers, 48 threads: the partial warp holds a whole warp's registers,
    # 65536/(128*32*2) = 8 blocks -> floor(8*48/32) = 12 of 64 warps
    (HW_W32, 128, 0, 1, 48, 0.1875),
    # 100.5 LDS bytes count as 101: 98304/101 = 973 blocks, the block limit 32 wins
    (HW_W32, 32, 100.5, 8, 8, 1.0),
    # 65 registers x 1024 threads: 65536/(65*32*32) < 1, no block fits
    (HW_W32, 65, 0, 32, 32, -math.inf),
    # more threads than a block may hold
    (HW_W32, 16, 0, 64, 32, -math.inf),
    # 64-wide: 256 threads = 4 waves, 131072/(128*64*4) = 4 blocks -> 16 of 32 waves
    (HW_W64, 128, 0, 16, 16, 0.5),
    # 64 threads, 64 KiB LDS: 163840/65536 = 2 blocks -> 2 of 32 waves
    (HW_W64, 64, 65536, 8, 8, 0.0625),
    # 96 threads = 2 waves: 16 blocks by waves, 131072/(32*64*2) = 32 by registers,
    # floor(16*96/64) = 24 waves
    (HW_W64, 32, 0, 96, 1, 0.75),
])
def test_occupancy_hand_worked(orc, hw, regs, lds, bx, by, want):
    assert orc.occupancy(regs, lds, _hwd(hw), bx, by) == want


def _occupancy_program(orc, hw, regs_coef, lds_coef=(0.0,), dn_regs=1):
    """Occupancy program over u = (n, bx, by) unscaled: registers per thread a
    polynomial of degree dn_regs, LDS bytes per block a constant."""
    coef = np.concatenate([np.asarray(regs_coef, float), np.asarray(lds_coef, float)])
    return orc.Program(orc.TEMPLATE_OCCUPANCY, 3, [dn_regs, 0], [0, 0], coef,
                       [0, len(regs_coef), len(coef)], hw=_hwd(hw), hw_stride=len(W.HW_NAMES),
                       scale=[1.0, 1.0, 1.0])


def _product_program(orc):
    """E = bx * by: every block format with the same thread count ties."""
    E = orc.monomials(3, 2)
    coef = np.array([1.0 if tuple(int(t) for t in e) == (0, 1, 1) else 0.0 for e in E])
    return orc.Program(orc.TEMPLATE_SINGLE, 3, [2], [0], coef, [0, len(coef)], scale=[1.0, 1.0, 1.0])


def test_select_sense_and_occupancy_tie_break(orc):
    cand = np.array([(8, 8), (4, 16), (2, 32), (1, 64), (16, 8)], np.int32)
    prim = _product_program(orc)
    # registers = 24 + 8 bx; 64 threads = 2 warps:
    #   (8,8): 88 regs -> floor(65536/(88*64)) = 11 blocks -> 22 warps
    #   (4,16): 56 -> 18 -> 36;  (2,32): 40 -> 25 -> 50;  (1,64): 32 -> 32 -> 64
    occ = _occupancy_program(orc, HW_W32, [24.0, 0.0, 8.0, 0.0])
    vals = [occ.value(0, 1.0, c) for c in cand[:4]]
    assert vals == [22 / 64, 36 / 64, 50 / 64, 1.0]
    ch, best, second = orc.select(prim, [1.0], cand)                   # plain argmin
    assert ch.tolist() == [[0]] and best[0, 0] == 64.0 and second[0, 0] == 64.0
    ch, _, _ = orc.select(prim, [1.0], cand, tie=occ, tie_sense=-1)    # highest occupancy
    assert ch.tolist() == [[3]]
    ch, _, _ = orc.select(prim, [1.0], cand, tie=occ, tie_sense=1)     # lowest occupancy
    assert ch.tolist() == [[0]]
    ch, best, second = orc.select(prim, [1.0], cand, sense=-1)         # largest E
    assert ch.tolist() == [[4]] and best[0, 0] == 128.0 and second[0, 0] == 64.0
    # the occupancy program maximised: (1, 64) is alone at 1.0; the second best is 50/64
    ch, best, second = orc.select(occ, [1.0], cand, sense=-1)
    assert ch.tolist() == [[3]] and best[0, 0] == 1.0 and second[0, 0] == 50 / 64
    # argmin is select with sense +1 and no tie program
    am, b2, s2 = orc.argmin(prim, [1.0], cand)
    assert am.tolist() == [[0]] and b2[0, 0] == 64.0 and s2[0, 0] == 64.0


def test_select_infeasible_and_tie_values_ranked_last(orc):
    cand = np.array([(32, 32), (64, 32), (2, 32), (1, 64)], np.int32)
    occ = _occupancy_program(orc, HW_W32, [24.0, 0.0, 8.0, 0.0])
    # (64, 32) exceeds 1024 threads; (32, 32): 280 registers x 1024 threads cannot fit
    ch, best, second = orc.select(occ, [1.0], cand, sense=-1)
    assert ch.tolist() == [[3]] and best[0, 0] == 1.0 and second[0, 0] == 50 / 64
    none = _occupancy_program(orc, HW_W32, [5000.0, 0.0, 0.0, 0.0])
    ch, best, second = orc.select(none, [1.0], cand, sense=-1)
    assert ch.tolist() == [[-1]] and best[0, 0] == -math.inf and second[0, 0] == -math.inf
    # a tie program that is infeasible on the lower index ranks it last
    prim = _product_program(orc)
    cand = np.array([(64, 1), (1, 64)], np.int32)
    occ2 = _occupancy_program(orc, dict(HW_W32, max_threads_per_block=1024), [-1000.0, 0.0, 1100.0, 0.0])
    # registers = 1100 bx - 1000: (64,1) -> 69400 (no block fits), (1,64) -> 100 -> 10 blocks
    assert occ2.value(0, 1.0, cand[0]) == -math.inf and occ2.value(0, 1.0, cand[1]) == 20 / 64
    ch, _, _ = orc.select(prim, [1.0], cand, tie=occ2, tie_sense=-1)
    assert ch.tolist() == [[1]]


def test_select_brute_force_lexicographic(orc):
    """Random integer-valued primary (many exact ties) and a random tie
    program, against a plain sort of (key1, key2, index) tuples."""
    rng = np.random.default_rng(17)
    cand = np.array([(bx, by) for bx in (1, 2, 4, 8, 16) for by in (1, 2, 4, 8, 16, 32)], np.int32)
    E = orc.monomials(3, 2)
    for trial in range(20):
        # primary: small integer combination of bx*by, bx, by -> exact ties
        w = rng.integers(0, 3, size=3).astype(float)
        coef = np.zeros(len(E))
        for k, e in enumerate(E):
            t = tuple(int(x) for x in e)
            coef[k] = {(0, 1, 1): w[0], (0, 1, 0): w[1], (0, 0, 1): w[2]}.get(t, 0.0)
        prim = orc.Program(orc.TEMPLATE_SINGLE, 3, [2], [0], coef, [0, len(coef)], scale=[1.0, 1.0, 1.0])
        occ = _occupancy_program(orc, HW_W32, [rng.uniform(16, 64), 0.0, rng.uniform(0, 16),
                                               rng.uniform(0, 16)], [rng.uniform(0, 8192)])
        sense, tsense = int(rng.choice([1, -1])), int(rng.choice([1, -1]))
        v1 = [prim.value(0, 3.0, c) for c in cand]
        v2 = [occ.value(0, 3.0, c) for c in cand]
        keys = []
        for i, (a, b) in enumerate(zip(v1, v2)):
            if not np.isfinite(a):
                continue
            keys.append((sense * a, tsense * b if np.isfinite(b) else math.inf, i))
        want = min(keys)[2]
        ch, best, second = orc.select(prim, [3.0], cand, sense=sense, tie=occ, tie_sense=tsense)
        assert ch[0, 0] == want, trial
        assert best[0, 0] == v1[want]
        others = sorted(sense * a for i, a in enumerate(v1) if i != want and np.isfinite(a))
        assert second[0, 0] == sense * others[0]


# --------------------------------------------------------------------------
# loss, gradient and refinement
# --------------------------------------------------------------------------

def test_loss_zero_at_planted_and_matches_tuple_evaluation(orc):
    b = W.uniform_batch(1, 200, 3, 2, 0.02, seed=41)
    u, y = b.fit_samples(0)
    pl = b.planted[0]
    c = planted_vector(orc, pl)
    L, _ = orc.loss_grad(u, y, 2, 2, c)
    np.testing.assert_allclose(L, np.sum((pl.value(u) - y) ** 2), rtol=1e-12)
    L0, _ = orc.loss_grad(u, pl.value(u), 2, 2, c)
    assert L0 <= 1e-28 * np.sum(y ** 2)


def test_gradient_central_differences(orc):
    b = W.uniform_batch(2, 150, 3, 2, 0.01, seed=43)
    for f in range(2):
        u, y = b.fit_samples(f)
        c = planted_vector(orc, b.planted[f]) + 0.05
        L, g = orc.loss_grad(u, y, 2, 2, c)
        h = 1e-6
        fd = np.zeros_like(c)
        for k in range(len(c)):
            cp, cm = c.copy(), c.copy()
            cp[k] += h
            cm[k] -= h
            fd[k] = (orc.loss_grad(u, y, 2, 2, cp)[0] - orc.loss_grad(u, y, 2, 2, cm)[0]) / (2 * h)
        floor = 1e-12 * np.max(np.abs(g))
        assert np.all(np.abs(fd - g) <= 1e-6 * np.abs(g) + floor + 1e-6 * np.max(np.abs(g)) * 1e-3)


def test_refine_recovers_planted_from_perturbed_start(orc):
    b = W.uniform_batch(1, 300, 2, 2, 0.0, seed=45)
    u, y = b.fit_samples(0)
    want = planted_vector(orc, b.planted[0])
    c, L, it = orc.refine(u, y, 2, 2, want + 0.01, max_iter=50)
    assert L <= 1e-24 * np.sum(y ** 2)
    np.testing.assert_allclose(c, want, rtol=1e-8, atol=1e-10)


def test_refine_reaches_stationary_point(orc):
    b = W.uniform_batch(1, 400, 3, 2, 0.01, seed=47)
    u, y = b.fit_samples(0)
    c0, *_ = orc.fit(u, y, 2, 2)
    L0, g0 = orc.loss_grad(u, y, 2, 2, c0)
    c, L, it = orc.refine(u, y, 2, 2, c0)
    _, g = orc.loss_grad(u, y, 2, 2, c)
    assert L <= L0
    assert np.max(np.abs(g)) <= 1e-6 * np.max(np.abs(g0))


# --------------------------------------------------------------------------
# the paper's "Error" (Section 5, Table 3)
# --------------------------------------------------------------------------

def _half_ulp(s: str) -> float:
    s = s.strip()
    return 0.5 * 10.0 ** (-(len(s.split(".")[1]) if "." in s else 0))


def test_error_formula_reproduces_table3(orc):
    rows = []
    with open(os.path.join(GOLDEN, "table3_error.csv")) as fh:
        rows = [r for r in csv.DictReader(line for line in fh if not line.startswith("#"))]
    assert len(rows) == 50
    for r in rows:
        c, bt, wt, err = (float(r[k]) for k in ("C_rt", "B_t", "W_t", "error"))
        dc, db, dw, de = (_half_ulp(r[k]) for k in ("C_rt", "B_t", "W_t", "error"))
        lo = orc.regret(c - dc, bt + db, wt + dw)
        hi = orc.regret(c + dc, bt - db, wt - dw)
        assert lo - de <= err <= hi + de, r
    # the two rows quoted most often, at their printed precision
    assert round(orc.regret(0.16, 0.15, 1.31), 2) == 0.86
    assert round(orc.regret(968, 143, 2802), 2) == 31.03


def test_coefficient_length_is_checked(orc):
    """A coefficient vector of the wrong length is an error, not a silent
    truncation (a mistake that mixes up the variable count and the degrees)."""
    import numpy as np
    import pytest
    u = np.random.default_rng(0).uniform(size=(3, 50))
    y = np.ones(50)
    c = np.zeros(orc.num_coefs(3, 4, 4))
    orc.loss_grad(u, y, 4, 4, c)
    with pytest.raises(ValueError):
        orc.loss_grad(u, y, 3, 4, c)
    with pytest.raises(ValueError):
        orc.refine(u, y, 3, 3, c)
    with pytest.raises(ValueError):
        orc.eval_rational(3, 3, 3, c, u)


# ---------------------------------------------------------------------------
# one decision node fitted from the samples (Section 3.2, third consequence)
# ---------------------------------------------------------------------------

def test_split_recovers_planted_node(orc):
    # noise-free piecewise rational with a sample-free band around theta: the
    # planted split has zero residual on both sides, every other split not
    sb = W.split_batch(6, 220, 2, 2, split_var=1, sigma=0.0, gap=0.02, seed=21)
    b = sb.batch
    nc = orc.num_coefs(2, 2, 2)
    for f in range(b.num_fits):
        u, y = b.fit_samples(f)
        r = orc.split_fit(u, y, 2, 1, nc)
        s = np.sort(u[1])
        kk = int((u[1] <= sb.theta[f]).sum())
        assert r["k"] == kk
        assert s[kk - 1] < r["theta"] < s[kk] and r["theta"] == 0.5 * (s[kk - 1] + s[kk])
        assert r["obj"] <= 1e-20 * float(y @ y)
        from tests.conftest import planted_in_order
        np.testing.assert_allclose(r["coef_l"], planted_in_order(orc, sb.left[f]), rtol=1e-8, atol=1e-10)
        np.testing.assert_allclose(r["coef_r"], planted_in_order(orc, sb.right[f]), rtol=1e-8, atol=1e-10)


def test_split_objective_brute_force_with_lapack(orc):
    # every candidate's objective from LAPACK least squares on each side's
    # design, the minimum and its position
    sb = W.split_batch(3, 48, 1, 1, split_var=0, sigma=0.02, seed=22)
    b = sb.batch
    for f in range(b.num_fits):
        u, y = b.fit_samples(f)
        r = orc.split_fit(u, y, 1, 0, 3, want_all=True)
        order = np.lexsort((np.arange(u.shape[1]), u[0]))
        us, uy = u[:, order], y[order]
        want = np.full(u.shape[1] + 1, np.inf)
        for k in range(3, u.shape[1] - 3 + 1):
            if not us[0, k - 1] < us[0, k]:
                continue
            tot = 0.0
            for lo, hi in ((0, k), (k, u.shape[1])):
                A, rhs = orc.design(us[:, lo:hi], uy[lo:hi], 1, 1)
                x = np.linalg.lstsq(A, rhs, rcond=None)[0]
                tot += float(np.sum((rhs - A @ x) ** 2))
            want[k] = tot
        fin = np.isfinite(want)
        assert np.array_equal(np.isfinite(r["obj_all"]), fin)
        np.testing.assert_allclose(r["obj_all"][fin], want[fin], rtol=1e-9)
        assert r["k"] == int(np.argmin(want)) and r["obj"] == r["obj_all"][r["k"]]


def test_split_keeps_equal_values_together_and_ignores_order(orc):
    rng = np.random.default_rng(23)
    u = np.round(rng.uniform(0, 1, size=(2, 90)) * 12) / 12      # many equal values
    y = np.where(u[0] <= 0.5, 1.0 + u[1], 2.0 - u[0] * u[1]) * (1 + 0.01 * rng.normal(size=90))
    r = orc.split_fit(u, y, 1, 0, 5, want_all=True)
    s = np.sort(u[0])
    for k in np.flatnonzero(np.isfinite(r["obj_all"])):
        assert s[k - 1] < s[k]
    p = rng.permutation(90)
    r2 = orc.split_fit(u[:, p], y[p], 1, 0, 5)
    assert r2["k"] == r["k"] and r2["theta"] == r["theta"]
    # the same minimiser (the samples are summed in another order)
    np.testing.assert_allclose(r2["coef_l"], r["coef_l"], rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(r2["coef_r"], r["coef_r"], rtol=1e-9, atol=1e-14)
    r3 = orc.split_fit(u, y, 1, 0, 60)          # no split leaves 60 on each side
    assert r3["k"] == -1 and np.isnan(r3["theta"]) and r3["obj"] == np.inf
