"""Pins of oracle.bspline: the interpolation matrices M_(N) and M^(l).

Pins: the matrices printed in Section 7 (golden file), the textbook
truncated-power B-spline (each row of M_(N) is one polynomial piece of B_(N),
Section 7), partition of unity / symmetry / positivity, Strang-Fix moments,
C^(N-2) continuity (Section 7: B_(N) is C^(N-2)), and the derivative identity
B_N' = B_{N-1}(.+1/2) - B_{N-1}(.-1/2) for M^(1) = M D and M^(2) = M D^2.
"""
import os
from fractions import Fraction

import pytest

from oracle.bspline import bspline_matrix, derivative_matrix
from pins import bspline_exact, bspline_deriv_exact, bspline_float

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bspline_matrices_printed.txt")


def _read_printed():
    mats = {}
    with open(GOLDEN) as fh:
        lines = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    i = 0
    while i < len(lines):
        _, order, _, scale = lines[i]
        order, scale = int(order), int(scale)
        rows = [[Fraction(int(v), scale) for v in lines[i + 1 + r]] for r in range(order)]
        mats[order] = rows
        i += 1 + order
    return mats


def _poly(row, x):
    return sum(c * x ** i for i, c in enumerate(row))


SAMPLES = [Fraction(k, 13) for k in range(13)] + [Fraction(1, 3), Fraction(999, 1000)]


def test_printed_matrices_reproduced_exactly():
    printed = _read_printed()
    assert sorted(printed) == [1, 2, 3, 4]
    for N, M in printed.items():
        assert bspline_matrix(N) == M, f"M_({N}) differs from the printed matrix"


@pytest.mark.parametrize("N", range(1, 9))
def test_rows_are_pieces_of_the_bspline(N):
    # Row j (0-based) is B_N(x + N/2 - 1 - j) on 0 <= x < 1 (Section 7 relation
    # between B_(N) and M_(N), with the Section 5 stencil).  15 sample points
    # > degree N-1 make this a polynomial identity.
    M = bspline_matrix(N)
    for j in range(N):
        for x in SAMPLES:
            assert _poly(M[j], x) == bspline_exact(N, x + Fraction(N, 2) - 1 - j)


@pytest.mark.parametrize("N", range(2, 9))
def test_derivative_rows_match_bspline_derivatives(N):
    M = bspline_matrix(N)
    for l in (1, 2):
        if l >= N:
            continue
        Ml = derivative_matrix(M, l)
        for j in range(N):
            for x in SAMPLES[1:-2]:          # interior points (no breakpoints)
                y = x + Fraction(N, 2) - 1 - j
                assert _poly(Ml[j], x) == bspline_deriv_exact(N, y, l)


@pytest.mark.parametrize("N", [2, 4, 6, 8])
def test_partition_of_unity_symmetry_positivity(N):
    M = bspline_matrix(N)
    M1 = derivative_matrix(M, 1)
    for t in SAMPLES:
        w = [_poly(M[j], t) for j in range(N)]
        wd = [_poly(M1[j], t) for j in range(N)]
        assert sum(w) == 1
        assert sum(wd) == 0
        assert all(v >= 0 for v in w)
        w_mirror = [_poly(M[N - 1 - j], 1 - t) for j in range(N)]
        assert w == w_mirror


@pytest.mark.parametrize("N", [4, 6])
def test_strang_fix_moments(N):
    # sum_j w_j(t) (j_rel - t)^d equals the d-th moment of B_N for d <= N-1,
    # independent of t.  B_N is the density of a sum of N independent uniforms
    # on [-1/2, 1/2): mu_2 = N/12, mu_4 = N/80 + N(N-1)/48, odd moments 0.
    M = bspline_matrix(N)
    mu = {0: Fraction(1), 1: Fraction(0), 2: Fraction(N, 12), 3: Fraction(0),
          4: Fraction(N, 80) + Fraction(N * (N - 1), 48), 5: Fraction(0)}
    for d in range(N):
        for t in SAMPLES:
            m = sum(_poly(M[j], t) * (Fraction(j - N // 2 + 1) - t) ** d for j in range(N))
            assert m == mu[d], (N, d, t)
    # order N moment depends on t: the reproduction (and convergence) order is N
    vals = {sum(_poly(M[j], t) * (Fraction(j - N // 2 + 1) - t) ** N for j in range(N))
            for t in SAMPLES}
    assert len(vals) > 1


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 8])
def test_continuity_order(N):
    # The spline is C^(N-2): the weight of one grid point leaving cell f at t=1
    # continues as the previous stencil slot of cell f+1 at t=0, through the
    # (N-2)-th derivative, and the (N-1)-th derivative jumps somewhere.
    M = bspline_matrix(N)
    jumped = False
    for r in range(N):
        Mr = derivative_matrix(M, r) if r else M
        for j in range(N):
            left = _poly(Mr[j], Fraction(1))
            right = _poly(Mr[j - 1], Fraction(0)) if j >= 1 else Fraction(0)
            if r <= N - 2:
                assert left == right, (N, r, j)
            elif left != right:
                jumped = True
        if r <= N - 2:
            assert _poly(Mr[N - 1], Fraction(0)) == 0
    assert jumped


def test_recursion_matches_truncated_power():
    for N in range(1, 9):
        for y in [-4.2, -2.5, -1.0, -0.3, 0.0, 0.25, 0.5, 1.7, 3.0]:
            assert abs(bspline_float(N, y) - float(bspline_exact(N, Fraction(y)))) < 1e-14


def test_bspline_integer_samples():
    # known values of the centred cubic and quintic B-splines at the integers
    assert [bspline_exact(4, k) for k in (0, 1, 2)] == [Fraction(2, 3), Fraction(1, 6), 0]
    assert [bspline_exact(6, k) for k in (0, 1, 2, 3)] == \
        [Fraction(11, 20), Fraction(13, 60), Fraction(1, 120), 0]


@pytest.mark.parametrize("N,want", [(4, Fraction(3, 2)), (6, Fraction(115, 96))])
def test_derivative_weight_l1_at_half(N, want):
    # sum_j |w'_j(t)| is largest at t = 1/2 (used to bound BF16 storage error
    # of the gradient); exact value there and not exceeded on a fine grid
    M1 = derivative_matrix(bspline_matrix(N), 1)
    l1 = lambda t: sum(abs(_poly(M1[j], t)) for j in range(N))
    assert l1(Fraction(1, 2)) == want
    assert all(l1(Fraction(k, 200)) <= want for k in range(201))
