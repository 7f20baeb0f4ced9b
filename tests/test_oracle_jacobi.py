"""Pins for the Jacobi/Laplace oracle: fields the iteration must leave exactly
unchanged, a hand-computed step, convergence to the closed-form harmonic
solution, symmetry, and the max-change bookkeeping."""
import numpy as np

from oracle import jacobi as oj


def test_linear_and_constant_fields_are_fixed_points():
    i, j = np.mgrid[0:9, 0:12]
    for u in (2.0 * i + 3.0 * j + 1.0, np.full((9, 12), 7.5)):
        v, ch = oj.step(u)
        np.testing.assert_array_equal(v, u)
        assert ch == 0.0


def test_hand_computed_step():
    u = np.zeros((3, 4))
    u[0, :] = [1, 2, 3, 4]
    u[2, :] = [5, 6, 7, 8]
    u[:, 0] = [1, 9, 5]
    u[:, 3] = [4, 10, 8]
    v, ch = oj.step(u)
    # interior (1,1): (2 + 6 + 9 + 0) / 4; (1,2): (3 + 7 + 0 + 10) / 4
    assert v[1, 1] == 17 / 4 and v[1, 2] == 20 / 4
    np.testing.assert_array_equal(v[0], u[0])
    np.testing.assert_array_equal(v[:, 0], u[:, 0])
    assert ch == 5.0


def test_converges_to_the_harmonic_solution():
    n, m = 10, 7
    i, j = np.mgrid[0:n, 0:m]
    exact = 0.5 * i - 1.5 * j + 2.0          # linear: harmonic, the unique solution
    u = exact.copy()
    u[1:-1, 1:-1] = 0.0
    v, ch = oj.solve(u, 2000)
    np.testing.assert_allclose(v, exact, atol=1e-9)
    assert ch < 1e-9


def test_symmetric_boundary_gives_symmetric_iterates():
    rng = np.random.default_rng(4)
    b = rng.uniform(-1, 1, (8, 8))
    u = b + b.T
    u[1:-1, 1:-1] = 0.0
    v, _ = oj.solve(u, 17)
    np.testing.assert_allclose(v, v.T, rtol=0, atol=1e-15)


def test_max_change_first_step():
    u = np.zeros((6, 6))
    u[0, :] = 1.0
    _, ch = oj.step(u)
    assert ch == 0.25
    v, ch = oj.solve(u, 3)
    assert 0 < ch < 0.25
