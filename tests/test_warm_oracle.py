"""Pins of the warm-start state map's reference (oracle/warm.py): hand values
whose arithmetic is exact in binary, the floors, the far-field and wall
conditions, and the fallback for non-finite network outputs."""
import numpy as np

from oracle.warm import freestream_cons, warm_state

G = 1.5  # gamma - 1 = 1/2: every value below is exact in binary


def _one(y, kind=0, nx=0.0, ny=1.0, mean=(1.25, 0.5, -0.25, 0.75), std=(0.5, 1.0, 2.0, 0.25),
         floor=0.0625, mach=0.5, alpha=0.0):
    Y = np.array([y], np.float32)
    return warm_state(Y, mean, std, floor, np.array([kind]), np.array([nx]), np.array([ny]),
                      mach, alpha, gamma=G)[:, 0]


def test_zero_output_gives_the_mean_state():
    # rho 1.25, u (0.5, -0.25), p 0.75: E = p/(gamma-1) + rho |u|^2/2 = 1.5 + 0.1953125
    np.testing.assert_array_equal(_one([0, 0, 0, 0]), [1.25, 0.625, -0.3125, 1.6953125])


def test_scaling_of_the_outputs():
    # prim = mean + std y = (1.25 + 0.5, 0.5 + 1, -0.25 - 2, 0.75 + 0.25 * 2)
    U = _one([1, 1, -1, 2])
    rho, u1, u2, p = 1.75, 1.5, -2.25, 1.25
    np.testing.assert_array_equal(U, [rho, rho * u1, rho * u2,
                                      p / (G - 1) + 0.5 * rho * (u1 * u1 + u2 * u2)])


def test_floors_on_density_and_pressure():
    # rho = 1.25 + 0.5 (-10) < 0 -> floor * rho_inf; p = 0.75 - 0.25 * 20 < 0 -> floor * p_inf
    U = _one([-10, 0, 0, -20])
    rho, p = 0.0625, 0.0625 / G
    assert U[0] == rho
    np.testing.assert_allclose(U[3], p / (G - 1) + 0.5 * rho * 0.3125, rtol=1e-15)


def test_outer_points_keep_the_freestream():
    Uinf = freestream_cons(0.5, 3.0, G)
    for y in ([0, 0, 0, 0], [5, -5, 1, 1], [np.inf, 0, 0, 0], [np.nan, 1, 1, 1]):
        np.testing.assert_array_equal(_one(y, kind=2, alpha=3.0), Uinf)


def test_non_finite_outputs_fall_back_to_the_freestream():
    Uinf = freestream_cons(0.5, 0.0, G)
    for y in ([np.inf, 0, 0, 0], [0, np.nan, 0, 0], [0, 0, -np.inf, 0], [0, 0, 0, np.nan]):
        np.testing.assert_array_equal(_one(y), Uinf)
    # an output so large that the energy overflows
    np.testing.assert_array_equal(_one([0, 3e38, 3e38, 0], std=(1, 1e300, 1e300, 1)), Uinf)


def test_wall_points_are_projected():
    n = np.array([0.6, 0.8])
    U = _one([1, 1, -1, 2], kind=1, nx=n[0], ny=n[1])
    Ui = _one([1, 1, -1, 2])
    m, mi = U[1:3], Ui[1:3]
    t = np.array([n[1], -n[0]])
    assert abs(m @ n) <= 1e-15 * np.abs(mi).max()
    np.testing.assert_allclose(m @ t, mi @ t, rtol=1e-15)
    assert U[0] == Ui[0] and U[3] == Ui[3]
