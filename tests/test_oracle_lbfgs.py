"""Pins of the L-BFGS baseline oracle (the paper's comparison optimiser):
the adjoint gradient against central finite differences, and the
optimiser against problems whose minimiser is known."""
import numpy as np
import pytest
from scipy.optimize import rosen, rosen_der

import synthetic
from oracle import lbfgs, metric
from oracle.admm import objectives, resimulate
from oracle.grid import Grid


def _tiny(seed=0):
    w = synthetic.small_problem((8, 8), 3, seed=seed, r=1e-2)
    rng = np.random.default_rng(seed + 10)
    w["keys"][2] = synthetic.smooth_noise_density((8, 8), rng, 1.0)
    return w


@pytest.mark.parametrize("velocity", ["sl", "vorticity"])
def test_gradient_matches_finite_differences(velocity):
    w = _tiny()
    g = Grid(w["n"])
    N, dt, r = w["num_steps"], w["dt"], w["r"]
    levels = metric.default_levels(w["n"])
    rng = np.random.default_rng(1)
    u = 0.05 * np.stack([synthetic.random_faces(w["n"], rng) for _ in range(N)])

    def J(x):
        rho, _ = resimulate(g, w["rho0"], x, dt, velocity=velocity)
        return objectives(g, rho, w["keys"], x, r, levels)[0]

    rho, v = resimulate(g, w["rho0"], u, dt, velocity=velocity)
    gr = lbfgs.gradient(g, rho, v, u, w["keys"], r, dt, levels, velocity=velocity)
    for k in range(3):
        d = np.stack([synthetic.random_faces(w["n"], rng) for _ in range(N)])
        eps = 1e-6
        fd = (J(u + eps * d) - J(u - eps * d)) / (2 * eps)
        assert abs(fd - np.sum(gr * d)) <= 1e-6 * max(abs(fd), 1e-12), k


def test_minimize_quadratic_reaches_solution():
    rng = np.random.default_rng(2)
    n = 30
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.logspace(0, 2, n)) @ Q.T
    b = rng.standard_normal(n)
    x, hist, done = lbfgs.minimize(lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b), np.zeros(n), 200)
    xs = np.linalg.solve(A, b)
    # an Armijo search on f resolves x to about sqrt(machine epsilon) times the conditioning
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)
    assert all(hist[i + 1] <= hist[i] for i in range(len(hist) - 1))


def test_minimize_rosenbrock():
    x, hist, done = lbfgs.minimize(lambda x: (rosen(x), rosen_der(x)), np.array([-1.2, 1.0]), 200)
    assert np.allclose(x, [1.0, 1.0], atol=1e-6)
    assert done < 200


@pytest.mark.parametrize("velocity", ["sl", "vorticity"])
def test_solve_decreases_objective(velocity):
    w = _tiny(3)
    g = Grid(w["n"])
    levels = metric.default_levels(w["n"])
    u, hist, done = lbfgs.solve(g, w["rho0"], w["keys"], w["num_steps"], w["r"], w["dt"], levels, 6,
                                velocity=velocity)
    assert done == 6
    assert all(hist[i + 1] <= hist[i] for i in range(len(hist) - 1))
    assert hist[-1] < hist[0]
    # the history is the objective of the returned controls under the same simulation
    rho, _ = resimulate(g, w["rho0"], u, w["dt"], velocity=velocity)
    assert abs(objectives(g, rho, w["keys"], u, w["r"], levels)[0] - hist[-1]) <= 1e-12 * hist[-1]


def test_visual_difference_stop_by_brute_force():
    """The stop after an accepted iterate: brute force over the iterates of
    unstopped runs (the method is deterministic, so k iterations give the
    k-th iterate) finds the first k whose trajectory change is at most eps;
    the stopped run must end exactly there, on that iterate."""
    w = _tiny(2)
    g = Grid(w["n"])
    N, dt, r = w["num_steps"], w["dt"], w["r"]
    levels = metric.default_levels(w["n"])
    K = 6
    xs = [lbfgs.solve(g, w["rho0"], w["keys"], N, r, dt, levels, k)[0] for k in range(K + 1)]
    traj = [resimulate(g, w["rho0"], x, dt)[0] for x in xs]
    diffs = [float(np.max(np.abs(traj[k] - traj[k - 1]))) for k in range(1, K + 1)]
    # a threshold between the smallest and largest change so that the stop
    # fires before K iterations
    eps = 0.5 * (min(diffs) + max(diffs))
    first = next(k + 1 for k, d in enumerate(diffs) if d <= eps)
    assert first < K
    x, hist, done = lbfgs.solve(g, w["rho0"], w["keys"], N, r, dt, levels, K, eps_stop=eps)
    assert done == first and len(hist) == first + 1
    assert np.array_equal(x, xs[first])
    # eps = 0 never stops early, a huge eps stops after the first iterate
    assert lbfgs.solve(g, w["rho0"], w["keys"], N, r, dt, levels, 3, eps_stop=0.0)[2] == 3
    assert lbfgs.solve(g, w["rho0"], w["keys"], N, r, dt, levels, 3, eps_stop=1e30)[2] == 1


@pytest.mark.parametrize("velocity", ["sl", "vorticity"])
def test_gradient_matches_finite_differences_3d(velocity):
    """The same pin on a 3D grid (vorticity on edges for the rotational form)."""
    w = synthetic.small_problem((5, 4, 4), 2, seed=12, r=1e-2)
    g = Grid(w["n"])
    N, dt, r = w["num_steps"], w["dt"], w["r"]
    levels = metric.default_levels(w["n"])
    rng = np.random.default_rng(13)
    u = 0.05 * np.stack([synthetic.random_faces(w["n"], rng) for _ in range(N)])

    def J(x):
        rho, _ = resimulate(g, w["rho0"], x, dt, velocity=velocity)
        return objectives(g, rho, w["keys"], x, r, levels)[0]

    rho, v = resimulate(g, w["rho0"], u, dt, velocity=velocity)
    gr = lbfgs.gradient(g, rho, v, u, w["keys"], r, dt, levels, velocity=velocity)
    for k in range(2):
        d = np.stack([synthetic.random_faces(w["n"], rng) for _ in range(N)])
        eps = 1e-6
        fd = (J(u + eps * d) - J(u - eps * d)) / (2 * eps)
        assert abs(fd - np.sum(gr * d)) <= 1e-6 * max(abs(fd), 1e-12), k
