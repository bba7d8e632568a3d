"""Seeded synthetic inputs shaped like the paper's workloads.

Shared by the tests, the oracle checks and the benchmark.  It holds none of
the method's arithmetic: it only draws densities, keyframes, velocity fields
and forces with NumPy's default_rng and blurs them with scipy.ndimage.
Lengths are in cell units; arrays use the C-order layout of the MAC grid
(cells (n2, n1, n0); faces x | y | z flattened).

The paper's keyframes (letter glyphs, bunny, armadillo, motion capture) are
not available; blobs, strokes and ellipsoids stand in for them at the same
grid sizes and step counts.
"""
import math

import numpy as np
from scipy import ndimage


def _coords(n):
    shape = tuple(reversed(n))
    g = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    return [g[len(n) - 1 - a] for a in range(len(n))]      # x, y[, z]


def gaussian_ball(n, centre, sigma):
    X = _coords(n)
    r2 = sum((X[a] - centre[a]) ** 2 for a in range(len(n)))
    return np.exp(-r2 / (2.0 * sigma * sigma)).ravel()


def blurred_ball(n, centre, radius, blur=1.0):
    X = _coords(n)
    r2 = sum((X[a] - centre[a]) ** 2 for a in range(len(n)))
    m = (r2 <= radius * radius).astype(np.float64)
    return ndimage.gaussian_filter(m, blur, mode="constant").ravel()


def blobs(n, rng, count, sig_lo=2.0, sig_hi=5.0):
    out = np.zeros(int(np.prod(n)))
    for _ in range(count):
        c = rng.uniform(np.array(n) / 4.0, 3.0 * np.array(n) / 4.0)
        s = rng.uniform(sig_lo, sig_hi)
        out = np.maximum(out, gaussian_ball(n, c, s))
    return out


def strokes(n, rng, count, width=6.0, blur=1.0):
    """Union of straight strokes (axis-aligned and diagonal), 2D only."""
    X = _coords(n)
    m = np.zeros(tuple(reversed(n)))
    half = width / 2.0
    for _ in range(count):
        p0 = rng.uniform(np.array(n) / 4.0, 3.0 * np.array(n) / 4.0)
        ang = math.radians(45.0 * rng.integers(0, 4))
        length = rng.uniform(n[0] / 8.0, n[0] / 3.0)
        dvec = np.array([math.cos(ang), math.sin(ang)])
        rx, ry = X[0] - p0[0], X[1] - p0[1]
        t = np.clip(rx * dvec[0] + ry * dvec[1], 0.0, length)
        dist2 = (rx - t * dvec[0]) ** 2 + (ry - t * dvec[1]) ** 2
        m = np.maximum(m, (dist2 <= half * half).astype(np.float64))
    return ndimage.gaussian_filter(m, blur, mode="constant").ravel()


def ellipsoids(n, rng, count, semi_lo, semi_hi, blur=1.0):
    X = _coords(n)
    m = np.zeros(tuple(reversed(n)))
    for _ in range(count):
        c = rng.uniform(np.array(n) / 4.0, 3.0 * np.array(n) / 4.0)
        s = rng.uniform(semi_lo, semi_hi, size=len(n))
        q = sum(((X[a] - c[a]) / s[a]) ** 2 for a in range(len(n)))
        m = np.maximum(m, (q <= 1.0).astype(np.float64))
    return ndimage.gaussian_filter(m, blur, mode="constant").ravel()


# ---------------------------------------------------------------- workloads
def c1_plain_2d_32(seed=0):
    """32x32, 10 steps, one keyframe at t = 10 (3 blobs, sigma 2..5);
    initial Gaussian ball sigma = 4."""
    rng = np.random.default_rng(seed)
    n = (32, 32)
    rho0 = gaussian_ball(n, rng.uniform(8.0, 24.0, size=2), 4.0)
    key = blobs(n, rng, 3)
    return dict(n=n, num_steps=10, dt=1.0 / 32, r=1e-3, rho0=rho0, keys={10: key})


def c2_plain_2d_128(seed=0):
    """128x128, 40 steps; disk of radius 12 to a union of 4-8 strokes at t = 40."""
    rng = np.random.default_rng(seed)
    n = (128, 128)
    rho0 = blurred_ball(n, rng.uniform(32.0, 96.0, size=2), 12.0)
    key = strokes(n, rng, int(rng.integers(4, 9)))
    return dict(n=n, num_steps=40, dt=1.0 / 128, r=1e-4, rho0=rho0, keys={40: key})


def c3_precision_3d(seed=0, scale=1):
    """64^3, 60 steps; sphere of radius 12 to ellipsoid unions at t = 30, 60.
    scale = 4 gives the 16^3 instance (all lengths divided by 4)."""
    rng = np.random.default_rng(seed)
    m = 64 // scale
    n = (m, m, m)
    rho0 = blurred_ball(n, (m / 2.0 - 0.5,) * 3, 12.0 / scale, 1.0)
    k30 = ellipsoids(n, rng, int(rng.integers(3, 7)), 6.0 / scale, 16.0 / scale, 1.0)
    k60 = ellipsoids(n, rng, int(rng.integers(3, 7)), 6.0 / scale, 16.0 / scale, 1.0)
    return dict(n=n, num_steps=60, dt=1.0 / m, r=1e-3, rho0=rho0, keys={30: k30, 60: k60})


def small_problem(n=(8, 8), N=4, seed=0, r=1e-2):
    """A tiny instance for brute-force checks."""
    rng = np.random.default_rng(seed)
    nn = tuple(n)
    c = np.array(nn) / 2.0 + rng.uniform(-1.0, 1.0, size=len(nn))
    rho0 = gaussian_ball(nn, c, max(nn) / 6.0)
    key = gaussian_ball(nn, c + rng.uniform(-1.5, 1.5, size=len(nn)), max(nn) / 6.0)
    return dict(n=nn, num_steps=N, dt=1.0 / nn[0], r=r, rho0=rho0, keys={N: key})


# ---------------------------------------------------------------- fields
def face_counts(n):
    d = len(n)
    out = []
    for a in range(d):
        c = 1
        for b in range(d):
            c *= n[b] + (1 if b == a else 0)
        out.append(c)
    return out


def random_faces(n, rng, scale=1.0):
    """Random face field with zero walls (not divergence free)."""
    d = len(n)
    parts = []
    for a in range(d):
        shape = list(reversed(n))
        shape[d - 1 - a] += 1
        x = rng.standard_normal(shape) * scale
        sl = [slice(None)] * d
        sl[d - 1 - a] = 0
        x[tuple(sl)] = 0.0
        sl[d - 1 - a] = -1
        x[tuple(sl)] = 0.0
        parts.append(x.ravel())
    return np.concatenate(parts)


def curl_noise_velocity(n, rng, sigma=4.0, max_cells_per_step=2.0, dt_over_h=1.0):
    """Divergence-free MAC velocity: the discrete curl of a blurred random
    potential that vanishes on the boundary.  2D: scalar stream function at
    nodes; 3D: vector potential on edges.  Scaled so max|v| dt/h is just
    below max_cells_per_step (by 2^-10 relative), so that no backtrace of
    the fastest face starts exactly on a lattice node when the bound is an
    integer."""
    d = len(n)
    if d == 2:
        n0, n1 = n
        psi = ndimage.gaussian_filter(rng.standard_normal((n1 + 1, n0 + 1)), sigma, mode="constant")
        psi[0, :] = psi[-1, :] = 0.0
        psi[:, 0] = psi[:, -1] = 0.0
        vx = psi[1:, :] - psi[:-1, :]          # (n1, n0+1): d psi / dy
        vy = -(psi[:, 1:] - psi[:, :-1])       # (n1+1, n0): -d psi / dx
        parts = [vx, vy]
    else:
        n0, n1, n2 = n
        # edge potentials: A_x on x-edges (n2+1, n1+1, n0), A_y (n2+1, n1, n0+1), A_z (n2, n1+1, n0+1)
        Ax = ndimage.gaussian_filter(rng.standard_normal((n2 + 1, n1 + 1, n0)), sigma, mode="constant")
        Ay = ndimage.gaussian_filter(rng.standard_normal((n2 + 1, n1, n0 + 1)), sigma, mode="constant")
        Az = ndimage.gaussian_filter(rng.standard_normal((n2, n1 + 1, n0 + 1)), sigma, mode="constant")
        # zero the potentials on boundary edges (edges lying in a wall plane)
        Ax[0], Ax[-1] = 0.0, 0.0
        Ax[:, 0], Ax[:, -1] = 0.0, 0.0
        Ay[0], Ay[-1] = 0.0, 0.0
        Ay[:, :, 0], Ay[:, :, -1] = 0.0, 0.0
        Az[:, 0], Az[:, -1] = 0.0, 0.0
        Az[:, :, 0], Az[:, :, -1] = 0.0, 0.0
        vx = (Az[:, 1:, :] - Az[:, :-1, :]) - (Ay[1:, :, :] - Ay[:-1, :, :])
        vy = (Ax[1:, :, :] - Ax[:-1, :, :]) - (Az[:, :, 1:] - Az[:, :, :-1])
        vz = (Ay[:, :, 1:] - Ay[:, :, :-1]) - (Ax[:, 1:, :] - Ax[:, :-1, :])
        parts = [vx, vy, vz]
    flat = np.concatenate([p.ravel() for p in parts])
    m = np.max(np.abs(flat))
    if m > 0:
        flat = flat * ((1.0 - 2.0 ** -10) * max_cells_per_step / (m * dt_over_h))
    return flat


def smooth_noise_density(n, rng, sigma=2.0):
    shape = tuple(reversed(n))
    x = ndimage.gaussian_filter(rng.uniform(0.0, 1.0, shape), sigma, mode="constant")
    ones = ndimage.gaussian_filter(np.ones(shape), sigma, mode="constant")
    return (x / ones).ravel()


# ---------------------------------------------------------------- serving stream
def c5_requests(seed=0, count=64, rate=1.0, sizes2d=(64, 128, 256), sizes3d=(32, 64, 96),
                steps2d=(20, 80), steps3d=(20, 60), r=1e-3):
    """Control requests arriving by a Poisson process of the given rate (per
    second): 2D grids from sizes2d with N ~ U{steps2d}, or 3D grids from
    sizes3d with N ~ U{steps3d}, each with probability 1/2; 1-3 keyframes at
    distinct steps, the last at N (blobs, or strokes in 2D); dt = 1/n.
    Returns dicts with the fields of a serving request."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        if rng.uniform() < 0.5:
            m = int(rng.choice(sizes2d))
            n = (m, m)
            N = int(rng.integers(steps2d[0], steps2d[1] + 1))
        else:
            m = int(rng.choice(sizes3d))
            n = (m, m, m)
            N = int(rng.integers(steps3d[0], steps3d[1] + 1))
        nk = int(rng.integers(1, 4))
        steps = sorted(set(rng.choice(np.arange(1, N), size=nk - 1, replace=False).tolist()) | {N}) if N > 1 else [N]
        c = np.array(n) / 2.0 + rng.uniform(-m / 8.0, m / 8.0, size=len(n))
        rho0 = gaussian_ball(n, c, m / 10.0)
        keys = []
        for _ in steps:
            if len(n) == 2 and rng.uniform() < 0.5:
                keys.append(strokes(n, rng, int(rng.integers(2, 5)), width=max(2.0, m / 20.0)))
            else:
                keys.append(blobs(n, rng, int(rng.integers(1, 4)), m / 16.0, m / 8.0))
        out.append(dict(rid=rid, arrival=t, n=n, num_steps=N, r=r, rho0=rho0, key_steps=steps,
                        key_rho=np.stack(keys), dt=1.0 / m))
    return out
