"""Seeded synthetic inputs: point clouds on closed surfaces and CN(0,1) right-hand sides.

This module only draws inputs. It holds none of the method's arithmetic (no kernel
evaluation, no tree, no compression, no product), so both the product path and the
CPU oracle may consume what it returns.

The paper's experiments use Galerkin meshes of several shapes (section 6.1); those
meshes are not available, so quasi-uniform point clouds on a sphere, an ellipsoid and
a cube surface stand in for them, discretised Nystrom-style (one point per unknown,
which section 3.1 lists as an admissible discretisation).

Recipes
-------
sphere     Fibonacci lattice z_i = 1-(2i+1)/N, phi_i = i*pi*(3-sqrt 5), jittered by
           0.1*h*xi with xi ~ U[-1,1]^3, then projected back onto the unit sphere.
ellipsoid  the jittered sphere points scaled by the semi-axes (1, 0.5, 0.25).
cube       surface of [0,1]^3: 6 faces, each an n x n grid of cell centres
           (n = round(sqrt(N/6)), so the actual count is 6 n^2), jittered in-plane by
           0.1*h*xi with xi ~ U[-1,1]^2.
h          sqrt(area / N): the mean spacing of the points on the surface.
kappa      kappa_h / h (kappa_h = 0.6 by default: about 10.5 points per wavelength).

Every draw uses numpy's PCG64 through ``numpy.random.default_rng`` with an explicit
(seed, stream) pair, so a cloud and its right-hand sides never share a stream.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_STREAM_POINTS = 1
_STREAM_RHS = 2

SURFACES = ("sphere", "ellipsoid", "cube")
ELLIPSOID_AXES = (1.0, 0.5, 0.25)


@dataclass(frozen=True)
class PointCloud:
    """Points in user order (row i is unknown i) plus the spacing and wavenumber."""

    surface: str
    points: np.ndarray  # (N, 3) float64, C-contiguous
    h: float
    kappa: float
    seed: int

    @property
    def n(self) -> int:
        return int(self.points.shape[0])


def _fibonacci_sphere(n: int) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def ellipsoid_area(axes=ELLIPSOID_AXES, nq: int = 400) -> float:
    """Surface area of an ellipsoid by tensor quadrature (Gauss-Legendre in cos(theta),
    trapezoid in phi, which is spectrally accurate for the periodic direction)."""
    a, b, c = axes
    t, w = np.polynomial.legendre.leggauss(nq)  # t = cos(theta) in [-1, 1]
    phi = np.linspace(0.0, 2.0 * math.pi, 2 * nq, endpoint=False)
    ct = t[:, None]
    st = np.sqrt(1.0 - ct * ct)
    cp, sp = np.cos(phi)[None, :], np.sin(phi)[None, :]
    # r(theta, phi) = (a st cp, b st sp, c ct); |r_theta x r_phi| / st is smooth in ct
    nx = b * c * st * cp
    ny = a * c * st * sp
    nz = a * b * ct
    dens = np.sqrt(nx * nx + ny * ny + nz * nz)  # = |r_theta x r_phi| / sin(theta)
    return float((w[:, None] * dens).sum() * (2.0 * math.pi / (2 * nq)))


def make_cloud(surface: str, n: int, seed: int = 0, kappa_h: float = 0.6) -> PointCloud:
    """Seeded point cloud on one of the synthetic surfaces (see the module recipes)."""
    if n < 1:
        raise ValueError("n must be positive")
    rng = np.random.default_rng([seed, _STREAM_POINTS])
    if surface in ("sphere", "ellipsoid"):
        h_unit = math.sqrt(4.0 * math.pi / n)
        p = _fibonacci_sphere(n) + 0.1 * h_unit * rng.uniform(-1.0, 1.0, size=(n, 3))
        p /= np.linalg.norm(p, axis=1)[:, None]
        if surface == "sphere":
            area = 4.0 * math.pi
        else:
            p = p * np.asarray(ELLIPSOID_AXES)[None, :]
            area = ellipsoid_area()
    elif surface == "cube":
        m = max(1, int(round(math.sqrt(n / 6.0))))
        n = 6 * m * m
        area = 6.0
        hh = 1.0 / m
        g = (np.arange(m) + 0.5) / m
        ga, gb = np.meshgrid(g, g, indexing="ij")
        ga, gb = ga.ravel(), gb.ravel()
        faces = []
        for axis in range(3):
            for side in (0.0, 1.0):
                uv = np.stack([ga, gb], 1) + 0.1 * hh * rng.uniform(-1.0, 1.0, size=(m * m, 2))
                uv = np.clip(uv, 0.0, 1.0)
                f = np.empty((m * m, 3))
                others = [a for a in range(3) if a != axis]
                f[:, axis] = side
                f[:, others[0]] = uv[:, 0]
                f[:, others[1]] = uv[:, 1]
                faces.append(f)
        p = np.concatenate(faces, 0)
    else:
        raise ValueError(f"unknown surface {surface!r}; expected one of {SURFACES}")
    h = math.sqrt(area / n)
    return PointCloud(surface, np.ascontiguousarray(p, dtype=np.float64), h, kappa_h / h, seed)


def make_rhs(n: int, nrhs: int = 1, seed: int = 0, dtype=np.complex128) -> np.ndarray:
    """x ~ CN(0,1): real and imaginary parts i.i.d. N(0, 1/2). Column-major (n, nrhs)."""
    rng = np.random.default_rng([seed, _STREAM_RHS])
    s = math.sqrt(0.5)
    x = rng.normal(0.0, s, size=(nrhs, n)) + 1j * rng.normal(0.0, s, size=(nrhs, n))
    return np.asfortranarray(x.T.astype(dtype))


def log_uniform_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """N = round(exp(U[ln lo, ln hi])) for a mixed-size operator population."""
    rng = np.random.default_rng([seed, 3])
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)
