"""Seeded synthetic inputs for the MLFMA matvec (point clouds and charges).

This module only draws random numbers; it holds none of the method's
arithmetic, so both the HIP path's tests and the FP64 oracle may use it.
Every generator uses ``numpy.random.default_rng(seed)`` and draws the
positions first, then the charges, from the same stream.

Workloads (wavelength 1, so k = 2 pi; leaf box side 0.25):

  sphere4k      N = 4,096 points area-uniform on a sphere of radius 1
                (diameter 2 wavelengths), complex128 charges, 1 RHS.
  sphere262k    N = 262,144 points area-uniform on a sphere of radius 8
                (diameter 16 wavelengths), complex64 charges, 1 RHS.
  spheroid1m    N = 1,048,576: 90% area-uniform on a prolate spheroid with
                semi-axes (3.2, 3.2, 32) (aspect 10:1, length 64), 10% in a
                Gaussian cluster (sigma 0.5) at the tip (0, 0, 32), redrawn
                while |z| > 32; complex64 charges, 1 RHS.
  sphere262k_r64  the sphere262k cloud with 64 right-hand sides.
  cube1m_r16    N = 1,048,576 uniform in [-8, 8]^3 with 16 right-hand
                sides; a second, independent charge set (seed 1) drives the
                target potential of the differentiation workload.

Charges are complex normal: real and imaginary parts N(0, 1).
"""
import math

import numpy as np

K_WAVENUMBER = 2.0 * math.pi
LEAF_SIZE = 0.25
DIGITS = 3


def _charges(rng, n, nrhs, dtype):
    shape = (n,) if nrhs == 1 else (n, nrhs)
    q = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return q.astype(dtype)


def sphere_points(rng, n, radius):
    """Area-uniform points on a sphere: normalised 3-D normal vectors."""
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return radius * v


def spheroid_points(rng, n, semi=(3.2, 3.2, 32.0)):
    """Area-uniform points on an ellipsoid by rejection: map a uniform
    sphere point u to (a u_x, b u_y, c u_z) and keep it with probability
    proportional to the local area stretch."""
    a, b, c = semi
    gmax = max(b * c, a * c, a * b)
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = 2 * (n - out.shape[0]) + 1024
        u = sphere_points(rng, m, 1.0)
        g = np.sqrt((b * c * u[:, 0]) ** 2 + (a * c * u[:, 1]) ** 2
                    + (a * b * u[:, 2]) ** 2)
        keep = rng.random(m) * gmax < g
        out = np.concatenate([out, u[keep] * np.array(semi)])
    return out[:n]


def tip_cluster(rng, n, tip=(0.0, 0.0, 32.0), sigma=0.5, zmax=32.0):
    """Isotropic Gaussian cluster at the tip, redrawn while |z| > zmax."""
    pts = tip + sigma * rng.standard_normal((n, 3))
    bad = np.abs(pts[:, 2]) > zmax
    while np.any(bad):
        pts[bad] = tip + sigma * rng.standard_normal((int(bad.sum()), 3))
        bad = np.abs(pts[:, 2]) > zmax
    return pts


WORKLOADS = {
    "sphere4k": dict(n=4096, shape="sphere", radius=1.0, nrhs=1,
                     dtype=np.complex128),
    "sphere262k": dict(n=262144, shape="sphere", radius=8.0, nrhs=1,
                       dtype=np.complex64),
    "spheroid1m": dict(n=1048576, shape="spheroid", nrhs=1,
                       dtype=np.complex64),
    "sphere262k_r64": dict(n=262144, shape="sphere", radius=8.0, nrhs=64,
                           dtype=np.complex64),
    "cube1m_r16": dict(n=1048576, shape="cube", half=8.0, nrhs=16,
                       dtype=np.complex64),
}


def make(name, seed=0, n=None, nrhs=None):
    """Positions [n, 3] float64 and charges [n] or [n, nrhs] for a workload.

    ``n`` and ``nrhs`` override the workload's sizes (same recipe, smaller
    or larger instance)."""
    spec = dict(WORKLOADS[name])
    n = spec["n"] if n is None else int(n)
    nrhs = spec["nrhs"] if nrhs is None else int(nrhs)
    rng = np.random.default_rng(seed)
    if spec["shape"] == "sphere":
        xyz = sphere_points(rng, n, spec["radius"])
    elif spec["shape"] == "spheroid":
        ntip = int(round(0.1 * n))
        body = spheroid_points(rng, n - ntip)
        xyz = np.concatenate([body, tip_cluster(rng, ntip)])
    elif spec["shape"] == "cube":
        h = spec["half"]
        xyz = rng.uniform(-h, h, size=(n, 3))
    else:
        raise ValueError(spec["shape"])
    q = _charges(rng, n, nrhs, spec["dtype"])
    return np.ascontiguousarray(xyz), q


def charges(n, nrhs, seed, dtype=np.complex64):
    """An independent complex-normal charge set (e.g. the target set)."""
    rng = np.random.default_rng(seed)
    return _charges(rng, n, nrhs, dtype)
