"""Seeded synthetic inputs for the near-field (P2P) operator.

This module only draws random numbers and lays them out. It holds none of the
operator's arithmetic (no keys, no trees, no kernels), so that the FP64 oracle
and the GPU path can both be fed from it without sharing any method code.

Every generator takes an explicit seed and uses ``numpy.random.default_rng``.
The order of the draws is part of the recipe and must not change.

Workloads (the paper has no public inputs; these stand in for its two case
studies, Sec. 4 and Sec. 5):

* ``uniform_particles``   -- particles uniform in the unit cube (gravity, uniform tree).
* ``plummer_mixture``     -- clustered particles from a mixture of Plummer spheres.
  It stands in for the PhotoNs-2.0 stellar-dynamics data set, which is not
  available (Sec. 5.2).
* ``grid_rhs``            -- complex64 source strengths on regular grids with
  i.i.d. N(0,1) real and imaginary parts.  DBIM drives its MLFMA calls with
  random input vectors (Sec. 5.1.3); these stand in for them.
* ``batched_grid_sides``  -- uneven grid edge lengths for a batch of instances.
"""
from __future__ import annotations

import numpy as np


def uniform_particles(n: int, seed: int):
    """Positions uniform in [0,1)^3 and masses uniform in [0.5,1.5]/n.

    Draw order: positions ``rng.random((n, 3))``, then masses.
    Returns float64 arrays x, y, z, m (each contiguous, length n).
    """
    rng = np.random.default_rng(seed)
    p = rng.random((n, 3))
    m = rng.uniform(0.5, 1.5, n) / n
    return (np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]),
            np.ascontiguousarray(p[:, 2]), m.astype(np.float64))


def slab_particles(n_slab: int, n_sparse: int, width: float, seed: int):
    """A thin dense slab against a sparse half-space: n_slab points uniform in
    [0.5, 0.5 + width) x [0,1)^2 and n_sparse uniform in [0, 0.5) x [0,1)^2,
    masses uniform in [0.5,1.5]/n.  Large sparse leaves then touch hundreds of
    small slab leaves (long near lists).

    Draw order: slab x, sparse x, then y, z of all points, then masses.
    """
    rng = np.random.default_rng(seed)
    n = n_slab + n_sparse
    x = np.concatenate([0.5 + rng.random(n_slab) * width, rng.random(n_sparse) * 0.5])
    y = rng.random(n)
    z = rng.random(n)
    m = rng.uniform(0.5, 1.5, n) / n
    return x, y, z, m.astype(np.float64)


def plummer_scale_radii(n_spheres: int = 8):
    """Scale radii a_s = 0.01 * 10**(s/(n_spheres-1)), geometric from 0.01 to 0.1."""
    s = np.arange(n_spheres, dtype=np.float64)
    return 0.01 * 10.0 ** (s / (n_spheres - 1))


def plummer_mixture(n: int, seed: int, n_spheres: int = 8):
    """Mixture of Plummer spheres inside the unit cube.

    Recipe: centres ``rng.random((n_spheres, 3))``; then, sphere by sphere, the
    particles of sphere s (n // n_spheres each, the first n % n_spheres spheres
    take one more) are drawn in rounds: a radius by the inverse Plummer mass
    profile r = a (u^{-2/3} - 1)^{-1/2} with u uniform in (0,1], and an
    isotropic direction (cos(theta) uniform in [-1,1], phi uniform in
    [0, 2 pi)).  Points that fall outside [0,1)^3 are rejected and redrawn in
    the next round.  Masses follow the uniform recipe, uniform in [0.5,1.5]/n,
    drawn last.
    """
    rng = np.random.default_rng(seed)
    centres = rng.random((n_spheres, 3))
    radii = plummer_scale_radii(n_spheres)
    counts = np.full(n_spheres, n // n_spheres, dtype=np.int64)
    counts[: n % n_spheres] += 1
    out = np.empty((n, 3), dtype=np.float64)
    pos = 0
    for s in range(n_spheres):
        need = int(counts[s])
        got = []
        while need > 0:
            k = max(need, 1024)
            u = 1.0 - rng.random(k)                      # (0, 1]
            r = radii[s] / np.sqrt(u ** (-2.0 / 3.0) - 1.0 + 1e-300)
            ct = rng.uniform(-1.0, 1.0, k)
            ph = rng.uniform(0.0, 2.0 * np.pi, k)
            st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
            p = np.stack([centres[s, 0] + r * st * np.cos(ph),
                          centres[s, 1] + r * st * np.sin(ph),
                          centres[s, 2] + r * ct], axis=1)
            ok = np.all((p >= 0.0) & (p < 1.0), axis=1)
            p = p[ok][:need]
            got.append(p)
            need -= p.shape[0]
        blk = np.concatenate(got, axis=0)
        out[pos: pos + blk.shape[0]] = blk
        pos += blk.shape[0]
    m = rng.uniform(0.5, 1.5, n) / n
    return (np.ascontiguousarray(out[:, 0]), np.ascontiguousarray(out[:, 1]),
            np.ascontiguousarray(out[:, 2]), m.astype(np.float64))


def grid_rhs(n_points: int, nrhs: int, seed: int):
    """Complex64 array [n_points, nrhs] with i.i.d. N(0,1) real and imaginary parts.

    Draw order: all real parts, then all imaginary parts.
    """
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((n_points, nrhs)).astype(np.float32)
    im = rng.standard_normal((n_points, nrhs)).astype(np.float32)
    q = np.empty((n_points, nrhs), dtype=np.complex64)
    q.real = re
    q.imag = im
    return q


def batched_grid_sides(n_instances: int, seed: int, lo: int = 4, hi: int = 13):
    """Edge lengths n_i = 4 * rng.integers(lo, hi): multiples of 4 in [4 lo, 4 (hi-1)]."""
    rng = np.random.default_rng(seed)
    return (4 * rng.integers(lo, hi, size=n_instances)).astype(np.int32)


def normal_like(shape, seed: int, dtype=np.float64):
    """i.i.d. N(0,1) values (upstream gradients); complex dtypes get N(0,1) parts."""
    rng = np.random.default_rng(seed)
    if np.issubdtype(np.dtype(dtype), np.complexfloating):
        re = rng.standard_normal(shape)
        im = rng.standard_normal(shape)
        return (re + 1j * im).astype(dtype)
    return rng.standard_normal(shape).astype(dtype)


# ---------------------------------------------------------------------------
# The five workloads.  Sizes and seeds are fixed here; tests and the benchmark
# read them from this table.
# ---------------------------------------------------------------------------
WORKLOADS = {
    # gravity, uniform particles, uniform octree depth 3, FP64
    "gravity_uniform_4096": dict(kind="gravity", gen="uniform", n=4096, seed=1,
                                 depth=3, leaf_cap=0, eps=1e-3, prec="fp64"),
    # Helmholtz, 64^3 grid, single RHS, FP32 vs FP64 oracle
    "helmholtz_grid_64": dict(kind="helmholtz", n_side=64, nrhs=1, seed=2, prec="fp32"),
    # gravity, 2^21 Plummer-mixture particles, adaptive octree cap 64, FP32-mixed
    "gravity_plummer_2m": dict(kind="gravity", gen="plummer", n=1 << 21, seed=3,
                               depth=20, leaf_cap=64, eps=1e-3, prec="fp32"),
    # Helmholtz, 128 grids of edge 16..48, 64 RHS, FP32 MFMA, one persistent launch
    "helmholtz_batched_128x64": dict(kind="helmholtz_batched", n_instances=128,
                                     nrhs=64, seed=4, prec="fp32"),
    # differentiated: gravity 2^18 Plummer (cap 64) and Helmholtz 48^3
    "adjoint_gravity_256k": dict(kind="gravity", gen="plummer", n=1 << 18, seed=5,
                                 depth=20, leaf_cap=64, eps=1e-3, prec="fp64"),
    "adjoint_helmholtz_48": dict(kind="helmholtz", n_side=48, nrhs=1, seed=5, prec="fp64"),
}


def grid_geometry(n_side: int):
    """Spacing h = 1/n_side (unit cube, cell-centred points) and wavenumber k for
    10 points per wavelength, k = 2 pi / (10 h)."""
    h = 1.0 / n_side
    return h, 2.0 * np.pi / (10.0 * h)


def particles(name: str):
    w = WORKLOADS[name]
    if w["gen"] == "uniform":
        return uniform_particles(w["n"], w["seed"])
    return plummer_mixture(w["n"], w["seed"])
