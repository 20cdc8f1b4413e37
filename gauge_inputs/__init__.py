"""Seeded synthetic SU(3) gauge configurations.

This module only *makes inputs*; it holds none of the gauge-fixing arithmetic
(no local functional, no subgroup maximiser, no overrelaxation, no gauge
condition).  Both the FP64 CPU oracle and the HIP library receive the arrays
produced here, so the two sides never share anything else.

Canonical host layout (what every entry point of the library and of the
oracle takes and returns): a C-contiguous float64 array of shape
``(V, 4, 3, 3, 2)`` = ``[site][mu][row][col][re, im]`` where the site index
is lexicographic with x fastest, ``site = x + Nx*(y + Ny*(z + Nz*t))``, and
``mu = 0..3`` is the x, y, z, t direction.  ``U[site, mu]`` is the link
``U_mu(x)`` that starts at ``x`` and points to ``x + mu^``.

Recipe (the lattice workloads are stated as: links ``exp(i eps H)`` with
``H`` random traceless Hermitian with N(0,1) entries, followed by a
Haar-random SU(3) gauge transformation at every site):

* ``H``: diagonal entries N(0,1) minus their mean, off-diagonal entries
  ``(a + i b)/sqrt(2)`` with ``a, b ~ N(0,1)``, Hermitian.
* ``exp(i eps H)`` by the float64 matrix exponential of ``torch.linalg``
  (CPU); ``det = exp(i eps tr H) = 1``.
* Haar SU(3) ``h(x)``: two complex Gaussian rows, Gram-Schmidt, third row the
  conjugated cross product (the unique unit-determinant completion).
* ``U_mu(x) <- h(x) U_mu(x) h(x + mu^)^dagger`` (periodic).

The random stream is numpy's PCG64 seeded with ``seed``; all draws happen in
one fixed order, and every matrix is computed independently of the others,
so the output does not depend on the thread count.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "volume",
    "lex_coords",
    "complex_view",
    "to_canonical",
    "random_traceless_hermitian",
    "expi_hermitian",
    "haar_su3",
    "identity_links",
    "gen_links",
    "pure_gauge_links",
    "su2_embedded_links",
    "random_traceless_hermitian2",
    "haar_su2",
    "gen_links_su2",
    "identity_links_su2",
    "pure_gauge_links_su2",
]


def volume(dims) -> int:
    nx, ny, nz, nt = (int(d) for d in dims)
    return nx * ny * nz * nt


def lex_coords(dims) -> np.ndarray:
    """(V, 4) int array of (x, y, z, t) for every lexicographic site."""
    nx, ny, nz, nt = (int(d) for d in dims)
    s = np.arange(volume(dims), dtype=np.int64)
    x = s % nx
    y = (s // nx) % ny
    z = (s // (nx * ny)) % nz
    t = s // (nx * ny * nz)
    return np.stack([x, y, z, t], axis=1)


def complex_view(links: np.ndarray) -> np.ndarray:
    """View a canonical (..., 3, 3, 2) float64 array as (..., 3, 3) complex128."""
    a = np.ascontiguousarray(links, dtype=np.float64)
    return a.view(np.complex128)[..., 0]


def to_canonical(u: np.ndarray) -> np.ndarray:
    """(..., 3, 3) complex128 -> (..., 3, 3, 2) float64 (copy, C-contiguous)."""
    u = np.ascontiguousarray(u, dtype=np.complex128)
    return np.ascontiguousarray(u.view(np.float64).reshape(u.shape + (2,)))


def random_traceless_hermitian(rng: np.random.Generator, n: int) -> np.ndarray:
    """n random traceless Hermitian 3x3 matrices (complex128)."""
    d = rng.standard_normal((n, 3))
    d -= d.mean(axis=1, keepdims=True)
    off = rng.standard_normal((n, 3, 2)) / math.sqrt(2.0)
    off_c = off[..., 0] + 1j * off[..., 1]
    h = np.zeros((n, 3, 3), dtype=np.complex128)
    h[:, 0, 0] = d[:, 0]
    h[:, 1, 1] = d[:, 1]
    h[:, 2, 2] = d[:, 2]
    for k, (i, j) in enumerate(((0, 1), (0, 2), (1, 2))):
        h[:, i, j] = off_c[:, k]
        h[:, j, i] = np.conj(off_c[:, k])
    return h


def expi_hermitian(h: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*H) for a stack of Hermitian matrices (float64 matrix exponential)."""
    import torch

    out = np.empty_like(h)
    for lo in range(0, h.shape[0], 1 << 21):
        hi = min(lo + (1 << 21), h.shape[0])
        a = torch.from_numpy(np.ascontiguousarray(h[lo:hi])) * (1j * float(eps))
        out[lo:hi] = torch.linalg.matrix_exp(a).numpy()
    return out


def haar_su3(rng: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-distributed SU(3) matrices (complex128)."""
    g = rng.standard_normal((n, 2, 3, 2))
    rows = g[..., 0] + 1j * g[..., 1]
    r0 = rows[:, 0]
    r1 = rows[:, 1]
    r0 = r0 / np.linalg.norm(r0, axis=1, keepdims=True)
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=1)


def identity_links(dims) -> np.ndarray:
    v = volume(dims)
    u = np.zeros((v, 4, 3, 3), dtype=np.complex128)
    u[:, :, 0, 0] = u[:, :, 1, 1] = u[:, :, 2, 2] = 1.0
    return to_canonical(u)


def _forward_site(dims, mu: int) -> np.ndarray:
    c = lex_coords(dims)
    nx, ny, nz, nt = (int(d) for d in dims)
    n = (nx, ny, nz, nt)
    c[:, mu] = (c[:, mu] + 1) % n[mu]
    return c[:, 0] + nx * (c[:, 1] + ny * (c[:, 2] + nz * c[:, 3]))


def _gauge_rotate(u: np.ndarray, h: np.ndarray, dims) -> np.ndarray:
    """u[s, mu] <- h[s] u[s, mu] h[s + mu^]^dagger (input construction only)."""
    import torch

    out = np.empty_like(u)
    th = torch.from_numpy(np.ascontiguousarray(h))
    for mu in range(4):
        fwd = torch.from_numpy(_forward_site(dims, mu))
        hd = th[fwd].transpose(-1, -2).conj()
        um = torch.from_numpy(np.ascontiguousarray(u[:, mu]))
        out[:, mu] = torch.matmul(torch.matmul(th, um), hd).numpy()
    return out


def gen_links(dims, eps: float, seed: int, gauge_rotate: bool = True) -> np.ndarray:
    """The synthetic configuration: exp(i eps H) links, then a Haar gauge rotation.

    Returns the canonical (V, 4, 3, 3, 2) float64 array.
    """
    dims = tuple(int(d) for d in dims)
    v = volume(dims)
    rng = np.random.default_rng(int(seed))
    h = random_traceless_hermitian(rng, 4 * v)
    u = expi_hermitian(h, float(eps)).reshape(v, 4, 3, 3)
    del h
    if gauge_rotate:
        g = haar_su3(rng, v)
        u = _gauge_rotate(u, g, dims)
    return to_canonical(u)


def pure_gauge_links(dims, seed: int) -> np.ndarray:
    """U_mu(x) = h(x) h(x+mu^)^dagger with Haar h: a gauge copy of the unit field."""
    dims = tuple(int(d) for d in dims)
    rng = np.random.default_rng(int(seed))
    g = haar_su3(rng, volume(dims))
    u = complex_view(identity_links(dims)).copy()
    return to_canonical(_gauge_rotate(u, g, dims))


def su2_embedded_links(dims, seed: int, eps: float = 0.8) -> np.ndarray:
    """Links diag(u, 1) with u a random SU(2) matrix in the (0,1) block."""
    dims = tuple(int(d) for d in dims)
    v = volume(dims)
    rng = np.random.default_rng(int(seed))
    a = rng.standard_normal((v * 4, 4))
    a[:, 0] += 1.0 / max(eps, 1e-12)
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    u = np.zeros((v * 4, 3, 3), dtype=np.complex128)
    u[:, 0, 0] = a[:, 0] + 1j * a[:, 3]
    u[:, 0, 1] = a[:, 2] + 1j * a[:, 1]
    u[:, 1, 0] = -a[:, 2] + 1j * a[:, 1]
    u[:, 1, 1] = a[:, 0] - 1j * a[:, 3]
    u[:, 2, 2] = 1.0
    return to_canonical(u.reshape(v, 4, 3, 3))


# ------------------------------------------------------------- SU(2) links --
# Canonical SU(2) layout: (V, 4, 2, 2, 2) float64 = [site][mu][row][col][re, im].


def random_traceless_hermitian2(rng: np.random.Generator, n: int) -> np.ndarray:
    """n random traceless Hermitian 2x2 matrices: diagonal N(0,1) minus the mean,
    off-diagonal (a + i b)/sqrt(2)."""
    d = rng.standard_normal((n, 2))
    d -= d.mean(axis=1, keepdims=True)
    off = rng.standard_normal((n, 2)) / math.sqrt(2.0)
    h = np.zeros((n, 2, 2), dtype=np.complex128)
    h[:, 0, 0] = d[:, 0]
    h[:, 1, 1] = d[:, 1]
    h[:, 0, 1] = off[:, 0] + 1j * off[:, 1]
    h[:, 1, 0] = off[:, 0] - 1j * off[:, 1]
    return h


def haar_su2(rng: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-distributed SU(2) matrices: a normalised Gaussian 4-vector (r0, r1, r2, r3) as
    [[r0 + i r3, r2 + i r1], [-r2 + i r1, r0 - i r3]]."""
    r = rng.standard_normal((n, 4))
    r /= np.linalg.norm(r, axis=1, keepdims=True)
    g = np.empty((n, 2, 2), dtype=np.complex128)
    g[:, 0, 0] = r[:, 0] + 1j * r[:, 3]
    g[:, 0, 1] = r[:, 2] + 1j * r[:, 1]
    g[:, 1, 0] = -r[:, 2] + 1j * r[:, 1]
    g[:, 1, 1] = r[:, 0] - 1j * r[:, 3]
    return g


def identity_links_su2(dims) -> np.ndarray:
    v = volume(dims)
    u = np.zeros((v, 4, 2, 2), dtype=np.complex128)
    u[:, :, 0, 0] = u[:, :, 1, 1] = 1.0
    return to_canonical(u)


def gen_links_su2(dims, eps: float, seed: int, gauge_rotate: bool = True) -> np.ndarray:
    """SU(2) configuration of the same recipe: exp(i eps H), H random traceless Hermitian 2x2,
    then a Haar SU(2) gauge rotation h(x) U_mu(x) h(x+mu^)^dag.  (V, 4, 2, 2, 2) float64."""
    dims = tuple(int(d) for d in dims)
    v = volume(dims)
    rng = np.random.default_rng(int(seed))
    h = random_traceless_hermitian2(rng, 4 * v)
    u = expi_hermitian(h, float(eps)).reshape(v, 4, 2, 2)
    if gauge_rotate:
        u = _gauge_rotate(u, haar_su2(rng, v), dims)
    return to_canonical(u)


def pure_gauge_links_su2(dims, seed: int) -> np.ndarray:
    """U_mu(x) = h(x) h(x+mu^)^dagger with Haar SU(2) h."""
    dims = tuple(int(d) for d in dims)
    rng = np.random.default_rng(int(seed))
    u = complex_view(identity_links_su2(dims)).copy()
    return to_canonical(_gauge_rotate(u, haar_su2(rng, volume(dims)), dims))
