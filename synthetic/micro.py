"""Synthetic periodic polycrystals (stand-ins for the paper's Neper RVEs).

The paper's RVEs are weighted Voronoi tessellations built with an external
tool (Sec. 3.1 and Sec. 4.1) and its second phase is a population of stiff
spherical carbides (Sec. 4.4).  Neither the tool nor its RVEs are available,
so the workloads use the plain periodic Voronoi construction below, with the
grain counts, particle fractions and radii of the benchmark configurations.

Conventions
-----------
* Grid of ``n**3`` voxels on the unit cube; voxel ``(a, b, c)`` (0-based) has
  its centre at ``((a+1/2)/n, (b+1/2)/n, (c+1/2)/n)``.  Flattened voxel index
  is ``(a*n + b)*n + c`` (z fastest), the layout used across the C ABI.
* Voronoi: each voxel belongs to the seed at the smallest periodic
  (minimum-image) Euclidean distance from its centre; exact ties go to the
  lowest seed index.
* Orientations: unit quaternions ``(w, x, y, z)`` drawn with Shoemake's
  subgroup algorithm, which is uniform on SO(3).
* Particles: spheres placed one after another with centre uniform in
  ``[0, n)^3`` (voxel units) and radius uniform in ``[rmin, rmax]`` voxels,
  periodic, overlaps allowed.  A voxel is inside when its centre lies within
  the radius.  Placement stops as soon as the particle voxel fraction reaches
  the target; particles override grains.
* Draw order from one ``numpy.random.Generator(PCG64(seed))``: seeds (G x 3),
  orientation uniforms (G x 3), then per particle (centre x 3, radius).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree


def voxel_centres(n: int) -> np.ndarray:
    """Centres of the ``n**3`` voxels of the unit cube, shape (n**3, 3)."""
    t = (np.arange(n, dtype=np.float64) + 0.5) / n
    a, b, c = np.meshgrid(t, t, t, indexing="ij")
    return np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1)


def voronoi_periodic(n: int, seeds: np.ndarray) -> np.ndarray:
    """Label every voxel with its nearest seed on the periodic unit cube.

    ``seeds`` has shape (G, 3) with entries in [0, 1).  Returns int32 labels of
    shape (n**3,) in [0, G).  Exact distance ties go to the lowest seed index.
    """
    seeds = np.asarray(seeds, dtype=np.float64)
    pts = voxel_centres(n)
    G = seeds.shape[0]
    if G == 1:
        return np.zeros(n ** 3, dtype=np.int32)
    tree = cKDTree(np.mod(seeds, 1.0), boxsize=1.0)
    d, idx = tree.query(pts, k=2)
    lab = idx[:, 0].copy()
    tie = d[:, 0] == d[:, 1]
    lab[tie] = np.minimum(idx[tie, 0], idx[tie, 1])
    return lab.astype(np.int32)


def shoemake_quaternions(u: np.ndarray) -> np.ndarray:
    """Uniform random unit quaternions from uniforms ``u`` of shape (G, 3).

    Shoemake (1992), "Uniform random rotations": with u1, u2, u3 ~ U[0,1),
    q = (sqrt(1-u1) sin 2pi u2, sqrt(1-u1) cos 2pi u2,
         sqrt(u1) sin 2pi u3, sqrt(u1) cos 2pi u3).
    Returned in (w, x, y, z) order with w = sqrt(u1) cos 2pi u3.
    """
    u = np.asarray(u, dtype=np.float64)
    u1, u2, u3 = u[:, 0], u[:, 1], u[:, 2]
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    x = a * np.sin(2 * np.pi * u2)
    y = a * np.cos(2 * np.pi * u2)
    z = b * np.sin(2 * np.pi * u3)
    w = b * np.cos(2 * np.pi * u3)
    q = np.stack([w, x, y, z], axis=1)
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def place_particles(rng: np.random.Generator, n: int, target: float,
                    rmin: float = 2.0, rmax: float = 4.0,
                    max_particles: int = 100000):
    """Stiff spherical particles until the voxel fraction reaches ``target``.

    Returns (mask of shape (n**3,), number of spheres, achieved fraction).
    """
    mask = np.zeros((n, n, n), dtype=bool)
    if target <= 0:
        return mask.ravel(), 0, 0.0
    count = 0
    total = n ** 3
    inside = 0
    while inside < target * total and count < max_particles:
        c = rng.random(3) * n
        r = rmin + (rmax - rmin) * rng.random()
        count += 1
        lo = np.floor(c - r - 1).astype(int)
        hi = np.ceil(c + r + 1).astype(int)
        ia = np.arange(lo[0], hi[0] + 1)
        ib = np.arange(lo[1], hi[1] + 1)
        ic = np.arange(lo[2], hi[2] + 1)
        # distance from voxel centres (index + 1/2) to the centre; the box is
        # taken around the centre, so the unwrapped offsets are already the
        # minimum-image ones as long as r < n/2.
        da = (ia + 0.5 - c[0])[:, None, None]
        db = (ib + 0.5 - c[1])[None, :, None]
        dc = (ic + 0.5 - c[2])[None, None, :]
        sel = da * da + db * db + dc * dc <= r * r
        A, B, C = np.nonzero(sel)
        mask[ia[A] % n, ib[B] % n, ic[C] % n] = True
        inside = int(mask.sum())
    return mask.ravel(), count, inside / total


@dataclass
class Microstructure:
    """One RVE: voxel labels plus per-label orientation and law.

    ``phase[v]`` indexes the label tables; labels ``0..grains-1`` are FCC
    grains (law 0) and, when particles are present, label ``grains`` is the
    stiff isotropic particle phase (law 1, identity orientation).
    """
    n: int
    phase: np.ndarray          # int32 (n**3,)
    quat: np.ndarray           # float64 (labels, 4) (w, x, y, z)
    law: np.ndarray            # int32 (labels,) 0 = FCC CP, 1 = isotropic SVK
    grains: int
    particle_fraction: float = 0.0
    particles: int = 0
    seeds: np.ndarray = field(default=None, repr=False)

    @property
    def labels(self) -> int:
        return int(self.quat.shape[0])


def make_microstructure(n: int, grains: int, seed: int,
                        particle_fraction: float = 0.0,
                        rng: np.random.Generator | None = None,
                        rmin: float = 2.0, rmax: float = 4.0) -> Microstructure:
    """Draw one synthetic RVE in the documented draw order."""
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    seeds = rng.random((grains, 3))
    quat = shoemake_quaternions(rng.random((grains, 3)))
    phase = voronoi_periodic(n, seeds)
    law = np.zeros(grains, dtype=np.int32)
    achieved, count = 0.0, 0
    if particle_fraction > 0:
        mask, count, achieved = place_particles(rng, n, particle_fraction,
                                                rmin, rmax)
        phase = phase.copy()
        phase[mask] = grains
        quat = np.concatenate([quat, np.array([[1.0, 0.0, 0.0, 0.0]])], axis=0)
        law = np.concatenate([law, np.array([1], dtype=np.int32)])
    return Microstructure(n=n, phase=phase.astype(np.int32),
                          quat=np.ascontiguousarray(quat), law=law,
                          grains=grains, particle_fraction=achieved,
                          particles=count, seeds=seeds)
