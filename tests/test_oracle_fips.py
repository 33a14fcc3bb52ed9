"""Pins of the non-local fatigue indicators (oracle/fips.py; Sec. 3.3,
Eqs. 25-26), CPU only."""

import numpy as np

from oracle import fips

IDQ = np.array([[1.0, 0.0, 0.0, 0.0]])


def test_grain_average_constant_and_per_grain_fields():
    rng = np.random.default_rng(0)
    n = 6
    phase = rng.integers(0, 5, n ** 3)
    law = np.array([0, 0, 1, 0, 0])          # label 2 is a particle
    m, g, means = fips.pcyc_grain(np.full(n ** 3, 2.5), phase, law)
    assert m == 2.5 and means[2] == 0.0
    f = np.array([1.0, 4.0, 99.0, 3.0, 2.0])
    m, g, means = fips.pcyc_grain(f[phase], phase, law)
    assert m == 4.0 and g == 1
    assert np.array_equal(means, np.where(law == 0, f, 0.0))


def test_grain_average_is_the_mean_and_ignores_empty_labels():
    phase = np.array([0, 0, 0, 2, 2, 0, 2, 0])
    law = np.zeros(3, dtype=np.int64)
    v = np.arange(8.0)
    m, g, means = fips.pcyc_grain(v, phase, law)
    assert means[0] == (0 + 1 + 2 + 5 + 7) / 5 and means[2] == (3 + 4 + 6) / 3
    assert means[1] == 0.0 and m == means[2] and g == 2


def _wrapped(a, n):
    # minimal-image offset (in voxels) from voxel 0 of a cell of n voxels
    return a if a < n // 2 else a - n


def _int_band(k):
    # floor(k / 3 + 1/2) in integer arithmetic
    return (2 * k + 3) // 6


def test_bands_of_a_single_grain_match_enumeration():
    # one grain fills an 8^3 cell, identity orientation; width sqrt(3) h
    # makes s / w = (a' + b' + c') / 3 (plane 0) with a' the wrapped offset
    n, L = 8, (1.0, 1.0, 1.0)
    h = 1.0 / n
    phase = np.zeros(n ** 3, dtype=np.int64)
    bl = fips.bands((n, n, n), L, phase, IDQ, np.array([0]), np.sqrt(3.0) * h)
    signs = [(1, 1, 1), (-1, 1, 1), (1, -1, 1), (1, 1, -1)]
    for p, sg in enumerate(signs):
        ref = {}
        for a in range(n):
            for b in range(n):
                for c in range(n):
                    k = (sg[0] * _wrapped(a, n) + sg[1] * _wrapped(b, n)
                         + sg[2] * _wrapped(c, n))
                    ref.setdefault(_int_band(k), []).append((a * n + b) * n + c)
        got = {j: list(v) for (g, pp, j, v) in bl if pp == p}
        assert got == ref


def test_band_values_of_band_constant_fields_and_off_plane_systems():
    n, L = 8, (1.0, 1.0, 1.0)
    h = 1.0 / n
    phase = np.zeros(n ** 3, dtype=np.int64)
    rng = np.random.default_rng(1)
    W = rng.random((n ** 3, 12))              # arbitrary on planes 1-3
    f = {j: 10.0 + j * j for j in range(-10, 11)}
    for a in range(n):
        for b in range(n):
            for c in range(n):
                j = _int_band(_wrapped(a, n) + _wrapped(b, n) + _wrapped(c, n))
                W[(a * n + b) * n + c, 0:3] = [f[j], 0.5 * f[j], -f[j]]
    mx, bi, vals, bl, syst = fips.wcyc_band(W, (n, n, n), L, phase, IDQ,
                                            np.array([0]), np.sqrt(3.0) * h)
    for v, (g, p, j, vox), s in zip(vals, bl, syst):
        if p == 0:
            assert v == f[j] and s == 0
    W2 = W.copy()
    W2[:, 0:3] = rng.random((n ** 3, 3))      # planes 1-3 bands unchanged
    _, _, vals2, _, _ = fips.wcyc_band(W2, (n, n, n), L, phase, IDQ,
                                       np.array([0]), np.sqrt(3.0) * h)
    plane = np.array([p for (_, p, _, _) in bl])
    assert np.array_equal(vals[plane > 0], vals2[plane > 0])
    assert mx == max(vals) and vals[bi] == mx


def test_relabelling_invariance():
    from synthetic import make_microstructure
    micro = make_microstructure(12, 6, 3)
    rng = np.random.default_rng(2)
    W = rng.random((12 ** 3, 12))
    P = rng.random(12 ** 3)
    law = np.zeros(6, dtype=np.int64)
    perm = rng.permutation(6)
    inv = np.argsort(perm)
    phase2 = perm[micro.phase]                 # label g becomes perm[g]
    quat2 = micro.quat[inv]
    a = fips.wcyc_band(W, (12,) * 3, (1, 1, 1), micro.phase, micro.quat, law, 0.1)
    b = fips.wcyc_band(W, (12,) * 3, (1, 1, 1), phase2, quat2, law, 0.1)
    assert a[0] == b[0]
    assert np.array_equal(np.sort(a[2]), np.sort(b[2]))
    pa = fips.pcyc_grain(P, micro.phase, law)
    pb = fips.pcyc_grain(P, phase2, law)
    assert pa[0] == pb[0] and pb[1] == perm[pa[1]]


def test_wide_bands_reduce_to_grain_averages():
    # a width wider than any grain puts a whole grain in band 0 of every
    # plane: band value = max over the plane's systems of the grain mean
    from synthetic import make_microstructure
    micro = make_microstructure(12, 5, 4)
    rng = np.random.default_rng(5)
    W = rng.random((12 ** 3, 12))
    law = np.zeros(5, dtype=np.int64)
    _, _, vals, bl, _ = fips.wcyc_band(W, (12,) * 3, (1, 1, 1), micro.phase,
                                       micro.quat, law, 10.0)
    assert len(bl) == 4 * 5
    for v, (g, p, j, vox) in zip(vals, bl):
        assert j == 0
        gm = [fips.grain_means(W[:, 3 * p + k], micro.phase, law)[0][g]
              for k in range(3)]
        assert np.isclose(v, max(gm), rtol=1e-14)
