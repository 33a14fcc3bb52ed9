"""Non-local fatigue indicator parameters (oracle; test infrastructure).

Sec. 3.3 of the paper, Eqs. 25-26: the local indicators P_cyc (Eq. 23) and
W_cyc^a (Eq. 24) are averaged over an integration volume and the largest
average in the RVE represents it.

* Eq. 25: the volume of a grain; P_cyc^g = max over grains of the grain
  average of P_cyc.
* Eq. 26: bands of a given width inside each grain, parallel to one of its
  slip planes; for a band the value is the largest, over the slip systems of
  that plane, of the band average of W_cyc^a; W_cyc^b = max over bands.

Readings (the paper gives neither the band width nor the band origin):

* A grain is a microstructure label of the crystal law; labels of the
  second phase and labels without voxels have no average (reported as 0 and
  left out of the maxima).  Every voxel has the same volume, so a volume
  average is a plain mean over the grain's voxels.
* Voxel (a, b, c) has its centre at ((a + 1/2) L0/n0, (b + 1/2) L1/n1,
  (c + 1/2) L2/n2).  The reference point of a grain is the centre of its
  voxel of lowest linear index; a voxel's offset d from it is taken as the
  periodic minimal image, d <- d - L floor(d / L + 1/2) per axis (grains are
  assumed to span less than half the cell along each axis).
* Band coordinate along plane p: s = (d0 n0 + d1 n1) + d2 n2 with n the
  sample-frame unit normal of the plane (the normal of the plane's first
  slip system); band index j = floor(s / w + 1/2), so band 0 is centred on
  the reference point.  The decisions are taken in FP64 in this operation
  order.
* Slip systems 3p, 3p+1, 3p+2 lie on plane p (the order of the crystal
  geometry module).

Pins (tests/test_oracle_fips.py): constant and per-grain-constant fields;
fields constant on bands by construction (band averages exact); systems off
the plane not seen by its bands; band count and band membership of a
single grain of identity orientation by explicit enumeration; relabelling
invariance; a grain across the periodic boundary equal to its shifted copy.
Status: pinned.
"""

from __future__ import annotations

import numpy as np

from . import crystal


def grain_means(field, phase, law):
    """Per-label mean of a voxel field; 0 for particle and empty labels.
    Returns (means (G,), counts (G,), crystal mask (G,))."""
    phase = np.asarray(phase).reshape(-1)
    law = np.asarray(law)
    G = law.size
    means = np.zeros(G)
    counts = np.zeros(G, dtype=np.int64)
    for g in range(G):
        sel = phase == g
        counts[g] = int(np.count_nonzero(sel))
        if counts[g] and law[g] == 0:
            means[g] = float(np.mean(field[sel]))
    return means, counts, (law == 0) & (counts > 0)


def pcyc_grain(pcyc, phase, law):
    """Eq. 25: (max, label of the max, per-label means)."""
    means, counts, ok = grain_means(pcyc, phase, law)
    if not ok.any():
        return 0.0, -1, means
    idx = np.nonzero(ok)[0]
    best = idx[np.argmax(means[idx])]        # first of equal maxima
    return float(means[best]), int(best), means


def plane_normals(quat):
    """(G, 4, 3) sample-frame unit normals of the four slip planes."""
    _, m = crystal.fcc_slip_systems()
    out = np.zeros((len(quat), 4, 3))
    for g, q in enumerate(quat):
        R = crystal.quat_to_matrix(q)
        for p in range(4):
            mp = m[3 * p]
            for i in range(3):
                out[g, p, i] = (R[i, 0] * mp[0] + R[i, 1] * mp[1]) + R[i, 2] * mp[2]
    return out


def voxel_centres(shape, L):
    """(N, 3) voxel centres, voxel index (a*n1 + b)*n2 + c."""
    n0, n1, n2 = shape
    a, b, c = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2),
                          indexing="ij")
    x = np.stack([(a + 0.5) * (L[0] / n0), (b + 0.5) * (L[1] / n1),
                  (c + 0.5) * (L[2] / n2)], axis=-1)
    return x.reshape(-1, 3)


def bands(shape, L, phase, quat, law, width):
    """List of bands (label, plane, j, voxel indices ascending), sorted by
    (label, plane, j)."""
    phase = np.asarray(phase).reshape(-1)
    x = voxel_centres(shape, L)
    normals = plane_normals(quat)
    out = []
    for g in range(len(law)):
        if law[g] != 0:
            continue
        vox = np.nonzero(phase == g)[0]
        if vox.size == 0:
            continue
        d = x[vox] - x[vox[0]]
        for a in range(3):
            d[:, a] = d[:, a] - L[a] * np.floor(d[:, a] / L[a] + 0.5)
        for p in range(4):
            n = normals[g, p]
            s = (d[:, 0] * n[0] + d[:, 1] * n[1]) + d[:, 2] * n[2]
            j = np.floor(s / width + 0.5).astype(np.int64)
            for jj in np.unique(j):
                out.append((g, p, int(jj), vox[j == jj]))
    return out


def band_values(wcyc, band_list):
    """Per band: max over the plane's three systems of the band mean of
    W_cyc (wcyc: (N, 12)); also the system attaining it."""
    vals = np.zeros(len(band_list))
    syst = np.zeros(len(band_list), dtype=np.int64)
    for b, (g, p, j, vox) in enumerate(band_list):
        m = [float(np.mean(wcyc[vox, 3 * p + k])) for k in range(3)]
        k = int(np.argmax(m))
        vals[b] = m[k]
        syst[b] = 3 * p + k
    return vals, syst


def wcyc_band(wcyc, shape, L, phase, quat, law, width):
    """Eq. 26: (max, index of the band of the max, band values, band list,
    system of each band's value)."""
    bl = bands(shape, L, phase, quat, law, width)
    vals, syst = band_values(wcyc, bl)
    if not bl:
        return 0.0, -1, vals, bl, syst
    b = int(np.argmax(vals))
    return float(vals[b]), b, vals, bl, syst
