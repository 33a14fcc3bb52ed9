"""Helpers shared by the GPU tests (not collected by pytest)."""

import numpy as np

from synthetic import material_params


def make_rve(micro, operator="discrete", precision="fp64", **kw):
    from paper_1806_10599_amd.binding import Rve
    r = Rve(micro.n, projection=operator, precision=precision, **kw)
    r.set_microstructure(micro.phase, micro.quat, micro.law, material_params())
    return r


def oracle_for(micro, operator):
    from oracle.solver import OracleRVE
    return OracleRVE((micro.n,) * 3, micro.phase, micro.quat, micro.law,
                     material_params(), operator)


def to_soa(A):
    """(N,3,3) voxel-major -> (9, N)."""
    return np.ascontiguousarray(A.reshape(A.shape[0], 9).T)


def rel_maxnorm(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
