"""ctypes binding of the C ABI in include/rve.h (argument marshalling only).

Every step of the solver runs in the HIP library; this module only converts
Python/NumPy arguments to the C structs and pointers.  PyTorch provides the
device memory (its caching allocator, through the ABI's allocator hooks) and
the HIP stream.  Importing fails loudly when the built library is missing:
there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libpaper_1806_10599_amd.so")

RVE_OK, RVE_EINVAL, RVE_ENOMEM, RVE_EDEVICE = 0, -1, -2, -3
RVE_ENOTCONV, RVE_ELOCAL, RVE_ESTATE = -4, -5, -6
STATUS_NAMES = {0: "RVE_OK", -1: "RVE_EINVAL", -2: "RVE_ENOMEM",
                -3: "RVE_EDEVICE", -4: "RVE_ENOTCONV", -5: "RVE_ELOCAL",
                -6: "RVE_ESTATE"}
PROJ = {"continuous": 0, "discrete": 1}
PREC = {"fp64": 0, "mixed": 1}
FIELDS = {"F": (0, 9), "P": (1, 9), "sigma": (2, 9), "Fpinv": (3, 9),
          "chi": (4, 12), "dgamma": (5, 12), "pcyc": (6, 1),
          "pcyc_lit": (7, 1), "wcyc": (8, 12), "statev": (9, None)}
NPARAMS = 10
MAX_NEWTON_LOG = 64
KERNEL_CLASSES = ("matvec_pass_a", "matvec_pass_b", "matvec_pass_c",
                  "cg_update", "return_map", "tangent", "residual_fp64",
                  "matvec_kp")

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
# user material (Appendix A form): (user, F1, F0, statev_old, statev_new,
# nstatev, sigma, ddsdde, fails, n, dt, stream) -> 0 when enqueued
UMAT_FN = C.CFUNCTYPE(C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                      C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                      C.c_void_p, C.c_void_p, C.c_int64, C.c_double,
                      C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class RveConfig(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("L", C.c_double * 3),
                ("projection", C.c_int32), ("precision", C.c_int32),
                ("warm_start", C.c_int32), ("use_graph", C.c_int32),
                ("newton_tol", C.c_double), ("newton_max_iter", C.c_int32),
                ("cg_tol", C.c_double), ("cg_max_iter", C.c_int32),
                ("cg_chunk", C.c_int32), ("stream", C.c_void_p),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN),
                ("alloc_ctx", C.c_void_p), ("cg_forcing", C.c_int32)]


class RveIncrementInfo(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("cg_iters_total", C.c_int32),
                ("local_failures", C.c_int32), ("used_learned", C.c_int32),
                ("cg_breakdowns", C.c_int32), ("status", C.c_int32),
                ("residual_rel", C.c_double),
                ("predictor_residual", C.c_double),
                ("plain_predictor_residual", C.c_double),
                ("P_bar", C.c_double * 9), ("sigma_bar", C.c_double * 9),
                ("residual_history", C.c_double * MAX_NEWTON_LOG),
                ("cg_iters", C.c_int32 * MAX_NEWTON_LOG),
                ("seconds", C.c_double)]


class RveNonlocalFips(C.Structure):
    _fields_ = [("band_width", C.c_double), ("grains", C.c_int32),
                ("pcyc_label", C.c_int32), ("pcyc_g", C.c_double),
                ("pcyc_lit_g", C.c_double), ("pcyc_lit_label", C.c_int32),
                ("wcyc_label", C.c_int32), ("bands", C.c_int64),
                ("wcyc_b", C.c_double), ("wcyc_band", C.c_int64),
                ("wcyc_plane", C.c_int32), ("wcyc_j", C.c_int32),
                ("wcyc_system", C.c_int32), ("wcyc_voxels", C.c_int32)]


class RveAdaptiveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("substeps", C.c_int32),
                ("cutbacks", C.c_int32), ("newton_iters_total", C.c_int32),
                ("cg_iters_total", C.c_int32), ("pad", C.c_int32),
                ("min_fraction", C.c_double), ("seconds", C.c_double),
                ("last", RveIncrementInfo)]


class RveWsConfig(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("dev_alloc", ALLOC_FN),
                ("dev_free", FREE_FN), ("alloc_ctx", C.c_void_p)]


def _load():
    if not os.path.exists(LIBPATH):
        raise ImportError(
            f"{LIBPATH} is missing: build it with "
            "`python -m paper_1806_10599_amd.build` (there is no CPU fallback)")
    lib = C.CDLL(LIBPATH)
    P = C.POINTER
    sig = {
        "rve_config_default": (C.c_int, [P(RveConfig)]),
        "rve_create": (C.c_int, [P(RveConfig), P(C.c_void_p)]),
        "rve_destroy": (C.c_int, [C.c_void_p]),
        "rve_set_microstructure": (C.c_int, [C.c_void_p, P(C.c_int32),
                                             C.c_int32, P(C.c_double),
                                             P(C.c_int32), P(C.c_double),
                                             C.c_int32]),
        "rve_apply_macro_strain_increment": (
            C.c_int, [C.c_void_p, P(C.c_double), C.c_double,
                      P(RveIncrementInfo)]),
        "rve_apply_macro_strain_increment_adaptive": (
            C.c_int, [C.c_void_p, P(C.c_double), C.c_double, C.c_int32,
                      C.c_int32, P(RveAdaptiveInfo)]),
        "rve_reset_fips": (C.c_int, [C.c_void_p]),
        "rve_get_fields": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p,
                                     C.c_size_t, C.c_int32]),
        "rve_get_macro": (C.c_int, [C.c_void_p, P(C.c_double)]),
        "rve_get_nonlocal_fips": (C.c_int, [C.c_void_p, C.c_double,
                                            P(RveNonlocalFips), C.c_void_p,
                                            C.c_void_p, C.c_int32,
                                            C.c_void_p, C.c_void_p,
                                            C.c_int64]),
        "rve_fip_band_lists": (C.c_int, [C.c_int32, P(C.c_double),
                                         P(C.c_int32), C.c_int32,
                                         P(C.c_double), P(C.c_int32),
                                         C.c_double, P(C.c_int64),
                                         P(C.c_int64), C.c_void_p,
                                         C.c_void_p, C.c_int64, C.c_int64]),
        "rve_batch_get_nonlocal_fips": (C.c_int, [C.c_void_p, C.c_int32,
                                                  C.c_double,
                                                  P(RveNonlocalFips),
                                                  C.c_void_p, C.c_void_p,
                                                  C.c_int32, C.c_void_p,
                                                  C.c_void_p, C.c_int64]),
        "rve_state_size": (C.c_int, [C.c_void_p, P(C.c_size_t)]),
        "rve_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
        "rve_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
        "rve_last_error": (C.c_char_p, [C.c_void_p]),
        "rve_debug_apply_G": (C.c_int, [C.c_void_p, P(C.c_double),
                                        P(C.c_double), C.c_int32]),
        "rve_debug_constitutive": (C.c_int, [C.c_void_p, P(C.c_double),
                                             C.c_double, P(C.c_double),
                                             P(C.c_double), P(C.c_double),
                                             P(C.c_int32)]),
        "rve_debug_set_field": (C.c_int, [C.c_void_p, C.c_int32,
                                          P(C.c_double), C.c_size_t]),
        "rve_bench_kernels": (C.c_int, [C.c_void_p, C.c_int32,
                                        P(C.c_double), C.c_int32]),
        "rve_set_kernel_timing": (C.c_int, [C.c_void_p, C.c_uint32]),
        "rve_set_kernel_timing_stride": (C.c_int, [C.c_void_p, C.c_int32]),
        "rve_get_kernel_launches": (C.c_int, [C.c_void_p, P(C.c_int64),
                                              C.c_int32, C.c_int32]),
        "rve_get_kernel_timing": (C.c_int, [C.c_void_p, P(C.c_double),
                                            P(C.c_int64), C.c_int32,
                                            C.c_int32]),
        "rve_get_return_map_counts": (C.c_int, [C.c_void_p, P(C.c_int64),
                                                C.c_int32]),
        "rve_set_fft_schedule": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32,
                                           C.c_int32]),
        "rve_get_fft_schedule": (C.c_int, [C.c_void_p, P(C.c_int32),
                                           P(C.c_double)]),
        "rve_ws_create": (C.c_int, [P(RveWsConfig), P(C.c_void_p)]),
        "rve_ws_destroy": (C.c_int, [C.c_void_p]),
        "rve_ws_param_count": (C.c_int, [C.c_void_p, P(C.c_int64)]),
        "rve_ws_set_params": (C.c_int, [C.c_void_p, P(C.c_float), C.c_int64]),
        "rve_ws_get_params": (C.c_int, [C.c_void_p, P(C.c_float), C.c_int64]),
        "rve_ws_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32,
                                     C.c_void_p]),
        "rve_ws_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_int32, C.c_float, P(C.c_double),
                                        P(C.c_float)]),
        "rve_ws_loss": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_int32, P(C.c_double)]),
        "rve_ws_last_error": (C.c_char_p, [C.c_void_p]),
        "rve_attach_warm_start": (C.c_int, [C.c_void_p, C.c_void_p]),
        "rve_ws_features": (C.c_int, [C.c_void_p, P(C.c_double), C.c_void_p]),
        "rve_ws_target": (C.c_int, [C.c_void_p, C.c_void_p]),
        "rve_set_user_material": (C.c_int, [C.c_void_p, UMAT_FN, C.c_void_p,
                                            C.c_int32, P(C.c_double)]),
        "rve_umat_neo_hooke": (C.c_int32, [C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_int32,
                                           C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_int64,
                                           C.c_double, C.c_void_p]),
        "rve_umat_bridge": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_int64, C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
        "rve_batch_create": (C.c_int, [P(RveConfig), C.c_int32, P(C.c_int32),
                                       P(C.c_void_p)]),
        "rve_batch_destroy": (C.c_int, [C.c_void_p]),
        "rve_batch_set_microstructure": (
            C.c_int, [C.c_void_p, C.c_int32, P(C.c_int32), C.c_int32,
                      P(C.c_double), P(C.c_int32), P(C.c_double), C.c_int32]),
        "rve_batch_apply_macro_strain_increment": (
            C.c_int, [C.c_void_p, P(C.c_double), C.c_double,
                      P(RveIncrementInfo)]),
        "rve_batch_reset_fips": (C.c_int, [C.c_void_p]),
        "rve_batch_get_fields": (C.c_int, [C.c_void_p, C.c_int32, C.c_uint32,
                                           C.c_void_p, C.c_size_t, C.c_int32]),
        "rve_batch_debug_apply_G": (C.c_int, [C.c_void_p, P(C.c_double),
                                              P(C.c_double)]),
        "rve_tune_fft_schedule": (C.c_int, [C.c_void_p]),
        "rve_batch_tune_fft_schedule": (C.c_int, [C.c_void_p]),
        "rve_batch_set_fft_schedule": (C.c_int, [C.c_void_p, C.c_int32,
                                                 C.c_int32, C.c_int32]),
        "rve_batch_get_fft_schedule": (C.c_int, [C.c_void_p, C.c_int32,
                                                 P(C.c_int32), P(C.c_double)]),
        "rve_apply_G_noalloc": (C.c_int, [C.c_int32, P(C.c_double), C.c_int32,
                                          C.c_void_p, C.c_void_p,
                                          C.c_void_p]),
        "rve_batch_get_macro": (C.c_int, [C.c_void_p, C.c_int32,
                                          P(C.c_double)]),
        "rve_batch_last_error": (C.c_char_p, [C.c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()
# the example user material of the library, as a function pointer
NEO_HOOKE_UMAT = UMAT_FN(("rve_umat_neo_hooke", LIB))


class RveError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _info_dict(info, rc):
    k = info.newton_iters
    nlog = min(k + 1, MAX_NEWTON_LOG)
    return dict(status=rc, newton_iters=k,
                cg_iters_total=info.cg_iters_total,
                cg_iters=list(info.cg_iters[:min(k, MAX_NEWTON_LOG)]),
                residuals=list(info.residual_history[:nlog]),
                local_failures=info.local_failures,
                used_learned=info.used_learned,
                cg_breakdowns=info.cg_breakdowns,
                residual_rel=info.residual_rel,
                predictor_residual=info.predictor_residual,
                plain_predictor_residual=info.plain_predictor_residual,
                P_bar=np.array(info.P_bar).reshape(3, 3),
                sigma_bar=np.array(info.sigma_bar).reshape(3, 3),
                seconds=info.seconds)


def _nonlocal_fips(call, labels, band_width, arrays):
    """Runs a get_nonlocal_fips entry point (``call(width, out, gp, gpl,
    labels, bw, bd, cap)`` returning a status) and converts the result."""
    out = RveNonlocalFips()
    call(band_width, C.byref(out), None, None, 0, None, None, 0)
    res = {k: getattr(out, k) for k, _ in RveNonlocalFips._fields_}
    if arrays:
        gp = np.zeros(labels)
        gpl = np.zeros(labels)
        nb = out.bands
        bw = np.zeros(max(nb, 1))
        bd = np.zeros((max(nb, 1), 5), dtype=np.int32)
        call(band_width, C.byref(out), _dptr(gp), _dptr(gpl), labels,
             _dptr(bw), bd.ctypes.data_as(C.c_void_p), nb)
        res.update(grain_pcyc=gp, grain_pcyc_lit=gpl, band_wcyc=bw[:nb],
                   band_desc=bd[:nb])
    return res


def fip_band_lists(n, phase, quat, law, band_width, L=(1.0, 1.0, 1.0)):
    """The slip bands of Eq. 26 as the library builds them (host code, no
    GPU needed): a list of (label, plane, j, voxel indices) in (label,
    plane, j) order."""
    phase = np.ascontiguousarray(phase, dtype=np.int32).reshape(-1)
    quat = np.ascontiguousarray(quat, dtype=np.float64).reshape(-1, 4)
    law = np.ascontiguousarray(law, dtype=np.int32).reshape(-1)
    Lc = np.ascontiguousarray(L, dtype=np.float64)
    nb, ne = C.c_int64(), C.c_int64()
    args = (int(n), _dptr(Lc), _iptr(phase), quat.shape[0], _dptr(quat),
            _iptr(law), float(band_width))
    rc = LIB.rve_fip_band_lists(*args, C.byref(nb), C.byref(ne), None, None,
                                0, 0)
    if rc != RVE_OK:
        raise RveError(rc, LIB.rve_last_error(None).decode())
    desc = np.zeros((max(nb.value, 1), 4), dtype=np.int32)
    vox = np.zeros(max(ne.value, 1), dtype=np.int32)
    rc = LIB.rve_fip_band_lists(*args, C.byref(nb), C.byref(ne),
                                desc.ctypes.data_as(C.c_void_p),
                                vox.ctypes.data_as(C.c_void_p), nb.value,
                                ne.value)
    if rc != RVE_OK:
        raise RveError(rc, LIB.rve_last_error(None).decode())
    out, e = [], 0
    for g, p, j, cnt in desc[:nb.value]:
        out.append((int(g), int(p), int(j), vox[e:e + cnt].copy()))
        e += cnt
    return out


def _make_config(L, projection, precision, newton_tol, newton_max_iter, cg_tol,
                 cg_max_iter, cg_chunk, use_graph, warm_start, stream, device,
                 torch_allocator, cg_forcing=False):
    cfg = RveConfig()
    LIB.rve_config_default(C.byref(cfg))
    cfg.L[:] = tuple(float(x) for x in L)
    cfg.projection = PROJ[projection]
    cfg.precision = PREC[precision]
    cfg.newton_tol = newton_tol
    cfg.newton_max_iter = newton_max_iter
    cfg.cg_tol = cg_tol
    cfg.cg_max_iter = cg_max_iter
    cfg.cg_chunk = cg_chunk
    cfg.use_graph = 1 if use_graph else 0
    if warm_start not in (0, 1, 2, 3):
        raise ValueError("warm_start must be False/0, True/1, 2 or 3 "
                         "(extrapolation)")
    cfg.warm_start = int(warm_start)
    if cg_forcing not in (0, 1, 2):
        raise ValueError("cg_forcing must be False/0, True/1 or 2")
    cfg.cg_forcing = int(cg_forcing)
    torch.cuda.set_device(device)
    stream = stream if stream is not None else torch.cuda.current_stream()
    cfg.stream = C.c_void_p(stream.cuda_stream or None)
    alloc = None
    if torch_allocator:
        alloc = _TorchAllocator(device)
        cfg.dev_alloc = alloc.alloc_fn
        cfg.dev_free = alloc.free_fn
    return cfg, stream, alloc


class _TorchAllocator:
    """Allocator hooks that draw device memory from torch's caching allocator."""

    def __init__(self, device):
        self.device = device

        def alloc(size, stream, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(
                    int(size), self.device, stream or 0)
            except Exception:  # out of memory -> NULL -> RVE_ENOMEM
                return None

        def free(ptr, ctx):
            torch.cuda.caching_allocator_delete(ptr)

        self.alloc_fn = ALLOC_FN(alloc)
        self.free_fn = FREE_FN(free)


class Rve:
    """One periodic RVE on the GPU (a handle of the C ABI)."""

    def __init__(self, n, L=(1.0, 1.0, 1.0), projection="discrete",
                 precision="fp64", newton_tol=1e-6, newton_max_iter=25,
                 cg_tol=1e-4, cg_max_iter=2000, cg_chunk=8, use_graph=False,
                 warm_start=False, stream=None, device=0,
                 torch_allocator=True, cg_forcing=False):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the library runs on the GPU only")
        self._lib = LIB
        self._h = None
        cfg, self.stream, self._alloc = _make_config(
            L, projection, precision, newton_tol, newton_max_iter, cg_tol,
            cg_max_iter, cg_chunk, use_graph, warm_start, stream, device,
            torch_allocator, cg_forcing)
        nn = (n, n, n) if np.isscalar(n) else tuple(n)
        cfg.n[:] = nn
        self.cfg = cfg
        self.n = nn[0]
        self.N = nn[0] * nn[1] * nn[2]
        h = C.c_void_p()
        rc = LIB.rve_create(C.byref(cfg), C.byref(h))
        if rc != RVE_OK:
            raise RveError(rc, LIB.rve_last_error(None).decode())
        self._h = h

    # ------------------------------------------------------------ lifecycle
    def close(self):
        if self._h is not None:
            self._lib.rve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc, ok=(RVE_OK,)):
        if rc not in ok:
            raise RveError(rc, self._lib.rve_last_error(self._h).decode())
        return rc

    # ------------------------------------------------------------- calls
    def set_microstructure(self, phase, quat, law, params):
        phase = np.ascontiguousarray(phase, dtype=np.int32).reshape(-1)
        quat = np.ascontiguousarray(quat, dtype=np.float64).reshape(-1, 4)
        law = np.ascontiguousarray(law, dtype=np.int32).reshape(-1)
        params = np.ascontiguousarray(params, dtype=np.float64).reshape(-1)
        if phase.size != self.N:
            raise ValueError("phase must have n^3 entries")
        self._check(LIB.rve_set_microstructure(
            self._h, _iptr(phase), quat.shape[0], _dptr(quat), _iptr(law),
            _dptr(params), params.size))
        self._nsv = 0
        self._labels = quat.shape[0]

    def set_user_material(self, material, statev0=None, user=None):
        """Use a user material of the Appendix A form for every voxel.

        ``material``: "neo_hooke" (the library's example material, whose
        state variables are mu, lambda and the accumulated |dJ|), a
        ``UMAT_FN`` function pointer, or a Python callable with the
        ``UMAT_FN`` arguments (device pointers as integers) that enqueues its
        work on the given stream.  ``statev0``: (nstatev, N) initial state
        variables."""
        if isinstance(material, str):
            if material != "neo_hooke":
                raise ValueError(f"unknown built-in user material {material!r}")
            fn = NEO_HOOKE_UMAT
        elif isinstance(material, UMAT_FN):
            fn = material
        elif callable(material):
            fn = UMAT_FN(material)
        else:
            raise TypeError("material must be a name, a UMAT_FN or a callable")
        if statev0 is None:
            sv = np.zeros((0, self.N))
        else:
            sv = np.ascontiguousarray(statev0, dtype=np.float64)
            if sv.ndim != 2 or sv.shape[1] != self.N:
                raise ValueError("statev0 must have shape (nstatev, N)")
        self._check(LIB.rve_set_user_material(
            self._h, fn, C.c_void_p(user), sv.shape[0],
            _dptr(sv) if sv.size else None))
        self._umat = fn          # keep the callback alive
        self._nsv = sv.shape[0]

    def increment(self, F_bar, dt):
        """One load increment; returns a dict (status included, no raise on
        ENOTCONV / ELOCAL, which leave the committed state unchanged)."""
        Fb = np.ascontiguousarray(F_bar, dtype=np.float64).reshape(9)
        info = RveIncrementInfo()
        rc = LIB.rve_apply_macro_strain_increment(self._h, _dptr(Fb),
                                                  float(dt), C.byref(info))
        self._check(rc, ok=(RVE_OK, RVE_ENOTCONV, RVE_ELOCAL))
        return _info_dict(info, rc)

    def increment_adaptive(self, F_bar, dt, max_cutbacks=6, grow_after=2):
        """A load step with automatic time incrementation (cutbacks on
        ENOTCONV / ELOCAL); returns a dict (status included)."""
        Fb = np.ascontiguousarray(F_bar, dtype=np.float64).reshape(9)
        info = RveAdaptiveInfo()
        rc = LIB.rve_apply_macro_strain_increment_adaptive(
            self._h, _dptr(Fb), float(dt), int(max_cutbacks), int(grow_after),
            C.byref(info))
        self._check(rc, ok=(RVE_OK, RVE_ENOTCONV, RVE_ELOCAL))
        return dict(status=rc, substeps=info.substeps, cutbacks=info.cutbacks,
                    newton_iters_total=info.newton_iters_total,
                    cg_iters_total=info.cg_iters_total,
                    min_fraction=info.min_fraction, seconds=info.seconds,
                    last=_info_dict(info.last, info.last.status))

    def reset_fips(self):
        self._check(LIB.rve_reset_fips(self._h))

    def field(self, name):
        return self.fields(name)[name]

    def fields(self, *names):
        """Several committed fields in one rve_get_fields call (bit mask of
        their ids); returns {name: array}, one component per row."""
        order = sorted(set(names), key=lambda k: FIELDS[k][0])
        comps = [FIELDS[k][1] if FIELDS[k][1] is not None
                 else getattr(self, "_nsv", 0) for k in order]
        out = np.empty((sum(comps), self.N), dtype=np.float64)
        mask = 0
        for k in order:
            mask |= 1 << FIELDS[k][0]
        self._check(LIB.rve_get_fields(self._h, mask, out.ctypes.data_as(
            C.c_void_p), out.nbytes, 0))
        res, row = {}, 0
        for k, c in zip(order, comps):
            blk = out[row:row + c]
            res[k] = blk[0].copy() if FIELDS[k][1] == 1 else blk.copy()
            row += c
        return res

    def field_device(self, name, out):
        """Copy a field into a torch tensor on the GPU (float64, contiguous)."""
        fid, comps = FIELDS[name]
        assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
        self._check(LIB.rve_get_fields(self._h, 1 << fid,
                                       C.c_void_p(out.data_ptr()),
                                       out.numel() * 8, 1))
        return out

    def macro(self):
        out = np.empty(29)
        self._check(LIB.rve_get_macro(self._h, _dptr(out)))
        return dict(F_bar=out[:9].reshape(3, 3), P_bar=out[9:18].reshape(3, 3),
                    sigma_bar=out[18:27].reshape(3, 3), t=out[27],
                    increments=int(out[28]))

    def nonlocal_fips(self, band_width=None, arrays=True):
        """Eqs. 25-26 on the committed indicator fields; band_width defaults
        to two voxel edges (along the first axis)."""
        w = 2.0 * self.cfg.L[0] / self.n if band_width is None else band_width

        def call(*a):
            self._check(LIB.rve_get_nonlocal_fips(self._h, *a))
        return _nonlocal_fips(call, getattr(self, "_labels", 0), float(w), arrays)

    def get_state(self) -> bytes:
        sz = C.c_size_t()
        self._check(LIB.rve_state_size(self._h, C.byref(sz)))
        buf = C.create_string_buffer(sz.value)
        self._check(LIB.rve_get_state(self._h, buf, sz.value))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(LIB.rve_set_state(self._h, buf, len(blob)))

    # --------------------------------------------------------------- hooks
    def debug_apply_G(self, A, precision="fp64"):
        A = np.ascontiguousarray(A, dtype=np.float64).reshape(9, self.N)
        out = np.empty_like(A)
        self._check(LIB.rve_debug_apply_G(self._h, _dptr(A), _dptr(out),
                                          PREC[precision]))
        return out

    def debug_constitutive(self, F, dt, tangent=True):
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(9, self.N)
        P = np.empty((9, self.N))
        dg = np.empty((12, self.N))
        K = np.empty((81, self.N)) if tangent else None
        fails = C.c_int32()
        self._check(LIB.rve_debug_constitutive(
            self._h, _dptr(F), float(dt), _dptr(P),
            _dptr(K) if tangent else None, _dptr(dg), C.byref(fails)))
        return dict(P=P, K=K, dg=dg, fails=fails.value)

    def debug_set_field(self, name, values):
        fid, comps = FIELDS[name]
        v = np.ascontiguousarray(values, dtype=np.float64).reshape(comps, self.N)
        self._check(LIB.rve_debug_set_field(self._h, fid, _dptr(v), v.nbytes))

    def bench_kernels(self, reps=20):
        """Average ms per launch of the hot-path kernels (see rve.h)."""
        out = np.zeros(len(KERNEL_CLASSES))
        self._check(LIB.rve_bench_kernels(self._h, int(reps), _dptr(out),
                                          len(KERNEL_CLASSES)))
        return dict(zip(KERNEL_CLASSES, out.tolist()))

    # --------------------------------------------------- learned warm start
    def set_kernel_timing(self, classes, cg_stride=1):
        """Time the given kernel classes live (names of KERNEL_CLASSES);
        the CG-iteration classes one launch in every cg_stride."""
        mask = 0
        for c in classes:
            mask |= 1 << KERNEL_CLASSES.index(c)
        self._check(LIB.rve_set_kernel_timing_stride(self._h, int(cg_stride)))
        self._check(LIB.rve_set_kernel_timing(self._h, mask))

    def kernel_timing(self, reset=False):
        """{class: (total ms, launches)} since the last reset."""
        n = len(KERNEL_CLASSES)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        self._check(LIB.rve_get_kernel_timing(self._h, ms, cnt, n,
                                              1 if reset else 0))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_CLASSES)}

    def kernel_launches(self, reset=False):
        """{class: every launch since the last reset, timed or skipped by the
        CG stride} for the timed classes."""
        n = len(KERNEL_CLASSES)
        cnt = (C.c_int64 * n)()
        self._check(LIB.rve_get_kernel_launches(self._h, cnt, n,
                                                1 if reset else 0))
        return {k: cnt[i] for i, k in enumerate(KERNEL_CLASSES)}

    def return_map_counts(self, reset=False):
        """Local Newton steps, residual evaluations, crystal and particle
        voxel visits of the return mappings timed live."""
        out = (C.c_int64 * 4)()
        self._check(LIB.rve_get_return_map_counts(self._h, out,
                                                  1 if reset else 0))
        return dict(steps=out[0], evals=out[1], crystal=out[2],
                    particle=out[3])

    def set_fft_schedule(self, cpb=0, tt=0, fused=0):
        """Force the CG-matvec schedule (fused: the direction step and K:p
        inside the first transform pass); (0, 0) tunes it again."""
        self._check(LIB.rve_set_fft_schedule(self._h, int(cpb), int(tt),
                                             int(fused)))

    def tune_fft_schedule(self):
        """Tune the CG-matvec schedule now (outside a timed run)."""
        self._check(LIB.rve_tune_fft_schedule(self._h))

    def fft_schedule(self):
        out = (C.c_int32 * 3)()
        ms = C.c_double()
        self._check(LIB.rve_get_fft_schedule(self._h, out, C.byref(ms)))
        return dict(cpb=out[0], tt=out[1], fused=out[2], tuned_ms=ms.value)

    def attach_warm_start(self, net):
        self._check(LIB.rve_attach_warm_start(self._h, net._h if net else None))
        self._net = net

    def features(self, F_bar_new, out=None):
        """Network input for the increment to F_bar_new (bf16 as int16 tensor
        [N][48] on the GPU)."""
        Fb = np.ascontiguousarray(F_bar_new, dtype=np.float64).reshape(9)
        if out is None:
            out = torch.empty((self.N, WS_FEAT), dtype=torch.int16,
                              device="cuda")
        self._check(LIB.rve_ws_features(self._h, _dptr(Fb),
                                        C.c_void_p(out.data_ptr())))
        return out

    def target(self, out=None):
        """Target of the last committed increment ([N][16] float32, GPU)."""
        if out is None:
            out = torch.empty((self.N, WS_OUT), dtype=torch.float32,
                              device="cuda")
        self._check(LIB.rve_ws_target(self._h, C.c_void_p(out.data_ptr())))
        return out


WS_FEAT = 48
WS_OUT = 16


def umat_bridge(F, sigma, ddsdde, stream=None):
    """Appendix A: P and K from the Cauchy stress and the Jaumann-rate tangent
    of a commercial-FE-style user material.  Inputs: float64 CUDA tensors of
    shapes (9, n), (6, n), (36, n); returns P (9, n) and K (81, n)."""
    for t, rows in ((F, 9), (sigma, 6), (ddsdde, 36)):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.dim() == 2 and t.shape[0] == rows):
            raise ValueError("expected contiguous float64 CUDA tensors of "
                             "shapes (9, n), (6, n), (36, n)")
    n = F.shape[1]
    if sigma.shape[1] != n or ddsdde.shape[1] != n:
        raise ValueError("inconsistent voxel counts")
    P = torch.empty((9, n), dtype=torch.float64, device=F.device)
    K = torch.empty((81, n), dtype=torch.float64, device=F.device)
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = LIB.rve_umat_bridge(C.c_void_p(F.data_ptr()),
                             C.c_void_p(sigma.data_ptr()),
                             C.c_void_p(ddsdde.data_ptr()), n,
                             C.c_void_p(P.data_ptr()), C.c_void_p(K.data_ptr()),
                             C.c_void_p(st.cuda_stream or None))
    if rc != RVE_OK:
        raise RveError(rc, LIB.rve_last_error(None).decode())
    return P, K


def apply_G_noalloc(n, field, out, L=(1.0, 1.0, 1.0), projection="discrete",
                    stream=None):
    """out = G(field) (Eq. 11, FP64) through rve_apply_G_noalloc, which
    allocates nothing; field, out: contiguous float64 CUDA tensors of shape
    (9, n^3).  Enqueued on the stream; no synchronization."""
    for t in (field, out):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.dim() == 2 and t.shape[0] == 9 and t.shape[1] == n ** 3):
            raise ValueError("expected contiguous float64 CUDA tensors of "
                             "shape (9, n^3)")
    Lc = np.ascontiguousarray(L, dtype=np.float64)
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = LIB.rve_apply_G_noalloc(int(n), _dptr(Lc), PROJ[projection],
                                 C.c_void_p(field.data_ptr()),
                                 C.c_void_p(out.data_ptr()),
                                 C.c_void_p(st.cuda_stream or None))
    if rc != RVE_OK:
        raise RveError(rc, LIB.rve_last_error(None).decode())
    return out


class BatchRve:
    """A batch of independent RVEs of mixed grid edges solved together (one
    handle of the batch C ABI); one macro gradient per RVE."""

    def __init__(self, ns, L=(1.0, 1.0, 1.0), projection="discrete",
                 precision="fp64", newton_tol=1e-6, newton_max_iter=25,
                 cg_tol=1e-4, cg_max_iter=2000, cg_chunk=8, use_graph=False,
                 stream=None, device=0, torch_allocator=True, cg_forcing=False):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the library runs on the GPU only")
        self._lib = LIB
        self._h = None
        cfg, self.stream, self._alloc = _make_config(
            L, projection, precision, newton_tol, newton_max_iter, cg_tol,
            cg_max_iter, cg_chunk, use_graph, False, stream, device,
            torch_allocator, cg_forcing)
        self.cfg = cfg
        self.ns = [int(x) for x in ns]
        arr = np.ascontiguousarray(self.ns, dtype=np.int32)
        h = C.c_void_p()
        rc = LIB.rve_batch_create(C.byref(cfg), len(self.ns), _iptr(arr),
                                  C.byref(h))
        if rc != RVE_OK:
            raise RveError(rc, LIB.rve_batch_last_error(None).decode())
        self._h = h

    def __len__(self):
        return len(self.ns)

    def close(self):
        if self._h is not None:
            self._lib.rve_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc, ok=(RVE_OK,)):
        if rc not in ok:
            raise RveError(rc, self._lib.rve_batch_last_error(self._h).decode())
        return rc

    def set_microstructure(self, b, phase, quat, law, params):
        phase = np.ascontiguousarray(phase, dtype=np.int32).reshape(-1)
        quat = np.ascontiguousarray(quat, dtype=np.float64).reshape(-1, 4)
        law = np.ascontiguousarray(law, dtype=np.int32).reshape(-1)
        params = np.ascontiguousarray(params, dtype=np.float64).reshape(-1)
        if phase.size != self.ns[b] ** 3:
            raise ValueError("phase must have n^3 entries")
        self._check(LIB.rve_batch_set_microstructure(
            self._h, b, _iptr(phase), quat.shape[0], _dptr(quat), _iptr(law),
            _dptr(params), params.size))
        if not hasattr(self, "_labels"):
            self._labels = [0] * len(self.ns)
        self._labels[b] = quat.shape[0]

    def increment(self, F_bar, dt):
        """One increment of every RVE; F_bar is (3, 3) for all or (B, 3, 3).
        Returns one dict per RVE (status included)."""
        B = len(self.ns)
        Fb = np.asarray(F_bar, dtype=np.float64)
        Fb = np.ascontiguousarray(np.broadcast_to(Fb.reshape(-1, 9), (B, 9)))
        info = (RveIncrementInfo * B)()
        rc = LIB.rve_batch_apply_macro_strain_increment(self._h, _dptr(Fb),
                                                        float(dt), info)
        self._check(rc, ok=(RVE_OK, RVE_ENOTCONV, RVE_ELOCAL))
        return [_info_dict(info[b], info[b].status) for b in range(B)]

    def reset_fips(self):
        self._check(LIB.rve_batch_reset_fips(self._h))

    def field(self, b, name):
        fid, comps = FIELDS[name]
        out = np.empty((comps, self.ns[b] ** 3), dtype=np.float64)
        self._check(LIB.rve_batch_get_fields(self._h, b, 1 << fid,
                                             out.ctypes.data_as(C.c_void_p),
                                             out.nbytes, 0))
        return out if comps > 1 else out[0]

    def debug_apply_G(self, fields):
        """G (Eq. 11) of one [9][n_b^3] field per RVE through the batched
        passes, in the batch's precision."""
        flat = np.concatenate([np.ascontiguousarray(f, dtype=np.float64)
                               .reshape(-1) for f in fields])
        assert flat.size == sum(9 * n ** 3 for n in self.ns)
        out = np.empty_like(flat)
        self._check(LIB.rve_batch_debug_apply_G(self._h, _dptr(flat),
                                                _dptr(out)))
        res, pos = [], 0
        for n in self.ns:
            res.append(out[pos:pos + 9 * n ** 3].reshape(9, n ** 3))
            pos += 9 * n ** 3
        return res

    def tune_fft_schedules(self):
        """Tune every edge's CG-matvec schedule now (outside a timed run)."""
        self._check(LIB.rve_batch_tune_fft_schedule(self._h))

    def set_fft_schedule(self, edge, cpb=0, tt=0):
        """Force the CG-matvec schedule of one grid edge; (0, 0) tunes it
        again at the next increment."""
        self._check(LIB.rve_batch_set_fft_schedule(self._h, int(edge),
                                                   int(cpb), int(tt)))

    def fft_schedules(self):
        """{edge: dict(cpb, tt, tuned_ms)} for every edge of the batch."""
        res = {}
        for e in sorted(set(self.ns)):
            out = (C.c_int32 * 2)()
            ms = C.c_double()
            self._check(LIB.rve_batch_get_fft_schedule(self._h, e, out,
                                                       C.byref(ms)))
            res[e] = dict(cpb=out[0], tt=out[1], tuned_ms=ms.value)
        return res

    def macro(self, b):
        out = np.empty(29)
        self._check(LIB.rve_batch_get_macro(self._h, b, _dptr(out)))
        return dict(F_bar=out[:9].reshape(3, 3), P_bar=out[9:18].reshape(3, 3),
                    sigma_bar=out[18:27].reshape(3, 3), t=out[27],
                    increments=int(out[28]))

    def nonlocal_fips(self, b, band_width=None, arrays=True):
        """Eqs. 25-26 for RVE b; band_width defaults to two voxel edges."""
        w = (2.0 * self.cfg.L[0] / self.ns[b] if band_width is None
             else band_width)

        def call(*a):
            self._check(LIB.rve_batch_get_nonlocal_fips(self._h, b, *a))
        labels = getattr(self, "_labels", [0] * len(self.ns))[b]
        return _nonlocal_fips(call, labels, float(w), arrays)


class WarmStartNet:
    """Handle of the warm-start network (parameters, Adam state, kernels)."""

    def __init__(self, stream=None, device=0):
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        cfg = RveWsConfig()
        cfg.stream = C.c_void_p(self.stream.cuda_stream or None)
        self._alloc = _TorchAllocator(device)
        cfg.dev_alloc = self._alloc.alloc_fn
        cfg.dev_free = self._alloc.free_fn
        h = C.c_void_p()
        rc = LIB.rve_ws_create(C.byref(cfg), C.byref(h))
        if rc != RVE_OK:
            raise RveError(rc, LIB.rve_ws_last_error(None).decode())
        self._h = h
        n = C.c_int64()
        self._check(LIB.rve_ws_param_count(self._h, C.byref(n)))
        self.param_count = n.value

    def _check(self, rc):
        if rc != RVE_OK:
            raise RveError(rc, LIB.rve_ws_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) is not None:
            LIB.rve_ws_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32).reshape(-1)
        self._check(LIB.rve_ws_set_params(
            self._h, p.ctypes.data_as(C.POINTER(C.c_float)), p.size))

    def get_params(self):
        p = np.empty(self.param_count, dtype=np.float32)
        self._check(LIB.rve_ws_get_params(
            self._h, p.ctypes.data_as(C.POINTER(C.c_float)), p.size))
        return p

    def forward(self, X, n, out=None):
        if out is None:
            out = torch.empty((n ** 3, WS_OUT), dtype=torch.float32,
                              device="cuda")
        self._check(LIB.rve_ws_forward(self._h, C.c_void_p(X.data_ptr()), n,
                                       C.c_void_p(out.data_ptr())))
        return out

    def train_step(self, X, T, n, lr, want_grad=False):
        loss = C.c_double()
        g = np.empty(self.param_count, dtype=np.float32) if want_grad else None
        self._check(LIB.rve_ws_train_step(
            self._h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()), n,
            float(lr), C.byref(loss),
            g.ctypes.data_as(C.POINTER(C.c_float)) if want_grad else None))
        return (loss.value, g) if want_grad else loss.value

    def loss(self, X, T, n):
        """Loss of one sample; no training step."""
        out = C.c_double()
        self._check(LIB.rve_ws_loss(self._h, C.c_void_p(X.data_ptr()),
                                    C.c_void_p(T.data_ptr()), n,
                                    C.byref(out)))
        return out.value
