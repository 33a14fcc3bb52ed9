"""The C-ABI library loads and exports every entry point rve.h declares.

CPU only: the library is loaded with ctypes but no compute call is made.
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rve.h")
LIB = os.path.join(ROOT, "paper_1806_10599_amd", "libpaper_1806_10599_amd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:rve_status|const char\s*\*)\s+(rve_\w+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_core_entry_points():
    names = declared_functions()
    for core in ("rve_create", "rve_destroy", "rve_set_microstructure",
                 "rve_apply_macro_strain_increment", "rve_get_fields"):
        assert core in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    # the binding has no CPU fallback: a missing library is an ImportError
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "rve_binding_probe",
        os.path.join(ROOT, "paper_1806_10599_amd", "binding.py"))
    mod = importlib.util.module_from_spec(spec)
    src = open(spec.origin).read().replace(
        'LIBPATH = os.path.join(_HERE, "libpaper_1806_10599_amd.so")',
        f'LIBPATH = {str(tmp_path / "missing.so")!r}')
    with pytest.raises(ImportError):
        exec(compile(src, spec.origin, "exec"), mod.__dict__)


def test_binding_rejects_bad_solver_modes_before_touching_a_device():
    # argument checks of the binding run on the host (no GPU needed)
    from paper_1806_10599_amd import binding
    args = dict(L=(1.0, 1.0, 1.0), projection="discrete", precision="mixed",
                newton_tol=1e-6, newton_max_iter=25, cg_tol=1e-4,
                cg_max_iter=500, cg_chunk=8, use_graph=False, stream=None,
                device=0, torch_allocator=False)
    with pytest.raises(ValueError, match="cg_forcing"):
        binding._make_config(warm_start=0, cg_forcing=3, **args)
    with pytest.raises(ValueError, match="warm_start"):
        binding._make_config(warm_start=5, cg_forcing=1, **args)
