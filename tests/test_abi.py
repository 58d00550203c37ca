"""The C-ABI library loads and exports every entry point of include/*.h (CPU only).

Also checks host-side argument validation, which returns before any device call.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1703_01202_amd", "libpfc.so")


def _declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for h in sorted(os.listdir(inc)):
        if h.endswith(".h"):
            text = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, h)).read(), flags=re.S)
            names.update(re.findall(r"\b(pfc_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libpfc.so is not built: run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_header_declares_the_hot_path():
    names = _declared_functions()
    for required in ("pfc_residual", "pfc_jv", "pfc_ras_setup", "pfc_ras_apply", "pfc_step",
                     "pfc_energy", "pfc_gmres", "pfc_newton", "pfc_create", "pfc_destroy",
                     "pfc_net_create", "pfc_net_forward", "pfc_net_gradient", "pfc_net_adam", "pfc_attach_net"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_1703_01202_amd import _lib
    assert set(_declared_functions()) <= set(_lib.SIGNATURES)


def _create(lib, n=(64, 64, 1), sub=(4, 4, 1), overlap=2, dim=2, **kw):
    from paper_1703_01202_amd import _lib
    for name, (res, args) in _lib.SIGNATURES.items():
        getattr(lib, name).restype = res
        getattr(lib, name).argtypes = args
    g = _lib.PfcGrid()
    g.dim = dim
    for a in range(3):
        g.n[a] = n[a]
        g.L[a] = 10.0
    m = _lib.PfcModel(gamma=0.25, mobility=kw.pop("mobility", 0), boundary=kw.pop("boundary", 0))
    o = _lib.PfcOpts()
    lib.pfc_default_opts(ctypes.byref(o))
    for a in range(3):
        o.sub[a] = sub[a]
    o.overlap = overlap
    for k, v in kw.items():
        setattr(o, k, v)
    ctx = ctypes.c_void_p()
    return lib.pfc_create(ctypes.byref(g), ctypes.byref(m), ctypes.byref(o), None, ctypes.byref(ctx))


@pytest.mark.parametrize("kw,status", [
    (dict(sub=(3, 4, 1)), -1),                  # 3 does not divide 64
    (dict(sub=(1, 4, 1)), -1),                  # fewer than two boxes
    (dict(overlap=30), -1),                     # extended box wider than n - 3
    (dict(n=(4, 64, 1)), -1),                   # grid too small
    (dict(gmres_restart=0), -1),
    (dict(gmres_restart=100), -1),
    (dict(mobility=2), -1),                     # M = 1 and M = 1 - phi^2 only
    (dict(boundary=2), -1),                     # periodic and Neumann-type only
    (dict(sub_solver=2, ilu_level=5), -1),      # ILU(k) up to k = 4
    (dict(sub_solver=3), -1),                   # no such subdomain solver
    (dict(precond_lag=-2), -1),
    (dict(dt_min=0.0), -1),
    (dict(sub_solver=1, dim=3, n=(32, 32, 32), sub=(4, 4, 4)), -8),   # exact LU is 2-D only
    (dict(ras_kind=3), -1),                     # no such Schwarz variant
    (dict(ras_kind=1, sub=(32, 32, 1), overlap=20), -1),   # AS sum over more than 16 boxes per axis
    (dict(guess=3), -1),                        # no such guess
    (dict(guess=2, dim=3, n=(32, 32, 32), sub=(4, 4, 4)), -8),       # learned guess is 2-D only
])
def test_create_rejects_bad_arguments(lib, kw, status):
    assert _create(lib, **kw) == status


def test_default_opts_match_paper_tolerances(lib):
    from paper_1703_01202_amd import _lib
    lib.pfc_default_opts.argtypes = [ctypes.POINTER(_lib.PfcOpts)]
    o = _lib.PfcOpts()
    lib.pfc_default_opts(ctypes.byref(o))
    # Sec. 5: eps_r = 1e-8, eps_a = 1e-10, xi_r = 1e-3, xi_a = 1e-11
    assert (o.newton_rtol, o.newton_atol, o.lin_rtol, o.lin_atol) == (1e-8, 1e-10, 1e-3, 1e-11)
    assert o.gmres_restart == 30 and o.mass_project == 1
    assert o.precond_lag == 0 and o.newton_rel_ref == 1


def test_opts_struct_size_matches_header():
    # the ctypes mirror must have the C layout: compile a probe of sizeof/offsetof with gcc
    import os
    import subprocess
    import tempfile
    from paper_1703_01202_amd import _lib
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = ('#include <stdio.h>\n#include <stddef.h>\n#include "pfc.h"\n'
           'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(pfc_opts), offsetof(pfc_opts, newton_rel_ref),'
           ' sizeof(pfc_step_stats), sizeof(pfc_grid), sizeof(pfc_model), offsetof(pfc_model, boundary),'
           ' offsetof(pfc_opts, ilu_level)); return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        cpath, exe = os.path.join(d, "p.c"), os.path.join(d, "p")
        open(cpath, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(root, "include"), cpath, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    assert int(out[0]) == ctypes.sizeof(_lib.PfcOpts)
    assert int(out[1]) == _lib.PfcOpts.newton_rel_ref.offset
    assert int(out[2]) == ctypes.sizeof(_lib.PfcStepStats)
    assert int(out[3]) == ctypes.sizeof(_lib.PfcGrid)
    assert int(out[4]) == ctypes.sizeof(_lib.PfcModel)
    assert int(out[5]) == _lib.PfcModel.boundary.offset
    assert int(out[6]) == _lib.PfcOpts.ilu_level.offset


def test_autotune_box_candidates_tile_the_grid():
    from paper_1703_01202_amd import autotune as A
    cands = A.box_candidates((1024, 1024))
    assert ((16, 64), 4) in cands and ((32, 64), 4) in cands
    for (sy, sx), ov in cands:
        assert 1024 % sy == 0 and 1024 % sx == 0
        assert 1024 // sx + 2 * ov in (24, 28, 32, 40)  # extended box widths asked for
    assert A.box_candidates((100, 100)) == []            # nothing divides: no candidates
