"""Host-side checks of the C-ABI library (no GPU): it loads, exports every symbol that
include/scola.h declares, validates plans, and its FP64 scalar tables match the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2003_04925_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libscola.so not built")
    return _lib


def declared_functions():
    src = open(os.path.join(ROOT, "include", "scola.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(scola_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    L = _lib()
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.exported_symbols()) == names


def test_status_strings():
    lib = _lib().lib()
    assert lib.scola_status_string(0) == b"SCOLA_OK"
    assert lib.scola_status_string(-5) == b"SCOLA_EUNSUPPORTED"


def test_uniform_tiling():
    from paper_2003_04925_amd import uniform_tiling
    t = uniform_tiling(64, 2, 8)
    assert len(t) == 8 and t[0] == ((0, 0, 0), 32, 8) and t[7] == ((32, 32, 32), 32, 8)
    with pytest.raises(Exception):
        uniform_tiling(64, 3, 8)


def _plan_status(L_, Np=32, tiles=None, mesh=0, tile_a_f=None, **kw):
    cfg = L_.make_config(kw.get("L", 100.0), Np, kw.get("n_steps", 4), 0.05, kw.get("a_f", 1.0),
                         kw.get("precision", 0), 0, 0, N_lpt=kw.get("N_lpt", 0),
                         fda_order=kw.get("fda_order", 0), n_lpt=kw.get("n_lpt", 0.0),
                         discretisation=kw.get("discretisation", 0))
    cos = L_.Cosmology(0.31, 0.0486, 0.6774, 0.9667, 0.81, 2.7255)
    tiles = tiles or [((0, 0, 0), Np, 0)]
    arr = (L_.Tile * len(tiles))()
    for i, (lo, n, b) in enumerate(tiles):
        arr[i].core_lo[:] = lo
        arr[i].core_n = n
        arr[i].buffer = b
        arr[i].mesh[:] = (mesh,) * 3 if isinstance(mesh, int) else mesh
        arr[i].a_f = tile_a_f[i] if tile_a_f else 0.0
    plan = ctypes.c_void_p()
    st = L_.lib().scola_plan_create(ctypes.byref(cfg), ctypes.byref(cos), arr, len(tiles),
                                    ctypes.byref(plan))
    if plan.value:
        L_.lib().scola_plan_destroy(plan)
    return st, L_.lib().scola_last_error().decode()


def test_plan_validation_errors():
    L_ = _lib()
    st, msg = _plan_status(L_, Np=24)
    assert st == -1 and "power of two" in msg
    st, msg = _plan_status(L_, a_f=0.01)
    assert st == -1
    st, msg = _plan_status(L_, tiles=[((0, 0, 0), 16, 8), ((16, 0, 0), 16, 8)])
    assert st == -1 and "cover" in msg
    st, msg = _plan_status(L_, tiles=[((0, 0, 0), 32, 3)])
    assert st == -5 and "one of 16" in msg
    over = [((0, 0, 0), 16, 8)] * 8
    st, msg = _plan_status(L_, tiles=over)
    assert st == -1 and "overlap" in msg


def _validated(st):
    """The plan passed validation: created (GPU) or stopped at the first HIP call (CPU)."""
    return st in (0, -3)


def test_config_and_tile_fields_accept_and_refuse():
    L_ = _lib()
    # mesh: 0 or M per axis accepted, any other size unsupported, negative invalid
    assert _validated(_plan_status(L_, mesh=0)[0])
    assert _validated(_plan_status(L_, mesh=32)[0])
    st, msg = _plan_status(L_, mesh=(32, 32, 33))
    assert st == -5 and "mesh[2]" in msg
    assert _plan_status(L_, mesh=-1)[0] == -1
    # box sizes of the form 2^a {1,3,5,7} outside 16 R, R = 1..8
    st, msg = _plan_status(L_, Np=16, tiles=[((0, 0, 0), 16, 4)])      # M = 24
    assert st == -5 and "one of 16" in msg
    st, msg = _plan_status(L_, Np=256, tiles=[((0, 0, 0), 256, 0)])    # M = 256
    assert st == -5
    # fda_order: 0, 2, 4 and 6 accepted, others invalid
    for o in (0, 2, 4, 6):
        assert _validated(_plan_status(L_, fda_order=o)[0])
    for o in (3, 8, -2):
        assert _plan_status(L_, fda_order=o)[0] == -1
    # N_lpt: 0, Np and power-of-two divisors of Np >= 8 accepted, anything else invalid
    for n in (0, 32, 16, 8):
        assert _validated(_plan_status(L_, N_lpt=n)[0])
    for n in (7, 4, 64, 24, -16):
        st, msg = _plan_status(L_, N_lpt=n)
        assert st == -1 and "N_lpt" in msg
    # n_lpt: any finite value; the discretisation switch
    assert _validated(_plan_status(L_, n_lpt=-1.5)[0])
    assert _plan_status(L_, n_lpt=float("nan"))[0] == -1
    assert _validated(_plan_status(L_, discretisation=1)[0])
    assert _plan_status(L_, discretisation=2)[0] == -1
    assert L_.lib().scola_status_string(-6) == b"SCOLA_EOVERFLOW"
    # per-tile final scale factor: 0 or > a_i
    tl = [((0, 0, 0), 16, 8), ((16, 0, 0), 16, 8), ((0, 16, 0), 16, 8), ((16, 16, 0), 16, 8),
          ((0, 0, 16), 16, 8), ((16, 0, 16), 16, 8), ((0, 16, 16), 16, 8), ((16, 16, 16), 16, 8)]
    assert _validated(_plan_status(L_, tiles=tl, tile_a_f=[0.5] + [0.0] * 7)[0])
    st, msg = _plan_status(L_, tiles=tl, tile_a_f=[0.01] + [0.0] * 7)
    assert st == -1 and "a_f" in msg


def test_schedule_table_matches_oracle():
    from oracle.cosmology import Cosmology, cola_schedule
    from paper_2003_04925_amd import schedule_table
    for n in (1, 10, 20):
        t = schedule_table(n)
        steps, final = cola_schedule(Cosmology(), 0.05, 1.0, n, want_final_kick=True)
        o = np.array([[s["a_D"], s["beta"], s["alpha"], s["D1"], s["D2"], s["D1_next"],
                       s["D2_next"], s["a_next"]] for s in steps])
        np.testing.assert_allclose(t[:n], o, rtol=1e-10)
        inv = final["inv_drift"]
        np.testing.assert_allclose(t[n, :6], [final["a_D"], final["beta"], final["D1"],
                                              final["D2"], -final["dD1"] * inv,
                                              final["dD2"] * inv], rtol=1e-10)


def test_standard_and_modified_schedules_match_oracle():
    from oracle.cosmology import Cosmology, cola_schedule
    from paper_2003_04925_amd import schedule_table
    for disc, nl in (("standard", 0.0), ("modified", -1.5)):
        t = schedule_table(10, discretisation=disc, n_lpt=nl)
        steps, final = cola_schedule(Cosmology(), 0.05, 1.0, 10, want_final_kick=True,
                                     discretisation=disc, n_lpt=nl if nl else -2.5)
        o = np.array([[s["beta"], s["alpha"]] for s in steps])
        np.testing.assert_allclose(t[:10, 1:3], o, rtol=1e-10)
        assert t[10, 1] == pytest.approx(final["beta"], rel=1e-10)
    # the two discretisations differ
    assert abs(schedule_table(10, discretisation="standard")[3, 2] /
               schedule_table(10)[3, 2] - 1) > 1e-3


def test_linear_power_matches_oracle():
    from oracle.cosmology import Cosmology
    from oracle.lpt import linear_power as oracle_power
    from paper_2003_04925_amd import linear_power
    k = np.logspace(-4, 1.5, 64)
    np.testing.assert_allclose(linear_power(k), oracle_power(k, Cosmology()), rtol=1e-11)


def test_product_package_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2003_04925_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.replace("oracle-free", ""), f
