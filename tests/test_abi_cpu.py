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


def _plan_status(L_, Np=32, tiles=None, **kw):
    cfg = L_.Config(kw.get("L", 100.0), Np, 0, kw.get("n_steps", 4), 0.05, kw.get("a_f", 1.0),
                    kw.get("precision", 0), 0, 0)
    cos = L_.Cosmology(0.31, 0.0486, 0.6774, 0.9667, 0.81, 2.7255)
    tiles = tiles or [((0, 0, 0), Np, 0)]
    arr = (L_.Tile * len(tiles))()
    for i, (lo, n, b) in enumerate(tiles):
        arr[i].core_lo[:] = lo
        arr[i].core_n = n
        arr[i].buffer = b
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
    assert st == -5 and "multiple of 16" in msg
    over = [((0, 0, 0), 16, 8)] * 8
    st, msg = _plan_status(L_, tiles=over)
    assert st == -1 and "overlap" in msg


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
