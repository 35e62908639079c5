"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every
function the headers under include/ declare, and rejects bad configurations before touching
the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1812_10375_amd import lbm, scenarios as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    """Every function any header under include/ declares."""
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_function():
    L = lbm.library()
    names = declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(L, n), n


def test_struct_layout_matches_header():
    # lbm_config: 2 uint32 + 9 int32/uint32 + 25 doubles + int32 + 3 pointers
    assert C.sizeof(lbm.LbmConfig) == 8 + 36 + 4 + 25 * 8 + 8 + 24
    assert C.sizeof(lbm.LbmObs) == 8 + 12 * 8 + 8 + 8


def test_workspace_bytes_for_the_full_boiling_workload():
    sc = S.pool_boiling(steps=1)
    nb = lbm.workspace_bytes(sc)
    nodes = 1024 * 1024
    # two population copies, two T copies, rho/u; then per-tile partials and the
    # 256-step history of per-tile energy partials (bounded by 32 MiB)
    fields = (2 * 9 + 3) * nodes * 4 + 2 * 1049 * 1024 * 4
    assert fields < nb < fields + (32 << 20)


@pytest.mark.parametrize("change", [
    {"nx": 0}, {"ny": 0}, {"n_sub": 0}, {"heater_rows": -1}, {"precision": "f16"},
    {"ny": 1, "top_bc": "convective"}, {"G": 1.0}, {"tau_l": 0.5}, {"s_q": 2.0},
    {"rho_v": 7.0}, {"k": 0.0}, {"g": float("nan")}, {"flags": ("two_launches", "one_launch")},
])
def test_invalid_configurations_are_rejected(change):
    sc = S.film_evaporation(nx=16, ny=16, film=4)
    sc.update(change)
    if sc["precision"] not in ("f32", "f64"):
        c, keep = lbm.make_config(dict(sc, precision="f32"))
        c.precision = 7
    else:
        c, keep = lbm.make_config(sc)
    assert lbm.library().lbm_workspace_bytes(C.byref(c)) == 0
    h = C.c_void_p()
    rho = np.zeros((1,))
    fake = C.c_void_p(1 << 20)  # never dereferenced: the call fails before any device work
    rc = lbm.library().lbm_init(C.byref(c), fake, 1 << 30, None, lbm._dptr(rho), lbm._dptr(rho), C.byref(h))
    assert rc == -1


def test_small_or_misaligned_workspace_is_rejected():
    sc = S.film_evaporation(nx=16, ny=16, film=4)
    c, keep = lbm.make_config(sc)
    need = lbm.library().lbm_workspace_bytes(C.byref(c))
    rho = np.ascontiguousarray(sc["rho0"])
    T = np.ascontiguousarray(sc["T0"])
    h = C.c_void_p()
    L = lbm.library()
    assert L.lbm_init(C.byref(c), C.c_void_p(1 << 20), need - 1, None, lbm._dptr(rho), lbm._dptr(T), C.byref(h)) == -2
    assert L.lbm_init(C.byref(c), C.c_void_p((1 << 20) + 4), need, None, lbm._dptr(rho), lbm._dptr(T), C.byref(h)) == -1
    assert L.lbm_step(None, 1) == -1
    assert L.lbm_strerror(-2) == b"workspace too small"


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1812_10375_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, re.M), fn
                assert "liboracle" not in text and "lbm_oracle" not in text, fn


def test_batch_rejects_incompatible_domains():
    L = lbm.library()
    a = S.film_evaporation(nx=16, ny=16, film=4, precision="f32")
    b = S.film_evaporation(nx=24, ny=12, film=4, precision="f32")
    good = lbm._BatchInputs([a, b])
    assert L.lbm_batch_workspace_bytes(good.cfgs, 2) >= (lbm.workspace_bytes(a) + lbm.workspace_bytes(b))
    for change in ({"precision": "f64"}, {"n_sub": 2}, {"flags": ("diff_isotropic",)}, {"tile_rows": -1}):
        bad = lbm._BatchInputs([a, dict(b, **change)])
        assert L.lbm_batch_workspace_bytes(bad.cfgs, 2) == 0, change
        h = C.c_void_p()
        fake = C.c_void_p(1 << 20)  # never dereferenced: the call fails before any device work
        rc = L.lbm_batch_init(bad.cfgs, 2, fake, 1 << 30, None, bad.rho0, bad.T0, C.byref(h))
        assert rc == -1 and not h.value, change
    assert L.lbm_batch_workspace_bytes(good.cfgs, 0) == 0


def test_autotuners_reject_bad_arguments_before_any_device_work():
    L = lbm.library()
    a = S.film_evaporation(nx=16, ny=16, film=4, precision="f32")
    inp = lbm._BatchInputs([a, a])
    need = L.lbm_batch_workspace_bytes(inp.cfgs, 2)
    fake = C.c_void_p(1 << 20)  # never dereferenced: the calls fail before any device work
    rows, flags, ms = (C.c_int32 * 2)(), (C.c_uint32 * 2)(), C.c_double()
    r1, ms1 = C.c_int(), C.c_double()
    # missing outputs, no steps, a workspace too small, incompatible domains
    assert L.lbm_autotune(inp.cfgs, 2, fake, need, None, inp.rho0, inp.T0, 5, None, flags, C.byref(ms)) == -1
    assert L.lbm_autotune(inp.cfgs, 2, fake, need, None, inp.rho0, inp.T0, 0, rows, flags, C.byref(ms)) == -1
    assert L.lbm_autotune(inp.cfgs, 2, fake, need - 1, None, inp.rho0, inp.T0, 5, rows, flags, C.byref(ms)) == -2
    assert L.lbm_autotune_tile_rows(inp.cfgs, 2, fake, need, None, inp.rho0, inp.T0, 5, None, C.byref(ms1)) == -1
    bad = lbm._BatchInputs([a, dict(a, precision="f64")])
    assert L.lbm_autotune(bad.cfgs, 2, fake, 1 << 30, None, bad.rho0, bad.T0, 5, rows, flags, C.byref(ms)) == -1
    assert L.lbm_autotune_tile_rows(bad.cfgs, 2, fake, 1 << 30, None, bad.rho0, bad.T0, 5, C.byref(r1),
                                    C.byref(ms1)) == -1
