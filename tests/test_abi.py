"""The C-ABI library loads, exports every symbol its header declares, and its
host-side logic (parameter rule, Alpert rule, shape helper, argument checks)
agrees with the oracle and the paper.  No device calls."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from conftest import ROOT, golden

fb = pytest.importorskip("paper_1709_01480_amd")
from oracle import alpert as OA  # noqa: E402
from oracle import fbim as OF  # noqa: E402
import workloads as W  # noqa: E402

PAPER = golden("paper_values.txt")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fbim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fbim_[A-Za-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(fb.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("order", [4, 8])
def test_alpert_rule_matches_oracle(order):
    # the library solves the moment system in long double; for order 8 its
    # conditioning (powers up to chi^6 with chi near 4) limits agreement to ~1e-11
    chi, w, a = fb.alpert_rule(order)
    ochi, ow, oa = OA.alpert_rule(order)
    tol = 1e-13 if order == 4 else 5e-11
    assert a == oa
    assert np.allclose(chi, ochi, rtol=0, atol=tol)
    assert np.allclose(w, ow, rtol=0, atol=tol)


def test_parameter_rule_printed_value():
    d = fb.derive_params(L=1.0, tol_ewald=1e-9, n_box=4)
    v, tol, _ = PAPER["xiL_nbox4_eps1e-9"]
    assert abs(d["xi"] - v) / v < tol
    assert d["P"] == 15 and d["r_c"] == 0.25


@pytest.mark.parametrize("name", ["starfish4", "starfish100", "starfish10k", "tiny2", "small12"])
def test_parameter_rule_matches_oracle(name):
    wl = W.make(name) if name != "starfish10k" else W.Workload(name=name, **W.CONFIGS[name])
    d = fb.derive_params(**wl.params())
    o = OF.derive_params(wl.L, wl.tol_ewald, n_box=wl.n_box, grid_M=wl.grid_M, xi=wl.xi, P=wl.P)
    assert d["n_box"] == o["n_box"] and d["grid_M"] == o["grid_M"] and d["P"] == o["P"]
    assert abs(d["xi"] - o["xi"]) <= 1e-12 * o["xi"]
    assert abs(d["eta_s"] - o["eta_s"]) <= 1e-12 * o["eta_s"]
    # the spreading tile divides the grid and covers the stencil half-width
    assert d["grid_M"] % d["tile"] == 0 and d["tile"] >= (d["P"] - 1) // 2


def test_starfish_helper_matches_oracle_curve():
    ref = fb.starfish(0.05, 0.3, 5, 64)
    sh = OF.Shape(0.05, 0.3, 5, 64)
    assert np.allclose(ref.reshape(-1, 2), sh.gamma(2 * np.pi * np.arange(64) / 64), atol=1e-16)


def test_invalid_parameters_rejected():
    with pytest.raises(fb.FbimError):
        fb.derive_params(L=1.0, tol_ewald=1e-9, n_box=2)
    # cutoff cell wider than the real-space E1 series covers (xi r_c = 10 > 8)
    with pytest.raises(fb.FbimError):
        fb.derive_params(L=1.0, tol_ewald=1e-9, n_box=3, xi=30.0, grid_M=64)
    fb.derive_params(L=1.0, tol_ewald=1e-9, n_box=4, xi=30.0, grid_M=64)  # xi r_c = 7.5
    with pytest.raises(fb.FbimError):
        fb.derive_params(L=1.0, tol_ewald=1e-9, n_box=4, grid_M=63)
    with pytest.raises(fb.FbimError):
        fb.derive_params(L=-1.0, tol_ewald=1e-9, n_box=4)
    with pytest.raises(fb.FbimError):
        fb.alpert_rule(6)


def test_uneven_suspension_draws_are_valid_systems():
    """The uneven-batch workload: sizes in range, node counts from the set, the
    library's parameter rule accepts every suspension with a power-of-two grid,
    and the bounding circles of each suspension do not overlap."""
    wls = W.uneven_suspensions(16)
    assert len(wls) == 16
    for w in wls:
        assert 16 <= w.n_bodies <= 512 and w.n_p in (64, 128, 256)
        d = fb.derive_params(**w.params())
        assert d["grid_M"] == w.grid_M and (w.grid_M & (w.grid_M - 1)) == 0
        dq = w.q[:, None, :] - w.q[None, :, :]
        dq -= w.L * np.round(dq / w.L)
        dist = np.sqrt((dq ** 2).sum(-1)) + np.eye(w.n_bodies) * 1e9
        assert dist.min() > 2 * w.a
    # the draw is seeded: the same call gives the same systems
    again = W.uneven_suspensions(16)
    assert all(np.array_equal(a.q, b.q) and a.n_p == b.n_p for a, b in zip(wls, again))


def test_params_struct_layout_matches_header(tmp_path):
    # the binding's ctypes structures have the C compiler's size and field offsets
    src = tmp_path / "layout.c"
    fields = [f for f, _ in fb.Params._fields_]
    body = "\n".join('  printf("%%zu ", offsetof(fbim_params, %s));' % f for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "fbim.h"\nint main(void) {\n%s\n'
                   '  printf("%%zu %%zu %%zu %%zu\\n", sizeof(fbim_params), sizeof(fbim_info), sizeof(fbim_derived), sizeof(fbim_tune_report));\n'
                   '  return 0;\n}\n' % body)
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    offs = [getattr(fb.Params, f).offset for f in fields]
    assert vals[:len(fields)] == offs
    assert vals[len(fields):] == [ctypes.sizeof(fb.Params), ctypes.sizeof(fb.Info), ctypes.sizeof(fb.Derived),
                                  ctypes.sizeof(fb.TuneReport)]


def test_autotune_cache_lookup(tmp_path):
    # the JSON-lines cache the autotuner reads and appends to: exact key match, the
    # last matching line wins, malformed lines and other keys are skipped
    path = tmp_path / "tune.jsonl"
    key = "arch=gfx950:cu=256|prec=1|N=640000|bodies=64x10000|what=1"
    path.write_text(
        '{"key": "%s", "n_box": 201, "grid_M": 2048, "tile": 16, "ms": 0.31}\n' % key
        + '{"key": "%s|extra", "n_box": 5, "grid_M": 64, "tile": 8, "ms": 0.1}\n' % key
        + '{"key": "%s", "n_box": "oops", "grid_M": 2048}\n' % key
        + 'not json at all\n'
        + '{"key": "%s", "n_box": 201, "grid_M": 2048, "tile": 32, "ms": 0.29}\n' % key
        + '{"key": "arch=gfx950:cu=256", "n_box": 7, "grid_M": 128, "tile": 32, "ms": 1}\n')
    assert fb.autotune_lookup(str(path), key) == (201, 2048, 32)
    assert fb.autotune_lookup(str(path), key + "|extra") == (5, 64, 8)
    assert fb.autotune_lookup(str(path), key[:-1]) is None
    assert fb.autotune_lookup(str(tmp_path / "missing.jsonl"), key) is None
