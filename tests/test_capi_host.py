"""Host-only checks of the C-ABI library (no GPU: nothing here launches a kernel).

* the library loads and exports every function include/nedner.h declares;
* descriptor validation returns the documented status codes;
* the sizes reported by nedner_query follow from the descriptor;
* calls that need a plan fail cleanly without one.
"""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1501_02946_amd as N
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nedner.h")
E_ARG, E_ALIAS, E_WORKSPACE, E_UNSUPPORTED = 1, 2, 4, 6


def _header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nedner_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = _header_functions()
    assert len(names) >= 15
    L = N.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", N.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_version_and_status_strings():
    L = N.lib()
    assert L.nedner_version() == 100
    for st in range(8):
        assert L.nedner_status_string(st)
    assert L.nedner_status_string(0) == b"ok"


def _desc(**kw):
    base = dict(xy=np.array([[0.25, 0.5], [0.75, 0.1]]), h=None, nt=64, dt=1 / 64, n1=8, n2=8,
                n3=32)
    base.update(kw)
    xy, h, nt, dt, n1, n2, n3 = (base.pop(k) for k in ("xy", "h", "nt", "dt", "n1", "n2", "n3"))
    return N._make_desc(xy, h, nt, dt, n1, n2, n3, **base)


def _validate(**kw):
    d, keep = _desc(**kw)
    st = N.lib().nedner_validate(ctypes.byref(d))
    return st, N.lib().nedner_last_error().decode()


def test_valid_descriptor():
    assert _validate()[0] == 0


def test_two_dimensional_descriptor():
    """n2 = 1: sensors on a line, one voxel across the second axis (d = 2)."""
    assert _validate(n2=1)[0] == 0
    info = N.query(np.array([[0.25, 0.5], [0.75, 0.5]]), 64, 1 / 64, (8, 1, 32))
    assert info["n2_os"] == 2 and info["columns"] == 9


@pytest.mark.parametrize("kw,status", [
    (dict(xy=np.zeros((0, 2))), E_ARG),                        # no sensors
    (dict(xy=np.array([[np.nan, 0.5]])), E_ARG),               # non-finite position
    (dict(xy=np.array([[1.0, 0.5]])), E_ARG),                  # outside [a, a+L)
    (dict(xy=np.array([[-0.01, 0.5]])), E_ARG),
    (dict(n1=9), E_ARG),                                       # odd grid
    (dict(n1=1), E_ARG),                                       # one voxel: only across axis 2
    (dict(n2=3), E_ARG),
    (dict(n3=1), E_ARG),
    (dict(n2=1, xy=np.array([[0.25, 0.5], [0.5, 0.5]]), flags=["equispaced"]), E_ARG),
    (dict(n3=7), E_ARG),
    (dict(nt=63), E_ARG),                                      # odd time count
    (dict(c=0.0), E_ARG),
    (dict(c=-1.0), E_ARG),
    (dict(dt=0.0), E_ARG),
    (dict(w=13), E_ARG),                                       # odd taps
    (dict(w=18), E_ARG),
    (dict(w=0), E_ARG),
    (dict(sigma=1.0), E_ARG),
    (dict(sigma=1.3), E_ARG),                                  # sigma*n not an even integer
    (dict(tau_scale=0.0), E_ARG),
    (dict(precision=7), E_ARG),
    (dict(flags=64), E_ARG),
    (dict(time_per_lane=3), E_ARG),
    (dict(h=np.array([1.0, -0.5])), E_ARG),
    (dict(d3=-1.0), E_ARG),
    (dict(window=2), E_ARG),                                   # unknown window
    (dict(window="kaiser_bessel", w=14), E_UNSUPPORTED),       # KB built for 4..12 taps
    (dict(window="kaiser_bessel", w=2), E_UNSUPPORTED),
    (dict(n1=14), E_UNSUPPORTED),                              # 28 is not 5-smooth
    (dict(nt=14 * 8), E_UNSUPPORTED),
    (dict(nt=16, dt=1 / 16, n3=32), E_ALIAS),                  # |omega| dt >= pi
])
def test_invalid_descriptors(kw, status):
    st, msg = _validate(**kw)
    assert st == status, (st, msg)
    assert msg


def test_flags_lift_checks():
    assert _validate(nt=16, dt=1 / 16, n3=32, flags=["allow_alias"])[0] == 0
    assert _validate(xy=np.array([[1.25, -0.5]]), flags=["wrap"])[0] == 0


def _expected_segments_and_entries(p, info, W=12):
    """Sweep segments and (sensor, column, sweep cell) list entries from their
    definition: per group of four columns of the oversampled grid, segments
    of rows [S0, S1) cut in order so that each costs (entries in the cell rows
    S0 - W/2 .. S1 + W/2 - 2 over the group's columns) at most what S + W - 1
    rows cost at the mean density, but keeps at least min(W, S) rows and at
    most 4 S."""
    n1, n2 = info["n1_os"], info["n2_os"]
    S = info["rows_per_wave"]
    u1 = n1 * (p.xy[:, 0] - p.a1) / (p.n1 * p.d1)
    u2 = n2 * (p.xy[:, 1] - p.a2) / (p.n2 * p.d2)
    c1 = np.floor(u1).astype(int) % n1
    c2 = np.floor(u2).astype(int) % n2
    # per column: entries per first-axis cell (a sensor enters each distinct column its taps reach)
    count = np.zeros((n2, n1), dtype=np.int64)
    for m in range(p.m):
        for col in set(((c2[m] + np.arange(W) - W // 2 + 1) % n2).tolist()):
            count[col, c1[m]] += 1
    ncg = (n2 + 3) // 4
    target = count.sum() / (ncg * n1) * (S + W - 1)
    minlen, maxlen = max(1, min(W, S)), min(n1, 4 * S)
    segments = entries = 0
    for cg in range(ncg):
        cost = count[4 * cg:4 * cg + 4].sum(axis=0)
        s0 = 0
        while s0 < n1:
            s1 = min(s0 + minlen, n1)
            c = sum(cost[v % n1] for v in range(s0 - W // 2, s1 + W // 2 - 1))
            while s1 < n1 and s1 - s0 < maxlen and c + cost[(s1 + W // 2 - 1) % n1] <= target:
                c += cost[(s1 + W // 2 - 1) % n1]
                s1 += 1
            segments += 1
            entries += int(c)
            s0 = s1
    return segments, entries


@pytest.mark.parametrize("name", ["c1", "c5sub"])
def test_query_sizes(name):
    p = synth.config(name)
    kw = p.geometry_kwargs()
    info = N.query(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), h=p.h, c=p.c, t0=p.t0, a1=p.a1,
                   a2=p.a2, d1=p.d1, d2=p.d2, d3=p.d3, precision="fp32c")
    assert (info["n1_os"], info["n2_os"], info["nt_os"]) == (2 * p.n1, 2 * p.n2, 2 * p.nt)
    K2, J1 = p.n2 // 2 + 1, p.n1 + 1
    assert info["columns"] == K2 * J1
    rs, cs = 4, 8
    U = 4 * p.n1 * p.n2 * p.nt * rs
    V = 2 * p.n1 * K2 * p.nt * cs
    G = K2 * J1 * p.nt * cs
    Z1 = K2 * J1 * p.n3 * cs
    Z2 = K2 * p.n1 * p.n3 * cs
    up = lambda b: (b + 255) // 256 * 256
    assert info["workspace_bytes"] == up(max(U, G, Z2)) + up(max(V, Z1))
    beta = math.pi * 1.5 / (2 * 6)
    assert abs(info["beta"] - beta) < 1e-15
    k = math.pi * np.array([p.n1 / (p.n1 * p.d1), p.n2 / (p.n2 * p.d2), 1.0 / p.d3])
    assert abs(info["max_abs_theta"] - p.c * p.dt * np.linalg.norm(k)) < 1e-12
    assert (info["segments"], info["list_entries"]) == _expected_segments_and_entries(p, info)
    info64 = N.query(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), h=p.h, precision="fp64")
    assert info64["workspace_bytes"] == up(2 * max(U, G, Z2)) + up(2 * max(V, Z1))


def test_calls_without_plan_fail_cleanly():
    L = N.lib()
    assert L.nedner_execute(None, None, None, 0, None) == E_ARG
    assert L.nedner_execute_adjoint(None, None, 0, None, None) == E_ARG
    assert L.nedner_execute_q(None, None, None, None) == E_ARG
    assert L.nedner_execute_q_adjoint(None, None, None, None) == E_ARG
    assert L.nedner_mip(None, 2, 2, 2, 0, 0, None, None) == E_ARG
    assert L.nedner_corrcoef(None, None, None, 4, 0, None, None, 0, None) == E_ARG
    assert L.nedner_tenenbaum(None, 4, 4, 0, 4, 0, 4, 0, None, None, 0, None) == E_ARG
    assert L.nedner_metrics_workspace_size() >= 8 * (3 * 512 + 2)
    assert L.nedner_set_workspace(None, None, 0) == E_ARG
    sz = ctypes.c_size_t(0)
    assert L.nedner_workspace_size(None, ctypes.byref(sz)) == E_ARG
    assert L.nedner_destroy(None) == 0
    assert L.nedner_plan_create(None, 0, None, None) == E_ARG


def test_product_path_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(N, "_LIB", None)
    monkeypatch.setattr(N, "LIB_PATH", os.path.join(ROOT, "nonexistent", "libnedner.so"))
    with pytest.raises(N.NednerError):
        N.lib()


def test_plan_refuses_to_run_without_gpu():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = synth.config("c5sub")
    with pytest.raises(N.NednerError):
        N.Plan(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3))


def test_binding_struct_layout_matches_header():
    """Field order of the ctypes mirror equals the C struct declaration order."""
    text = open(HEADER).read()
    body = text[text.index("typedef struct {\n  int64_t m;"):text.index("} nedner_desc;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl or decl.startswith("typedef"):
            decl = decl.split("{", 1)[-1].strip()
            if not decl:
                continue
        names = decl.split(None, 1)[1] if " " in decl else ""
        for part in names.replace("*", " ").split(","):
            part = part.strip().split()[-1] if part.strip() else ""
            if part:
                fields.append(part)
    assert fields == [f for f, _ in N.desc_struct._fields_]


def test_batch_descriptor_checks_before_any_device_work():
    L = N.lib()
    d0, k0 = _desc()
    d1, k1 = _desc(precision="fp64")
    arr = (N.desc_struct * 2)(d0, d1)
    plan = ctypes.c_void_p()
    assert L.nedner_plan_create_many(arr, 2, 0, None, ctypes.byref(plan)) == E_ARG
    assert b"precision" in L.nedner_last_error()
    d2, k2 = _desc(w=8)
    arr = (N.desc_struct * 2)(d0, d2)
    assert L.nedner_plan_create_many(arr, 2, 0, None, ctypes.byref(plan)) == E_ARG
    assert L.nedner_plan_create_many(arr, 0, 0, None, ctypes.byref(plan)) == E_ARG
    assert L.nedner_execute_many(None, None, None, 0, None) == E_ARG
    t = N.tuning_struct()
    assert L.nedner_get_tuning(None, ctypes.byref(t)) == E_ARG
    assert L.nedner_set_tuning(None, ctypes.byref(t)) == E_ARG
    assert L.nedner_autotune(None, None, None, ctypes.byref(t)) == E_ARG


def test_injected_hip_error_needs_a_plan():
    L = N.lib()
    assert L.nedner_debug_inject_hip_error(None, 1) == E_ARG
