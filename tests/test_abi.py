"""The C interface: the library loads, exports every function the header
declares, the ctypes mirror matches the C struct layouts, and host-side
argument checks behave as documented (no GPU work is launched here)."""
import ctypes as ct
import os
import re
import subprocess

import pytest

from paper_2008_13461_amd import _abi as A
from synth import config as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pixeltrack.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z_]+)\s*\(", text)))


def test_header_functions_are_exported():
    L = A.load()
    names = _declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
        assert n in A.SIGNATURES, f"{n} has no ctypes signature"


def test_abi_version():
    assert A.load().pt_abi_version() == A.PT_ABI_VERSION


_STRUCTS = {
    "pt_config": ["bfield", "n_pairs", "pair_inner", "pair_dphi", "pt_min", "cut_mask", "ca_rmax_other",
                  "root_always_mask", "min_hits", "layer_barrel", "x_over_x0", "p_cap", "n_modules", "n_phi_bins",
                  "block_links", "f64_solve_threshold", "vtx_min_hits", "vtx_kmeans_iter", "vtx_pt_min",
                  "vtx_pt_cap", "fishbone_theta", "exclusive_hits"],
    "pt_hits": ["n_hits", "n_events", "event_offsets", "dtype", "x", "layer", "module"],
    "pt_workspace": ["ptr", "bytes"],
    "pt_cells": ["cap", "inner", "pair", "count", "inner_first", "inner_count"],
    "pt_links": ["cap", "in_cell", "count", "out_start", "out_count", "has_inner"],
    "pt_ntuplets": ["cap", "hits", "n", "count_raw", "kept", "count"],
    "pt_tracks": ["cap", "params", "chi2", "status", "cov"],
    "pt_vertices": ["cap", "z", "var", "chi2", "ndf", "n_tracks", "sum_pt2", "event_first", "count", "track_vertex"],
}


def test_struct_layouts_match_the_header(tmp_path):
    src = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for s, fields in _STRUCTS.items():
        src.append(f'  printf("{s} size %zu\\n", sizeof({s}));')
        for f in fields:
            src.append(f'  printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    src += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(c)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in out:
        if not line:
            continue
        key, val = line.rsplit(" ", 1)
        val = int(val)
        if key.endswith(" size"):
            s = key.split()[0]
            assert ct.sizeof(getattr(A, s)) == val, key
        else:
            s, f = key.split(".")
            assert getattr(getattr(A, s), f).offset == val, key


def test_workspace_size_and_config_checks():
    L = A.load()
    cfg = A.make_config(C.default_config())
    n = L.pt_workspace_size(ct.byref(cfg), 100_000, 4, 1_000_000, 250_000, 100_000)
    assert n > 100_000 * 32
    # invalid settings are rejected without touching the device
    bad = A.make_config(C.default_config(min_hits=2))
    assert L.pt_workspace_size(ct.byref(bad), 10, 1, 10, 10, 10) == 0
    bad = A.make_config(C.default_config(pt_min=0.0))
    assert L.pt_workspace_size(ct.byref(bad), 10, 1, 10, 10, 10) == 0
    bad = A.make_config(C.default_config(max_hits=9))
    assert L.pt_workspace_size(ct.byref(bad), 10, 1, 10, 10, 10) == 0
    assert L.pt_workspace_size(None, 10, 1, 10, 10, 10) == 0
    assert L.pt_workspace_size(ct.byref(cfg), -1, 1, 10, 10, 10) == 0


def test_argument_errors_are_synchronous():
    L = A.load()
    cfg = A.make_config(C.default_config())
    ws = A.pt_workspace()
    cells = A.pt_cells()
    hits = A.pt_hits()
    hits.n_hits = 10
    hits.n_events = 1
    hits.dtype = 7                      # not a valid dtype
    assert L.pt_build_doublets(ct.byref(hits), ct.byref(cfg), ct.byref(cells), None, ws, None) == A.PT_ERR_ARG
    assert L.pt_build_doublets(None, ct.byref(cfg), ct.byref(cells), None, ws, None) == A.PT_ERR_ARG
    t = A.pt_ntuplets()
    tr = A.pt_tracks()
    assert L.pt_fit_broken_line(ct.byref(hits), ct.byref(cfg), ct.byref(t), None, 9, ct.byref(tr), None, ws,
                                None) == A.PT_ERR_ARG
    assert L.pt_err_string(A.PT_ERR_WORKSPACE).decode().startswith("workspace")
    # argument errors leave no device error behind
    assert L.pt_last_device_error() == b""


def test_python_package_fails_loudly_without_library(tmp_path):
    with pytest.raises(A.LibraryMissing):
        A._lib, saved = None, A._lib
        try:
            A.load(str(tmp_path / "missing.so"))
        finally:
            A._lib = saved
