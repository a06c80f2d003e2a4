"""The C ABI without a GPU: the library loads, exports every declared entry
point, and its host-side argument validation returns the documented codes."""
import ctypes as C
import glob
import os
import re
import subprocess

import numpy as np
import pytest

from conftest import ROOT

INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(INCLUDE, "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(tpc_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("tpc_track_event", "tpc_ctx_create", "tpc_ctx_destroy", "tpc_params_default",
                 "tpc_last_error", "tpc_validate"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1712_09407_amd import tpc
    out = subprocess.run(["nm", "-D", "--defined-only", tpc.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (tpc_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        getattr(tpc.lib, n)          # resolvable through ctypes as well
    assert set(tpc.EXPORTS) <= exported


def test_library_is_built_for_gfx950():
    from paper_1712_09407_amd import tpc
    out = subprocess.run(["strings", tpc.LIB_PATH], capture_output=True, text=True).stdout
    assert "gfx950" in out


def test_default_params_match_the_paper():
    from paper_1712_09407_amd import tpc
    p = tpc.default_params()
    assert p.alpha == 6.0 and p.min_clusters == 30
    assert p.max_tracklets == 0


def _valid_host_structs():
    from paper_1712_09407_amd import synth, tpc
    geo = tpc.make_geometry(synth.ROW_X, synth.TAN_HALF, synth.Z_MAX)
    # validation never dereferences device pointers: any non-null value will do
    ev = tpc.Event(36, 0x1000, 1000, 0x2000, 0x3000, 0x4000)
    return tpc, geo, ev


def test_validation_accepts_a_valid_call():
    tpc, geo, ev = _valid_host_structs()
    assert tpc.validate(ev, geo) == tpc.TPC_OK


@pytest.mark.parametrize("case", [
    "rows_small", "rows_big", "rows_not_increasing", "sectors_zero", "clusters_negative",
    "y_null", "offsets_null", "sigma_zero", "gate_zero", "sinphi_one", "beta_zero",
    "min_clusters_small", "seed_len_one", "seed_window_one", "min_pt_zero", "prior_zero", "nan_window",
    "tan_half_zero", "max_tracklets_negative"])
def test_validation_rejects(case):
    tpc, geo, ev = _valid_host_structs()
    p = tpc.default_params()
    if case == "rows_small":
        geo.n_rows = 2
    elif case == "rows_big":
        geo = tpc.make_geometry(np.arange(1, 200, dtype=np.float32), 0.17, 250)
    elif case == "rows_not_increasing":
        rx = np.arange(100, 259, dtype=np.float32)
        rx[50] = rx[49]
        geo = tpc.make_geometry(rx, 0.17, 250)
    elif case == "sectors_zero":
        ev.n_sectors = 0
    elif case == "clusters_negative":
        ev.n_clusters = -1
    elif case == "y_null":
        ev.y = None
    elif case == "offsets_null":
        ev.row_offsets = None
    elif case == "sigma_zero":
        p.sigma_y = 0.0
    elif case == "gate_zero":
        p.chi2_gate = 0.0
    elif case == "sinphi_one":
        p.max_sinphi = 1.0
    elif case == "beta_zero":
        p.beta = 0.0
    elif case == "min_clusters_small":
        p.min_clusters = 2
    elif case == "seed_len_one":
        p.min_seed_len = 1
    elif case == "seed_window_one":
        p.seed_window = 1
    elif case == "min_pt_zero":
        p.min_pt = 0.0
    elif case == "prior_zero":
        p.prior_qpt = 0.0
    elif case == "nan_window":
        p.nf_win_z = float("nan")
    elif case == "tan_half_zero":
        geo.tan_half_angle = 0.0
    elif case == "max_tracklets_negative":
        p.max_tracklets = -5
    assert tpc.validate(ev, geo, p) == tpc.TPC_ERR_INVALID_ARG
    assert tpc.last_error() != ""


def test_empty_event_is_valid():
    tpc, geo, ev = _valid_host_structs()
    ev.n_clusters = 0
    ev.y = None
    ev.z = None
    assert tpc.validate(ev, geo) == tpc.TPC_OK


def test_null_context_is_an_error_not_a_crash():
    tpc, geo, ev = _valid_host_structs()
    nt, nc = C.c_int32(0), C.c_int32(0)
    tr = tpc.Tracks(0, 0, C.pointer(nt), C.pointer(nc), None, None, None, None)
    rc = tpc.lib.tpc_track_event(None, C.byref(ev), C.byref(geo), 0.5,
                                 C.byref(tpc.default_params()), C.byref(tr), None)
    assert rc == tpc.TPC_ERR_INVALID_ARG


def test_global_entry_rejects_null_arguments():
    tpc, geo, ev = _valid_host_structs()
    nt, nc = C.c_int32(0), C.c_int32(0)
    tr = tpc.Tracks(0, 0, C.pointer(nt), C.pointer(nc), None, None, None, None)
    n, m = C.c_int32(0), C.c_int32(0)
    pr = tpc.Prolongations(0, 0, C.pointer(n), C.pointer(m), None, None, None)
    rc = tpc.lib.tpc_track_event_global(None, C.byref(ev), C.byref(geo), 0.5,
                                        C.byref(tpc.default_params()), C.byref(tr), C.byref(pr),
                                        None)
    assert rc == tpc.TPC_ERR_INVALID_ARG


def test_oracle_library_exports(orc):
    out = subprocess.run(["nm", "-D", "--defined-only", orc.LIB], capture_output=True, text=True,
                         check=True).stdout
    hdr = open(os.path.join(ROOT, "oracle", "tpc_oracle.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    for name in set(re.findall(r"\b(orc_\w+)\s*\(", hdr)):
        assert f" T {name}" in out, name


def test_oracle_and_gpu_library_share_nothing():
    """The oracle is independent of the HIP path: no shared sources or headers."""
    import oracle
    from paper_1712_09407_amd import build
    osrc = open(os.path.join(ROOT, "oracle", "tpc_oracle.c")).read()
    assert "tpc_track.h" not in osrc and "tpc_internal.h" not in osrc
    for s in build.SOURCES:
        src = open(os.path.join(build.CSRC, s)).read()
        assert "tpc_oracle" not in src and "oracle/" not in src
    psrc = open(os.path.join(ROOT, "paper_1712_09407_amd", "tpc.py")).read()
    assert "import oracle" not in psrc and "from oracle" not in psrc


STRUCTS = {  # C type name -> ctypes mirror in the binding
    "tpc_geometry": "Geometry", "tpc_event": "Event", "tpc_params": "Params",
    "tpc_tracks": "Tracks", "tpc_tuning": "Tuning", "tpc_server_config": "ServerConfig",
    "tpc_server_done": "ServerDone", "tpc_prolongations": "Prolongations",
    "tpc_merged": "Merged"}


def test_struct_layouts_match_the_header(tmp_path):
    """The Python binding's ctypes structs have the header's sizes and field
    offsets (a C program built from include/tpc_track.h prints them)."""
    from paper_1712_09407_amd import tpc
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "tpc_track.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in getattr(tpc, pyname)._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", INCLUDE, str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, pyname in STRUCTS.items():
        cls = getattr(tpc, pyname)
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU: --gpus above 1 exits with a message."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "single GPU" in r.stderr
