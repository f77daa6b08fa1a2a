"""Host-side tests of the HIP library (no GPU): symbols, argument handling and
the nested-dissection / supernodal analysis."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from paper_2306_06946_amd import icr
from paper_2306_06946_amd.scenes import make_scene

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "icr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(icr_[a-z_A-Z0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = icr.lib()
    names = _declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_binding_covers_the_header():
    assert set(_declared_symbols()) == set(icr._SIGS)


def _true_fill(perm, nodes, tets):
    """Node-level structure of L for P A P^T by symbolic elimination (sets)."""
    N = len(nodes)
    iperm = np.empty(N, dtype=np.int64)
    iperm[perm] = np.arange(N)
    adj = [set() for _ in range(N)]
    for t in tets:
        p = iperm[t]
        for a in p:
            for b in p:
                if a != b:
                    adj[a].add(b)
    struct = [None] * N
    children = [[] for _ in range(N)]
    for j in range(N):
        s = {i for i in adj[j] if i > j}
        for c in children[j]:
            s |= struct[c]
        s.discard(j)
        struct[j] = s
        if s:
            children[min(s)].append(j)
        struct[j] = s
    return struct


@pytest.mark.parametrize("cfg", ["tiny", "medium"])
def test_supernodal_structure_contains_true_fill(cfg):
    sc = make_scene(cfg, 0)
    a = icr.analyze(sc["nodes"], sc["tets"])
    perm, sup, rp, rows = a["perm"], a["sup"], a["rows_ptr"], a["rows"]
    N = len(sc["nodes"])
    assert np.array_equal(np.sort(perm), np.arange(N))
    # supernodes tile the permuted order, parents come after children
    col0, ncol, parent, first = sup[:, 0], sup[:, 1], sup[:, 2], sup[:, 3]
    assert col0[0] == 0 and np.all(col0[1:] == col0[:-1] + ncol[:-1]) and col0[-1] + ncol[-1] == N
    assert np.all((parent == -1) | (parent > np.arange(len(sup))))
    owner = np.repeat(np.arange(len(sup)), ncol)
    fill = _true_fill(perm, sc["nodes"], sc["tets"])
    for j in range(N):
        s = owner[j]
        allowed = set(range(j + 1, col0[s] + ncol[s])) | set(rows[rp[s]:rp[s + 1]].tolist())
        assert fill[j] <= allowed, (j, s)


def test_analyze_rejects_bad_ids():
    L = icr.lib()
    nodes = np.zeros((4, 3))
    tets = np.array([[0, 1, 2, 9]], dtype=np.int32)
    perm = np.zeros(4, dtype=np.int32)
    st = L.icr_analyze(nodes.ctypes.data_as(ctypes.c_void_p), 4, tets.ctypes.data_as(ctypes.c_void_p), 1,
                       perm.ctypes.data_as(ctypes.c_void_p), None, 0, None, None, 0, None, None)
    assert st == icr.E_ARG


def test_null_scene_is_rejected():
    L = icr.lib()
    assert L.icr_factor(None) == icr.E_ARG
    assert L.icr_last_error(None) == b"null scene"


def test_analysis_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The host analysis (graph, nested dissection, supernodal structure,
    consistency check) built with -fsanitize=address,undefined and run on the
    tiny and medium meshes and on two stacked bodies (two components)."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    from paper_2306_06946_amd.scenes import stacked_grids
    exe = str(tmp_path / "analysis_check")
    csrc = os.path.join(ROOT, "paper_2306_06946_amd", "csrc")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(csrc, "analysis.cpp"), os.path.join(ROOT, "tests", "host", "analysis_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    meshes = [make_scene("tiny", 0), make_scene("medium", 0)]
    nodes, tets, _, _, _ = stacked_grids(6, 5, 4, 3, 0.01, 0.2, np.random.default_rng(3))
    meshes.append(dict(nodes=nodes, tets=tets))
    for k, sc in enumerate(meshes):
        path = tmp_path / f"mesh{k}.bin"
        with open(path, "wb") as f:
            f.write(np.array([len(sc["nodes"]), len(sc["tets"])], dtype=np.int32).tobytes())
            f.write(np.ascontiguousarray(sc["nodes"], dtype=np.float64).tobytes())
            f.write(np.ascontiguousarray(sc["tets"], dtype=np.int32).tobytes())
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe, str(path)], capture_output=True, text=True, env=env)
        assert r.returncode == 0 and r.stdout.startswith("ok "), (r.stdout, r.stderr[-2000:])
        a = icr.analyze(sc["nodes"], sc["tets"])
        assert r.stdout.split()[1:] == [str(len(a["sup"])), str(len(a["rows"]))]
