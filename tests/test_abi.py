"""The C-ABI library loads and exports every call declared in include/gid.h; the
binding's struct layouts match the header; argument errors are reported without
touching a GPU; default parameters are the paper's.  CPU only (no compute)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

import paper_1908_01961_amd as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gid.h")
GOLDEN = os.path.join(ROOT, "tests", "golden", "paper_parameters.txt")


def declared_calls():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gid_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_call():
    lib = G.load_library()
    names = declared_calls()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in G.SIGNATURES}
    assert set(names) == bound


def test_struct_layout_matches_header():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "gid.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(gid_params), sizeof(gid_frame_stats),
         offsetof(gid_params, chroma_gate), offsetof(gid_params, use_graph),
         offsetof(gid_frame_stats, n_half));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == ctypes.sizeof(G.GidParams)
    assert vals[1] == ctypes.sizeof(G.GidFrameStats)
    assert vals[2] == G.GidParams.chroma_gate.offset
    assert vals[3] == G.GidParams.use_graph.offset
    assert vals[4] == G.GidFrameStats.n_half.offset


def test_default_params_are_the_papers():
    p = G.default_params(6)
    want = {}
    for line in open(GOLDEN):
        f = line.split("#")[0].split()
        if f:
            want[f[0]] = float(f[1])
    lam = p.lambda_
    assert lam.data == want["lam_data"] and lam.cluster == want["lam_cluster"]
    assert lam.r_sparsity == want["lam_rsparsity"] and lam.p == want["p"]
    assert lam.r_consistency == want["lam_rconsistency"] and lam.monochrome == want["lam_mono"]
    assert lam.i_sparsity == want["lam_isparsity"] and lam.smoothness == want["lam_smooth"]
    assert lam.non_neg == want["lam_nonneg"] and lam.ir == want["lam_ir"] and lam.cr == want["lam_cr"]
    assert p.eps_nonneg == pytest.approx(want["eps_nonneg"]) and p.retinex_k == want["retinex_k"]
    assert p.struct_size == ctypes.sizeof(G.GidParams)


def test_argument_errors_without_gpu():
    lib = G.load_library()
    p = G.GidParams()
    assert lib.gid_default_params(0, ctypes.byref(p)) == 1
    assert lib.gid_default_params(17, ctypes.byref(p)) == 1
    assert lib.gid_default_params(4, None) == 1
    assert lib.gid_default_params(4, ctypes.byref(p)) == 0
    h = ctypes.c_void_p()
    bad = G.default_params(4)
    bad.struct_size = 4
    assert lib.gid_create(ctypes.byref(bad), 64, 48, None, ctypes.byref(h)) == 1
    good = G.default_params(4)
    assert lib.gid_create(ctypes.byref(good), 1, 48, None, ctypes.byref(h)) == 1
    assert lib.gid_create(ctypes.byref(good), 64, 48, None, None) == 1
    g2 = G.default_params(4, gn_iters=0)
    assert lib.gid_create(ctypes.byref(g2), 64, 48, None, ctypes.byref(h)) == 1
    assert lib.gid_destroy(None) == 0
    for call in ("gid_synchronize", "gid_reset_clip", "gid_layer_step"):
        assert getattr(lib, call)(None, *([None] if call == "gid_layer_step" else [])) == 1
    assert lib.gid_status_string(4) == b"non-finite value"
    assert lib.gid_last_error(None) == b"no context"


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1908_01961_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower().replace("oracles", ""), f
