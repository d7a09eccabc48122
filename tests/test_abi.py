"""The C-ABI library loads and exports every entry point include/imloc.h
declares; the ctypes structures of the binding match the C layout (checked
against a probe compiled by gcc from the header); host-side argument checks
reject bad calls without touching a device."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "imloc.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(imloc_\w+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2601_04185_amd as pk
    L = C.CDLL(pk.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(L, nm), nm
    assert sorted(pk.EXPORTED) == names


def test_struct_layout_matches_header(tmp_path):
    import paper_2601_04185_amd as pk
    src = tmp_path / "probe.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "imloc.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(imloc_ransac_params), sizeof(imloc_stats), sizeof(imloc_camera),
         sizeof(imloc_pose), sizeof(imloc_corr), sizeof(imloc_corr_out), sizeof(imloc_matches));
  printf("%zu %zu %zu %zu %zu\n", offsetof(imloc_ransac_params, precision), offsetof(imloc_ransac_params, seed),
         offsetof(imloc_stats, score_launches), offsetof(imloc_stats, ms_total), sizeof(imloc_server_config));
  printf("%zu %zu %zu\n", sizeof(imloc_dense_matches), sizeof(imloc_triangulation_params),
         offsetof(imloc_triangulation_params, max_refine_iters));
  printf("%zu %zu\n", sizeof(imloc_rig_camera), offsetof(imloc_rig_camera, cam_from_rig));
  return 0;
}
''')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    got = [int(x) for x in out]
    want = [C.sizeof(pk.RansacParams), C.sizeof(pk.Stats), C.sizeof(pk.Camera), C.sizeof(pk.Pose),
            C.sizeof(pk.Corr), C.sizeof(pk.CorrOut), C.sizeof(pk.Matches),
            pk.RansacParams.precision.offset, pk.RansacParams.seed.offset, pk.Stats.score_launches.offset,
            pk.Stats.ms_total.offset, C.sizeof(pk.ServerConfig), C.sizeof(pk.DenseMatches),
            C.sizeof(pk.TriangulationParams), pk.TriangulationParams.max_refine_iters.offset,
            C.sizeof(pk.RigCamera), pk.RigCamera.cam_from_rig.offset]
    assert got == want


def test_host_side_checks_without_device():
    import paper_2601_04185_amd as pk
    L = pk.lib()
    p = pk.make_params(threshold_px=4.0, fixed_samples=1024)
    # null context
    assert L.imloc_lo_ransac_pnp(None, None, 0, None, C.byref(p), None, None, None) == pk.IMLOC_EINVAL
    assert L.imloc_score(None, None, 0, None, None, 0, 4.0, 0, None, None) == pk.IMLOC_EINVAL
    assert L.imloc_set_workspace(None, None, 0) == pk.IMLOC_EINVAL
    # workspace sizing is host arithmetic
    b1 = L.imloc_workspace_bytes(2000, C.byref(p))
    b2 = L.imloc_workspace_bytes(50000, C.byref(p))
    assert 0 < b1 < b2
    big = pk.make_params(threshold_px=6.0, fixed_samples=10000, batch=10000)
    assert L.imloc_workspace_bytes(50000, C.byref(big)) > b2
    assert L.imloc_score_workspace_bytes(1000, 10, 0) > 0
    assert L.imloc_lift_workspace_bytes(160000, 20) > 0
    ns = (C.c_int64 * 3)(100, 5000, 200)
    assert L.imloc_batch_workspace_bytes(3, ns, C.byref(p), 1) >= L.imloc_workspace_bytes(5000, C.byref(p))
    assert L.imloc_sample_workspace_bytes(2000, 1024) > 0
    cfg = pk.ServerConfig(64, 8, 200000, 64 * 4096, 64 * 200256)
    assert L.imloc_server_workspace_bytes(C.byref(cfg)) > 0
    bad = pk.ServerConfig(0, 8, 200000, 64 * 4096, 64 * 200256)
    assert L.imloc_server_workspace_bytes(C.byref(bad)) == 0
    # mapping depth: the view table plus a 16-byte refinement-queue entry per pixel
    t1 = L.imloc_triangulate_workspace_bytes(480, 640, 10)
    assert t1 >= 16 * 480 * 640 + 11 * 16 * 8
    assert L.imloc_triangulate_workspace_bytes(480, 640, 32) > t1
    assert L.imloc_triangulate_workspace_bytes(960, 640, 10) > t1
    assert L.imloc_triangulate_workspace_bytes(0, 640, 10) < t1


def test_paper_params():
    """imloc_paper_params fills the settings Sec. 3.3 "Pose Estimation" gives:
    batches of 1,000, scoring subsample of at most 10,000, stop at a 1e-4
    chance of having missed the best model or 100,000 samples, local
    optimisation of a new best (top 1), Cauchy refinement over the full set."""
    import paper_2601_04185_amd as pk
    p = pk.paper_params(6.0)
    assert p.threshold_px == 6.0 and p.fixed_samples == 0
    assert p.batch == 1000 and p.min_iters == 1000 and p.max_iters == 100000
    assert abs((1.0 - p.confidence) - 1e-4) < 1e-15
    assert p.max_score_points == 10000 and p.lo_top_k == 1
    assert p.final_iters > 0 and p.cauchy_scale_px == 3.0 and p.exhaustive == 0
    assert pk.paper_params(4.0, seed=7).seed == 7
    L = pk.lib()
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        assert L.imloc_paper_params(bad, C.byref(pk.RansacParams())) == pk.IMLOC_EINVAL
    assert L.imloc_paper_params(4.0, None) == pk.IMLOC_EINVAL
    with pytest.raises(TypeError):
        pk.paper_params(4.0, no_such_field=1)
