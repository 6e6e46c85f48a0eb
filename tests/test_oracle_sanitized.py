"""The oracle's C source under AddressSanitizer and UBSan (CPU): a second
build of the same file, loaded by a child process with the ASan runtime
preloaded, runs every entry point on small cases -- rendering, colour,
scoring in each mode, ICP, GICP, normals and the tree -- and must finish
without a report."""
import os
import subprocess
import sys
import textwrap

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SCRIPT = textwrap.dedent("""
    import sys
    sys.path.insert(0, {tests!r}); sys.path.insert(0, {root!r})
    import numpy as np
    import oracle
    from random_cases import random_case
    from test_oracle_icp import K_HI, _scene_and_gt, _yaw_shift
    from test_oracle_msg import DELTA, _world
    for seed in range(4):
        mesh, scene, poses, p = random_case(seed)
        for flags in (0, oracle.MARK_OCCLUDERS | (oracle.USE_RGB if p["rgb"] else 0), oracle.VOL_CYL,
                      oracle.JO_NN | oracle.MARK_OCCLUDERS):
            oracle.score(mesh, scene, poses[:4], delta_mm=p["delta"], tau_c=p["tau"], flags=flags,
                         stride=p["stride"], threads=2)
        oracle.score_detail(mesh, scene, poses[0], delta_mm=p["delta"], flags=oracle.MARK_OCCLUDERS)
    m, scene, gt = _scene_and_gt(1, K_HI)
    starts = np.stack([_yaw_shift(gt, 0.04, 3.0, -2.0)]).astype(np.float32)
    oracle.icp(m, scene, starts, delta_mm=5.0, flags=0, rho_mm=10.0, iterations=3, stride=2, dof=3, threads=2)
    oracle.icp(m, scene, starts, delta_mm=5.0, flags=0, rho_mm=10.0, iterations=3, stride=2, dof=6, threads=2)
    oracle.gicp(m, scene, starts, delta_mm=5.0, flags=0, rho_mm=10.0, iterations=3, stride=2, threads=2)
    oracle.normal_image(scene.depth, K_HI, 10)
    meshes, wscene, wgt, cands = _world()
    oracle.msg_search(wscene, [(meshes[o], o + 1, cands[o][:2]) for o in range(3)], beam=2, delta_mm=DELTA,
                      tau_c=20.0, flags=oracle.MARK_OCCLUDERS | oracle.USE_RGB, threads=2)
    print("sanitized oracle run ok")
""")


def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime for the host compiler")
    from oracle import build as oracle_build
    lib = oracle_build.build_sanitized(str(tmp_path / "liboracle_asan.so"))
    env = dict(os.environ, LD_PRELOAD=asan, PERCH_ORACLE_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(tests=HERE, root=ROOT)], env=env, capture_output=True,
                       text=True, timeout=600)
    report = r.stdout[-3000:] + r.stderr[-6000:]
    assert r.returncode == 0 and "sanitized oracle run ok" in r.stdout, report
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
