"""Seeded random cases against the oracle: small procedural meshes, random
intrinsics, image sizes, delta, tau_c, flags and strides, an occluded scene
with sensor noise, and candidate poses spread around the true one.  L, Q and
every depth-only count are bit-exact; counts with the colour term are within
0.1 % of the points per pose."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2008_00326_amd as pk  # noqa: E402
from random_cases import random_case  # noqa: E402

CASES = 24


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pk.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("seed", range(CASES))
def test_random_case_matches_oracle(ctx, seed):
    mesh, scene, poses, p = random_case(seed)
    say(f"case {seed}: image {scene.K[0]}x{scene.K[1]}, {mesh.tri.shape[0]} tris, {p}")
    sid = ctx.set_scene(scene.K, scene.depth, scene.rgb, delta_mm=p["delta"], tau_c=p["tau"], use_rgb=p["rgb"],
                        mark_occluders=p["occl"], stride=p["stride"])
    mid = ctx.load_mesh(mesh.xyz, mesh.tri, mesh.rgb)
    t = torch.from_numpy(poses).cuda()
    jr, jo, nr, nq = ctx.score_poses(sid, mid, t)
    torch.cuda.synchronize()
    got = [a.cpu().numpy() for a in (jr, jo, nr, nq)]
    ctx.drop_scene(sid)
    ctx.unload_mesh(mid)
    flags = (oracle.USE_RGB if p["rgb"] else 0) | (oracle.MARK_OCCLUDERS if p["occl"] else 0)
    exp = oracle.score(mesh, scene, poses, delta_mm=p["delta"], tau_c=p["tau"], flags=flags, stride=p["stride"],
                       threads=8)
    assert np.array_equal(got[2], exp[2]), f"L differs at {np.flatnonzero(got[2] != exp[2])[:8]}"
    assert np.array_equal(got[3], exp[3]), f"Q differs at {np.flatnonzero(got[3] != exp[3])[:8]}"
    if p["rgb"]:
        assert np.all(np.abs(got[0] - exp[0]) <= np.ceil(0.001 * exp[2]))
        assert np.all(np.abs(got[1] - exp[1]) <= np.ceil(0.001 * exp[3]))
    else:
        assert np.array_equal(got[0], exp[0]) and np.array_equal(got[1], exp[1])
    assert exp[2].sum() > 0    # the cases render something
