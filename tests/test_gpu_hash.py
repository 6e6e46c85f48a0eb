"""The uniform-grid voxel hash search (PERCH_HASH) against the neighbour
table and the oracle.

The hash changes how J_r finds each rendered point's nearest observed point
(Eq. 2, Eq. 4), not what it finds: every output must equal the table's bit
for bit -- on every pose of the 640x480 RGB workload and of the 6-DoF
workload, through the tree's successor scoring, in every scoring mode on
seeded random cases -- and the oracle's on a sample, while the scene holds no
table.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2008_00326_amd as pk  # noqa: E402
from paper_2008_00326_amd.workloads import make_config  # noqa: E402
from random_cases import random_case  # noqa: E402

THREADS = 0


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


def score_all(ctx, w, search):
    w.search = search
    sid, mids = pk.load_workload(ctx, w)
    info = ctx.scene_info(sid)
    items = []
    for o in w.objects:
        p = torch.from_numpy(np.ascontiguousarray(o.poses)).cuda()
        n = p.shape[0]
        items.append({"scene": sid, "mesh": mids[o.mesh], "label": o.label, "poses": p,
                      "nr": torch.empty(n, dtype=torch.int32, device="cuda"),
                      "nq": torch.empty(n, dtype=torch.int32, device="cuda")})
    out = ctx.score_batch(items)
    torch.cuda.synchronize()
    got = [tuple(it[k].cpu().numpy() for k in ("jr", "jo", "nr", "nq")) for it in out]
    return sid, mids, info, got


@pytest.mark.parametrize("cfg", [2, 3])
def test_hash_equals_table_every_pose(ctx, cfg):
    w = make_config(cfg, 0)
    say(f"voxel hash vs table, config {cfg}")
    sid_t, mids_t, info_t, ref = score_all(ctx, w, "table")
    sid_h, mids_h, info_h, got = score_all(ctx, w, "hash")
    assert info_h["table_entries"] == 0 and info_t["table_entries"] > 0
    assert info_h["device_bytes"] < info_t["device_bytes"] / 3
    say(f"  scene memory: table {info_t['device_bytes'] / 2**20:.1f} MB, hash {info_h['device_bytes'] / 2**20:.1f} MB")
    for k, (a, b) in enumerate(zip(ref, got)):
        for name, x, y in zip(("J_r", "J_o", "L", "Q"), a, b):
            assert np.array_equal(x, y), f"object {k}: {name} differs at {np.flatnonzero(x != y)[:8]}"
    # and against the oracle on a sample
    rng = np.random.default_rng(cfg)
    for k, o in enumerate(w.objects[:3]):
        sel = np.unique(np.concatenate([rng.choice(o.poses.shape[0], 6, replace=False),
                                        np.argsort(np.abs(o.poses - o.gt_pose).sum(1))[:2]]))
        exp = oracle.score(w.meshes[o.mesh], w.scene, o.poses[sel], delta_mm=w.delta_mm, tau_c=w.tau_c,
                           flags=oracle.USE_RGB | oracle.MARK_OCCLUDERS, label=o.label, threads=THREADS,
                           search="window")
        g = [x[sel] for x in got[k]]
        assert np.array_equal(g[2], exp[2]) and np.array_equal(g[3], exp[3])
        assert np.all(np.abs(g[0] - exp[0]) <= np.ceil(0.001 * exp[2]))
        assert np.all(np.abs(g[1] - exp[1]) <= np.ceil(0.001 * exp[3]))
    for sid, mids in ((sid_t, mids_t), (sid_h, mids_h)):
        ctx.drop_scene(sid)
        for m in mids:
            ctx.unload_mesh(m)


@pytest.mark.parametrize("seed", range(8))
def test_hash_random_cases_against_the_oracle(ctx, seed):
    mesh, scene, poses, p = random_case(seed)
    jo = "nn" if seed % 3 == 2 else "exact"
    volume = "cyl" if seed % 4 == 1 else "aabb"
    say(f"voxel hash, random case {seed} ({p}, jo={jo}, volume={volume})")
    sid = ctx.set_scene(scene.K, scene.depth, scene.rgb, delta_mm=p["delta"], tau_c=p["tau"], use_rgb=p["rgb"],
                        mark_occluders=p["occl"], stride=p["stride"], search="hash", jo=jo, volume=volume)
    mid = ctx.load_mesh(mesh.xyz, mesh.tri, mesh.rgb if p["rgb"] else None)
    t = torch.from_numpy(poses).cuda()
    got = [x.cpu().numpy() for x in ctx.score_poses(sid, mid, t)]
    flags = (oracle.USE_RGB if p["rgb"] else 0) | (oracle.MARK_OCCLUDERS if p["occl"] else 0)
    flags |= (oracle.JO_NN if jo == "nn" else 0) | (oracle.VOL_CYL if volume == "cyl" else 0)
    exp = oracle.score(mesh, scene, poses, delta_mm=p["delta"], tau_c=p["tau"], flags=flags, stride=p["stride"],
                       threads=THREADS)
    assert np.array_equal(got[2], exp[2]) and np.array_equal(got[3], exp[3])
    if p["rgb"]:
        tol_o = np.ceil(0.001 * exp[3]) + (np.ceil(0.001 * exp[2]) if jo == "nn" else 0)
        assert np.all(np.abs(got[0] - exp[0]) <= np.ceil(0.001 * exp[2]))
        assert np.all(np.abs(got[1] - exp[1]) <= tol_o)
    else:
        assert np.array_equal(got[0], exp[0]) and np.array_equal(got[1], exp[1])
    ctx.drop_scene(sid)
    ctx.unload_mesh(mid)


def test_hash_tree_successors_equal_table(ctx):
    w = make_config(2, 0)
    w.volume = "label"
    say("voxel hash in the tree's successor scoring")
    outs = []
    for search in ("table", "hash"):
        w.search = search
        sid, mids = pk.load_workload(ctx, w)
        a, b = w.objects[0], w.objects[1]
        state = [(mids[a.mesh], a.label, a.gt_pose)]
        t = torch.from_numpy(np.ascontiguousarray(b.poses[::16])).cuda()
        r = ctx.msg_expand(sid, state, mids[b.mesh], t, label=b.label)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in r if x is not None])
        ctx.drop_scene(sid)
        for m in mids:
            ctx.unload_mesh(m)
    for x, y in zip(*outs):
        assert np.array_equal(x, y)


def test_hash_flag_combinations_refused(ctx):
    K = (64, 48, 50.0, 50.0, 32.0, 24.0)
    d = np.full((48, 64), 800, np.uint16)
    for other in ("knn1", "knn2"):
        flags = pk.HASH | (pk.KNN1 if other == "knn1" else pk.KNN2) | pk.MARK_OCCLUDERS
        with pytest.raises(pk.PerchError) as e:
            ctx.set_scene(K, d, delta_mm=10.0, flags=flags)
        assert e.value.status == -1
