"""GPU parity of the paper-faithful variants against the oracle: the
inscribed-cylinder volume V(O) (Table I's conservative volume), J_o by
nearest-neighbour marking and the kNN II search (Sec. IV-A, parallel cost
computation).

L, Q and every depth-only count are bit-exact.  With the colour term, J_r is
within ceil(0.001 L) as elsewhere; under nearest-neighbour marking an
inlier's colour decision also decides whether its neighbour is marked, so
J_o is within ceil(0.001 Q) + ceil(0.001 L).
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
from tiny_meshes import TScene  # noqa: E402

THREADS = 16
VARIANTS = {"cyl": ("cyl", "exact"), "nn": ("aabb", "nn"), "cyl+nn": ("cyl", "nn")}


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


def oflags(rgb, occl, volume, jo):
    f = (oracle.USE_RGB if rgb else 0) | (oracle.MARK_OCCLUDERS if occl else 0)
    f |= {"aabb": oracle.VOL_AABB, "cyl": oracle.VOL_CYL}[volume]
    return f | (oracle.JO_NN if jo == "nn" else 0)


def gpu_score(ctx, sid, mid, poses, label=0):
    t = torch.from_numpy(np.ascontiguousarray(poses, np.float32)).cuda()
    jr, jo, nr, nq = ctx.score_poses(sid, mid, t, label=label)
    torch.cuda.synchronize()
    return jr.cpu().numpy(), jo.cpu().numpy(), nr.cpu().numpy(), nq.cpu().numpy()


def check(got, exp, rgb, jo_mode, what):
    jr, jo, nr, nq = got
    ejr, ejo, enr, enq = exp
    assert np.array_equal(nr, enr), f"{what}: L differs at {np.flatnonzero(nr != enr)[:8]}"
    assert np.array_equal(nq, enq), f"{what}: Q differs at {np.flatnonzero(nq != enq)[:8]}"
    if not rgb:
        assert np.array_equal(jr, ejr), f"{what}: J_r differs at {np.flatnonzero(jr != ejr)[:8]}"
        assert np.array_equal(jo, ejo), f"{what}: J_o differs at {np.flatnonzero(jo != ejo)[:8]}"
        return
    tol_r = np.ceil(0.001 * enr).astype(int)
    tol_o = np.ceil(0.001 * enq).astype(int) + (tol_r if jo_mode == "nn" else 0)
    assert np.all(np.abs(jr - ejr) <= tol_r), f"{what}: J_r beyond tolerance {np.abs(jr - ejr).max()}"
    assert np.all(np.abs(jo - ejo) <= tol_o), f"{what}: J_o beyond tolerance {np.abs(jo - ejo).max()}"


@pytest.mark.parametrize("seed", range(12))
def test_random_case_variants(ctx, seed):
    mesh, scene, poses, p = random_case(seed)
    mid = ctx.load_mesh(mesh.xyz, mesh.tri, mesh.rgb)
    t = torch.from_numpy(poses).cuda()
    for name, (volume, jo) in VARIANTS.items():
        say(f"case {seed} {name}: image {scene.K[0]}x{scene.K[1]}, {mesh.tri.shape[0]} tris, {p}")
        sid = ctx.set_scene(scene.K, scene.depth, scene.rgb, delta_mm=p["delta"], tau_c=p["tau"], use_rgb=p["rgb"],
                            mark_occluders=p["occl"], stride=p["stride"], volume=volume, jo=jo)
        got = [a.cpu().numpy() for a in ctx.score_poses(sid, mid, t)]
        torch.cuda.synchronize()
        ctx.drop_scene(sid)
        exp = oracle.score(mesh, scene, poses, delta_mm=p["delta"], tau_c=p["tau"],
                           flags=oflags(p["rgb"], p["occl"], volume, jo), stride=p["stride"], threads=THREADS)
        check(got, exp, p["rgb"], jo, f"case {seed} {name}")
        assert exp[2].sum() > 0
    ctx.unload_mesh(mid)


@pytest.mark.parametrize("variant", ["cyl", "nn", "cyl+nn"])
def test_cfg2_full_size_variant(ctx, variant):
    """All 32,000 cfg2 poses (640x480, RGB) under the variant, in the launch
    shape of the benchmark; the oracle checks two poses of every footprint
    class and the true pose of every object.  J_r is that of the exact test;
    the cylinder lies inside the box."""
    volume, jo = VARIANTS[variant]
    w = make_config(2, 0)
    say(f"cfg2 full size {variant}")
    s = w.scene
    sid_x = ctx.set_scene(s.K, s.depth, s.rgb, delta_mm=w.delta_mm, tau_c=w.tau_c, use_rgb=True)
    sid_v = ctx.set_scene(s.K, s.depth, s.rgb, delta_mm=w.delta_mm, tau_c=w.tau_c, use_rgb=True, volume=volume, jo=jo)
    mids = [ctx.load_mesh(m.xyz, m.tri, m.rgb) for m in w.meshes]
    rng = np.random.default_rng(7)
    for o in w.objects:
        got = gpu_score(ctx, sid_v, mids[o.mesh], o.poses, label=o.label)
        cls = ctx.last_classes(o.poses.shape[0])
        ref = gpu_score(ctx, sid_x, mids[o.mesh], o.poses, label=o.label)
        jr, jv, nr, nq = got
        assert np.array_equal(nr, ref[2])
        assert np.all((jr >= 0) & (jr <= nr)) and np.all((jv >= 0) & (jv <= nq))
        assert np.array_equal(jr, ref[0])                  # J_r does not depend on either variant
        if volume == "aabb":
            assert np.array_equal(nq, ref[3])
        else:
            assert np.all(nq <= ref[3])
        sel = [rng.choice(np.flatnonzero(cls == c), min(2, int((cls == c).sum())), replace=False)
               for c in np.unique(cls)]
        sel = np.unique(np.concatenate(sel + [np.array([0])]))
        poses = np.concatenate([o.gt_pose[None], o.poses[sel]])
        g = gpu_score(ctx, sid_v, mids[o.mesh], poses, label=o.label)
        exp = oracle.score(w.meshes[o.mesh], TScene(s.K, s.depth, s.rgb, None), poses, delta_mm=w.delta_mm,
                           tau_c=w.tau_c, flags=oflags(True, w.mark_occluders, volume, jo), label=o.label,
                           threads=THREADS)
        check(g, exp, True, jo, f"cfg2 {variant} object {o.label}")
        # scoring a subset gives the same outputs as the full launch
        for a, b in zip(g, got):
            assert np.array_equal(a[1:], b[sel])
    ctx.drop_scene(sid_x)
    ctx.drop_scene(sid_v)
    for mid in mids:
        ctx.unload_mesh(mid)


def test_batch_mixes_variants(ctx):
    """One batched launch over scenes with different volume and J_o modes
    gives each item the outputs of its own score_poses call."""
    items, refs = [], []
    sids, mids = [], []
    for seed, (volume, jo) in zip(range(20, 24), [("aabb", "exact"), ("cyl", "exact"), ("aabb", "nn"), ("cyl", "nn")]):
        mesh, scene, poses, p = random_case(seed)
        sid = ctx.set_scene(scene.K, scene.depth, scene.rgb, delta_mm=p["delta"], tau_c=p["tau"], use_rgb=p["rgb"],
                            mark_occluders=p["occl"], stride=p["stride"], volume=volume, jo=jo)
        mid = ctx.load_mesh(mesh.xyz, mesh.tri, mesh.rgb)
        sids.append(sid)
        mids.append(mid)
        t = torch.from_numpy(poses).cuda()
        refs.append(gpu_score(ctx, sid, mid, poses))
        n = poses.shape[0]
        items.append({"scene": sid, "mesh": mid, "label": 0, "poses": t,
                      **{k: torch.empty(n, dtype=torch.int32, device="cuda") for k in ("jr", "jo", "nr", "nq")}})
    say("batch of four variant scenes")
    out = ctx.score_batch(items)
    torch.cuda.synchronize()
    for it, ref in zip(out, refs):
        for key, r in zip(("jr", "jo", "nr", "nq"), ref):
            assert np.array_equal(it[key].cpu().numpy(), r)
    for sid in sids:
        ctx.drop_scene(sid)
    for mid in mids:
        ctx.unload_mesh(mid)


@pytest.mark.parametrize("seed", range(6))
def test_knn2_scan_equals_table(ctx, seed):
    """The paper's kNN II search (every rendered point scans the whole
    observed cloud) gives the outputs of the neighbour table, bit for bit,
    under both J_o modes; and the oracle's counts."""
    mesh, scene, poses, p = random_case(40 + seed)
    mid = ctx.load_mesh(mesh.xyz, mesh.tri, mesh.rgb)
    t = torch.from_numpy(poses).cuda()
    for jo in ("exact", "nn"):
        outs = []
        for search in ("table", "knn2"):
            say(f"case {40 + seed} {jo} {search}: image {scene.K[0]}x{scene.K[1]}, {p}")
            sid = ctx.set_scene(scene.K, scene.depth, scene.rgb, delta_mm=p["delta"], tau_c=p["tau"],
                                use_rgb=p["rgb"], mark_occluders=p["occl"], stride=p["stride"], jo=jo, search=search)
            outs.append([a.cpu().numpy() for a in ctx.score_poses(sid, mid, t)])
            torch.cuda.synchronize()
            ctx.drop_scene(sid)
        for a, b in zip(*outs):
            assert np.array_equal(a, b)
        exp = oracle.score(mesh, scene, poses, delta_mm=p["delta"], tau_c=p["tau"],
                           flags=oflags(p["rgb"], p["occl"], "aabb", jo), stride=p["stride"], threads=THREADS)
        check(outs[1], exp, p["rgb"], jo, f"case {40 + seed} {jo} knn2")
    ctx.unload_mesh(mid)


def test_knn2_full_size_sample(ctx):
    """kNN II on the 640x480 cfg2 scene for a few poses per object (each
    rendered point scans all 307,200 pixels): the table's outputs exactly."""
    w = make_config(2, 0)
    s = w.scene
    say("cfg2 kNN II sample")
    sids = [ctx.set_scene(s.K, s.depth, s.rgb, delta_mm=w.delta_mm, tau_c=w.tau_c, use_rgb=True, jo="nn", search=x)
            for x in ("table", "knn2")]
    rng = np.random.default_rng(11)
    for o in w.objects:
        mid = ctx.load_mesh(w.meshes[o.mesh].xyz, w.meshes[o.mesh].tri, w.meshes[o.mesh].rgb)
        poses = np.concatenate([o.gt_pose[None], o.poses[rng.choice(o.poses.shape[0], 3, replace=False)]])
        a, b = (gpu_score(ctx, sid, mid, poses, label=o.label) for sid in sids)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        assert a[2].min() > 0
        ctx.unload_mesh(mid)
    for sid in sids:
        ctx.drop_scene(sid)


@pytest.mark.parametrize("seed", range(6))
def test_knn1_array_equals_table(ctx, seed):
    """The paper's kNN I search (every rendered-observed distance in one
    array, reduced by rows and columns) gives the neighbour table's outputs
    bit for bit, under both J_o modes and all three volumes; and the
    oracle's counts."""
    mesh, scene, poses, p = random_case(60 + seed)
    volume = ("aabb", "cyl", "aabb")[seed % 3]
    mid = ctx.load_mesh(mesh.xyz, mesh.tri, mesh.rgb)
    t = torch.from_numpy(poses[:12]).cuda()
    for jo in ("exact", "nn"):
        outs = []
        for search in ("table", "knn1"):
            say(f"case {60 + seed} {jo} {search} {volume}: image {scene.K[0]}x{scene.K[1]}, {p}")
            sid = ctx.set_scene(scene.K, scene.depth, scene.rgb, delta_mm=p["delta"], tau_c=p["tau"],
                                use_rgb=p["rgb"], mark_occluders=p["occl"], stride=p["stride"], jo=jo, search=search,
                                volume=volume)
            outs.append([a.cpu().numpy() for a in ctx.score_poses(sid, mid, t)])
            torch.cuda.synchronize()
            ctx.drop_scene(sid)
        for a, b in zip(*outs):
            assert np.array_equal(a, b)
        exp = oracle.score(mesh, scene, poses[:12], delta_mm=p["delta"], tau_c=p["tau"],
                           flags=oflags(p["rgb"], p["occl"], volume, jo), stride=p["stride"], threads=THREADS)
        check(outs[1], exp, p["rgb"], jo, f"case {60 + seed} {jo} knn1")
    ctx.unload_mesh(mid)


@pytest.mark.parametrize("volume", ["aabb", "label"])
def test_knn1_full_size_sample(ctx, volume):
    """kNN I on the 640x480 cfg2 scene, two poses per object (each pose's
    distance array holds L x ~300,000 entries, gigabytes): the table's
    outputs exactly."""
    w = make_config(2, 0)
    s = w.scene
    say(f"cfg2 kNN I sample, {volume}")
    sids = [ctx.set_scene(s.K, s.depth, s.rgb, s.labels, delta_mm=w.delta_mm, tau_c=w.tau_c, use_rgb=True,
                          volume=volume, search=x) for x in ("table", "knn1")]
    rng = np.random.default_rng(12)
    for o in w.objects:
        mid = ctx.load_mesh(w.meshes[o.mesh].xyz, w.meshes[o.mesh].tri, w.meshes[o.mesh].rgb)
        poses = np.concatenate([o.gt_pose[None], o.poses[rng.choice(o.poses.shape[0], 1, replace=False)]])
        a, b = (gpu_score(ctx, sid, mid, poses, label=o.label) for sid in sids)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        assert a[2].min() > 0
        ctx.unload_mesh(mid)
    for sid in sids:
        ctx.drop_scene(sid)


def test_knn1_scored_by_score_poses_only(ctx):
    mesh, scene, poses, p = random_case(70)
    mid = ctx.load_mesh(mesh.xyz, mesh.tri, mesh.rgb)
    sid = ctx.set_scene(scene.K, scene.depth, scene.rgb, delta_mm=p["delta"], search="knn1")
    t = torch.from_numpy(poses[:4]).cuda()
    with pytest.raises(pk.PerchError, match="KNN1"):
        ctx.best_poses(sid, [mid], [0], [t])
    with pytest.raises(pk.PerchError, match="KNN1"):
        ctx.msg_expand(sid, [], mid, t)
    ctx.drop_scene(sid)
    ctx.unload_mesh(mid)


def test_flag_validation(ctx):
    K = (32, 24, 30.0, 30.0, 16.0, 12.0)
    depth = np.zeros((24, 32), np.uint16)
    with pytest.raises(pk.PerchError):
        ctx.set_scene(K, depth, flags=3 << 4)             # no such volume mode
    with pytest.raises(pk.PerchError):
        ctx.set_scene(K, depth, flags=1 << 12)            # unknown bit
    with pytest.raises(pk.PerchError):
        ctx.set_scene(K, depth, flags=pk.KNN1 | pk.KNN2)  # two searches
    with pytest.raises(pk.PerchError):
        ctx.set_scene(K, depth, flags=pk.KNN2 | pk.HASH)  # two searches
    with pytest.raises(ValueError):
        ctx.set_scene(K, depth, volume="sphere")
    with pytest.raises(ValueError):
        ctx.set_scene(K, depth, search="kd-tree")
    sid = ctx.set_scene(K, depth, flags=pk.VOL_CYL | pk.JO_NN | pk.KNN2 | pk.MARK_OCCLUDERS)
    ctx.drop_scene(sid)


def test_knn1_array_beyond_the_budget_is_refused():
    """kNN I with a distance array larger than the context's HBM budget (a
    320x240 self-render: 4,798 x 4,798 pairs, 88 MB, against 48 MB): a
    clean PERCH_ENOMEM naming the array; the context then scores a farther
    pose, whose array fits, as the oracle does."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from test_oracle_icp import K_HI, _scene_and_gt
    m, scene, gt = _scene_and_gt(0, K_HI)
    with pk.Context(0, hbm_budget_bytes=48 << 20) as small:
        mid = small.load_mesh(m.xyz, m.tri, m.rgb)
        sid = small.set_scene(scene.K, scene.depth, delta_mm=5.0, mark_occluders=False, search="knn1")
        say("kNN I under a 48 MB budget")
        t = torch.from_numpy(gt.reshape(1, 12).astype(np.float32)).cuda()
        with pytest.raises(pk.PerchError, match="does not fit"):
            small.score_poses(sid, mid, t)
        # the context goes on: a pose 3 m further back has a small array
        far = gt.reshape(1, 12).astype(np.float32).copy()
        far[0, 11] += 3000.0
        got = [a.cpu().numpy() for a in small.score_poses(sid, mid, torch.from_numpy(far).cuda())]
        exp = oracle.score(m, scene, far, delta_mm=5.0, flags=0)
        for a, b in zip(got, exp):
            assert np.array_equal(a, b)
        assert 0 < got[2][0] < 1000
