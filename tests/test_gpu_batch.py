"""Batched render of several poses in one HIP graph: every pose's image must
equal the same pose rendered alone (bit for bit: the per-sample work is the
same, only the schedule differs), on every replay, for any stream count and
for the persistent kernel under every tile shape; one pose is also checked
against the FP64 oracle at the reduced-precision pixel bar."""
import numpy as np
import pytest
import torch

from paper_2212_10550_amd import synth

pytestmark = pytest.mark.gpu


def _params():
    p = synth.make_rootinit_params(seed=4).astype(np.float32)
    p[-27:-3] += np.linspace(0, 0.5, 24, dtype=np.float32)
    return p


@pytest.fixture(scope="module")
def small_batch():
    # three poses of the batch (270^2 at 5 %, 540^2 and 1080^2), every 37th ray
    ws = []
    for k in (0, 4, 2):
        w = synth.batch_pose(k)
        ws.append(synth.ray_subset(w, np.arange(0, w.R, 37)))
    return ws


_OUTS = ("color", "opacity", "n_used", "T_final")


def _single_refs(ws, params, poses):
    """Every pose rendered alone by the staged path: outputs and fallback count."""
    from paper_2212_10550_amd import lib as K
    from paper_2212_10550_amd.pipeline import Pipeline
    refs = []
    for w, p in zip(ws, poses):
        single = Pipeline(w, table_dtype=torch.float16, mlp_dtype=K.BF16, rootinit_params=params, device_count=True)
        single.forward()
        torch.cuda.synchronize()
        assert single.read_count() == p.S
        refs.append({k: getattr(single, k).clone() for k in _OUTS})
        refs[-1]["n_fallback"] = int(single.guided.n_fallback.item())
        del single
    return refs


def _check_replays(br, refs, what):
    """Two replays: every output bit equal to the reference's.  The staged
    kernels solve every sample; the persistent kernel stops evaluating a ray
    after the group where it terminates, so it evaluates at most the posed
    samples and at least the used ones, with at most the staged fallbacks."""
    for rep in range(2):
        for p in br.poses:
            p.color.fill_(float("nan"))
            p.opacity.fill_(float("nan"))
            p.T_final.fill_(float("nan"))
            p.n_used.fill_(-1)
            p.n_fallback.fill_(-1)
            p.n_evaluated.fill_(-1)
        br.render()
        torch.cuda.synchronize()
        for i, p in enumerate(br.poses):
            for k in _OUTS:
                assert torch.equal(getattr(p, k), refs[i][k]), (what, rep, i, k)
            fb = int(p.n_fallback.item())
            if br.persistent is None:
                assert fb == refs[i]["n_fallback"], (what, rep, i)
            else:
                ev = int(p.n_evaluated.item())
                assert int(p.n_used.sum().item()) <= ev <= p.S, (what, rep, i, ev, p.S)
                assert 0 <= fb <= refs[i]["n_fallback"], (what, rep, i)


@pytest.mark.parametrize("n_streams", [1, 2])
def test_batch_matches_single_pose(small_batch, n_streams):
    from paper_2212_10550_amd.batch import BatchRenderer
    params = _params()
    br = BatchRenderer(small_batch, params, n_streams=n_streams)
    br.capture()
    refs = _single_refs(small_batch, params, br.poses)
    _check_replays(br, refs, f"{n_streams} streams")
    print(f"batch ({n_streams} streams): samples {[p.S for p in br.poses]}")


# schedules: rays per tile (ragged last tiles, 64 = one lane per ray),
# samples per segment (256: a 64-ray tile splits into several segments),
# waves per workgroup, workgroups per CU (every kernel instantiation)
@pytest.mark.parametrize("sched", [(64, 256, 4, 2), (13, 256, 4, 1), (32, 384, 4, 3), (1, 256, 4, 4),
                                   (32, 256, 8, 1), (32, 256, 8, 2)])
def test_persistent_matches_single_pose(small_batch, sched):
    from paper_2212_10550_amd.batch import BatchRenderer
    params = _params()
    br = BatchRenderer(small_batch, params, n_streams=1)
    br.set_persistent(*sched)
    br.capture()
    refs = _single_refs(small_batch, params, br.poses)
    _check_replays(br, refs, f"persistent {sched}")
    used = [int(p.n_used.sum().item()) for p in br.poses]
    ev = [int(p.n_evaluated.item()) for p in br.poses]
    print(f"persistent {sched}: samples {[p.S for p in br.poses]}, evaluated {ev}, used {used}, "
          f"fallback {[int(p.n_fallback.item()) for p in br.poses]} (staged {[r['n_fallback'] for r in refs]})")


def test_persistent_full_poses_match_staged():
    """Two whole poses of the batch (540^2 at 20 % and 270^2 at 5 %, the
    workload's own sizes): persistent and staged renders agree bit for bit,
    with the poses in one plan."""
    from paper_2212_10550_amd.batch import BatchRenderer
    ws = [synth.batch_pose(k) for k in (4, 3)]
    br = BatchRenderer(ws, _params(), n_streams=2)
    br.render()
    torch.cuda.synchronize()
    refs = [{k: getattr(p, k).clone() for k in _OUTS} for p in br.poses]
    for r, p in zip(refs, br.poses):
        r["n_fallback"] = int(p.n_fallback.item())
    br.set_persistent(32, 256, 8, 2)
    br.capture()
    _check_replays(br, refs, "full poses")
    print(f"full poses: rays {[p.R for p in br.poses]}, samples {[p.S for p in br.poses]}")


def test_persistent_rejects_bad_schedules(small_batch):
    from paper_2212_10550_amd import lib as K
    from paper_2212_10550_amd.batch import BatchRenderer
    br = BatchRenderer(small_batch[:1], _params(), n_streams=1)
    br.set_persistent(16, 256, 4, 1)
    with pytest.raises(RuntimeError, match="status 1"):
        K.batch_render(br._ws, 65, 256, 4, 1)  # more rays per tile than lanes
    with pytest.raises(RuntimeError, match="status 1"):
        K.batch_render(br._ws, 16, 128, 4, 1)  # a segment must hold two whole rays
    with pytest.raises(RuntimeError, match="status 1"):
        K.batch_render(br._ws, 16, 256, 4, 0)
    with pytest.raises(RuntimeError, match="status 1"):
        K.batch_render(br._ws, 16, 256, 6, 1)  # 4 or 8 waves
    with pytest.raises(RuntimeError, match="status 3"):
        K.batch_render(br._ws, 16, 256, 8, 3)  # no such instantiation
    with pytest.raises(RuntimeError, match="status 3"):
        K.batch_render(br._ws, 64, 8192, 8, 1)  # beyond the LDS of a workgroup


def test_batch_pose_against_oracle(orc, small_batch):
    from paper_2212_10550_amd.batch import BatchRenderer
    br = BatchRenderer(small_batch, _params(), n_streams=2)
    br.render()
    torch.cuda.synchronize()
    w = small_batch[1]
    idx = np.arange(0, w.R, 5)
    ref = orc.forward(synth.ray_subset(w, idx))["color"]
    got = br.poses[1].color.double().cpu().numpy()[idx]
    err = np.abs(got - ref)
    print(f"batch pose vs oracle: {len(idx)} rays, mean {err.mean():.2e} max {err.max():.2e}")
    assert err.max() <= 1e-3
    assert err.mean() <= 1e-4
