"""Batched render of several poses in one HIP graph: every pose's image must
equal the same pose rendered alone (bit for bit: the per-sample work is the
same, only the schedule differs), on every replay, for any stream count;
one pose is also checked against the FP64 oracle at the reduced-precision
pixel bar."""
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


@pytest.mark.parametrize("n_streams", [1, 2])
def test_batch_matches_single_pose(small_batch, n_streams):
    from paper_2212_10550_amd import lib as K
    from paper_2212_10550_amd.batch import BatchRenderer
    from paper_2212_10550_amd.pipeline import Pipeline
    params = _params()
    br = BatchRenderer(small_batch, params, n_streams=n_streams)
    br.capture()
    refs = []
    for w, p in zip(small_batch, br.poses):
        single = Pipeline(w, table_dtype=torch.float16, mlp_dtype=K.BF16, rootinit_params=params, device_count=True)
        single.forward()
        torch.cuda.synchronize()
        assert single.read_count() == p.S
        refs.append(single.color.clone())
    for rep in range(2):
        for p in br.poses:
            p.color.fill_(float("nan"))
        br.render()
        torch.cuda.synchronize()
        for i, p in enumerate(br.poses):
            assert torch.equal(p.color, refs[i]), (rep, i)
    print(f"batch ({n_streams} streams): samples {[p.S for p in br.poses]}")


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
