"""A full 540x540 frame through the library, checked on a seeded subset of
rays against the FP64 oracle: the FP32 path with the 24-init solve at the
FP32 bar, and the reduced-precision path (FP16 table, BF16 features and
MLP, learned root initialiser with multi-init fallback) at the 1e-3 pixel
bar."""
import numpy as np
import pytest
import torch

from paper_2212_10550_amd import synth
from tests.gpu_util import assert_mixed, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frame_and_ref(orc):
    w = synth.full_frame()
    sub = np.arange(0, w.R, 211)
    ref = orc.forward(synth.ray_subset(w, sub), details=True)
    return w, sub, ref


def _ok_rays(p, S, ref, sub, R):
    """Rays whose samples agree with the oracle on which samples found a
    root (a flip at the validity threshold changes the ray legitimately)."""
    ray = host(p.ray_id[:S]).astype(np.int64)
    gb = host(p.bone[:S]).astype(int)
    pos = np.searchsorted(sub, ray)
    keep = (pos < len(sub)) & (sub[np.minimum(pos, len(sub) - 1)] == ray)
    # samples of the subset rays, in march order (the march is exact)
    gsub = gb[keep]
    ob = ref["deform"]["bone"]
    assert len(gsub) == len(ob)
    flip = (gsub >= 0) != (ob >= 0)
    ok = np.ones(len(sub), bool)
    ok[np.unique(ref["march"]["ray_id"][flip])] = False
    return ok


def test_frame_f32_multi_init(frame_and_ref):
    from paper_2212_10550_amd.pipeline import Pipeline
    w, sub, ref = frame_and_ref
    p = Pipeline(w)
    S = p.forward()
    torch.cuda.synchronize()
    ok = _ok_rays(p, S, ref, sub, w.R)
    assert ok.mean() > 0.99
    err = assert_mixed(host(p.color)[sub][ok], ref["color"][ok], 1e-5, "pixel colour (FP32)")
    print(f"frame f32: S={S}, rays compared {ok.sum()} of {len(sub)}, max err {err:.2e}")


def test_frame_mixed_learned_init(frame_and_ref):
    from paper_2212_10550_amd import lib as K
    from paper_2212_10550_amd import rootinit
    from paper_2212_10550_amd.pipeline import Pipeline
    w, sub, ref = frame_and_ref
    data = rootinit.make_dataset(range(1000, 1032), 2048, device="cuda:0")
    params = rootinit.fit(data, epochs=6)
    p = Pipeline(w, table_dtype=torch.float16, mlp_dtype=K.BF16, rootinit_params=params)
    S = p.forward()
    torch.cuda.synchronize()
    c = host(p.color)[sub].astype(np.float64)
    err = np.abs(c - ref["color"])
    fb = int(p.guided.n_fallback.item())
    print(f"frame mixed: S={S}, fallback {fb}, pixel err mean {err.mean():.2e} max {err.max():.2e}")
    assert err.max() <= 1e-3
    assert err.mean() <= 1e-4
