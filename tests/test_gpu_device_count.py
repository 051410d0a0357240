"""Device-resident sample counts and graph capture.

Every stage called with S_dev (the count read on the device, S the
capacity) must give the same results as the same stage called with the
host count: bit for bit where the per-sample arithmetic is the same, to
summation-order rounding where partial sums are grouped differently.  A
captured training step replayed several times, with eager work between
the replays, must match the eager step every time."""
import numpy as np
import pytest
import torch

from paper_2212_10550_amd import synth
from tests.gpu_util import host

pytestmark = pytest.mark.gpu


def _pipes(w, **kw):
    from paper_2212_10550_amd.pipeline import Pipeline
    return Pipeline(w, **kw), Pipeline(w, device_count=True, **kw)


def _close(a, b, what, rtol=1e-5):
    a = host(a)
    b = host(b)
    scale = max(np.abs(a).max(), 1e-30)
    err = np.abs(a - b).max() / scale
    assert err <= rtol, f"{what}: {err:.2e}"
    return err


@pytest.mark.parametrize("mixed", [False, True])
def test_training_step_device_count_matches_host_count(mixed):
    from paper_2212_10550_amd import lib as K
    w = synth.train_step()
    kw = dict(table_dtype=torch.float16, mlp_dtype=K.BF16) if mixed else {}
    ph, pd = _pipes(w, **kw)
    S = ph.train_step()
    assert pd.train_step() is None
    torch.cuda.synchronize()
    assert pd.read_count() == S
    # forward: identical per-sample work
    for name in ("xc", "bone", "sigma", "rgb"):
        a, b = getattr(ph, name), getattr(pd, name)
        assert torch.equal(a[..., :S], b[..., :S]), name
    assert torch.equal(ph.color, pd.color)
    assert torch.equal(ph.loss, pd.loss)
    # backward: the same gradients up to the grouping of partial sums and the
    # order of atomic adds
    assert torch.equal(ph.grad_xp[:, :S], pd.grad_xp[:, :S])
    errs = [_close(ph.grad_params, pd.grad_params, "grad_params", 1e-4),
            _close(ph.grad_table, pd.grad_table, "grad_table"),
            _close(ph.grad_B, pd.grad_B, "grad_B"),
            _close(ph.grad_W, pd.grad_W, "grad_W")]
    print(f"device count vs host count (mixed={mixed}): S={S}, grad diffs {['%.1e' % e for e in errs]}")


def test_frame_device_count_learned_init():
    from paper_2212_10550_amd import lib as K
    from paper_2212_10550_amd import rootinit
    w = synth.ray_subset(synth.tiny_forward(), np.arange(512))
    params = synth.make_rootinit_params(seed=4).astype(np.float32)
    params[-27:-3] += np.linspace(0, 0.5, 24, dtype=np.float32)
    ph, pd = _pipes(w, table_dtype=torch.float16, mlp_dtype=K.BF16, rootinit_params=params)
    S = ph.forward()
    pd.forward()
    torch.cuda.synchronize()
    assert pd.read_count() == S
    assert torch.equal(ph.bone[:S], pd.bone[:S])
    assert torch.equal(ph.xc[:, :S], pd.xc[:, :S])
    assert torch.equal(ph.color, pd.color)
    assert int(ph.guided.n_fallback.item()) == int(pd.guided.n_fallback.item())


def test_graph_replay_matches_eager():
    from paper_2212_10550_amd.pipeline import Pipeline
    w = synth.train_step()
    eager = Pipeline(w)
    S = eager.train_step()
    torch.cuda.synchronize()
    ref = {k: getattr(eager, k).clone() for k in ("color", "loss", "grad_params", "grad_table", "grad_B", "grad_xp")}
    pg = Pipeline(w, device_count=True)
    pg.capture_train_step()
    for rep in range(3):
        # clobber the outputs and run unrelated eager work between replays
        for k in ref:
            getattr(pg, k).fill_(float("nan"))
        eager.train_step()
        torch.cuda.synchronize()
        pg.train_step()
        torch.cuda.synchronize()
        assert pg.read_count() == S
        assert torch.equal(pg.color, ref["color"]), rep
        assert torch.equal(pg.loss, ref["loss"]), rep
        assert torch.equal(pg.grad_xp[:, :S], ref["grad_xp"][:, :S]), rep
        _close(pg.grad_params, ref["grad_params"], f"grad_params replay {rep}", 1e-4)
        _close(pg.grad_table, ref["grad_table"], f"grad_table replay {rep}")
        _close(pg.grad_B, ref["grad_B"], f"grad_B replay {rep}")


def test_device_count_overflow_is_reported():
    """A capacity below the march's count: the device-count stages clamp to
    the capacity (no access past the buffers) and read_count reports it."""
    from paper_2212_10550_amd.pipeline import Pipeline
    w = synth.train_step()
    full = Pipeline(w)
    S = full.forward()
    small = Pipeline(w, cap=S // 2, device_count=True)
    small.train_step()
    torch.cuda.synchronize()
    assert int(small.n_samples.item()) == S
    with pytest.raises(RuntimeError):
        small.read_count()
    assert np.isfinite(host(small.color)).all()


def test_march_capacity_status():
    """ia355_occgrid_march with n_required: the kept count is returned, and a
    capacity below it gives IA355_ERR_CAPACITY with the count needed; the
    first cap samples equal those of a large enough buffer."""
    from paper_2212_10550_amd import lib as K
    from paper_2212_10550_amd.pipeline import Pipeline
    w = synth.train_step()
    p = Pipeline(w)
    S = K.occgrid_march(p.rays_o, p.rays_d, p.occ_bits, p.G, w.occ_aabb, w.dt, w.n_per_ray, w.max_steps, p.xs, p.ts,
                        p.ray_id, p.cap, p.ray_off, p.ray_cnt, p.ray_dt, p.n_samples, p.ws_march, check=True)
    assert S == int(p.n_samples.item()) and 0 < S <= p.cap
    cap = S // 3
    xs = torch.full((3, cap), 7.0, device=p.dev)
    ts = torch.empty(cap, device=p.dev)
    rid = torch.empty(cap, dtype=torch.int32, device=p.dev)
    with pytest.raises(K.CapacityError) as e:
        K.occgrid_march(p.rays_o, p.rays_d, p.occ_bits, p.G, w.occ_aabb, w.dt, w.n_per_ray, w.max_steps, xs, ts, rid,
                        cap, p.ray_off, p.ray_cnt, p.ray_dt, p.n_samples, p.ws_march, check=True)
    assert e.value.n_required == S and e.value.cap == cap
    torch.cuda.synchronize()
    assert np.array_equal(host(xs), host(p.xs[:, :cap]))
