"""A whole training step on the GPU, started from the oracle's roots, against
the FP64 oracle started from the same roots: every output element by element
(FP32 form), and the error of the FP16-table / BF16-MLP form against the
oracle on the FP32 master values (total error) and on the rounded table and
MLP weights (kernel error), stated per output.

Both sides take the oracle's canonical roots rounded to FP32 as the deform
stage's output (the root finding itself is checked against the oracle's
root set in the forward tests).  With identical points, the selection among
distinct valid roots and the root error drop out, and every later stage is
compared on identical inputs.  Nothing the HIP path computes is fed to the
oracle.
"""
import json

import numpy as np
import pytest
import torch

from paper_2212_10550_amd import synth
from tests import bounds
from tests.gpu_util import assert_mixed, dev, feat_host, host

pytestmark = pytest.mark.gpu

GTOL = 1e-4  # gradient bar of the FP32 path (per element, of the magnitude sum)
BF16_U = 2.0 ** -9  # unit roundoff of BF16 (8 significant bits, round to nearest)
FP16_U = 2.0 ** -11


def _K():
    from paper_2212_10550_amd import lib as K
    return K


def _workload(stride):
    w = synth.train_step()
    return w if stride == 1 else synth.ray_subset(w, np.arange(0, w.R, stride))


def _oracle_roots(orc, w):
    """The oracle's roots of the marched samples, rounded to FP32 (the form
    both sides take as the deform output)."""
    m = orc.march(w.rays_o, w.rays_d, w.occ, w.occ_aabb, w.dt, w.n_per_ray, w.max_steps)
    d = orc.deform(m["xs"], w.B, w.W, w.skin_aabb, w.hash_aabb, w.max_iter, w.tol_stop, w.tol_valid)
    return d["xc"].astype(np.float32), d["bone"].astype(np.int16)


def _gpu_step_from_roots(p, xc, bone):
    """March, then every later stage of a training step with the deform
    output set to (xc, bone)."""
    p.march()
    S = p.read_count()
    assert S == xc.shape[0], (S, xc.shape)
    p.xc[:, :S] = torch.as_tensor(np.ascontiguousarray(xc.T), device=p.dev)
    p.bone[:S] = torch.as_tensor(bone, device=p.dev)
    p._encode(S, None)
    p._mlp(S, None)
    p._render()
    p._last = (S, None)
    p.backward(S, None)
    torch.cuda.synchronize()
    return S


def _gpu_outputs(p, S, L):
    f = host(p.feat.float()).reshape(L, p.cap, 2)[:, :S, :].transpose(1, 0, 2).reshape(S, 2 * L)
    return dict(feat=f, sigma=host(p.sigma[:S]), rgb=p.soa(p.rgb, S), color=host(p.color), opacity=host(p.opacity),
                loss=np.array([float(p.loss.item())]), grad_sigma=host(p.grad_sigma[:S]), grad_rgb=p.soa(p.grad_rgb, S),
                grad_params=host(p.grad_params), grad_feat=feat_host(p.grad_feat, S, p.cap),
                grad_table=host(p.grad_table), grad_xc=p.soa(p.grad_xc, S), grad_xp=p.soa(p.grad_xp, S),
                grad_B=host(p.grad_B), grad_W=host(p.grad_W))


def _rows_close(got, ref, tol, what):
    """Per-sample 3-vectors: |gpu - oracle| <= tol * max(|oracle row|, 1e-3 max row)."""
    rn = np.linalg.norm(ref, axis=1, keepdims=True)
    floor = 1e-3 * rn.max() if rn.size else 1.0
    err = np.abs(got - ref) / np.maximum(np.maximum(rn, floor), 1e-300)
    assert (err <= tol).all(), f"{what}: max row-relative error {err.max():.3e} ({(err > tol).sum()} elements)"
    return float(err.max())


def test_train_step_from_oracle_roots_f32(orc):
    """FP32 training step (8192 rays, binned table gradient): every output
    element by element.  Sums over samples (parameter, table, bone and
    skinning-grid gradients) are held to 1e-4 of the sum of their terms'
    magnitudes, the error bound of any summation order."""
    from paper_2212_10550_amd.pipeline import Pipeline
    w = _workload(1)
    xc, bone = _oracle_roots(orc, w)
    p = Pipeline(w)
    S = _gpu_step_from_roots(p, xc, bone)
    ref = orc.train_step(w, roots=(xc, bone))
    g = _gpu_outputs(p, S, w.L)
    res, aabb = ref["res"], w.hash_aabb
    e = {}
    e["feat"] = bounds.check_scaled(g["feat"], ref["feat"], bounds.feature_magnitude(orc, xc, w.table, res, aabb, bone),
                                    1e-5, "features")
    e["sigma"] = assert_mixed(g["sigma"], ref["sigma"], 1e-5, "sigma")
    e["rgb"] = assert_mixed(g["rgb"], ref["rgb"], 1e-5, "rgb")
    e["color"] = assert_mixed(g["color"], ref["color"], 1e-5, "colour")
    e["opacity"] = assert_mixed(g["opacity"], ref["opacity"], 1e-5, "opacity")
    e["loss"] = assert_mixed(g["loss"], [ref["loss"]], 1e-5, "loss")
    gmax = lambda a: 1e-3 * np.abs(a).max()
    e["grad_sigma"] = assert_mixed(g["grad_sigma"], ref["grad_sigma"], GTOL, "grad_sigma", scale=gmax(ref["grad_sigma"]))
    e["grad_rgb"] = assert_mixed(g["grad_rgb"], ref["grad_rgb"], GTOL, "grad_rgb", scale=gmax(ref["grad_rgb"]))
    mag_p, mag_gf = bounds.mlp_grad_magnitude(ref["feat"], w.mlp, ref["grad_sigma"], ref["grad_rgb"], bone)
    e["grad_params"] = bounds.check_scaled(g["grad_params"], ref["grad_params"], mag_p, GTOL, "grad_params")
    e["grad_feat"] = bounds.check_scaled(g["grad_feat"], ref["grad_feat"], mag_gf, GTOL, "grad_feat")
    mag_t = bounds.table_grad_magnitude(orc, mag_gf, xc, w.table, res, aabb, bone)
    e["grad_table"] = bounds.check_scaled(g["grad_table"], ref["grad_table"], mag_t, GTOL, "grad_table (binned)")
    e["grad_xc"] = _rows_close(g["grad_xc"], ref["grad_xc"], GTOL, "grad_xc")
    e["grad_xp"] = _rows_close(g["grad_xp"], ref["grad_xp"], GTOL, "grad_xp")
    mag_B, mag_W, cnt_W = bounds.deform_grad_magnitude(ref["grad_xp"], xc, bone, w.B, w.W, w.skin_aabb)
    e["grad_B"] = bounds.check_scaled(g["grad_B"], ref["grad_B"], mag_B, GTOL, "grad_B")
    # a corner weight also carries the absolute error of the FP32 cell fractions
    ef = bounds.cell_fraction_error(w.W.shape[2::-1])
    e["grad_W"] = bounds.check_bound(g["grad_W"], ref["grad_W"], GTOL * mag_W + ef * cnt_W + 1e-10 * GTOL * mag_W.max(),
                                     "grad_W")
    assert (g["grad_xp"][bone < 0] == 0).all()
    print(f"f32 step from oracle roots: S={S}, valid {int((bone >= 0).sum())}; max errors (per bar): "
          + json.dumps({k: float(f"{v:.3g}") for k, v in e.items()}))


def _error_table(g, ref):
    return {k: bounds.error_stats(g[k], ref[k] if k != "loss" else [ref["loss"]]) for k in g}


def _normrel(got, ref):
    return float(np.linalg.norm(np.ravel(got) - np.ravel(ref)) / max(np.linalg.norm(np.ravel(ref)), 1e-300))


MIXED_KEYS = ("feat", "sigma", "rgb", "color", "opacity", "loss", "grad_sigma", "grad_rgb", "grad_params", "grad_feat",
              "grad_table", "grad_xc", "grad_xp", "grad_B", "grad_W")


def mixed_step_errors(orc, w, xc, bone, g, table_r):
    """Per-output error of a mixed-precision step's outputs g against three
    oracle runs from the same roots: "total" (FP32 master table and MLP,
    FP64 arithmetic), "rounded" (the FP16 table and BF16-rounded MLP
    weights, FP64 arithmetic: the error of the arithmetic alone) and
    "storage" (the FP16 table and the decoder in its BF16 storage form:
    what the kernels compute, up to FP32 accumulation).  Returns the three
    references and, per output, mean / p99.9 / max absolute error and the
    norm-wise relative error against each."""
    params_r = torch.as_tensor(w.mlp).bfloat16().double().numpy()
    refs = {"total": orc.train_step(w, roots=(xc, bone)),
            "rounded": orc.train_step(w, table=table_r, params=params_r, roots=(xc, bone)),
            "storage": orc.train_step(w, table=table_r, roots=(xc, bone), mlp_bf16=True)}
    table = {}
    for k in MIXED_KEYS:
        row = {}
        for name, ref in refs.items():
            rk = [ref["loss"]] if k == "loss" else ref[k]
            st = bounds.error_stats(g[k], rk)
            st["norm_rel"] = _normrel(g[k], rk)
            row[name] = st
        table[k] = row
    return refs, table


@pytest.mark.parametrize("stride", [4])
def test_mixed_step_error_vs_oracle(orc, stride):
    """FP16 table, BF16 features and MLP (MFMA, FP32 accumulate), FP32
    compositing and implicit-function-theorem backward, on a quarter of the
    training rays, against the oracle from the same roots: the total error
    (FP32 masters), the error of the arithmetic on the rounded table and
    weights, and the parity with the BF16 storage form.

    Bars (stated from the arithmetic, not fitted):
      * pixels, total and rounded: mean |dC| <= 1e-3 (the reduced-precision
        pixel bar), max <= 1e-2;
      * features: |d| <= 2^-8 of sum_c w_c |theta_c| against the rounded
        table (BF16 rounding of an FP32 interpolation); against the FP32
        masters add the FP16 rounding of the table, 2^-11 of the same sum
        plus 2^-25 (half the spacing of FP16 subnormals, below 2^-14, where
        most entries of a 1e-4-scale table lie);
      * parity with the storage form: every MLP parameter and feature
        gradient element within 2^-8 of the sum of its terms' magnitudes (a
        stored value may differ by one bfloat16 step where its FP32 value
        sits on a rounding boundary), every other gradient within 1e-3
        norm-wise;
      * total error of every gradient, norm-wise <= 0.1: the BF16 form flips
        the ReLU decisions of the hidden units whose pre-activation lies
        within a bfloat16 rounding of zero (a few per thousand), and each
        flip moves that sample's term by its full size (a sanity bar; the
        figures are reported per output)."""
    from paper_2212_10550_amd.pipeline import Pipeline
    K = _K()
    w = _workload(stride)
    xc, bone = _oracle_roots(orc, w)
    p = Pipeline(w, table_dtype=torch.float16, mlp_dtype=K.BF16)
    S = _gpu_step_from_roots(p, xc, bone)
    g = _gpu_outputs(p, S, w.L)
    table_r = host(p.table)  # the FP16 table the kernels read
    refs, tab = mixed_step_errors(orc, w, xc, bone, g, table_r)
    print(f"mixed step (1/{stride} of the rays, S={S}) error per output [mean / p99.9 / max abs; norm-rel]:")
    for k, row in tab.items():
        print(f"  {k:11s} " + " | ".join(f"{n} {v['mean']:.1e}/{v['p999']:.1e}/{v['max']:.1e}; {v['norm_rel']:.1e}"
                                         for n, v in row.items()) + f" (scale {row['total']['ref_max']:.1e})")
    for n in ("total", "rounded"):
        c = tab["color"][n]
        assert c["mean"] <= 1e-3 and c["max"] <= 1e-2, (n, c)
    res, aabb = refs["total"]["res"], w.hash_aabb
    fmag = bounds.feature_magnitude(orc, xc, table_r, res, aabb, bone)
    bounds.check_scaled(g["feat"], refs["rounded"]["feat"], fmag, 2.0 ** -8, "features (rounded table)")
    bounds.check_bound(g["feat"], refs["total"]["feat"], (2.0 ** -8 + FP16_U) * fmag + 2.0 ** -25,
                       "features (total error)")
    st = refs["storage"]
    feat_q = torch.as_tensor(st["feat"], dtype=torch.float32).bfloat16().double().numpy()
    mag_p, mag_gf = bounds.mlp_grad_magnitude(feat_q, w.mlp, st["grad_sigma"], st["grad_rgb"], bone)
    bounds.check_scaled(g["grad_params"], st["grad_params"], mag_p, 2.0 ** -8, "grad_params (storage form)")
    bounds.check_scaled(g["grad_feat"], st["grad_feat"], mag_gf, 2.0 ** -8, "grad_feat (storage form)")
    bad = {k: tab[k]["storage"]["norm_rel"] for k in ("grad_sigma", "grad_rgb", "grad_table", "grad_xc", "grad_xp",
                                                      "grad_B", "grad_W", "loss")
           if tab[k]["storage"]["norm_rel"] > 1e-3}
    assert not bad, f"norm-wise error against the storage form above 1e-3: {bad}"
    bad = {k: tab[k]["total"]["norm_rel"] for k in MIXED_KEYS if k.startswith("grad") and
           tab[k]["total"]["norm_rel"] > 0.1}
    assert not bad, f"total norm-wise error above 0.1: {bad}"
