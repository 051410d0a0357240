"""The oracle's chain with the deform output given (``roots``): fed the
solver's own roots it reproduces the full chain exactly, and it rejects a
root set that does not match the marched samples."""
import numpy as np
import pytest

from paper_2212_10550_amd import synth


def test_roots_given_equals_full_chain(orc):
    w = synth.ray_subset(synth.train_step(), np.arange(0, 8192, 32))
    full = orc.train_step(w)
    given = orc.train_step(w, roots=(full["deform"]["xc"], full["deform"]["bone"]))
    for k in ("feat", "sigma", "color", "opacity", "loss", "grad_params", "grad_table", "grad_xc", "grad_xp", "grad_B",
              "grad_W"):
        assert np.array_equal(np.asarray(given[k]), np.asarray(full[k])), k


def test_roots_given_rejects_wrong_count(orc):
    w = synth.ray_subset(synth.train_step(), np.arange(0, 8192, 256))
    with pytest.raises(ValueError):
        orc.forward(w, roots=(np.zeros((3, 3)), np.zeros(3, np.int16)))
