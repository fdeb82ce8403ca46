"""Host checks of the learned stage's stored weights (no GPU): the committed file
is raw float32 of exactly the network's parameter count, its description is
plain JSON with the training record, and the values are finite and not all
zero.  The parameter count comes from the library (stokes_unet_param_count)."""
import json
import os

import numpy as np
import pytest

from paper_1901_07892_amd import learned


def test_trained_weights_load_and_match_the_network():
    p, meta = learned.load_params()
    if p is None:
        pytest.skip("no trained weights in the package")
    import paper_1901_07892_amd as S
    assert p.dtype == np.float32 and p.size == S.stokes_unet_param_count() == meta["param_count"]
    assert np.all(np.isfinite(p)) and np.count_nonzero(p) > p.size // 2
    assert meta["grid"] == 32 and meta["instances"] >= 100
    hist = meta["history"]
    assert len(hist) == meta["epochs"] and hist[-1]["val_loss"] < hist[0]["val_loss"]


def test_load_rejects_a_mismatched_description(tmp_path):
    d = tmp_path / "m"
    os.makedirs(d)
    np.arange(10, dtype="<f4").tofile(str(d / (learned.MODEL_NAME + ".f32")))
    with open(d / (learned.MODEL_NAME + ".json"), "w") as f:
        json.dump({"param_count": 11}, f)
    with pytest.raises(ValueError):
        learned.load_params(str(d))
    assert learned.load_params(str(tmp_path / "absent")) == (None, None)
