"""What the trained warm-start network gains over the method without it.

The committed network (trained on the GPU by the library's own kernels on labels from the
float64 optimiser) picks initial log-hyperparameters for held-out mass-spring-damper
datasets; the default initialisation stays the fallback (used whenever its NLML is
lower).  After the same number of Adam steps, the warm-started NLML must on average be
below the default-initialised one, and the fallback guarantees it never starts worse.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from tests.test_gpu_parity import lib  # noqa: E402,F401


def test_warm_start_beats_default_on_heldout(lib):
    from paper_2505_00136_amd import warmstart as W
    if not os.path.exists(W.MODEL_PATH):
        pytest.skip("no trained warm-start network in the tree")
    model = W.WarmStartModel.load(W.MODEL_PATH)
    assert model.params.shape == (lib.gpr_mlp_nparams(),)
    runner = W.Runner()
    rows = W.evaluate(runner, model, [20000 + j for j in range(6)], steps=20)
    for r in rows:
        start = min(r["nlml0_learned"], r["nlml0_default"])
        # fallback: the chosen start is never worse than the default start
        assert start <= r["nlml0_default"] + 1e-12
    gain = np.mean([r["final_default"] - r["final_warm"] for r in rows])
    assert gain > 0.0, rows
