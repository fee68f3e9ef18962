"""Host-side logic of the learned setup: the fallback rule and the committed
weight file (plain .npz, loadable without pickle, shape of a 4-layer,
24-channel network)."""
import json

import numpy as np


def test_fallback_rule():
    from paper_1611_01034_amd.learned_setup import decide_fallback
    assert decide_fallback(float("nan"), 0.5)
    assert decide_fallback(0.7, 0.5, margin=1.25)
    assert not decide_fallback(0.6, 0.5, margin=1.25)
    assert not decide_fallback(0.4, 0.5)


def test_committed_weights_file():
    import os
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_1611_01034_amd", "weights",
                     "net_l4_c24.npz")
    with np.load(p, allow_pickle=False) as z:
        params, C, L = z["params"], int(z["C"]), int(z["L"])
        meta = json.loads(str(z["meta"]))
    assert (C, L) == (24, 4)
    assert params.size == 2 * L * 9 * C * C * 16 + 2 * (L - 1) * C
    assert np.all(np.isfinite(params))
    assert meta["loss_history"][-1] < meta["loss_history"][0]
