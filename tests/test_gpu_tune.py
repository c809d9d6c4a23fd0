"""The project's autotuner (slmc_autotune): every candidate it runs must give bitwise the
default's log-dets, signs and statuses (none rejected), and after tuning the evaluation
calls that pick up the choice return bitwise what they returned before."""

import numpy as np
import pytest

from synth import workload_item, workload_models

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1802_06177_amd as slmc  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("wl,lam_idx,items,prec", [("W2", 0, 16, "fp64"), ("W2", 0, 16, "int8x5"),
                                                   ("W4", 1, 8, "int8x5"), ("W4", 1, 8, "fp64")])
def test_autotune_candidates_are_bitwise_equal_and_choice_is_used(wl, lam_idx, items, prec):
    md = workload_models(wl, lam_idx)[0]
    m = slmc.model_from_dict(md)
    x = torch.tensor(np.stack([workload_item(wl, b, lam_idx)[1] for b in range(items)]),
                     dtype=torch.float64, device=DEV)
    opt = slmc.options(prec, 1)
    print("case: autotune %s items=%d prec=%s" % (wl, items, prec), flush=True)
    try:
        before = [t.cpu().numpy() for t in slmc.green(m, x, opt)]
        choice, tried, rejected = slmc.autotune(m, x, opt)
        print("  choice %s, %d candidates, %d rejected" % (choice, tried, rejected), flush=True)
        assert tried >= 9 and rejected == 0
        t, tuned = slmc.tuning(m, items, opt)
        assert tuned and t == choice
        after = [t.cpu().numpy() for t in slmc.green(m, x, opt)]
        for a, b in zip(before, after):
            assert np.array_equal(a, b)
    finally:
        slmc.cache_clear()
