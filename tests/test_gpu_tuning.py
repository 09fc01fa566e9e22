"""Tuned kernel settings: a table entry for the precision, width class and
reproducibility requirement of a factorization supplies the settings left
at their defaults, and the results stay what those settings compute."""
import json
import os
import sys

import numpy as np
import pytest

from paper_1908_10169_amd import matgen as mg

pytestmark = pytest.mark.gpu

SHIPPED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1908_10169_amd", "tuning", "gfx950.json")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_tuned_entry_applies(tmp_path):
    torch = _torch()
    from paper_1908_10169_amd import bilu
    w = mg.workload("cd3d_12_b4")
    table = {"version": 1, "entries": [
        dict(precision=0, width_class=0, reproducible=1, workers_per_cu=1, update_mfma=0,
             factor_path=2, apply_path=1, deterministic=1)]}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(table))
    x = torch.from_numpy(np.random.default_rng(5).standard_normal(w.a.n)).cuda()
    outs = []
    try:
        assert bilu.load_tuning(str(p)) == 1
        for use in (1, 0):
            h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_tuning=use)
            h.analyze(w.a, pre_perm=w.perm)
            h.factor(w.tau)
            assert h.stats()["tuning_applied"] == use
            assert h.stats()["max_width_initial"] <= 16
            y = torch.empty_like(x)
            h.apply(x, y)
            h.sync()
            f = h.export()
            outs.append((b"".join(v.tobytes() for v in f.L + f.W + f.D), y.cpu().numpy().tobytes()))
            h.close()
        print(f"[tuning] entry applied; identical bits with and without it", flush=True)
        sys.stdout.flush()
        # other settings compute the same bits (global staging, one worker per
        # CU, per-level apply)
        assert outs[0] == outs[1]
        # an entry for reproducible handles does not serve handles without
        # that requirement
        h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, deterministic=0)
        h.analyze(w.a, pre_perm=w.perm)
        h.factor(w.tau)
        assert h.stats()["tuning_applied"] == 0
        h.close()
    finally:
        bilu.load_tuning(SHIPPED if os.path.exists(SHIPPED) else None)
