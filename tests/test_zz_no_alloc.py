"""bilu_apply_noalloc through the C ABI: the allocation-free apply equals
bilu_apply bit for bit, on two calls in a row with different handles, the
second with fewer unknowns (the fixed device array keeps the first call's
contents, which must not leak into the second)."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_1908_10169_amd import matgen as mg

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def factored(name):
    from paper_1908_10169_amd import bilu
    w = mg.workload(name)
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL)
    h.analyze(w.a, pre_perm=w.perm)
    h.factor(w.tau)
    return w, h


def test_apply_noalloc_equals_apply():
    torch = _torch()
    from paper_1908_10169_amd import bilu
    lib = bilu.load()
    for name in ("cd3d_24_b4", "cd2d_32x32_b3"):  # 55,296 then 3,072 unknowns
        w, h = factored(name)
        print(f"[noalloc] {name} n={w.a.n}", flush=True)
        sys.stdout.flush()
        x = torch.from_numpy(np.random.default_rng(3).standard_normal(w.a.n)).cuda()
        y_ref = torch.empty_like(x)
        y_na = torch.full_like(x, float("nan"))
        assert lib.bilu_apply(h._h, C.c_void_p(x.data_ptr()), C.c_void_p(y_ref.data_ptr())) == 0
        st = lib.bilu_apply_noalloc(h._h, C.c_void_p(x.data_ptr()), C.c_void_p(y_na.data_ptr()))
        assert st == bilu.BILU_OK, lib.bilu_last_error(h._h)
        assert lib.bilu_sync(h._h) == 0
        assert y_ref.cpu().numpy().tobytes() == y_na.cpu().numpy().tobytes()
        assert h.stats()["apply_faults"] == 0
        h.close()


def test_apply_noalloc_errors():
    torch = _torch()
    from paper_1908_10169_amd import bilu
    lib = bilu.load()
    h = bilu.Bilu()
    x = torch.zeros(8, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    assert lib.bilu_apply_noalloc(h._h, C.c_void_p(x.data_ptr()),
                                  C.c_void_p(y.data_ptr())) == bilu.BILU_ERR_STATE
    assert lib.bilu_apply_noalloc(h._h, C.c_void_p(x.data_ptr()),
                                  C.c_void_p(x.data_ptr())) == bilu.BILU_ERR_INVALID
    h.close()
