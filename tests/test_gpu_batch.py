"""Batched factorization: independent matrices factored in one launch.

Each handle's factor must equal the one an individual bilu_factor computes
(bit for bit: the same arithmetic per block) and the oracle's (partition,
patterns, values within the tolerance, iteration counts)."""
import math
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


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def factor_bytes(f):
    return (f.starts.tobytes(), f.starts_initial.tobytes(), [r.tobytes() for r in f.R],
            [c.tobytes() for c in f.C], b"".join(x.tobytes() for x in f.L + f.W + f.D))


SMALL = [
    ("cd2d_24_b2", lambda: (mg.grid2d_random_blocks(24, 2, 3.5, seed=11), None), 1e-2, True),
    ("cd3d_10_b3", lambda: (mg.grid3d_convdiff(b=3, dims=(10, 10, 10), seed=12),
                            mg.node_perm_to_scalar(mg.grid_nd_node_order((10, 10, 10)), 3)), 1e-3,
     True),
    ("el3d_8_b3", lambda: (mg.grid3d_elasticity(side=8, b=3, seed=13), None), 5e-3, False),
    ("random", lambda: (mg.random_sparse(300, 0.02, seed=14, diag_shift=3.0), None), 1e-2, True),
    ("cd2d_12_b5", lambda: (mg.grid2d_random_blocks(12, 5, 6.0, seed=15), None), 1e-3, True),
    ("cd3d_6_b1", lambda: (mg.grid3d_convdiff(b=1, dims=(6, 6, 6), seed=16), None), 1e-2, False),
]


def test_batched_small_equals_individual_and_oracle():
    torch = _torch()
    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import bilu
    mats = [(name, *make(), tau, agg) for name, make, tau, agg in SMALL]
    hs = []
    for name, a, perm, tau, agg in mats:
        h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=agg)
        h.analyze(a, pre_perm=perm)
        hs.append(h)
    say(f"[batch] {len(hs)} small matrices, n = {[m[1].n for m in mats]}")
    bilu.factor_batched(hs, [m[3] for m in mats])
    for (name, a, perm, tau, agg), h in zip(mats, hs):
        fb = h.export()
        g = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=agg)
        g.analyze(a, pre_perm=perm)
        g.factor(tau)
        assert factor_bytes(fb) == factor_bytes(g.export()), name
        g.close()
        o = Oracle()
        assert o.run(a, OracleOptions(tau=tau, use_aggregation=agg), pre_perm=perm) == 0
        fo = o.factors()
        assert np.array_equal(fb.starts, fo.starts) and np.array_equal(fb.starts_initial,
                                                                       fo.starts_initial), name
        num = den = 0.0
        for k in range(len(fo.starts) - 1):
            assert np.array_equal(fb.R[k], fo.R[k]) and np.array_equal(fb.C[k], fo.C[k]), name
            for x, y in ((fb.L[k], fo.L[k]), (fb.W[k], fo.W[k]), (fb.D[k], fo.D[k])):
                num += float(np.sum((x - y) ** 2))
                den += float(np.sum(y ** 2))
        assert np.sqrt(num / den) <= 1e-10, name
        b = a.matvec(np.ones(a.n))
        _, info_o = o.fgmres(b, restart=30, rtol=1e-8)
        bd = torch.from_numpy(b).cuda()
        xd = torch.zeros_like(bd)
        info = h.fgmres(bd, xd, restart=30, rtol=1e-8)
        assert info["converged"] and info["iterations"] == info_o["iterations"], name
        say(f"[batch] {name}: n={a.n} blocks={len(fb.starts) - 1} iterations={info['iterations']}")
    for h in hs:
        h.close()


def test_batch64_one_launch():
    """The 64-matrix workload (2D/3D stencils, 1-6 unknowns per node, n
    log-uniform in [20k, 300k], tau in {1e-2, 1e-3}) in one launch; sampled
    handles equal their individual factorization bit for bit, and every
    system converges to 1e-8."""
    torch = _torch()
    from paper_1908_10169_amd import bilu
    descs = mg.batch_workloads(5, 64)
    ws = [mg.batch_matrix(d) for d in descs]
    say(f"[batch64] n total {sum(w.a.n for w in ws)}")
    hs = []
    for w in ws:
        h = bilu.Bilu(ordering=bilu.ORDER_NATURAL)
        h.analyze(w.a, pre_perm=w.perm)
        hs.append(h)
    bilu.factor_batched(hs, [w.tau for w in ws])
    say("[batch64] factored")
    for i in (0, 17, 63):
        g = bilu.Bilu(ordering=bilu.ORDER_NATURAL)
        g.analyze(ws[i].a, pre_perm=ws[i].perm)
        g.factor(ws[i].tau)
        assert factor_bytes(hs[i].export()) == factor_bytes(g.export()), i
        g.close()
    it64 = []
    for w, h in zip(ws, hs):
        b = w.a.matvec(np.ones(w.a.n))
        bd = torch.from_numpy(b).cuda()
        xd = torch.zeros_like(bd)
        info = h.fgmres(bd, xd, restart=30, rtol=1e-8)
        res = np.linalg.norm(b - w.a.matvec(xd.cpu().numpy())) / np.linalg.norm(b)
        assert info["converged"] and res <= 1e-8, w.name
        it64.append(info["iterations"])
    # a seeded sample of the batch against the oracle: partition, patterns,
    # values, iterations (the three smallest of eight drawn handles keep the
    # oracle's time bounded)
    from oracle import Oracle, OracleOptions
    rng = np.random.default_rng(64)
    drawn = sorted(rng.choice(64, size=8, replace=False), key=lambda i: ws[i].a.nnz)[:3]
    for i in drawn:
        w = ws[int(i)]
        o = Oracle()
        assert o.run(w.a, OracleOptions(tau=w.tau, use_aggregation=True), pre_perm=w.perm) == 0
        fb, fo = hs[int(i)].export(), o.factors()
        assert np.array_equal(fb.starts, fo.starts) and np.array_equal(fb.starts_initial,
                                                                       fo.starts_initial), w.name
        num = den = 0.0
        for k in range(len(fo.starts) - 1):
            assert np.array_equal(fb.R[k], fo.R[k]) and np.array_equal(fb.C[k], fo.C[k]), w.name
            for x, y in ((fb.L[k], fo.L[k]), (fb.W[k], fo.W[k]), (fb.D[k], fo.D[k])):
                num += float(np.sum((x - y) ** 2))
                den += float(np.sum(y ** 2))
        assert np.sqrt(num / den) <= 1e-10, w.name
        _, info_o = o.fgmres(w.a.matvec(np.ones(w.a.n)), restart=30, rtol=1e-8)
        assert it64[int(i)] == info_o["iterations"], w.name
        say(f"[batch64] {w.name} (n={w.a.n}) equals the oracle")
    for h in hs:
        h.close()
    # the configuration's arithmetic: FP32 updates in one launch, FP64 pivot
    # blocks and FGMRES; every system reaches 1e-8 within +10% of the FP64
    # iterations
    hs = []
    for w in ws:
        h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, update_precision=bilu.PREC_F32)
        h.analyze(w.a, pre_perm=w.perm)
        hs.append(h)
    bilu.factor_batched(hs, [w.tau for w in ws])
    say("[batch64] factored with FP32 updates")
    worst = 0.0
    for k, (w, h) in enumerate(zip(ws, hs)):
        b = w.a.matvec(np.ones(w.a.n))
        bd = torch.from_numpy(b).cuda()
        xd = torch.zeros_like(bd)
        info = h.fgmres(bd, xd, restart=30, rtol=1e-8)
        res = np.linalg.norm(b - w.a.matvec(xd.cpu().numpy())) / np.linalg.norm(b)
        assert info["converged"] and res <= 1e-8, w.name
        assert info["iterations"] <= math.ceil(1.1 * it64[k]), (w.name, info["iterations"], it64[k])
        worst = max(worst, info["iterations"] / it64[k])
        if k in (0, 31, 63):
            assert h.kept_residual() <= 1e-6, w.name
        h.close()
    say(f"[batch64] FP32: all converged; largest iteration ratio to FP64 {worst:.3f}")
