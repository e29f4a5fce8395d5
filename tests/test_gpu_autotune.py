"""The panel-width autotuner (krr_autotune): it picks one of its candidate
widths for a size class, fits then give each system the width of its own
class, and -- since the persistent factorisation runs every system with its
own width -- a system's alpha is the same bit for bit whether it is fitted
alone or in a ragged batch with systems of other classes.  Results stay
within the mixed-precision tolerance of the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_00569_amd import datagen, krr
from _parity import ew

pytestmark = pytest.mark.gpu


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def test_tuned_widths_alone_equal_batched(dev):
    ctx = krr.Context(0)
    try:
        w_small, ms_small = ctx.autotune("mixed", 300, 10, n_sys=4)
        w_large, ms_large = ctx.autotune("mixed", 2500, 10, n_sys=4)
        print(f"tuned: m=300 -> {w_small} tiles ({ms_small:.2f} ms), m=2500 -> {w_large} tiles ({ms_large:.2f} ms)",
              flush=True)
        assert w_small in (2, 4) and w_large in (2, 4, 6, 8, 12, 16, 20, 24, 32)
        # a ragged batch: partitions of about 300 and about 2,500 points
        g = np.random.default_rng(12)
        sizes = [300, 2500, 280, 2600]
        X = np.concatenate([g.standard_normal((m, 10)) + 6.0 * g.standard_normal(10) for m in sizes])
        perm = g.permutation(X.shape[0])
        X = X[perm]
        y = np.sin(X[:, 0] + X[:, 1]) + 0.1 * g.standard_normal(X.shape[0])
        part = np.repeat(np.arange(4), sizes)[perm].astype(np.int32)
        C = np.stack([X[part == j].mean(0) for j in range(4)])
        params = [krr.Params(sigma=3.0, lam=1e-2, prec="mixed", refine_tol=1e-8, max_refine=20)]
        Xd, yd, ad, Cd = _t(X, dev), _t(y, dev), _t(part, dev), _t(C, dev)
        mb, ib, sb = ctx.fit(Xd, yd, ad, Cd, 4, params)
        assert sb == 0
        om = O.fit(X, y, part, C, 4, 3.0, 1e-2)
        for j in range(4):
            sel = np.nonzero(part == j)[0]           # increasing original index: the order inside a partition
            ma, ia, sa = ctx.fit(_t(X[sel], dev), _t(y[sel], dev), _t(np.zeros(sel.size, np.int32), dev),
                                 _t(C[j:j + 1], dev), 1, params)
            assert sa == 0
            alone = ma[0].alpha(0).cpu().numpy()
            batched = mb[0].alpha(j).cpu().numpy()
            assert np.array_equal(alone, batched), j
            assert ew(batched, om.alphas[j]) < 1e-6
            ma[0].free()
        mb[0].free()
    finally:
        ctx.close()
