"""pixelsne_kl_noalloc (the KL without device allocation) against pixelsne_kl.

Both run the same kernels over the same grid and reduce the partial sums on
the device in the same fixed order, so the results are equal bit for bit.
Two calls in a row on two contexts, the second with fewer points, so that
stale partial sums of the first call are left in the shared fixed buffer;
then the first context again.  Both precisions; the oracle's KL of the same
state pins the value (1e-5, the KL parity bar).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1611_02568_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def psne():
    from paper_1611_02568_amd import pixelsne
    pixelsne.load()
    assert torch.cuda.is_available()
    return pixelsne


def _ctx(psne, n, prec, seed):
    X, _ = datagen.small_mixture(n=n, D=20, seed=seed)
    P = oracle.build_P(X, 20.0)
    ctx = psne.Context.from_P(*P, screen=512, precision=prec,
                              Y_init=torch.as_tensor(datagen.initial_embedding(n, seed=seed + 1)))
    ctx.step(60)
    return ctx, P


@pytest.mark.parametrize("prec", [0, 1])
def test_kl_noalloc_matches_kl(psne, prec):
    big, Pb = _ctx(psne, 3000, prec, seed=70)
    small, Ps = _ctx(psne, 1200, prec, seed=80)
    for ctx, P in ((big, Pb), (small, Ps), (big, Pb)):
        a = ctx.kl_noalloc()
        b = ctx.kl()
        assert a == b, (a, b)
        st = ctx.get_state()
        ref = oracle.kl(st["z"].double().cpu().numpy(), np.array(st["s"]), P)
        assert abs(a - ref) <= 1e-5 * ref
