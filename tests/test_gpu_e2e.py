"""Whole runs, GPU against oracle: independent setups (each side builds its
own kNN, P and initial scaling from the same X and y(0)), 1,000 iterations
each, final KL within 1% (both embeddings scored by the oracle's exact-Z KL
of Eq. 4 with the oracle's P).

* 2,000 x 50 float64 mixture, perplexity 30, screen 512 (the small workload),
  both precisions;
* 10,000 x 784 uint8 mixture, perplexity 30, screen 1024: the MNIST-shaped
  workload's recipe at a size the oracle runs in seconds, FP32 path;
* 20,000 x 128 Zipf(1.1) mixture, perplexity 50, k 150, screen 2048: the
  1M workload's recipe at reduced n, both precisions.

Slow (set PSNE_SLOW=1; each takes minutes of oracle time on the host):
* the full 70,000 x 784 uint8 workload, independent setups;
* 1,000,000 points at the benchmark's P size (258 nonzeros per row, a
  synthetic P from the generators: the oracle cannot build P from a million
  rows in test time), screen 2048, FP32 path.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1611_02568_amd import datagen

pytestmark = pytest.mark.gpu

slow = pytest.mark.skipif(os.environ.get("PSNE_SLOW") != "1",
                          reason="minutes of oracle time on the host; set PSNE_SLOW=1")


@pytest.fixture(scope="module")
def psne():
    from paper_1611_02568_amd import pixelsne
    pixelsne.load()
    assert torch.cuda.is_available()
    return pixelsne


_oracle_runs = {}


def _oracle_run(key, X, u, r, y0, k=None, iters=1000):
    """The oracle's own P and 1,000 iterations (cached per workload)."""
    if key not in _oracle_runs:
        P = oracle.build_P(X.astype(np.float64), u, k=k)
        st = oracle.State(y0, r)
        oracle.iterate(st, oracle.params(r), P, iters)
        _oracle_runs[key] = (P, st, oracle.kl(st.z, st.s, P))
    return _oracle_runs[key]


def _gpu_kl(psne, X, u, r, y0, prec, P, iters=1000):
    ctx = psne.Context.from_data(torch.as_tensor(X).cuda(), u, r, Y_init=torch.as_tensor(y0),
                                 precision=prec)
    ctx.step(iters)
    st = ctx.get_state()
    z = st["z"].double().cpu().numpy()
    kl_own = ctx.kl()
    kl = oracle.kl(z, np.array(st["s"]), P)
    # the library's own exact-Z KL agrees with the oracle's score of the same state
    assert abs(kl_own - kl) <= 1e-5 * kl
    return kl


@pytest.mark.parametrize("prec", [0, 1])
def test_e2e_small_mixture(psne, prec):
    X, _ = datagen.small_mixture(n=2000)
    y0 = datagen.initial_embedding(2000, seed=datagen.seed_for(0, 1))
    P, _, kl_o = _oracle_run("small", X, 30.0, 512, y0)
    kl_g = _gpu_kl(psne, X, 30.0, 512, y0, prec, P)
    assert abs(kl_g - kl_o) <= 0.01 * kl_o, (kl_g, kl_o)


def test_e2e_uint8_reduced(psne):
    X, _ = datagen.uint8_mixture(n=10000, D=784)
    y0 = datagen.initial_embedding(10000, seed=datagen.seed_for(1, 1))
    P, _, kl_o = _oracle_run("u8-10k", X, 30.0, 1024, y0)
    kl_g = _gpu_kl(psne, X, 30.0, 1024, y0, 0, P)
    assert abs(kl_g - kl_o) <= 0.01 * kl_o, (kl_g, kl_o)


@pytest.mark.parametrize("prec", [0, 1])
def test_e2e_zipf_reduced(psne, prec):
    X, _, _ = datagen.zipf_mixture_1m(n=20000)
    y0 = datagen.initial_embedding(20000, seed=datagen.seed_for(2, 1))
    P, _, kl_o = _oracle_run("zipf-20k", X, 50.0, 2048, y0, k=150)
    kl_g = _gpu_kl(psne, X, 50.0, 2048, y0, prec, P)
    assert abs(kl_g - kl_o) <= 0.01 * kl_o, (kl_g, kl_o)


@slow
def test_e2e_uint8_full(psne):
    X, _ = datagen.uint8_mixture(n=70000, D=784)
    y0 = datagen.initial_embedding(70000, seed=datagen.seed_for(1, 1))
    P, _, kl_o = _oracle_run("u8-70k", X, 30.0, 1024, y0)
    kl_g = _gpu_kl(psne, X, 30.0, 1024, y0, 0, P)
    print(f"70,000 x 784 uint8: KL gpu {kl_g:.6f} oracle {kl_o:.6f}", flush=True)
    assert abs(kl_g - kl_o) <= 0.01 * kl_o, (kl_g, kl_o)


@slow
def test_e2e_1m_synthetic_P(psne):
    n, r = 1_000_000, 2048
    P = datagen.circulant_affinities(n, 129, seed=datagen.seed_for(2, 5))
    y0 = datagen.initial_embedding(n, seed=datagen.seed_for(2, 1))
    ctx = psne.Context.from_P(*P, screen=r, Y_init=torch.as_tensor(y0), precision=0)
    ctx.step(1000)
    st = ctx.get_state()
    kl_g = oracle.kl(st["z"].double().cpu().numpy(), np.array(st["s"]), P)
    del ctx
    ost = oracle.State(y0, r)
    oracle.iterate(ost, oracle.params(r), P, 1000)
    kl_o = oracle.kl(ost.z, ost.s, P)
    print(f"1M synthetic P: KL gpu {kl_g:.6f} oracle {kl_o:.6f}", flush=True)
    assert abs(kl_g - kl_o) <= 0.01 * kl_o, (kl_g, kl_o)
