"""Batched Lanczos: many windows of different shape in one set of launches.

With the plans' own tile shapes (tuning off) each instance of a batch runs exactly the
arithmetic of its single-plan solve (same kernels per tile, same fixed-order
reductions): energies, step counts and Ritz vectors equal the single-plan results bit
for bit.  With the tuned shapes (default) the block GEMMs may sum in another order:
results agree to the precision's rounding.  Both match the FP64 oracle's Lanczos."""
import sys
import time

import numpy as np
import pytest

from oracle import blocksparse as bs
from oracle import lanczos as olz

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_03318_amd as pk  # noqa: E402
from gpu_helpers import WindowGPU, problem, to_dev  # noqa: E402

NAMES = ["ly3_chi16", "ly4_chi64", "ly6_chi200", "ly4_chi64", "ly3_chi16"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def starts(name, seed):
    wl, L, W1, W2, R, th, keys, mpo = problem(name)
    rng = np.random.default_rng(seed)
    v = bs.flatten(th, keys)
    return v + 0.3 * (rng.standard_normal(v.size) + 1j * rng.standard_normal(v.size))


# matvec tolerance of each precision (relative to the largest element)
TOL = {pk.DM_FP64: 1e-12, pk.DM_FP32: 2e-5, pk.DM_BF16X3: 1e-4}


@pytest.mark.parametrize("tuned", [False, True])
@pytest.mark.parametrize("prec", [pk.DM_FP64, pk.DM_FP32, pk.DM_BF16X3])
def test_batched_equals_single(prec, tuned, monkeypatch):
    say(f"batched vs single prec={prec} tuned={tuned}")
    monkeypatch.setenv("MRDMRG_TUNE", "1" if tuned else "0")
    gs, plans, x0 = [], [], []
    for i, name in enumerate(NAMES):
        wl, L, W1, W2, R, th, keys, mpo = problem(name)
        g = WindowGPU(wl, L, R, mpo)
        gs.append((g, keys))
        plans.append(g.plan(prec))
        x0.append(to_dev(g.pack_theta(bs.unflatten(starts(name, 10 + i), keys))))
    batch = pk.Batch(plans)
    for rep in range(2):
        xb = [x.clone() for x in x0]
        t0 = time.perf_counter()
        eb, kb, us = pk.lanczos_ground_batched(batch, xb, 30, 1e-14)
        wall_us = 1e6 * (time.perf_counter() - t0)
        for i, p in enumerate(plans):
            xs = x0[i].clone()
            es, ks = pk.lanczos_ground(p, xs, 30, 1e-14)
            assert kb[i] == ks, (rep, i)
            if tuned:
                assert abs(eb[i] - es) <= 100 * TOL[prec] * abs(es), (rep, i, eb[i], es)
                assert 1 - abs(complex(torch.vdot(xb[i], xs))) <= 100 * TOL[prec], (rep, i)
            else:
                assert eb[i] == es, (rep, i, eb[i], es)
                assert torch.equal(xb[i], xs)
            assert 0 < us[i] <= wall_us
    if tuned:
        say(batch.info())
        assert batch.info().count("bucket") >= 2
    if prec == pk.DM_FP64:
        for i, name in enumerate(NAMES):
            wl, L, W1, W2, R, th, keys, mpo = problem(name)
            mv = lambda v: bs.flatten(bs.heff_apply(L, W1, W2, R, bs.unflatten(v, keys)), keys)
            eo, vo, ko, _, _ = olz.lanczos(mv, starts(name, 10 + i), max_iter=30)
            assert kb[i] == ko and abs(eb[i] - eo) <= 1e-10 * abs(eo)


def test_batch_rejects_mixed_precision_and_repeats():
    wl, L, W1, W2, R, th, keys, mpo = problem("ly3_chi16")
    g = WindowGPU(wl, L, R, mpo)
    p64, p32 = g.plan(pk.DM_FP64), g.plan(pk.DM_FP32)
    with pytest.raises(pk.LibraryError):
        pk.Batch([p64, p32])
    with pytest.raises(pk.LibraryError):
        pk.Batch([p64, p64])
