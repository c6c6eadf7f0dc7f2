"""Cost-model kernels vs the fp64 reference, and the packed schedule.

Tolerance: fp32 sums of at most B + 64 products (B <= 256 here) carry a
relative rounding error of about (B + 64) * 2^-24 ~ 2e-5 of the sum of the
absolute terms; outputs use rel 1e-4, gradients abs 1e-5 x max|gradient|
(cancellation makes small entries' relative error meaningless).
"""
import numpy as np
import pytest

import oracle as O
import wpm_inputs as W
from oracle import mlp_ref as R

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def CM():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_00806_amd import costmodel
    return costmodel


def data(seed, B):
    rng = np.random.default_rng(seed)
    X = rng.normal(1.0, 2.0, (B, 16)).astype(np.float32)
    T = rng.normal(0.0, 1.5, (B, 2)).astype(np.float32)
    return X, T


def test_forward_matches_reference(CM):
    X, T = data(0, 300)
    p = CM.init_params(3)
    norm = CM.make_norm(X, T)
    m = CM.CostModel(p, norm)
    got = m.predict(X)
    want, _ = R.forward(p.astype(np.float64), norm.astype(np.float64), X.astype(np.float64))
    np.testing.assert_allclose(got, want, rtol=1e-4, atol=1e-5)


def test_gradient_and_loss_match_reference(CM):
    X, T = data(1, 256)
    p = CM.init_params(4)
    norm = CM.make_norm(X, T)
    m = CM.CostModel(p, norm)
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(T).cuda()
    from paper_2301_00806_amd import _lib as L
    work = torch.empty(int(L.lib().wpm_mlp_work_floats(len(X))), dtype=torch.float32, device="cuda")
    g = torch.empty(L.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    m.grad(Xd, Td, work, g, loss)
    lref, gref = R.loss_and_grad(p.astype(np.float64), norm.astype(np.float64), X.astype(np.float64),
                                 T.astype(np.float64))
    gg = g.cpu().numpy()
    assert abs(loss.item() - lref) <= 1e-4 * abs(lref)
    np.testing.assert_allclose(gg, gref, rtol=0, atol=1e-5 * np.abs(gref).max())
    # determinism: the fixed-order reduction gives identical bits
    g2 = torch.empty_like(g)
    m.grad(Xd, Td, work, g2, None)
    assert torch.equal(g, g2)


def test_adam_step_matches_reference(CM):
    X, T = data(2, 128)
    p = CM.init_params(5)
    norm = CM.make_norm(X, T)
    m = CM.CostModel(p, norm)
    from paper_2301_00806_amd import _lib as L
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    work = torch.empty(int(L.lib().wpm_mlp_work_floats(len(X))), dtype=torch.float32, device="cuda")
    g = torch.empty(L.MLP_PARAMS, dtype=torch.float32, device="cuda")
    pr, mr, vr = p.astype(np.float64), np.zeros(R.NPARAM), np.zeros(R.NPARAM)
    for step in range(1, 4):
        m.grad(Xd, Td, work, g, None)
        gcpu = g.cpu().numpy().astype(np.float64)
        m.adam(g, 1e-3, weight_decay=1e-4)
        pr, mr, vr = R.adam_step(pr, gcpu, mr, vr, step, 1e-3, weight_decay=1e-4)
        np.testing.assert_allclose(m.params.cpu().numpy(), pr, rtol=1e-5, atol=1e-6)
        pr = m.params.cpu().numpy().astype(np.float64)  # follow the device trajectory


def test_training_on_gpu_reduces_loss(CM):
    rng = np.random.default_rng(7)
    X = rng.normal(size=(2048, 16)).astype(np.float32)
    T = np.stack([np.sin(X[:, 0]) + 0.5 * X[:, 1] ** 2, X[:, 2] * X[:, 3]], 1).astype(np.float32)
    m = CM.CostModel(seed=1)
    m.norm = torch.from_numpy(CM.make_norm(X, T)).cuda()
    l0 = m.loss(X, T)
    m.fit(X, T, epochs=60, lr=3e-3, batch=256)
    l1 = m.loss(X, T)
    assert l1 < 0.2 * l0, (l0, l1)


def test_packed_schedule_counts_match(CM):
    from paper_2301_00806_amd import engine as E
    insts = W.batch(E.kdim, count=64)
    preps = E.prepare_many(insts)
    ref, _ = E.sweep(preps, mode=2, cbits=9, want_sets=False)
    batch = E.DeviceBatch(preps)
    sw = E.Sweeper(batch, cap=1 << 20)
    items = E.build_queue(batch.k, 9, 256)
    for bins in (1, 7, E.persistent_grid(batch, 256)):
        cost = np.random.default_rng(bins).uniform(0.1, 2.0, len(preps)).astype(np.float32)
        out, offs, _ = E.pack_bins(items, bins, cost)
        sw.set_items(out, bin_offsets=offs)
        sw.launch(3, wg_size=256)
        res = sw.result()
        assert np.array_equal(res.counts, ref.counts), bins
