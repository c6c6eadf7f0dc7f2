"""What the trained cost model gains over scheduling without it.

The network is trained on the GPU (the engine's own forward/backward/Adam
kernels) from timings of batch-workload instances, then used on fresh
learned-workload instances:
  - it must predict per-instance sweep cost better than the constant
    per-vector cost of the "cost is proportional to 2^k" heuristic;
  - the model-scheduled sweep must give bit-identical counts and must not be
    slower than the static round-robin fallback (the schedule without a model).
Timings are printed so the run records the size of the gain.
"""
import numpy as np
import pytest

import wpm_inputs as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_00806_amd import costmodel as CM, engine as E, scheduler as S
    return CM, E, S


def kernel_ms(E, S, batch, sw, plan, reps=3):
    sw.set_items(plan.items, segments=plan.segments)
    sw.launch(plan.mode, wg_size=256)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sw.launch(plan.mode, wg_size=256)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, sw.result()


def test_model_predicts_and_schedules_better_than_without(mods):
    CM, E, S = mods
    train = E.prepare_many(W.batch(E.kdim, count=1024))
    Xtr, Ttr, _ = S.measure_labels(train, cbits=12, wg=256, repeats=2)
    model = CM.CostModel(seed=0)
    model.fit(Xtr, Ttr, epochs=150, lr=3e-3, batch=256)

    fresh = E.prepare_many(W.learned(E.kdim, count=2048, start=20000))
    Xte, Tte, _ = S.measure_labels(fresh, cbits=12, wg=256, repeats=1)
    ok = np.isfinite(Tte[:, 0])
    pred = model.predict(Xte[ok])[:, 0]
    rmse_model = float(np.sqrt(np.mean((pred - Tte[ok, 0]) ** 2)))
    const = float(np.median(Ttr[np.isfinite(Ttr[:, 0]), 0]))
    rmse_const = float(np.sqrt(np.mean((const - Tte[ok, 0]) ** 2)))
    print(f"\nlog-RMSE of ns/vector on fresh instances: model {rmse_model:.3f}, constant {rmse_const:.3f}")
    assert rmse_model < rmse_const

    batch = E.DeviceBatch(fresh)
    sw = E.Sweeper(batch, cap=1 << 24)
    cost = S.per_vector_cost(model, CM.features_of(fresh))
    t_static, r_static = kernel_ms(E, S, batch, sw, S.make_plan(batch, "static", cbits=12, wg=256))
    t_model, r_model = kernel_ms(E, S, batch, sw, S.make_plan(batch, "dynamic", cost=cost, cbits=12, wg=256))
    t_pow2, r_pow2 = kernel_ms(E, S, batch, sw, S.make_plan(batch, "dynamic", cbits=12, wg=256))
    print(f"sweep ms: static round robin {t_static:.2f}, model LPT {t_model:.2f}, 2^k LPT {t_pow2:.2f}")
    assert np.array_equal(r_static.counts, r_model.counts)
    assert np.array_equal(r_static.counts, r_pow2.counts)
    assert t_model <= 1.02 * t_static
