"""What the trained cost model gains over scheduling without it.

The network is trained on the GPU (the engine's own forward/backward/Adam
kernels) from timings of batch-workload instances, then used on fresh
learned-workload instances:
  - it must predict per-instance sweep cost better than the constant
    per-vector cost of the "cost is proportional to 2^k" heuristic, over all
    instances and over the large ones that hold 90% of the vectors;
  - scheduled by the model, the sweep gives bit-identical counts and is
    compared with the same policy ordered by 2^k (the method without the
    model) and with static round robin (the fallback): the model's dynamic
    queue must be faster than static round robin, and within the run-to-run
    noise band (NOISE, 2% of the median) of the 2^k order or faster.  Medians
    of REPS timed launches each; the measured ratios are printed.
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


REPS = 5
NOISE = 0.02


def kernel_ms(E, S, batch, sw, plan, reps=REPS):
    sw.set_items(plan.items, segments=plan.segments)
    sw.launch(plan.mode, wg_size=256)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sw.launch(plan.mode, wg_size=256)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.median(ms)), sw.result()


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
    const = float(np.median(Ttr[np.isfinite(Ttr[:, 0]), 0]))
    rmse_model = float(np.sqrt(np.mean((pred - Tte[ok, 0]) ** 2)))
    rmse_const = float(np.sqrt(np.mean((const - Tte[ok, 0]) ** 2)))
    # the large instances: those holding 90% of the vectors
    vec = np.array([float(1 << p.k) for p in fresh])[ok]
    order = np.argsort(-vec)
    top = order[:int(np.searchsorted(np.cumsum(vec[order]) / vec.sum(), 0.9)) + 1]
    rmse_model_top = float(np.sqrt(np.mean((pred[top] - Tte[ok, 0][top]) ** 2)))
    rmse_const_top = float(np.sqrt(np.mean((const - Tte[ok, 0][top]) ** 2)))
    print(f"\nlog-RMSE of ns/vector on fresh instances: model {rmse_model:.3f}, constant {rmse_const:.3f}; "
          f"on the {len(top)} instances holding 90% of the vectors: model {rmse_model_top:.3f}, "
          f"constant {rmse_const_top:.3f}")
    assert rmse_model < rmse_const
    assert rmse_model_top < rmse_const_top

    batch = E.DeviceBatch(fresh)
    sw = E.Sweeper(batch, cap=1 << 24)
    cost = S.per_vector_cost(model, CM.features_of(fresh))
    t_static, r_static = kernel_ms(E, S, batch, sw, S.make_plan(batch, "static", cbits=12, wg=256))
    t_model, r_model = kernel_ms(E, S, batch, sw, S.make_plan(batch, "dynamic", cost=cost, cbits=12, wg=256))
    t_pow2, r_pow2 = kernel_ms(E, S, batch, sw, S.make_plan(batch, "dynamic", cbits=12, wg=256))
    p_model, r_pm = kernel_ms(E, S, batch, sw, S.make_plan(batch, "packed", cost=cost, cbits=12, wg=256))
    p_pow2, r_pp = kernel_ms(E, S, batch, sw, S.make_plan(batch, "packed", cbits=12, wg=256))
    print(f"sweep ms (medians of {REPS}): static round robin {t_static:.2f}, dynamic queue in model order "
          f"{t_model:.2f}, in 2^k order {t_pow2:.2f} (2^k / model = {t_pow2 / t_model:.3f}); packed bins "
          f"on model cost {p_model:.2f}, on 2^k {p_pow2:.2f} (2^k / model = {p_pow2 / p_model:.3f})")
    for r in (r_model, r_pow2, r_pm, r_pp):
        assert np.array_equal(r_static.counts, r.counts)
    assert t_model < t_static
    assert t_model <= (1 + NOISE) * t_pow2
