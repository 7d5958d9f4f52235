"""BF16-MFMA surrogate kernels: gradients against the FP64 CPU reference,
training, ensemble prediction, save/load, and graph-replayed training."""
import numpy as np
import pytest

from oracle import mlp_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sur():
    from paper_2408_13807_amd import surrogate
    return surrogate


def _data(n, seed=0):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(-1, 3, n), rng.uniform(0, 2, n), rng.uniform(-1, 2, n),
                         rng.uniform(-1, 2, n), rng.integers(0, 2, n), rng.uniform(0, 1, n)]).astype(np.float32)
    y = (1.2 + 0.3 * np.sin(X[:, 0]) - 0.2 * X[:, 5] * X[:, 1] + 0.1 * X[:, 4]).astype(np.float32)
    return X, y


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("depth", [1, 4])
def test_gradients_match_fp64_reference(sur, depth):
    net = sur.SurNet(members=2, depth=depth, seed=3)
    X, y = _data(1000, seed=1)
    xm, xs = X.mean(axis=0), X.std(axis=0)
    ym, ys = float(y.mean()), float(y.std())
    net.set_normalization(xm, xs, ym, ys)
    P = net.get_params()
    loss, G = net.gradients(X, y)
    for m in range(2):
        lr, gr = mlp_ref.loss_and_grad(P[m].astype(np.float64), depth, X, y, xm, xs, ym, ys)
        assert abs(loss[m] / lr - 1) < 2e-2, (loss[m], lr)
        # block by block: BF16 operands with FP32 accumulation against FP64
        o = 0
        blocks = [256 * 32] + [256 * 256] * (depth - 1) + [256] * depth + [256, 1]
        for k, size in enumerate(blocks):
            e = _rel(G[m, o:o + size].astype(np.float64), gr[o:o + size])
            assert e < 5e-2, (m, k, e)
            o += size
        cos = G[m] @ gr / (np.linalg.norm(G[m]) * np.linalg.norm(gr))
        assert cos > 0.999
    net.close()


@pytest.mark.parametrize("members,depth", [(3, 4), (3, 1), (2, 2), (1, 3)])
def test_prediction_matches_reference_forward(sur, members, depth):
    # depth 1: the first layer is also the last (its epilogue folds the output
    # layer); one member: zero spread; 3000 rows: 24 tiles, the last one ragged
    net = sur.SurNet(members=members, depth=depth, seed=5)
    X, y = _data(3000, seed=2)
    xm, xs = X.mean(axis=0), X.std(axis=0)
    net.set_normalization(xm, xs, 1.2, 0.25)
    P = net.get_params()
    mean, spread = net.predict(X)
    ref = np.stack([mlp_ref.predict_logT(P[m].astype(np.float64), depth, X, xm, xs, 1.2, 0.25)
                    for m in range(members)])
    assert np.max(np.abs(mean - ref.mean(axis=0))) < 2e-2
    if members > 1:
        T = 10.0 ** ref
        sp = T.std(axis=0, ddof=1) / T.mean(axis=0)
        assert np.max(np.abs(spread - sp)) < 5e-3 + 0.05 * sp.max()
    else:
        assert np.all(spread == 0.0)
    net.close()


@pytest.mark.parametrize("use_graph", [1, 0])
def test_training_reduces_loss(sur, use_graph):
    X, y = _data(50_000, seed=3)
    net = sur.SurNet(members=2, depth=4, seed=7)
    loss0, _ = net.gradients(X[:4096], y[:4096])
    loss = net.train(X, y, steps=300, batch=1024, lr=2e-3, use_graph=use_graph)
    assert np.all(loss < 0.05 * loss0), (loss0, loss)
    Xt, yt = _data(5000, seed=4)
    mean, spread = net.predict(Xt)
    assert np.sqrt(np.mean((mean - yt) ** 2)) < 0.05
    net.close()


def test_save_load_roundtrip(sur, tmp_path):
    net = sur.SurNet(members=2, depth=2, seed=9)
    X, y = _data(2000, seed=5)
    net.train(X, y, steps=20, batch=512)
    path = str(tmp_path / "net.sur")
    net.save(path)
    a = net.predict(X)
    other = sur.SurNet(members=2, depth=2, seed=10)
    other.load(path)
    b = other.predict(X)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    net.close()
    other.close()


def test_predict_models_matches_row_prediction(sur):
    from paper_2408_13807_amd import workloads as wl
    params = wl.batch_parameters(300, seed=8)
    X, offs = wl.study_features(params)
    net = sur.SurNet(members=3, depth=4, seed=11)
    net.set_normalization(X.mean(axis=0), X.std(axis=0), 1.3, 0.4)
    mean_r, spread_r = net.predict(X)
    q = wl.study_model_inputs(params)
    mean_m, spread_m, ms = net.predict_models(q["model_x"], q["row_off"], q["radius_off"], q["radius"])
    # the same normalised inputs reach the same kernels: identical results
    np.testing.assert_array_equal(mean_m, mean_r)
    np.testing.assert_array_equal(spread_m, spread_r)
    np.testing.assert_array_equal(ms, np.maximum.reduceat(spread_r, offs[:-1]))
    # and the FP64 reference forward on a few models
    P = net.get_params()
    for m in (0, 17, 299):
        rows = slice(offs[m], offs[m + 1])
        ref = np.stack([mlp_ref.predict_logT(P[k].astype(np.float64), 4, X[rows], X.mean(axis=0), X.std(axis=0),
                                             1.3, 0.4) for k in range(3)]).mean(axis=0)
        assert np.max(np.abs(mean_m[rows] - ref)) < 2e-2
    # a subset in another order, with an empty model in between
    sub = [5, 2, 250]
    q2 = wl.study_model_inputs(params, sub)
    ro = np.concatenate([q2["row_off"][:2], q2["row_off"][1:]])
    ra = np.concatenate([q2["radius_off"][:1], [0], q2["radius_off"][1:]])
    mx = np.concatenate([q2["model_x"][:1], np.zeros((1, 5), np.float32), q2["model_x"][1:]])
    mean_s, _, ms_s = net.predict_models(mx, ro, ra, q2["radius"])
    ref = np.concatenate([mean_r[offs[k]:offs[k + 1]] for k in sub])
    np.testing.assert_array_equal(mean_s, ref)
    assert ms_s[1] == 0.0 and ms_s[0] == ms[5] and ms_s[3] == ms[250]
    net.close()


def test_predict_models_tiles_over_many_models(sur):
    # models of 0-3 rows (a quarter empty), with a stretch of 0/1-row models so
    # that a 128-row tile spans more than the 64 model boundaries the kernel
    # stages: the 64-way search for a tile's first model, the bisection over the
    # staged boundaries and the walk beyond them, against the row path
    rng = np.random.default_rng(21)
    n_models = 3000
    rows = rng.integers(0, 4, n_models)
    rows[:400] = rng.integers(0, 2, 400)
    row_off = np.concatenate([[0], np.cumsum(rows)]).astype(np.int64)
    model_x = np.column_stack([rng.uniform(-1, 3, n_models), rng.uniform(0, 2, n_models), rng.uniform(-1, 2, n_models),
                               rng.uniform(-1, 2, n_models), rng.integers(0, 2, n_models)]).astype(np.float32)
    radius = rng.uniform(1e-3, 1.0, int(row_off[-1])).astype(np.float32)
    X = np.column_stack([np.repeat(model_x, rows, axis=0), radius]).astype(np.float32)
    net = sur.SurNet(members=3, depth=4, seed=4)
    net.set_normalization(X.mean(axis=0), X.std(axis=0), 1.3, 0.4)
    mean_r, spread_r = net.predict(X)
    mean_m, spread_m, ms = net.predict_models(model_x, row_off, row_off[:-1], radius)
    np.testing.assert_array_equal(mean_m, mean_r)
    np.testing.assert_array_equal(spread_m, spread_r)
    expect = np.zeros(n_models, np.float32)
    full = rows > 0
    expect[full] = np.maximum.reduceat(spread_r, row_off[:-1][full])
    np.testing.assert_array_equal(ms, expect)
    assert rows[:400].sum() < 256      # the first tiles hold more than 64 models each
    net.close()


def test_ire_profiles_in_several_launches(sur):
    # a long model list runs as several batched launches, each prepared on the
    # host while the previous one runs: every model gets its own temperatures, in
    # order (against one launch of all; independent realisations, but the models'
    # profiles differ by far more than their noise)
    from paper_2408_13807_amd import workloads as wl
    params = wl.batch_parameters(23, seed=17)
    one = sur.ire_profiles(params, range(23), package_scale=0.2)
    many = sur.ire_profiles(params, range(23), package_scale=0.2, chunk=5)
    np.testing.assert_array_equal(many["row_off"], one["row_off"])
    assert many["packages"] == one["packages"]
    for m in range(23):
        s = slice(one["row_off"][m], one["row_off"][m + 1])
        assert np.median(np.abs(many["T"][s] - one["T"][s]) / one["T"][s]) < 0.05, m


def test_full_size_whole_model_prediction_on_samples(sur):
    # the benchmark's inference: 10^6 study models (2.1e8 rows, 5 members) in one
    # launch, sampled models against the FP64 forward, and every model's largest
    # spread against its rows'
    from paper_2408_13807_amd import workloads as wl
    params = wl.batch_parameters(1_000_000, seed=303)
    q = wl.study_model_inputs(params)
    net = sur.SurNet(members=5, depth=4, seed=7)
    Xs, _ = wl.study_features(params, np.arange(0, 1_000_000, 997))
    xm, xs = Xs.mean(axis=0), Xs.std(axis=0)
    net.set_normalization(xm, xs, 1.3, 0.4)
    mean, spread, ms = net.predict_models(q["model_x"], q["row_off"], q["radius_off"], q["radius"])
    ro = q["row_off"]
    assert len(mean) == ro[-1] > 2e8
    assert np.isfinite(mean).all() and np.isfinite(spread).all()
    P = net.get_params()
    rng = np.random.default_rng(4)
    sample = np.concatenate([[0, 999_999], rng.choice(1_000_000, 30, replace=False)])
    for m in sample:
        X, _ = wl.study_features(params, [m])
        ref = np.stack([mlp_ref.predict_logT(P[k].astype(np.float64), 4, X, xm, xs, 1.3, 0.4) for k in range(5)])
        rows = slice(ro[m], ro[m + 1])
        assert np.max(np.abs(mean[rows] - ref.mean(axis=0))) < 2e-2, m
        assert ms[m] == spread[rows].max(), m
    net.close()


def test_predict_models_rejects_bad_offsets(sur):
    from paper_2408_13807_amd import ire
    net = sur.SurNet(members=2, depth=2, seed=1)
    x = np.zeros((2, 5), np.float32)
    r = np.linspace(0.1, 0.9, 10).astype(np.float32)
    for ro, ra in (([1, 3, 6], [0, 0]),       # row_off[0] != 0
                   ([0, 5, 3], [0, 0]),       # decreasing
                   ([0, 5, 12], [0, 4]),      # radius range beyond the table
                   ([0, 5, 8], [-1, 0])):     # negative radius offset
        with pytest.raises(ire.IREError) as e:
            net.predict_models(x, np.array(ro), np.array(ra), r)
        assert e.value.code == ire.IRE_E_INVALID
    net.close()


def test_trained_surrogate_gains_over_the_tracer(sur):
    # End to end on a small parameter study: train the ensemble on batched IRE
    # temperatures of 8000 study models, then, on 512 held-out models, compare
    # surrogate-with-fallback against the batched tracer at the same budgets,
    # both scored against IRE at 16x each model's package budget.  Every model
    # is scored by its worst shell, the 95th percentile of its shells and their
    # median.  The worst shell of a model is mostly the Monte Carlo noise of a
    # rarely hit shell (in IRE itself and in the reference), so the claim is
    # comparative there: the models the surrogate accepts are within 2 % at
    # least as often as the tracer's own runs.  The surrogate must also answer
    # in a fraction of the tracer's time.
    import time

    from paper_2408_13807_amd import workloads as wl
    train = wl.batch_parameters(8000, seed=11)
    r = sur.ire_profiles(train, range(8000), package_scale=0.5)
    X, y = sur.training_set(train, range(8000), r["T"])
    print(f"training rows {len(y)}", flush=True)
    net = sur.fit(X, y, steps=8000, batch=4096, seed=3)
    try:
        held = wl.batch_parameters(512, seed=12)
        ref = sur.ire_profiles(held, range(512), package_scale=16.0)
        other = dict(held, seed=held["seed"] + np.uint64(1 << 20))
        own = sur.ire_profiles(other, range(512), package_scale=1.0)
        sur.predict_models(net, held, range(8))        # warm-up
        t0 = time.perf_counter()
        p = sur.predict_models(net, held, range(512))
        t_pred = time.perf_counter() - t0
        out = sur.predict_with_fallback(net, held, range(512), threshold=0.02)
    finally:
        net.close()
    acc = p["model_spread"] <= 0.02
    Ts = 10.0 ** p["logT"].astype(np.float64)
    summ = sur.error_summary(Ts, ref["T"], ref["row_off"], acc, {"ire_1x": own["T"]})
    for stat, row in summ.items():
        print(f"{stat}: within 2 %: surrogate accepted {row['surrogate_accepted']:.3f}, all {row['surrogate_all']:.3f}, "
              f"after fallback {row['after_fallback']:.3f}, tracer {row['ire_1x']:.3f}", flush=True)
    print(f"accepted {acc.mean():.2f}; prediction {t_pred * 1e3:.1f} ms vs tracer {own['seconds'] * 1e3:.1f} ms",
          flush=True)
    assert acc.mean() > 0.3
    # worst shell and 95th percentile: the accepted models at least as often within 2 % as the tracer's runs
    assert summ["max"]["surrogate_accepted"] >= summ["max"]["ire_1x"]
    assert summ["p95"]["surrogate_accepted"] >= summ["p95"]["ire_1x"]
    # the typical shell: accepted models' median error well inside 2 %, and after the fallback
    assert summ["median"]["median_error_surrogate_accepted"] < 0.01
    assert summ["median"]["after_fallback"] > 0.85
    # the fallback's temperatures are the tracer's own
    err_f = sur.model_errors(out["T"], ref["T"], ref["row_off"], "p95")
    assert np.isfinite(err_f).all()
    # the prediction of every model takes a fraction of what the tracer needs for them
    assert t_pred < 0.2 * own["seconds"]
