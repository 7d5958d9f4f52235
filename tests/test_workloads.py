"""The batched study's inputs built for many models at once
(workloads.study_shells, study_features, study_model_inputs) against the
one-model builders (batch_model, surrogate_features): the batched tracer and
the surrogate see the clouds the per-model runs see."""
import numpy as np

from paper_2408_13807_amd import workloads as wl


def test_study_shells_equal_the_per_model_clouds():
    params = wl.batch_parameters(300, seed=11)
    idx = np.array([7, 0, 299, 7, 150, 151, 3])       # any order, repeats
    r_flat, rho_flat = wl.study_shells(params, idx)
    ro = rd = 0
    for m in idx:
        mm = wl.batch_model(params, int(m))
        n = len(mm["rho"])
        np.testing.assert_array_equal(r_flat[ro:ro + n + 1], mm["r_edges"])
        np.testing.assert_allclose(rho_flat[rd:rd + n], mm["rho"], rtol=1e-12)
        ro += n + 1
        rd += n
    assert ro == len(r_flat) and rd == len(rho_flat)
    # the whole study at once, and no models
    r_all, rho_all = wl.study_shells(params)
    assert len(r_all) == int(np.sum(params["n"].astype(np.int64) + 1)) and len(rho_all) == int(np.sum(params["n"]))
    r0, rho0 = wl.study_shells(params, [])
    assert len(r0) == 0 and len(rho0) == 0


def test_study_features_follow_the_shells():
    params = wl.batch_parameters(40, seed=12)
    X, offs = wl.study_features(params)
    assert offs[-1] == len(X) == int(np.sum(params["n"]))
    for m in (0, 17, 39):
        mm = wl.batch_model(params, m)
        np.testing.assert_allclose(X[offs[m]:offs[m + 1]], wl.surrogate_features(params, m, mm["r_edges"]), rtol=1e-6)
