"""ire_run_noalloc, the entry point for callers that cannot allocate device
memory, against ire_run + ire_get_results (the existing entry point) through
the C-ABI: two calls in a row, the second with a smaller model and fewer
packages, so that the second call starts from a scratch array that holds the
first call's larger contents."""
import json
import os

import numpy as np
import pytest

import mc_stats
from paper_2408_13807_amd import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ire():
    from paper_2408_13807_amd import ire as lib
    return lib


def golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        g = json.load(f)
    return {k: np.asarray(v) if isinstance(v, list) else v for k, v in g.items()}


def both_entry_points(ire, h, model, n_ext, seed, **opts):
    """ire_run's results and ire_run_noalloc's, on one handle."""
    import torch
    h.set_model(model)
    h.set_options(**opts)
    h.run(n_ext, 0, seed)               # also puts the model's tables on the device
    ref = h.results()
    n = len(model["rho"])
    A = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    T = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    print(f"noalloc call: {n} shells, {n_ext} packages, {opts}", flush=True)
    h.run_noalloc(n_ext, 0, seed, A.data_ptr(), T.data_ptr())
    torch.cuda.synchronize()
    # the handle's own run is untouched
    again = h.results()
    np.testing.assert_array_equal(again["A"], ref["A"])
    return ref, A.cpu().numpy(), T.cpu().numpy()


def test_noalloc_serial_fp64_equals_ire_run(ire):
    # serial FP64 runs are deterministic: the two entry points give the same bits
    with ire.IREModel(0) as h:
        for model, n_ext in ((wl.cfg_external_large(), 800), (wl.cfg_external_small(), 300)):
            ref, A, T = both_entry_points(ire, h, model, n_ext, 21, stepping=ire.IRE_FP64, max_lanes=1)
            np.testing.assert_array_equal(A, ref["A"])
            np.testing.assert_array_equal(T, ref["T"])


def test_noalloc_parallel_fp32_matches_oracle_ensembles(ire):
    # the parallel FP32 path: both entry points within the oracle ensembles'
    # statistical bound, the larger cloud first
    with ire.IREModel(0) as h:
        for model, n_ext, gold, opts in ((wl.cfg_external_large(), 1_000_000, "ext101_tau10_1e6", {}),
                                         (wl.cfg_external_small(), 100_000, "ext50_tau1_1e5", dict(replicas=2))):
            g = golden(gold)
            ref, A, T = both_entry_points(ire, h, model, n_ext, 22, **opts)
            for name, t in (("ire_run", ref["T"]), ("ire_run_noalloc", T)):
                ok, f = mc_stats.compare(t, g["T_mean"], g["T_std"], g["A_mean"], g["A_std"], len(g["seeds"]),
                                         name=f"{gold} {name}")
                print(f"{gold} {name}: {f * 100:.1f}% of shells within max(1%, 3 sigma)")
                assert ok
            # the total absorbed power of the two runs agrees to its Monte Carlo scatter
            assert abs(A.sum() / ref["A"].sum() - 1) < 0.05


def test_noalloc_rejects_what_it_cannot_hold(ire):
    import torch
    A = torch.zeros(1000, dtype=torch.float64, device="cuda")
    T = torch.zeros(1000, dtype=torch.float64, device="cuda")
    with ire.IREModel(0) as h:
        h.set_model(wl.cfg_external_small())
        # tables not yet on the device
        with pytest.raises(ire.IREError) as e:
            h.run_noalloc(1000, 0, 1, A.data_ptr(), T.data_ptr())
        assert e.value.code == ire.IRE_E_STATE
        h.run(1000, 0, 1)
        h.results()
        with pytest.raises(ire.IREError) as e:
            h.run_noalloc(1000, 0, 1, 0, T.data_ptr())
        assert e.value.code == ire.IRE_E_INVALID
        # 600 shells x 8 accumulator groups exceed the fixed scratch
        big = wl.external_sphere(n=600, tau_V=1.0, K=8)
        h.set_model(big)
        h.set_options(replicas=8)
        h.run(1000, 0, 1)
        h.results()
        with pytest.raises(ire.IREError) as e:
            h.run_noalloc(1000, 0, 1, A.data_ptr(), T.data_ptr())
        assert e.value.code == ire.IRE_E_INVALID and "4096" in str(e.value)
