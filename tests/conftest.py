import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU (runs the HIP path)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def pytest_terminal_summary(terminalreporter):
    # the parity comparisons' z-score distribution tests (named; the unnamed ones are
    # the statistics' own tests on synthetic draws, some shifted on purpose)
    mc = sys.modules.get("mc_stats")
    named = [x for x in mc.KS_PVALUES if x[0]] if mc is not None else []
    if named:
        name, p = min(named, key=lambda x: x[1])
        terminalreporter.write_line(f"z-score distribution tests: {len(named)}, smallest p = {p:.3g} ({name})")
