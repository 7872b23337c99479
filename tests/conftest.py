import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU-side check")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Report the worst gradient error seen against the oracle's conditioning
    (|g - g*| / (2^-24 kappa)), next to the constant the bar allows."""
    mod = sys.modules.get("test_gpu_parity")
    if mod is None or not getattr(mod, "KAPPA_RATIO", {}).get("n"):
        return
    k = mod.KAPPA_RATIO
    terminalreporter.write_line(
        f"gradient parity: worst |g - g*| / (2^-24 kappa) = {k['max']:.3g} over {k['n']} compared rows "
        f"(bar constant c(T) = {mod.gpu_rounding_constant(0.5):.0f} at T = 0.5)")


def pytest_runtest_setup(item):
    """With SSA_TEST_TRACE=1, name every test on stdout before it starts (a run
    that ends abruptly then still shows which test was running)."""
    if os.environ.get("SSA_TEST_TRACE") == "1":
        print(f"\n[start] {item.nodeid}", flush=True)
