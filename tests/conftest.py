import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def alpha_ref(orc):
    """(m, s) of the oracle's alpha_p rule with the information the library has when it
    selects: ||A||_1 always; ||A^2||_1 when the plain rule's degree forms A^2 (m >= 2, else its
    bound ||A||^2); ||A^3||_1 when it forms A^3 (m >= 12, else its bound).  nk: the oracle's
    [||A||, ||A^2||, ||A^3||]."""
    def f(nk, u=2.0 ** -53):
        n1 = float(nk[0])
        mp, _ = orc.select_plain(n1, u)
        n2 = float(nk[1]) if mp >= 2 else n1 * n1
        n3 = float(nk[2]) if mp >= 12 else None
        return orc.select_alpha(orc.alpha_bounds(n1, n2, n3), u)
    return f
