"""lbe_init_static (the context in the library's own device array, no device allocation) against
lbe_init with a caller workspace: same kernels, same launch plan, so the states agree bit for
bit; two static contexts in a row, the second on a smaller problem."""
import numpy as np
import pytest

from paper_2403_15051_amd import lbe, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lbe.load()


CASES = [
    ("fourier-cyl nr 96 + couette nr 40", [dict(W.FOURIER_CYL, nr=96), dict(W.COUETTE_SMALL, nr=40)], 120),
    ("couette nr 16", [dict(W.COUETTE_SMALL, nr=16)], 80),
]


def test_static_workspace_matches_caller_workspace():
    for name, ps, steps in CASES:
        print("case", name, flush=True)
        ref = lbe.Solver(ps)
        ref.step(steps)
        ref.sync()
        st = lbe.Solver(ps, static_ws=True)
        st.step(steps)
        st.sync()
        for k in range(len(ps)):
            a, b = st.get_state(k), ref.get_state(k)
            err = float(np.abs(a - b).max() / np.abs(b).max())
            print(name, "instance", k, "max rel diff", err, flush=True)
            assert err <= 1e-12
            ma, mb = st.moments(k), ref.moments(k)
            assert np.abs(ma["T"] - mb["T"]).max() <= 1e-12 * np.abs(mb["T"]).max()
        st.close()
        ref.close()


def test_static_workspace_limits():
    s1 = lbe.Solver(dict(W.COUETTE_SMALL, nr=16), static_ws=True)
    with pytest.raises(lbe.LbeError) as e:  # one static context per device at a time
        lbe.Solver(dict(W.COUETTE_SMALL, nr=16), static_ws=True)
    assert e.value.status == lbe.LBE_ESTATE
    s1.close()
    with pytest.raises(lbe.LbeError) as e:  # larger than the 64 MiB array
        lbe.Solver([dict(W.FOURIER_SPH)] * 2, static_ws=True)
    assert e.value.status == lbe.LBE_ENOMEM
    s2 = lbe.Solver(dict(W.COUETTE_SMALL, nr=12), static_ws=True)  # released: usable again
    s2.step(3)
    s2.sync()
    s2.close()
