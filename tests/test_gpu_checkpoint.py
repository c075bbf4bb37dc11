"""Checkpoint / resume through the C ABI.  lbe_checkpoint_save / lbe_checkpoint_load carry the exact
device state one step reads from the previous one, so stepping N, restoring into a fresh context and
stepping M equals stepping N + M bit for bit (FP64 and FP32 storage, across an FP32 mass fix, and
after the steady driver switched an FP32 instance to FP64 storage).  lbe_get_state / lbe_set_state
carry f only: the fresh context recomputes the moment sums from f with a different summation, so
that resume agrees to rounding."""
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


BATCH = [dict(W.COUETTE_SMALL, nr=16), dict(W.FOURIER_SPH, nr=24, q_radial=4, q_t1=4, q_t2=4),
         dict(W.FOURIER_CYL, nr=40, q_radial=6, q_t1=6, q_t2=4)]


@pytest.mark.parametrize("precision", [lbe.FP64, lbe.FP32_STORE])
def test_checkpoint_resume_is_bitwise(precision):
    ps = [dict(p, precision=precision) for p in BATCH]
    a = lbe.Solver(ps)
    a.step(37)
    blob = a.checkpoint()
    a.step(23)  # crosses the FP32 mass fix at step 50
    b = lbe.Solver(ps)
    b.restore(blob)
    assert [b.info(k)["steps"] for k in range(len(ps))] == [37] * len(ps)
    b.step(23)
    for k in range(len(ps)):
        assert np.array_equal(a.get_state(k), b.get_state(k)), k


def test_checkpoint_after_the_switch_to_fp64_storage():
    p = dict(W.FOURIER_CYL, nr=32, q_radial=4, q_t1=4, q_t2=4, precision=lbe.FP32_STORE)
    a = lbe.Solver(p)
    st, steps, res = a.run_to_steady(1e-8, 400000, 50)
    info = a.info(0)
    print("steps", steps[0], "residual", res[0], "switched at", info["promoted_at"], flush=True)
    assert st == lbe.LBE_OK and info["fp32_now"] == 0
    blob = a.checkpoint()
    b = lbe.Solver(p)
    b.restore(blob)
    assert b.info(0)["fp32_now"] == 0
    a.step(20)
    b.step(20)
    assert np.array_equal(a.get_state(0), b.get_state(0))


def test_checkpoint_of_other_problems_is_rejected():
    a = lbe.Solver(BATCH[:2])
    blob = a.checkpoint()
    b = lbe.Solver([BATCH[0], dict(BATCH[1], kn=0.06)])
    with pytest.raises(lbe.LbeError) as e:
        b.restore(blob)
    assert e.value.status == lbe.LBE_EINVAL
    with pytest.raises(lbe.LbeError):
        b.restore(blob[:100])


def test_state_resume_agrees_to_rounding():
    ps = BATCH
    a = lbe.Solver(ps)
    a.step(40)
    b = lbe.Solver(ps)
    for k in range(len(ps)):
        b.set_state(k, a.get_state(k))
    a.step(30)
    b.step(30)
    for k in range(len(ps)):
        fa, fb = a.get_state(k), b.get_state(k)
        assert np.abs(fa - fb).max() <= 1e-13 * np.abs(fa).max(), k
