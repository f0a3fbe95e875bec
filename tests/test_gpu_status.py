"""GPU checks of the device-side status words: a NaN or infinite value that
a launch stores is reported (GE_ERR_NONFINITE) by the plan's check call and
by its next call; a wave's wait for a neighbouring wave that gives up is
reported as GE_ERR_SYNC.  Both conditions are forced as data or from the
host (a poll bound of zero): every kernel still exits normally."""
import numpy as np
import pytest

from paper_1310_3422_amd import ge, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    ge.lib()


def _raises(status, fn):
    with pytest.raises(ge.GEError) as ei:
        fn()
    assert ei.value.status == status, str(ei.value)


@pytest.mark.parametrize("precision,k", [("fp64", 0), ("fp32", 0), ("fp32c", 0),
                                         ("fp64", 16), ("fp32", 4)])
def test_nonfinite_state_is_reported(precision, k):
    n = 131071                       # n + 1 a multiple of 2k for the sub-domain plans
    u0 = inputs.sine_rod(n, seed=5)
    plan = ge.Plan(n, 2.0, precision, k=k)
    ws = plan.new_workspace()
    # a clean run raises nothing
    u = ge.pack_state(u0, precision)
    plan.step_n(u, 0, 40, ws)
    plan.check()
    # a NaN in the state spreads and is stored
    bad = u0.copy()
    bad[70000] = np.nan
    u = ge.pack_state(bad, precision)
    plan.step_n(u, 0, 40, ws)
    _raises(ge.GE_ERR_NONFINITE, plan.check)
    plan.check()                     # reported once, then cleared
    # the next call reports a finished launch's condition and enqueues nothing
    plan.step_n(u, 40, 10, ws)
    torch.cuda.synchronize()
    before = u.clone()
    _raises(ge.GE_ERR_NONFINITE, lambda: plan.step_n(u, 50, 10, ws))
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(before), torch.nan_to_num(u))
    plan.check()


def test_infinite_wall_result_is_reported():
    n = 5000
    plan = ge.Plan(n, 1.0, "fp64")
    u = ge.pack_state(np.zeros(n), "fp64")
    gl = torch.zeros(11, dtype=torch.float64, device="cuda")
    gl[5] = float("inf")
    plan.step_n(u, 0, 10, g_left_t=gl)
    _raises(ge.GE_ERR_NONFINITE, plan.check)


@pytest.mark.parametrize("precision", ["fp32", "fp64", "fp32c"])
def test_batch_nonfinite_is_reported(precision):
    rb = inputs.rod_batch(seed=31, nrods=40, nmin=64, nmax=70000, align=4)
    b = ge.Batch.from_inputs(rb, precision)
    ws = b.new_workspace()
    u = ge.pack_batch_state(rb.u0, rb.offsets, rb.n, precision)
    b.solve(u, 0, 30, ws)
    b.check()
    bad = rb.u0.copy()
    bad[rb.offsets[7] + 3] = np.nan
    u = ge.pack_batch_state(bad, rb.offsets, rb.n, precision)
    b.solve(u, 0, 30, ws)
    _raises(ge.GE_ERR_NONFINITE, b.check)
    b.check()


def test_batch_wait_that_gives_up_is_reported():
    """Rods of several waves exchanging edge values every level (sync = 2):
    with a poll bound of zero every wait gives up at once; the run ends
    normally and reports GE_ERR_SYNC (to the next solve and to the check).
    With the bound restored the same plan gives the barrier form's bits."""
    rb = inputs.rod_batch(seed=32, nrods=24, nmin=3000, nmax=30000, align=4)
    ref = ge.Batch.from_inputs(rb, "fp32", sync=1)
    wref = ref.new_workspace()
    u_ref = ge.pack_batch_state(rb.u0, rb.offsets, rb.n, "fp32")
    ref.solve(u_ref, 0, 50, wref)
    ref.check()

    b = ge.Batch.from_inputs(rb, "fp32", sync=2)
    ws = b.new_workspace()
    b.set_wait_polls(0)

    def drain():
        # a wave that gave up read edge slots that may hold anything, NaN
        # included, so a non-finite report may follow the wait's
        for _ in range(2):
            try:
                b.check()
                return
            except ge.GEError as e:
                assert e.status == ge.GE_ERR_NONFINITE, str(e)

    u = ge.pack_batch_state(rb.u0, rb.offsets, rb.n, "fp32")
    b.solve(u, 0, 50, ws)
    torch.cuda.synchronize()
    _raises(ge.GE_ERR_SYNC, lambda: b.solve(u, 50, 10, ws))   # reported at the next call
    drain()
    u = ge.pack_batch_state(rb.u0, rb.offsets, rb.n, "fp32")
    b.solve(u, 0, 50, ws)
    _raises(ge.GE_ERR_SYNC, b.check)
    drain()

    b.set_wait_polls(1 << 16)
    u = ge.pack_batch_state(rb.u0, rb.offsets, rb.n, "fp32")
    b.solve(u, 0, 50, ws)
    b.check()
    assert torch.equal(u, u_ref)
    with pytest.raises(ge.GEError):
        b.set_wait_polls(-1)
