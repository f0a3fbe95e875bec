"""The allocation-free batch entry point (ge_solve_batch_static): called
through the C ABI, it must give ge_solve_batch's bits, on two calls in a
row, the second with a smaller batch (the scratch keeps the first call's
contents), with rods above the on-chip limit in the first."""
import ctypes

import numpy as np
import pytest

from paper_1310_3422_amd import ge, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run_both(rb, precision, step0, nsteps):
    b = ge.Batch.from_inputs(rb, precision)
    u0 = ge.pack_batch_state(rb.u0, rb.offsets, rb.n, precision)
    ua = u0.clone()
    b.solve(ua, step0, nsteps, b.new_workspace())
    ub = u0.clone()
    st = ge.lib().ge_solve_batch_static(b.handle, ctypes.c_void_p(ub.data_ptr()), step0, nsteps,
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == ge.GE_OK, ge.last_error()
    b.check()
    torch.cuda.synchronize()
    return b, ua, ub


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32"])
def test_static_scratch_matches_the_workspace_entry_point(precision):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    big = inputs.rod_batch(seed=51, nrods=300, nmin=200, nmax=90000, align=4)
    b1, ua, ub = _run_both(big, precision, 1, 77)
    if precision != "fp32":
        assert (big.n > 32768).any() and b1.workspace_bytes > 256
    assert torch.equal(ua, ub)
    small = inputs.rod_batch(seed=52, nrods=40, nmin=64, nmax=20000, align=4)
    b2, ua, ub = _run_both(small, precision, 0, 40)
    assert torch.equal(ua, ub)


def test_static_scratch_rejects_plans_beyond_its_size():
    """Rods above the on-chip limit needing more than 32 MiB of second level
    buffers are refused before anything is enqueued."""
    n = np.full(40, 120000, dtype=np.int64)      # 40 x 120000 doubles: 38 MB
    offs = np.zeros(41, dtype=np.int64)
    offs[1:] = np.cumsum(n)
    b = ge.Batch(n, offs, np.full(40, 1.0), np.zeros(40), np.zeros(40), precision="fp64")
    assert b.workspace_bytes > 32 << 20
    u = torch.zeros(b.state_elems, dtype=torch.float64, device="cuda")
    st = ge.lib().ge_solve_batch_static(b.handle, ctypes.c_void_p(u.data_ptr()), 0, 10, None)
    assert st == ge.GE_ERR_UNSUPPORTED
    assert "scratch" in ge.last_error()
