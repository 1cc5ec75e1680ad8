"""The allocation-free variant of the segment current deposit
(ecpic_deposit_current_noalloc): device arrays in and out, a fixed file-scope
scratch instead of allocated buffers, asynchronous on the context's stream.
Its output must equal the allocating entry point's (ecpic_deposit_current) to
the bar of that call's own parity test, on consecutive calls that reuse the
scratch with a smaller input the second time."""
import numpy as np
import pytest

import paper_2203_06513_amd as ec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _segments(L, dx, n, seed):
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0, L, n)
    x0[:10] = np.arange(10) * dx                 # exactly on knots
    x1 = x0 + rng.uniform(-0.95, 0.95, n) * dx
    x1[10:20] = x0[10:20]                        # zero length
    x0[20:25] = L - 1e-14; x1[20:25] = L + 0.3 * dx      # wrap right
    x0[25:30] = 1e-14; x1[25:30] = -0.4 * dx             # wrap left
    return x0, x1


def _call(c, x0, x1, J, flags):
    return c.deposit_current_noalloc(x0.data_ptr(), x1.data_ptr(), x0.numel(), J.data_ptr(), flags.data_ptr())


@pytest.mark.parametrize("p", [2, 3, 5])
def test_noalloc_deposit_matches_allocating_call(p):
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible to torch")
    dev = torch.device("cuda:0")
    M, L, w = 16, 3.0, 0.37
    dx = L / M
    stream = torch.cuda.current_stream(dev)
    with ec.Context(L=L, M=M, degree=p, n_particles=0, dt=0.01, tol=1e-12, weight=w,
                    stream=stream.cuda_stream) as c:
        for n, seed in ((20000, p), (3001, 10 + p)):      # the second call is smaller
            x0, x1 = _segments(L, dx, n, seed)
            ref = c.deposit_current(x0, x1)
            x0t = torch.from_numpy(x0).to(dev)
            x1t = torch.from_numpy(x1).to(dev)
            J = torch.full((M,), float("nan"), dtype=torch.float64, device=dev)
            flags = torch.full((1,), -1, dtype=torch.int32, device=dev)
            assert _call(c, x0t, x1t, J, flags) == ec.OK
            torch.cuda.synchronize()
            Jh = J.cpu().numpy()
            assert int(flags.cpu()[0]) == 0
            assert np.abs(Jh - ref).max() / np.abs(ref).max() <= 1e-13
            assert abs(Jh.sum() - w * (x1 - x0).sum()) <= 1e-12
        # a segment that leaves the neighbour cells is flagged, the others still deposit
        x0, x1 = _segments(L, dx, 500, 99)
        x1[3] = x0[3] + 2.5 * dx
        J = torch.empty((M,), dtype=torch.float64, device=dev)
        flags = torch.zeros((1,), dtype=torch.int32, device=dev)
        assert _call(c, torch.from_numpy(x0).to(dev), torch.from_numpy(x1).to(dev), J, flags) == ec.OK
        torch.cuda.synchronize()
        assert int(flags.cpu()[0]) == 2
        keep = np.ones(500, bool)
        keep[3] = False
        ref = c.deposit_current(x0[keep], x1[keep])
        assert np.abs(J.cpu().numpy() - ref).max() / np.abs(ref).max() <= 1e-13


def test_noalloc_rejects_more_cells_than_its_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible to torch")
    dev = torch.device("cuda:0")
    with ec.Context(L=1000.0, M=20000, degree=3, n_particles=0, dt=0.01, tol=1e-12, weight=1.0) as c:
        x = torch.zeros(4, dtype=torch.float64, device=dev)
        J = torch.zeros(20000, dtype=torch.float64, device=dev)
        flags = torch.zeros(1, dtype=torch.int32, device=dev)
        assert _call(c, x, x, J, flags) == ec.EINVAL
