"""restore_gmm_nll_noalloc: the weighted NLL of the learned regeneration
distribution for callers that cannot allocate device memory.  Its workspace
is a library-owned device array, so it must give exactly the result of
restore_gmm_nll with a caller workspace (the same kernels and grid), also
on a second call right after the first with a smaller input (the array
keeps the first call's partial sums, which the second must not read)."""
import numpy as np
import pytest

from tests.test_gpu_learned import _nll_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2409_07148_amd import restore
    return restore


def _call(R, fn, K, d, beta, tensors, ws=None):
    import torch
    t_row, t_x, t_w = tensors
    n = t_w.numel()
    dout = torch.full((t_row.numel(),), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    if ws is None:
        fn(K, d, beta, t_row.data_ptr(), t_x.data_ptr(), t_w.data_ptr(), n, dout.data_ptr(), loss.data_ptr())
    else:
        fn(K, d, beta, t_row.data_ptr(), t_x.data_ptr(), t_w.data_ptr(), n, dout.data_ptr(), loss.data_ptr(),
           ws.data_ptr(), ws.numel())
    torch.cuda.synchronize()
    return dout.cpu().numpy(), loss.cpu().numpy()


def test_noalloc_nll_equals_the_workspace_entry_point(R):
    import torch
    cases = [(64, 12, 0.1, 600_001), (5, 3, 0.25, 2_500)]   # the second smaller
    inputs = []
    for K, d, beta, n in cases:
        row, x, w = _nll_inputs(K, d, n, seed=K + d)
        inputs.append(tuple(torch.from_numpy(a.astype(np.float32)).cuda() for a in (row, x, w)))
    # two no-allocation calls in a row, the second with the smaller input
    got = [_call(R, R.restore_gmm_nll_noalloc, K, d, beta, t) for (K, d, beta, _), t in zip(cases, inputs)]
    ws = torch.empty(R.restore_gmm_nll_workspace_bytes(), dtype=torch.uint8, device="cuda")
    for (K, d, beta, n), t, (g_dout, g_loss) in zip(cases, inputs, got):
        r_dout, r_loss = _call(R, R.restore_gmm_nll, K, d, beta, t, ws)
        print(f"[nll noalloc] K {K} d {d} n {n}: loss {g_loss[0]:.9f} vs {r_loss[0]:.9f}", flush=True)
        assert np.all(np.isfinite(g_dout)) and np.isfinite(g_loss[0])
        assert np.array_equal(g_dout, r_dout) and np.array_equal(g_loss, r_loss)


def test_noalloc_nll_rejects_bad_arguments(R):
    import torch
    row, x, w = _nll_inputs(4, 2, 10, seed=1)
    t = tuple(torch.from_numpy(a.astype(np.float32)).cuda() for a in (row, x, w))
    for K, d, beta in ((0, 2, 0.1), (65, 2, 0.1), (4, 17, 0.1), (4, 2, 1.0)):
        with pytest.raises(R.RestoreError) as e:
            _call(R, R.restore_gmm_nll_noalloc, K, d, beta, t)
        assert e.value.status == R.E_INVALID_ARG
