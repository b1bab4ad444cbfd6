"""The controller exact stage's log, sine and cosine evaluated on the device
give the host's bits (aeb_ctl_math both ways): the host test's accuracy
measurement of that arithmetic then holds for the kernels."""
import numpy as np
import pytest

from test_ctl_math_host import _args

pytestmark = pytest.mark.gpu


def test_device_equals_host_bitwise():
    import torch
    from paper_2604_27193_amd import binding as B
    a, x = _args(1_000_000, 5)
    want = B.ctl_math(a, x)
    got = B.ctl_math(torch.from_numpy(a).cuda(), torch.from_numpy(x).cuda(), device=True)
    torch.cuda.synchronize()
    for g, w in zip(got, want):
        assert np.array_equal(g.cpu().numpy().view(np.uint64), w.view(np.uint64))


def test_empty_and_bad_arguments():
    import torch
    from paper_2604_27193_amd import binding as B
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    assert all(t.numel() == 0 for t in B.ctl_math(e, e, device=True))
    with pytest.raises(ValueError):
        B.ctl_math(torch.zeros(3, dtype=torch.float64, device="cuda"),
                   torch.zeros(4, dtype=torch.float64, device="cuda"), device=True)
