"""The controller exact stage's log, sine and cosine evaluated on the device
give the host's bits (aeb_ctl_math both ways): the host test's accuracy
measurement of that arithmetic then holds for the kernels.  Also the
counter-check kernel (aeb_valu_probe) that the VALU counters' accounting is
verified on."""
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


def test_counter_check_kernel():
    """aeb_valu_probe (the counter-check kernel) runs in both precisions and
    computes what its arithmetic says: 8 chains of x <- 0.999 x + 1e-3 from
    x = lane + c, summed."""
    import torch
    from paper_2604_27193_amd import binding as B
    for fp32 in (False, True):
        out = B.valu_probe(fp32, 1024, 10).cpu().numpy().astype(np.float64)
        lane = np.arange(1024) % 256
        x = np.stack([lane + c for c in range(8)]).astype(np.float64)
        for _ in range(10):
            x = 0.999 * x + 1e-3
        want = x.sum(axis=0)
        assert np.allclose(out, want, rtol=1e-5 if fp32 else 1e-12)
    with pytest.raises(B.AebError):
        B.valu_probe(False, 1000, 1)  # not a multiple of 256
