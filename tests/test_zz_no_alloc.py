"""qsv_norm_noalloc (the allocation-free variant of qsv_norm, for callers that cannot
allocate): through the C ABI, its result equals qsv_norm's bit for bit, on two calls in
a row that share the device scratch array, the second on a smaller state; and on a
tensor the library never allocated.  Both precisions."""
import ctypes

import pytest

from paper_2604_03816_amd import circuits as C

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_norm_noalloc_equals_norm_twice(dtype):
    import torch
    from paper_2604_03816_amd import qsv
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    for n, depth, seed in ((20, 12, 31), (13, 6, 32)):   # the second call is smaller
        s = qsv.State(n, dtype)
        s.apply(C.brickwork(n, depth, seed))
        # a slightly unnormalised state, so the value is not trivially 1
        s.tensor.mul_(1.0 + 1e-3 * (n - 12))
        s.sync()
        want = s.norm()
        qsv.norm_noalloc(s.tensor, out, stream=s.stream)
        s.sync()
        got = out.item()
        assert got == want, (dtype, n, got, want)
        s.free()
    torch.cuda.synchronize()


def test_norm_noalloc_on_a_torch_tensor():
    import torch
    from paper_2604_03816_amd import qsv
    g = torch.Generator(device="cpu").manual_seed(5)
    x = torch.randn(1 << 16, dtype=torch.complex128, generator=g).cuda()
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    qsv.norm_noalloc(x, out)
    torch.cuda.synchronize()
    ref = float((x.abs() ** 2).sum().item())
    assert abs(out.item() - ref) <= 1e-12 * ref
    # argument errors are reported, not faulted on
    with pytest.raises(qsv.QSVError):
        qsv.check(qsv.lib().qsv_norm_noalloc(None, 10, 1, None, None))
    with pytest.raises(qsv.QSVError):
        qsv.check(qsv.lib().qsv_norm_noalloc(ctypes.c_void_p(x.data_ptr()), 35, 1,
                                             ctypes.c_void_p(out.data_ptr()), None))
