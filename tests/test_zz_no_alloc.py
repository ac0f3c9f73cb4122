"""sd_inner_noalloc (static device scratch, no allocation) against sd_inner
(caller scratch) through the C ABI: two calls in a row, the second on a
smaller input, each bit-identical to sd_inner on the same inputs (same
kernels, same fixed summation order) and within FP64 rounding of the host
inner product."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
from paper_2206_11664_amd import sd  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_inner_noalloc_matches_inner(dtype):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    for call, (n, sa, sb) in enumerate(((20, 41, 42), (9, 43, 44))):
        print(f"[gpu] sd_inner_noalloc call {call} n={n} dtype={dtype}", flush=True)
        a_h = workloads.random_state(n, sa)
        b_h = workloads.random_state(n, sb)
        a = torch.from_numpy(a_h).to(dtype).cuda()
        b = torch.from_numpy(b_h).to(dtype).cuda()
        got = sd.sd_inner_noalloc(a, b, n)
        want = sd.sd_inner(a, b, n)
        assert got == want, (call, got, want)
        # and the value itself: the host FP64 inner product of the stored amplitudes
        ref = np.vdot(a.cpu().numpy().astype(np.complex128), b.cpu().numpy().astype(np.complex128))
        assert abs(got - ref) <= 1e-12, (call, got, ref)
        # the norm as <a|a>: real, equal to sd_norm2 within rounding
        got_aa = sd.sd_inner_noalloc(a, a, n)
        assert abs(got_aa.imag) <= 1e-15
        assert abs(got_aa.real - sd.sd_norm2(a, n)) <= 1e-13
