"""The allocation-free dot product (partial sums in the library's static device array)
against the entry point that takes a scratch buffer: equal bit for bit, on two calls
in a row with the second input smaller, in FP64 and FP32."""
import numpy as np
import pytest

from _support import ensure_built, gpu_available, print_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not gpu_available():
        pytest.skip("no GPU")
    ensure_built()


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_noalloc_dot_equals_scratch_dot(dtype):
    import torch
    from paper_2204_01722_amd.binding import hpmg_vec_dot, hpmg_vec_dot_noalloc
    print_case("noalloc_dot", dtype=dtype)
    dt = getattr(torch, dtype)
    rng = np.random.default_rng(31)
    for n in (3_000_003, 4_099):  # second call smaller: every partial is rewritten
        x = torch.from_numpy(rng.normal(size=n)).to(dt).cuda()
        y = torch.from_numpy(rng.normal(size=n)).to(dt).cuda()
        ref = hpmg_vec_dot(x, y)
        got = hpmg_vec_dot_noalloc(x, y)
        torch.cuda.synchronize()
        exact = float(np.dot(x.double().cpu().numpy(), y.double().cpu().numpy()))
        print(f"  n={n}: noalloc {float(got)!r} scratch {float(ref)!r} numpy {exact!r}", flush=True)
        assert torch.equal(got, ref)
        assert abs(float(got) - exact) <= 1e-12 * float(torch.linalg.norm(x.double()) * torch.linalg.norm(y.double()))
    # empty input: the sum of nothing
    e = torch.empty(0, dtype=dt, device="cuda")
    assert float(hpmg_vec_dot_noalloc(e, e)) == 0.0
