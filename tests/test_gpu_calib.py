"""Measurement helpers of the library: the calibration copy (known traffic
for the memory counters) and the FP32 multiply-add throughput kernel (the
ceiling of the ALU-bound kernels)."""
import numpy as np
import pytest

from paper_1702_06359_amd import abi, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_required):
    c = abi.Context(abi.config_from_geometry(synth.Geometry(), max_cands=1))
    yield c
    c.close()


def test_calib_copy_is_exact(ctx):
    import torch
    print("case calib copy 1 MiB + 16 B", flush=True)
    src = torch.arange((1 << 18) + 4, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    ctx.calib_copy(src.data_ptr(), dst.data_ptr(), src.numel() * 4)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_calib_fma_values_and_flop(ctx):
    """Every lane's 8 chains x <- x a + b (a = 0.999999, b = 1e-6 in FP32)
    against the closed form a^n x0 + b (1 - a^n) / (1 - a) in FP64: FP32
    rounding over n = 256 steps stays far below 1e-4 relative."""
    import torch
    n_blocks, iters = 6, 256
    out = torch.full((n_blocks * 256,), float("nan"), dtype=torch.float32, device="cuda")
    print(f"case calib fma {n_blocks} blocks x {iters} rounds", flush=True)
    ms, flop = ctx.calib_fma(out.data_ptr(), n_blocks, iters)
    got = out.cpu().numpy().astype(np.float64)
    assert ms > 0.0
    assert flop == 2.0 * 8 * iters * 256 * n_blocks
    a, b = float(np.float32(0.999999)), float(np.float32(1e-6))
    t = np.arange(n_blocks * 256)
    base = (t & 1023).astype(np.float32) * np.float32(1e-3)
    an = a ** iters
    want = sum(an * np.float64(base + np.float32(i)) + b * (1.0 - an) / (1.0 - a) for i in range(8))
    np.testing.assert_allclose(got, want, rtol=1e-4)


def test_calib_fma_rejects_bad_arguments(ctx):
    import torch
    out = torch.empty(256, dtype=torch.float32, device="cuda")
    for nb, it in ((0, 4), (1, 0), (1, 6)):
        with pytest.raises(abi.MkfError):
            ctx.calib_fma(out.data_ptr(), nb, it)
    with pytest.raises(abi.MkfError):
        ctx.calib_fma(0, 1, 4)
