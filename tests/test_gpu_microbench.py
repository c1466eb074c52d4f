"""The device-rate measurements (frt_microbench): a streaming copy's
bandwidth lies between a sliver of the published 8 TB/s and the peak itself
(the 2 GiB buffers are far larger than every cache), random FP32 atomics run
at a rate no slower than the march's deposits need (well above 1e9/s), the
arguments are checked, and every buffer goes back through the context's
allocator."""
import pytest

from paper_2409_04521_amd import frt

pytestmark = pytest.mark.gpu


def test_rates_are_plausible_and_nothing_stays_allocated():
    alloc = frt.TorchAllocator(0)
    ctx = frt.Context(0, allocator=alloc)
    mb = frt.microbench(ctx, 2 << 30, 1 << 24)
    print(f"copy {mb['copy_GBps']:.0f} GB/s, FP32 atomics {mb['atomic_per_s']:.3e}/s", flush=True)
    assert 500.0 < mb["copy_GBps"] <= 8000.0
    assert mb["atomic_per_s"] > 1e9
    assert mb["copy_bytes"] == 2 << 30 and mb["atomic_slots"] == 1 << 24
    assert alloc.bytes_out() == 0
    ctx.close()


def test_arguments_are_checked():
    ctx = frt.Context(0)
    for a, b in ((1000, 1 << 20), ((1 << 20) + 8, 1 << 20), (1 << 20, 10)):
        with pytest.raises(frt.FrtError) as e:
            frt.microbench(ctx, a, b)
        assert e.value.code == frt.FRT_EINVAL
    ctx.close()
