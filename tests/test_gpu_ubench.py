"""The device micro-benchmarks that give the Monte Carlo kernel its measured
ceilings do the work they claim: every atomic mode adds exactly
blocks x threads x per_thread ones, and the copy copies."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def soc():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1812_06632_amd import soc as m
    return m


_DTYPE = {4: torch.float32, 5: torch.int64, 6: torch.int32}


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 5, 6])
def test_atomic_modes_count_every_add(soc, mode):
    ctx = soc.Context(0)
    n = 1 << 16
    a = torch.zeros((8 if mode == 1 else 1) * n, dtype=_DTYPE.get(mode, torch.float64), device="cuda")
    blocks, threads, per = 64, 256, 5
    ms = soc.ubench(ctx, 0, a, None, n, per, mode, blocks, threads)
    assert ms > 0
    assert a.double().sum().item() == blocks * threads * per
    if mode == 2:
        # whole 64-double blocks: every block holds a multiple of 64 adds
        counts = a.view(-1, 64).sum(1).cpu()
        assert torch.all(torch.remainder(counts, 64) == 0)
    if mode == 3:
        assert a[4096:].abs().sum().item() == 0
    ctx.close()


def test_atomic_mode_bounds_rejected(soc):
    ctx = soc.Context(0)
    a = torch.zeros(100, dtype=torch.float64, device="cuda")
    with pytest.raises(soc.SocError):
        soc.ubench(ctx, 0, a, None, 100, 1, 3, 1, 64)   # LDS mode needs n >= 4096
    with pytest.raises(soc.SocError):
        soc.ubench(ctx, 0, a, None, 100, 1, 7, 1, 64)
    ctx.close()


def test_copy(soc):
    ctx = soc.Context(0)
    src = torch.arange(1 << 20, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    soc.ubench(ctx, 2, src, dst, src.numel() * 4, 1, 0, 256, 256)
    assert torch.equal(src, dst)
    ctx.close()
