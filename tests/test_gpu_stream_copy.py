"""The device bandwidth reference gplbm_stream_copy (bench.py's stream
ceiling): it copies exactly, for sizes below, at and above one grid pass,
and rejects misaligned or ragged requests."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available()
    from paper_2111_05960_amd import binding
    binding.load()
    return binding


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, 3 * (1 << 20) + 48, 256 << 20])
def test_stream_copy_copies(gp, nbytes):
    import torch
    print(f"case stream copy {nbytes} bytes", flush=True)
    g = torch.Generator(device="cuda").manual_seed(nbytes)
    a = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
    b = torch.zeros_like(a)
    s = torch.cuda.current_stream()
    gp.gplbm_stream_copy(a.data_ptr(), b.data_ptr(), nbytes, s.cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_stream_copy_rejects(gp):
    import torch
    a = torch.zeros(64, dtype=torch.uint8, device="cuda")
    b = torch.zeros_like(a)
    s = torch.cuda.current_stream().cuda_stream
    for src, dst, n in ((a.data_ptr() + 4, b.data_ptr(), 32), (a.data_ptr(), b.data_ptr(), 24),
                        (0, b.data_ptr(), 32)):
        with pytest.raises(gp.GplbmError):
            gp.gplbm_stream_copy(src, dst, n, s)
