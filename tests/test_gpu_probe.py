"""The stream-copy probe (the bench's achievable-HBM measurement) copies
every byte: sizes that are and are not whole strides of its grid, each
workgroups-per-CU setting the bench times, and a copy into the middle of a
larger buffer that leaves the bytes around it alone."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("nbytes", [16, 4096, (1 << 20) + 48, 3 * (1 << 22) + 16 * 37])
@pytest.mark.parametrize("per_cu", [1, 2, 4, 8, 16])
def test_stream_copy_copies_every_byte(nbytes, per_cu):
    from paper_2207_11328_amd import abi
    g = torch.Generator(device="cpu").manual_seed(nbytes + per_cu)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g).to("cuda:0")
    guard = 256
    dst = torch.full((nbytes + 2 * guard,), 0xA5, dtype=torch.uint8, device="cuda:0")
    abi.sph_stream_copy(src, dst[guard:guard + nbytes], nbytes, per_cu)
    torch.cuda.synchronize()
    out = dst.cpu()
    assert torch.equal(out[guard:guard + nbytes], src.cpu())
    assert (out[:guard] == 0xA5).all() and (out[guard + nbytes:] == 0xA5).all()
