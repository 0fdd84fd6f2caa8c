"""The streaming copy that bench.py times as the HBM reference: a
byte-exact copy for ragged sizes (a partial run of four 16-byte words, a
partial workgroup, more workgroups than the grid holds)."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_10148_amd import sss
    sss.lib()
    return sss


@pytest.mark.parametrize("n_words", [4, 4 * 1027 + 12, 4 * 256 * 4 * 32768 + 4 * 5])
def test_stream_copy_is_exact(sss, n_words):
    g = torch.Generator(device="cuda").manual_seed(n_words)
    a = torch.randint(-2 ** 31, 2 ** 31 - 1, (n_words,), dtype=torch.int32, device="cuda", generator=g)
    b = torch.full_like(a, 7)
    sss.stream_copy(a, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
