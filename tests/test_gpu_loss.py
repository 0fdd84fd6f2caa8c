"""sss_loss (L1 + D-SSIM and its image gradient) against the FP64 oracle."""
import numpy as np
import pytest

from oracle import loss as oloss
from paper_2503_10148_amd import scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_10148_amd import sss as binding
    binding.lib()
    return binding


@pytest.mark.parametrize("lam", [0.0, 0.2, 1.0])
def test_loss_matches_oracle_multiview(sss, lam):
    rng = np.random.default_rng(17)
    cams = [scenes.ring_camera(70, 45), scenes.ring_camera(16, 16), scenes.ring_camera(129, 33)]
    imgs = [rng.uniform(-0.2, 1.2, (c["height"], c["width"], 3)).astype(np.float32) for c in cams]
    tgts = [scenes.smooth_target(c["width"], c["height"], seed=i) for i, c in enumerate(cams)]
    P = sum(c["width"] * c["height"] for c in cams)
    # oracle over all views: means over all 3P values
    Ls, gs = [], []
    for im, tg in zip(imgs, tgts):
        L, g = oloss.loss_and_grad(im, tg, lam)
        w = im.size / (3.0 * P)
        Ls.append(L * w)
        gs.append((g * w).reshape(-1, 3))
    img = torch.as_tensor(np.concatenate([i.reshape(-1, 3) for i in imgs]), device="cuda")
    tgt = torch.as_tensor(np.concatenate([t.reshape(-1, 3) for t in tgts]), device="cuda")
    out = torch.zeros(1, device="cuda")
    dl = sss.loss(img, tgt, cams, lam, loss_out=out)
    torch.cuda.synchronize()
    assert out.item() == pytest.approx(sum(Ls), rel=1e-5)
    want = np.concatenate(gs)
    got = dl.cpu().numpy()
    scale = np.sqrt(np.mean(want ** 2))
    assert np.all(np.abs(got - want) <= 1e-3 * np.maximum(np.abs(want), scale))
