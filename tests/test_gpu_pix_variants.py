"""The raster kernels' other variants, chosen by environment variables read
once per process, against the oracle: pixels per lane (SSS_PIX_FWD,
SSS_PIX_BWD) and the persistent work-queue form of the recompute-mode
backward (SSS_BWD_PERSISTENT).  Each setting runs in a child process that
renders a small ragged case, back-propagates in the stored and recompute
modes and checks image and gradients at the parity bar of the defaults."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np, torch
import oracle
from paper_2503_10148_amd import scenes, sss
from tests._util import PARAMS, grad_close, to_device
s = scenes.make_scene(3000, 3, seed=7, neg_frac=0.3)
s["scales"] *= np.float32(2.0)
cams = [scenes.ring_camera(250, 190, angle=1.1)]
n = s["means"].shape[0]
ref = oracle.render(s, cams[0])
dev = to_device(s)
proj = sss.project(dev, cams)
bins = sss.BinSorter(1024)(proj, cams, n)
img, _, ncon = sss.render_fwd(bins, cams)
torch.cuda.synchronize()
diff = np.abs(img.cpu().numpy().reshape(ref["image"].shape) - ref["image"])
diff[ref["xflags"] != 0] = 0.0
assert diff.max() <= 1e-4, diff.max()
w = np.random.default_rng(78).standard_normal(ref["image"].shape)
w[ref["xflags"] != 0] = 0.0
gref = oracle.render_backward(s, cams[0], w, fwd=ref)
dl = torch.as_tensor(w.reshape(-1, 3), dtype=torch.float32, device="cuda")
keep = ref["proj"]["pflags"] == 0
for mode in (sss.BWD_STORED, sss.BWD_RECOMPUTE):
    g = sss.render_bwd(dev, proj, bins, cams, dl, mode=mode, image=img, n_contrib=ncon)
    torch.cuda.synchronize()
    for k in PARAMS:
        ok, worst = grad_close(g[k].cpu().numpy(), gref[k], mask=keep)
        assert ok, (mode, k, worst)
print("ok")
"""


@pytest.mark.parametrize("fwd,bwd,persistent", [("2", "1", "0"), ("4", "4", "0"), ("1", "1", "1"), ("1", "2", "1")])
def test_pixels_per_lane_variants_match_oracle(fwd, bwd, persistent):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    env = dict(os.environ, SSS_PIX_FWD=fwd, SSS_PIX_BWD=bwd, SSS_BWD_PERSISTENT=persistent)
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0 and "ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
