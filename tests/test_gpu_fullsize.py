"""Parity at the full workload sizes, in the configuration the benchmark
times (default pixels per lane, one launch over all views): the GPU image
and gradients are compared with the FP64 oracle on sampled 32x32 windows.

The oracle renders each window with the window's own camera (principal
point shifted, frustum clamp of the full image), which gives exactly the
full image's pixels there (pinned by test_window_render_equals_crop_of_full_render).
The loss weight is random inside the windows and zero elsewhere, so the
oracle's window gradients add up to the gradient of the GPU's whole-image
backward pass.  Explained pixels (a decision within its margin) get weight
zero and are not compared; components the oracle flags are not compared.
"""
import numpy as np
import pytest

import oracle
from paper_2503_10148_amd import scenes
from tests._util import PARAMS, grad_close, to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WIN = 32


@pytest.fixture(scope="module")
def sss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_10148_amd import sss as binding
    binding.lib()
    return binding


def _windows(cams, count, rng):
    """Disjoint windows (view, x0, y0), not aligned to tiles."""
    out = []
    while len(out) < count:
        v = int(rng.integers(0, len(cams)))
        c = cams[v]
        x0 = int(rng.integers(0, c["width"] - WIN))
        y0 = int(rng.integers(0, c["height"] - WIN))
        if all(w[0] != v or abs(w[1] - x0) >= WIN or abs(w[2] - y0) >= WIN for w in out):
            out.append((v, x0, y0))
    return out


@pytest.mark.parametrize("name,mode,count", [("m1", "stored", 6), ("large", "recompute", 4),
                                             ("multiview", "stored", 4), ("multiview", "recompute_l1", 4),
                                             ("m1", "stored_det", 4)])
def test_full_size_windows_match_oracle(sss, name, mode, count):
    """stored_det: the deterministic backward (no float atomics), which must
    also repeat bit for bit.
    recompute_l1: the configuration the multi-view workload is timed in,
    the forward pass recomputed per tile inside the backward launch with the
    L1 loss fused.  The target equals the image outside the windows (the L1
    gradient there is sign(0) = 0) and the image minus 0.5 sign(w) inside
    them, so the fused loss gradient is sign(w) / (3P) in the windows: the
    oracle gets that weight; the recomputed image must equal the forward
    pass's bit for bit, and the loss is 0.5 per weighted value / (3P)."""
    scene, cams = scenes.workload(name)
    n = scene["means"].shape[0]
    s64 = {k: np.asarray(scene[k], np.float64) for k in PARAMS}
    s64["sh_degree"] = scene["sh_degree"]
    dev = to_device(scene)
    del scene
    proj = sss.project(dev, cams)
    det = mode == "stored_det"
    bins = sss.BinSorter(0, keep_offsets=det)(proj, cams, n)
    img, _, ncon = sss.render_fwd(bins, cams)
    torch.cuda.synchronize()
    offs = np.cumsum([0] + [c["width"] * c["height"] for c in cams])
    img_np = img.cpu().numpy()
    dl = np.zeros_like(img_np)
    rng = np.random.default_rng(scenes.SEED_FD + 7)
    gref = {k: np.zeros_like(s64[k]) for k in PARAMS}
    flagged = np.zeros(n, bool)
    bad_total, explained_total = 0, 0
    for v, x0, y0 in _windows(cams, count, rng):
        cam = cams[v]
        wc = oracle.window_camera(cam, x0, y0, WIN, WIN)
        ref = oracle.render(s64, wc)
        W = cam["width"]
        rows = offs[v] + (y0 + np.arange(WIN))[:, None] * W + (x0 + np.arange(WIN))[None, :]
        got = img_np[rows.reshape(-1)].reshape(WIN, WIN, 3)
        explained = ref["xflags"] != 0
        bad = (np.abs(got - ref["image"]).max(axis=2) > 1e-4) & ~explained
        bad_total += int(bad.sum())
        explained_total += int(explained.sum())
        w = rng.standard_normal((WIN, WIN, 3)).astype(np.float32)
        w[explained] = 0.0
        if mode == "recompute_l1":
            w = np.sign(w) / np.float32(3 * img_np.shape[0])     # the fused L1 loss's weights
        dl[rows.reshape(-1)] = w.reshape(-1, 3)
        g = oracle.render_backward(s64, wc, w.astype(np.float64), fwd=ref)
        for k in PARAMS:
            gref[k] += g[k]
        flagged |= ref["proj"]["pflags"] != 0
    assert bad_total == 0, bad_total
    assert explained_total < 0.02 * count * WIN * WIN
    m = sss.BWD_RECOMPUTE if mode.startswith("recompute") else sss.BWD_STORED
    if mode == "recompute_l1":
        P = img_np.shape[0]
        sgn = np.sign(dl)
        target = torch.as_tensor((img_np - np.float32(0.5) * sgn).astype(np.float32), device="cuda")
        image_out = torch.empty_like(img)
        loss = torch.zeros(1, device="cuda")
        g = sss.render_bwd(dev, proj, bins, cams, target, mode=m, loss=sss.LOSS_L1, image_out=image_out,
                           loss_out=loss)
        torch.cuda.synchronize()
        assert torch.equal(image_out, img)
        assert abs(float(loss.item()) - 0.5 * float(np.abs(sgn).sum()) / (3.0 * P)) <= 1e-6 * float(loss.item())
    else:
        stored = m == sss.BWD_STORED
        dl_dev = torch.as_tensor(dl, device="cuda")
        g = sss.render_bwd(dev, proj, bins, cams, dl_dev, mode=m, image=img if stored else None,
                           n_contrib=ncon if stored else None, deterministic=det)
        torch.cuda.synchronize()
        if det:
            again = sss.render_bwd(dev, proj, bins, cams, dl_dev, mode=m, image=img, n_contrib=ncon, deterministic=True)
            torch.cuda.synchronize()
            for k in PARAMS:
                assert torch.equal(again[k], g[k]), k
    touched = np.abs(gref["opacity"]) > 0
    assert touched.sum() > 100
    fails = []
    for k in PARAMS:
        got = g[k].cpu().numpy()
        ok, worst = grad_close(got, gref[k], mask=~flagged)
        if not ok:
            a = got.reshape(n, -1).astype(np.float64)
            b = gref[k].reshape(n, -1)
            rms = np.sqrt(np.mean(b ** 2))
            ratio = np.where(flagged[:, None], 0.0, np.abs(a - b) / (1e-3 * np.maximum(np.abs(b), rms)))
            i, j = np.unravel_index(np.argmax(ratio), ratio.shape)
            detail = dict(i=int(i), j=int(j), got=float(a[i, j]), ref=float(b[i, j]), rms=float(rms),
                          nu=float(s64["nu"][i]), o=float(s64["opacity"][i]), n_over=int((ratio > 1).sum()))
            fails.append(f"{k}: worst {worst:.3f} {detail}")
    if fails:
        raise AssertionError(f"{name}: " + "; ".join(fails))


def test_sghmc_step_on_five_million_components(sss):
    """The sampler step over all 5M means of the multi-view workload's size
    (counters beyond 2^22 exercise the high words of the Philox counter's
    index), element by element against the oracle."""
    n = 5_000_000
    rng = np.random.default_rng(scenes.SEED_SGHMC)
    f = lambda a: a.astype(np.float32)
    mu, r, g = f(rng.standard_normal((n, 3))), f(rng.standard_normal((n, 3))), f(rng.standard_normal((n, 3)))
    o = f(rng.uniform(-1, 1, n))
    o[::7] = f(rng.uniform(-0.004, 0.004, o[::7].size))          # switch on
    sc, q = f(np.exp(rng.uniform(-4, -2, (n, 3)))), f(rng.standard_normal((n, 4)))
    ref_mu, ref_r = oracle.sghmc_step(mu, r, g, o, sc, q, 0.01, 0.1, 100.0, 0.995, False, True, seed=9, step=3)
    T = lambda a: torch.as_tensor(a, device="cuda")
    dmu, dr = T(mu.copy()), T(r.copy())
    sss.sghmc_step(dmu, dr, T(g), T(o), 0.01, 0.1, 100.0, 0.995, False, True, seed=9, step=3, scales=T(sc),
                   quats=T(q))
    torch.cuda.synchronize()
    np.testing.assert_allclose(dmu.cpu().numpy(), ref_mu, rtol=1e-5, atol=2e-6)
    np.testing.assert_allclose(dr.cpu().numpy(), ref_r, rtol=1e-5, atol=2e-6)


@pytest.mark.parametrize("name", ["m1", "large"])
def test_full_size_tile_lists_match_oracle(sss, name):
    """Every tile's list at the full workload size, in the binning the
    benchmark runs (no host wait, a second call with the capacity the first
    one sized), against the oracle's per-tile lists (box of pixel centres
    meets the ellipse; depth key, then index): the same components in the
    same order, except components whose rectangle decisions the oracle
    flags as within its margin, which are dropped from both sides."""
    scene, cams = scenes.workload(name)
    cam = cams[0]
    n = scene["means"].shape[0]
    o = oracle.project(scene, cam)
    tx, ty = oracle.tiles(cam)
    ost, olst = oracle.bin_tiles(o["touched"], o["rect"], o["key"], tx, ty, proj=o)
    dev = to_device(scene)
    proj = sss.project(dev, cams)
    binner = sss.BinSorter(0, no_wait=True)
    binner(proj, cams, n).resolve()                       # sizes the capacity (this call waits)
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    bins = binner(proj, cams, n, counts=counts)           # the no-wait call
    torch.cuda.synchronize()
    bins.resolve()
    assert bins.n_pairs == int(o["touched"].sum())
    T = tx * ty
    order = bins.order.cpu().numpy().view(np.uint32).astype(np.int64)
    start = bins.tile_start.cpu().numpy().astype(np.int64)
    assert start[0] == 0 and start[T] == bins.n_pairs
    ids = order[bins.pair_rank.cpu().numpy()[: bins.n_pairs].astype(np.int64)]
    tile = np.repeat(np.arange(T), np.diff(start[: T + 1]))
    ref_tile = np.repeat(np.arange(T), np.diff(ost.astype(np.int64)))
    flagged = (o["pflags"] & oracle.PF_RECT_EDGE) != 0
    keep, ref_keep = ~flagged[ids], ~flagged[olst]
    assert flagged.sum() < 0.001 * n
    np.testing.assert_array_equal(tile[keep], ref_tile[ref_keep])
    np.testing.assert_array_equal(ids[keep], olst[ref_keep].astype(np.int64))


def test_multiview_tile_lists_in_windows_match_oracle(sss):
    """The 8-view workload's tile lists (6e8 pairs, one binning over all
    views), compared with the oracle on two tile-aligned windows of 4 x 4
    tiles per view.  A window camera differs from its view only by a
    principal point moved by whole pixels and keeps the view's frustum
    clamp, so its tiles are the view's tiles and their lists the view's
    lists; components the oracle flags near a rectangle decision are
    dropped from both sides."""
    scene, cams = scenes.workload("multiview")
    n = scene["means"].shape[0]
    dev = to_device(scene)
    proj = sss.project(dev, cams)
    bins = sss.BinSorter(0)(proj, cams, n)
    torch.cuda.synchronize()
    offs = np.cumsum([0] + [oracle.tiles(c)[0] * oracle.tiles(c)[1] for c in cams])
    rng = np.random.default_rng(scenes.SEED_FD + 11)
    compared = 0
    for v, cam in enumerate(cams):
        txs, tys = oracle.tiles(cam)
        for _ in range(2):
            tx0 = int(rng.integers(0, txs - 4)) if txs > 4 else 0
            ty0 = int(rng.integers(0, tys - 4)) if tys > 4 else 0
            wc = oracle.window_camera(cam, 16 * tx0, 16 * ty0, 64, 64)
            o = oracle.project(scene, wc)
            ost, olst = oracle.bin_tiles(o["touched"], o["rect"], o["key"], 4, 4, proj=o)
            flagged = (o["pflags"] & oracle.PF_RECT_EDGE) != 0
            for j in range(4):
                for i in range(4):
                    t = int(offs[v] + (ty0 + j) * txs + tx0 + i)
                    s0, s1 = int(bins.tile_start[t].item()), int(bins.tile_start[t + 1].item())
                    ranks = bins.pair_rank[s0:s1].long()
                    ids = (bins.order[ranks].long() - v * n).cpu().numpy()
                    ref = olst[ost[4 * j + i]:ost[4 * j + i + 1]].astype(np.int64)
                    assert ((ids >= 0) & (ids < n)).all()
                    got = ids[~flagged[ids]]
                    want = ref[~flagged[ref]]
                    np.testing.assert_array_equal(got, want, err_msg=f"view {v} tile ({tx0 + i}, {ty0 + j})")
                    compared += len(want)
    assert compared > 10000
