"""Parity on the method's edge cases: the alpha clamp, the nu clamp and its
gradient gate, and nu up to the clamp bound 1e4, where the FP32 log2(1 + y)
correction and the dT2D/dnu series of the kernels matter most.

The "edges" scene has signed opacities up to |o| = 1 (an eighth at +0.999,
an eighth at -0.999, a few at exactly +-1), nu log-uniform over [1, 1e4] with
a sixteenth each at exactly 1, at 0.7 (clamped up to 1) and at 2e4 (clamped
down to 1e4), and large components (scales 0.04 .. 0.25), so that alphas
reach the 0.99 clamp at hundreds of (pixel, component) evaluations.

Bars as in test_gpu_parity: images 1e-4 per channel outside the oracle's
explained pixels, gradients 1e-3 max(|g|, rms(g)), tile lists bit-exact.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2503_10148_amd import scenes
from tests._util import PARAMS, decode_records, grad_close, to_device

torch = pytest.importorskip("torch")


def edges_case(n=600, seed=12):
    s = scenes.make_scene(n, 3, seed=seed, neg_frac=0.3, scale_range=(0.04, 0.25))
    rng = np.random.default_rng(seed + 1000)
    o = rng.uniform(-1.0, 1.0, n)
    k = rng.permutation(n)
    o[k[: n // 8]] = 0.999
    o[k[n // 8: n // 4]] = -0.999
    o[k[n // 4: n // 4 + 6]] = 1.0
    o[k[n // 4 + 6: n // 4 + 12]] = -1.0
    nu = np.exp(rng.uniform(0.0, math.log(1e4), n))
    j = rng.permutation(n)
    nu[j[: n // 16]] = 1.0
    nu[j[n // 16: n // 8]] = 0.7
    nu[j[n // 8: 3 * n // 16]] = 2e4
    s["opacity"] = o.astype(np.float32)
    s["nu"] = nu.astype(np.float32)
    return s, [scenes.ring_camera(233, 157, angle=0.6)]


def _alpha_maps(p, cam, i):
    H, W = cam["height"], cam["width"]
    ys, xs = np.mgrid[0:H, 0:W]
    a, b, c = p["conic"][i]
    dx, dy = xs + 0.5 - p["mean2d"][i, 0], ys + 0.5 - p["mean2d"][i, 1]
    h = a * dx * dx + 2 * b * dx * dy + c * dy * dy
    nu = p["nu_c"][i]
    return h, p["opacity"][i] * (1 + h / nu) ** (-(nu + 2) / 2)


def test_edges_case_reaches_every_edge():
    """CPU check of the input itself: the clamps really fire in this scene."""
    s, cams = edges_case()
    p = oracle.project(s, cams[0])
    vis = p["valid"] == 1
    assert ((s["nu"] == np.float32(0.7)) & vis).sum() >= 20
    assert ((s["nu"] == np.float32(2e4)) & vis).sum() >= 20
    assert ((s["nu"] == np.float32(1.0)) & vis).sum() >= 20
    assert p["nu_c"][vis].max() == 1e4 and p["nu_c"][vis].min() == 1.0
    assert ((p["nu_c"] > 1e3) & vis).sum() >= 40
    clamped = sum(int((np.abs(_alpha_maps(p, cams[0], i)[1]) > 0.99).sum()) for i in np.nonzero(vis)[0])
    assert clamped >= 200
    f = oracle.render(s, cams[0])
    assert f["tfinal"].max() > 1.5                 # negative components raise T above 1


@pytest.fixture(scope="module")
def sss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_10148_amd import sss as binding
    binding.lib()
    return binding


@pytest.mark.gpu
def test_edges_projection_and_lists_match_oracle(sss):
    s, cams = edges_case()
    cam = cams[0]
    n = s["means"].shape[0]
    o = oracle.project(s, cam)
    dev = to_device(s)
    proj = sss.project(dev, cams)
    bins = sss.BinSorter(1024)(proj, cams, n)
    torch.cuda.synchronize()
    rec = decode_records(proj.records.cpu().numpy())
    touched = proj.touched.cpu().numpy()
    flagged = o["pflags"] != 0
    m = (touched > 0) & (o["valid"] == 1)
    assert np.array_equal((touched > 0)[~flagged], (o["valid"] == 1)[~flagged])
    assert np.array_equal(touched[~flagged], o["touched"][~flagged])
    np.testing.assert_allclose(1.0 / rec["inv_nu"][m].astype(np.float64), o["nu_c"][m], rtol=2e-7)
    np.testing.assert_allclose(rec["nb"][m], -0.5 * (o["nu_c"][m] + 2.0), rtol=2e-7)
    np.testing.assert_allclose(rec["hs"][m], o["hstar"][m], rtol=2e-7)
    # tile lists: bit-exact (the oracle's lists map component -> the GPU's entry)
    start, lst = oracle.bin_tiles(o["touched"], o["rect"], o["key"], *oracle.tiles(cam), proj=o)
    ts = bins.tile_start.cpu().numpy()
    order = bins.order.cpu().numpy()
    pr = bins.pair_rank.cpu().numpy()
    for t in range(len(start) - 1):
        assert np.array_equal(order[pr[ts[t]:ts[t + 1]]], lst[start[t]:start[t + 1]]), t


@pytest.mark.gpu
def test_edges_forward_matches_oracle(sss):
    s, cams = edges_case()
    cam = cams[0]
    n = s["means"].shape[0]
    ref = oracle.render(s, cam)
    dev = to_device(s)
    proj = sss.project(dev, cams)
    bins = sss.BinSorter(1024)(proj, cams, n)
    img, tfin, ncon = sss.render_fwd(bins, cams)
    torch.cuda.synchronize()
    H, W = ref["xflags"].shape
    diff = np.abs(img.cpu().numpy().reshape(H, W, 3) - ref["image"]).max(axis=2)
    explained = ref["xflags"] != 0
    assert explained.mean() < 0.01
    assert not ((diff > 1e-4) & ~explained).any(), diff[~explained].max()
    nc = ncon.cpu().numpy().reshape(H, W)
    assert np.array_equal(nc[~explained], ref["ncontrib"][~explained])
    tf = tfin.cpu().numpy().reshape(H, W)
    assert np.all(np.abs(tf - ref["tfinal"])[~explained] <= 1e-4 * np.maximum(1.0, ref["tfinal"][~explained]))


@pytest.mark.gpu
@pytest.mark.parametrize("mode,det", [("stored", False), ("recompute", False), ("stored", True), ("recompute", True)])
def test_edges_backward_matches_oracle(sss, mode, det):
    s, cams = edges_case()
    cam = cams[0]
    n = s["means"].shape[0]
    ref = oracle.render(s, cam)
    w = np.random.default_rng(79).standard_normal(ref["image"].shape)
    w[ref["xflags"] != 0] = 0.0
    gref = oracle.render_backward(s, cam, w, fwd=ref)
    dev = to_device(s)
    proj = sss.project(dev, cams)
    bins = sss.BinSorter(1024, keep_offsets=det)(proj, cams, n)
    img, _, ncon = sss.render_fwd(bins, cams)
    dl = torch.as_tensor(w.reshape(-1, 3), dtype=torch.float32, device="cuda")
    m = sss.BWD_STORED if mode == "stored" else sss.BWD_RECOMPUTE
    g = sss.render_bwd(dev, proj, bins, cams, dl, mode=m, image=img, n_contrib=ncon, deterministic=det)
    torch.cuda.synchronize()
    keep = ref["proj"]["pflags"] == 0
    for k in PARAMS:
        ok, worst = grad_close(g[k].cpu().numpy(), gref[k], mask=keep)
        assert ok, (k, worst)
    # the nu gate: raw nu outside [1, 1e4] gets exactly zero gradient
    outside = (s["nu"] < 1.0) | (s["nu"] > 1e4)
    assert outside.sum() > 50
    assert np.all(g["nu"].cpu().numpy()[outside] == 0.0)
    assert np.abs(gref["g_nu"][outside]).max() > 0.0


def _one_component(nu, o, sigma_px, cam, colour=(0.8, 0.5, 0.3)):
    sc = sigma_px * 4.0 / cam["fx"]
    dc = (np.asarray(colour, np.float64) - 0.5) * 2.0 * math.sqrt(math.pi)
    return dict(means=np.zeros((1, 3), np.float32), scales=np.full((1, 3), sc, np.float32),
                quats=np.array([[0.9, 0.1, -0.3, 0.2]], np.float32), nu=np.array([nu], np.float32),
                opacity=np.array([o], np.float32), sh=dc.astype(np.float32).reshape(1, 1, 3), sh_degree=0)


@pytest.mark.gpu
@pytest.mark.parametrize("o", [0.999, -0.999, 1.0])
@pytest.mark.parametrize("nu", [1.0, 5.0, 1e4])
def test_clamped_alpha_passes_no_gradient_on_gpu(sss, o, nu):
    """One on-axis component with |o| near 1: the image matches the oracle
    (alpha clipped to +-0.99), and with loss weights only on pixels where its
    alpha is clamped (by a margin) every gradient but the colour's is exactly
    zero, as in the oracle."""
    cam = scenes.lookat_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 64, 64)
    s = _one_component(nu, o, 20.0, cam)
    ref = oracle.render(s, cam)
    h, a = _alpha_maps(ref["proj"], cam, 0)
    clamped = np.abs(a) > 0.991
    assert clamped.sum() >= 4
    w = np.zeros((64, 64, 3))
    w[clamped] = np.random.default_rng(3).standard_normal((clamped.sum(), 3))
    gref = oracle.render_backward(s, cam, w, fwd=ref)
    dev = to_device(s)
    cams = [cam]
    proj = sss.project(dev, cams)
    bins = sss.BinSorter(1024, keep_offsets=True)(proj, cams, 1)
    img, _, ncon = sss.render_fwd(bins, cams)
    diff = np.abs(img.cpu().numpy().reshape(64, 64, 3) - ref["image"]).max()
    assert diff <= 1e-4
    dl = torch.as_tensor(w.reshape(-1, 3), dtype=torch.float32, device="cuda")
    for mode in (sss.BWD_STORED, sss.BWD_RECOMPUTE):
        for det in (False, True):
            g = sss.render_bwd(dev, proj, bins, cams, dl, mode=mode, image=img, n_contrib=ncon, deterministic=det)
            torch.cuda.synchronize()
            for k in ("means", "scales", "quats", "nu", "opacity"):
                assert np.all(gref[k] == 0.0), k
                assert np.all(g[k].cpu().numpy() == 0.0), (k, mode, det)
            assert np.abs(gref["sh"]).max() > 0
            ok, worst = grad_close(g["sh"].cpu().numpy(), gref["sh"])
            assert ok, worst


@pytest.mark.gpu
def test_nu_1e4_within_the_gaussian_limit_bound(sss):
    """At nu = 1e4 (the clamp bound) the kernel's 2D t lies within the
    Gaussian-limit bound |ln T_nu + h/2| <= h/nu + (nu + 2) h^2 / (4 nu^2)
    for h <= 11.1 (plus FP32 rounding), and within 1e-5 (relative) of the
    FP64 oracle's T_nu."""
    cam = scenes.lookat_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 96, 96)
    s = _one_component(1e4, 0.8, 10.0, cam, colour=(1.0, 1.0, 1.0))
    opts = dict(alpha_min=0.0)
    ref = oracle.render(s, cam, opts)
    p = ref["proj"]
    h, a = _alpha_maps(p, cam, 0)
    dev = to_device(s)
    proj = sss.project(dev, [cam], opts)
    bins = sss.BinSorter(1 << 14)(proj, [cam], 1)
    img, _, _ = sss.render_fwd(bins, [cam], opts)
    torch.cuda.synchronize()
    col = p["rgb"][0, 0]
    T = img.cpu().numpy().reshape(96, 96, 3)[..., 0].astype(np.float64) / (col * p["opacity"][0])
    sel = h <= 11.1
    assert sel.sum() > 1000
    nu = 1e4
    bound = h / nu + (nu + 2) * h * h / (4 * nu * nu)
    assert np.all(np.abs(np.log(T[sel]) + h[sel] / 2) <= bound[sel] + 2e-6)
    Tref = a / p["opacity"][0]
    assert np.all(np.abs(T[sel] - Tref[sel]) <= 1e-5 * Tref[sel])
    # and the bound is not trivially loose: the Gaussian itself is off by more than FP32 noise
    assert np.abs(np.log(Tref[sel]) + h[sel] / 2).max() > 1e-4


@pytest.mark.gpu
@pytest.mark.parametrize("raw,bound", [(0.7, 1.0), (0.5, 1.0), (2e4, 1e4), (1e6, 1e4)])
def test_raw_nu_outside_the_clamp_renders_as_the_bound(sss, raw, bound):
    """Raw nu outside [1, 1e4]: the image is bit-identical to the one at the
    bound, and nu gets zero gradient while the other parameters get the
    bound's gradients."""
    cam = scenes.lookat_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 48, 48)
    out = {}
    w = torch.as_tensor(np.random.default_rng(9).standard_normal((48 * 48, 3)), dtype=torch.float32, device="cuda")
    for v in (raw, bound):
        s = _one_component(v, 0.6, 6.0, cam)
        dev = to_device(s)
        proj = sss.project(dev, [cam])
        bins = sss.BinSorter(1024, keep_offsets=True)(proj, [cam], 1)
        img, _, ncon = sss.render_fwd(bins, [cam])
        g = sss.render_bwd(dev, proj, bins, [cam], w, image=img, n_contrib=ncon, deterministic=True)
        torch.cuda.synchronize()
        out[v] = (img.cpu().numpy(), {k: g[k].cpu().numpy() for k in PARAMS})
    assert np.array_equal(out[raw][0], out[bound][0])
    assert out[raw][1]["nu"][0] == 0.0 and out[bound][1]["nu"][0] != 0.0
    for k in ("means", "scales", "quats", "opacity", "sh"):
        assert np.array_equal(out[raw][1][k], out[bound][1][k]), k


@pytest.mark.gpu
@pytest.mark.parametrize("opts", [dict(alpha_max=0.9999), dict(alpha_max=0.9999, t_min=0.0)],
                         ids=["alpha_max_0.9999", "t_min_0"])
def test_edges_extreme_compositing_options(sss, opts):
    """alpha_max just below 1 (1 - alpha down to 1e-4) and t_min = 0: a
    finished pixel keeps a negative transmittance that no later component
    may flip or feed.  t_min = 0 acts as the smallest normal float in the
    kernels, where the oracle never stops; what it adds beyond that point is
    below 1e-38, so images and gradients match at the usual bars and the
    contributor counts wherever the oracle's transmittance stays above
    1e-30."""
    s, cams = edges_case()
    cam = cams[0]
    n = s["means"].shape[0]
    ref = oracle.render(s, cam, opts)
    H, W = ref["xflags"].shape
    explained = ref["xflags"] != 0
    assert explained.mean() < 0.01
    assert (ref["tfinal"] < 1e-3).sum() > 200           # deep, saturated pixels
    dev = to_device(s)
    proj = sss.project(dev, cams, opts)
    bins = sss.BinSorter(1024)(proj, cams, n)
    img, tfin, ncon = sss.render_fwd(bins, cams, opts)
    torch.cuda.synchronize()
    diff = np.abs(img.cpu().numpy().reshape(H, W, 3) - ref["image"]).max(axis=2)
    assert not ((diff > 1e-4) & ~explained).any(), diff[~explained].max()
    tf = tfin.cpu().numpy().reshape(H, W)
    assert np.all(tf >= 0.0)
    assert np.all(np.abs(tf - ref["tfinal"])[~explained] <= 1e-4 * np.maximum(1.0, ref["tfinal"][~explained]))
    deep = ref["tfinal"] > 1e-30
    nc = ncon.cpu().numpy().reshape(H, W)
    assert np.array_equal(nc[~explained & deep], ref["ncontrib"][~explained & deep])
    w = np.random.default_rng(80).standard_normal(ref["image"].shape)
    w[explained] = 0.0
    gref = oracle.render_backward(s, cam, w, opts, fwd=ref)
    dl = torch.as_tensor(w.reshape(-1, 3), dtype=torch.float32, device="cuda")
    keep = ref["proj"]["pflags"] == 0
    for m in (sss.BWD_STORED, sss.BWD_RECOMPUTE):
        g = sss.render_bwd(dev, proj, bins, cams, dl, opts, mode=m, image=img, n_contrib=ncon)
        torch.cuda.synchronize()
        for k in PARAMS:
            ok, worst = grad_close(g[k].cpu().numpy(), gref[k], mask=keep)
            assert ok, (k, m, worst)
