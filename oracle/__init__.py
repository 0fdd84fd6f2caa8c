"""FP64 CPU oracle for the Student Splatting and Scooping rasterizer.

TEST INFRASTRUCTURE ONLY.  The product library never imports, links or calls
anything here; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` do.  The oracle shares no code with the
HIP library: the arithmetic lives in ``sss_oracle.c`` (plain C, FP64), this
module only marshals numpy arrays.

Method references (3D Student Splatting and Scooping, arXiv 2503.10148):
projection -- Sec. 3.2 eq. (t_2D) and SM "Forward Pass"; compositing --
Sec. 3.4 eq. (SSS_color); gradients -- SM "Backward Pass"; sampler --
Sec. 3.4 eq. (sigmoidUpdate) and SM "SGHMC Sampling".

Functions whose result has no independent pin are marked "parity unpinned"
in their docstring; every other function is pinned by tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sss_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

TILE = 16

# pixel / component explanation flags (see sss_oracle.c)
PF_RECT_EDGE, PF_DET, PF_RGB_CLAMP, PF_TX_CLAMP, PF_NU_CLAMP = 1, 2, 4, 8, 16
XF_ALPHA_MIN, XF_ALPHA_MAX, XF_T_MIN, XF_COMPONENT = 1, 2, 4, 8


def build(force: bool = True) -> str:
    """Compile sss_oracle.c into liboracle.so with gcc (FP64, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB_PATH)
        _lib.orc_bin.restype = ctypes.c_int64
        _lib.orc_tiles_x.restype = ctypes.c_int
        _lib.orc_tiles_y.restype = ctypes.c_int
        _lib.orc_lnbeta.restype = ctypes.c_double
        _lib.orc_lnbeta.argtypes = [ctypes.c_double, ctypes.c_double]
        _lib.orc_relocate_step.restype = ctypes.c_int64
    return _lib


def set_threads(k: int) -> None:
    """Thread count of the oracle's OpenMP loops (projection, compositing,
    raster backward)."""
    _load().orc_set_threads(ctypes.c_int(int(k)))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def cam_array(cam) -> np.ndarray:
    """cam dict (viewmat 3x4, fx, fy, cx, cy, width, height) -> 20 doubles.

    Every value is first rounded to FP32, because the library receives
    FP32 cameras.  A window cut out of a larger image (see `window_camera`)
    carries that image's size in 'clamp_size' for the EWA frustum clamp."""
    v = np.asarray(cam["viewmat"], dtype=np.float32).reshape(12)
    rest = np.array([cam["fx"], cam["fy"], cam["cx"], cam["cy"]], dtype=np.float32)
    cw, ch = cam.get("clamp_size", (cam["width"], cam["height"]))
    return np.concatenate([v.astype(np.float64), rest.astype(np.float64),
                           np.array([cam["width"], cam["height"], cw, ch], dtype=np.float64)])


def window_camera(cam, x0, y0, w, h):
    """The camera that renders pixels [x0, x0+w) x [y0, y0+h) of `cam`.

    The principal point moves by the window origin (exact in FP32 for
    integer offsets) and the frustum clamp keeps the full image's size, so
    every pixel of the window gets the same value as in the full render."""
    c = dict(cam)
    c["cx"] = float(np.float32(cam["cx"]) - np.float32(x0))
    c["cy"] = float(np.float32(cam["cy"]) - np.float32(y0))
    c["width"], c["height"] = int(w), int(h)
    c["clamp_size"] = cam.get("clamp_size", (cam["width"], cam["height"]))
    return c


DEFAULT_OPTS = dict(alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, z_near=0.2, nu_min=1.0,
                    nu_max=1e4, lowpass=0.0, bg=(0.0, 0.0, 0.0), family="student_t", trunc_mode=0)


def opts_array(opts=None) -> np.ndarray:
    o = dict(DEFAULT_OPTS)
    if opts:
        o.update(opts)
    vals = [o["alpha_min"], o["alpha_max"], o["t_min"], o["z_near"], o["nu_min"], o["nu_max"],
            o["lowpass"], *o["bg"]]
    fam = {"student_t": 0, "gaussian": 1}.get(o["family"], o["family"]) if isinstance(o["family"], str) \
        else int(o["family"])
    tm = {"alpha": 0, "coverage": 1}.get(o["trunc_mode"], o["trunc_mode"]) if isinstance(o["trunc_mode"], str) \
        else int(o["trunc_mode"])
    return np.concatenate([np.asarray(vals, dtype=np.float32).astype(np.float64), [float(fam), float(tm)]])


def tiles(cam):
    return (int(cam["width"]) + TILE - 1) // TILE, (int(cam["height"]) + TILE - 1) // TILE


def _scene64(scene):
    n = int(np.asarray(scene["means"]).shape[0])
    deg = int(scene["sh_degree"])
    K = (deg + 1) ** 2
    return dict(n=n, deg=deg, K=K,
                means=_f64(scene["means"]).reshape(n, 3), scales=_f64(scene["scales"]).reshape(n, 3),
                quats=_f64(scene["quats"]).reshape(n, 4), nu=_f64(scene["nu"]).reshape(n),
                opacity=_f64(scene["opacity"]).reshape(n), sh=_f64(scene["sh"]).reshape(n, K, 3))


# --------------------------------------------------------------------------
# spherical harmonics
# --------------------------------------------------------------------------
def sh_eval(degree: int, dirs: np.ndarray, grad: bool = False):
    """Real SH basis (Cartesian polynomial table) at unit directions [m,3]."""
    lib = _load()
    dirs = _f64(dirs).reshape(-1, 3)
    K = (degree + 1) ** 2
    Y = np.zeros((dirs.shape[0], K))
    dY = np.zeros((dirs.shape[0], K, 3))
    for j in range(dirs.shape[0]):
        yj = np.zeros(K)
        dj = np.zeros((K, 3))
        d = np.ascontiguousarray(dirs[j])
        lib.orc_sh_eval(ctypes.c_int(degree), _p(d), _p(yj), _p(dj))
        Y[j] = yj
        dY[j] = dj
    return (Y, dY) if grad else Y


def sh_eval_legendre(degree: int, dirs: np.ndarray):
    """Real SH basis from associated Legendre functions (pins sh_eval)."""
    lib = _load()
    dirs = _f64(dirs).reshape(-1, 3)
    K = (degree + 1) ** 2
    Y = np.zeros((dirs.shape[0], K))
    for j in range(dirs.shape[0]):
        yj = np.zeros(K)
        d = np.ascontiguousarray(dirs[j])
        lib.orc_sh_eval_legendre(ctypes.c_int(degree), _p(d), _p(yj))
        Y[j] = yj
    return Y


# --------------------------------------------------------------------------
# projection / binning / compositing
# --------------------------------------------------------------------------
def project(scene, cam, opts=None):
    """Per-component projection for one camera (FP64)."""
    lib = _load()
    s = _scene64(scene)
    n = s["n"]
    c = cam_array(cam)
    o = opts_array(opts)
    out = dict(valid=np.zeros(n, np.int32), mean2d=np.zeros((n, 2)), cov2d=np.zeros((n, 3)),
               conic=np.zeros((n, 3)), rgb=np.zeros((n, 3)), nu_c=np.zeros(n), hstar=np.zeros(n),
               hrect=np.zeros(n), rect=np.zeros((n, 4), np.int32), key=np.zeros(n, np.uint32),
               touched=np.zeros(n, np.int32), pflags=np.zeros(n, np.int32))
    lib.orc_project(ctypes.c_int(n), ctypes.c_int(s["deg"]), _p(s["means"]), _p(s["scales"]),
                    _p(s["quats"]), _p(s["nu"]), _p(s["opacity"]), _p(s["sh"]), _p(c), _p(o),
                    _p(out["valid"]), _p(out["mean2d"]), _p(out["cov2d"]), _p(out["conic"]),
                    _p(out["rgb"]), _p(out["nu_c"]), _p(out["hstar"]), _p(out["hrect"]), _p(out["rect"]),
                    _p(out["key"]), _p(out["touched"]), _p(out["pflags"]))
    out["opacity"] = s["opacity"]
    return out


def bin_tiles(touched, rect, key, tiles_x, tiles_y, proj=None):
    """Per-tile component lists in ascending (depth key, index) order.  With
    `proj` (a projection result) a tile of a component's rectangle is listed
    when its box of pixel centres meets the component's ellipse; without it
    whole rectangles are listed."""
    lib = _load()
    touched = np.ascontiguousarray(touched, dtype=np.int32)
    rect = np.ascontiguousarray(rect, dtype=np.int32)
    key = np.ascontiguousarray(key, dtype=np.uint32)
    n = touched.shape[0]
    m = int(np.clip(touched, 0, None).astype(np.int64).sum())
    start = np.zeros(tiles_x * tiles_y + 1, np.int32)
    lst = np.zeros(max(m, 1), np.int32)
    geo = (None, None, None) if proj is None else tuple(
        np.ascontiguousarray(proj[k], dtype=np.float64) for k in ("mean2d", "conic", "hrect"))
    got = lib.orc_bin(ctypes.c_int(n), _p(touched), _p(rect), _p(key), *(None if g is None else _p(g) for g in geo),
                      ctypes.c_int(tiles_x), ctypes.c_int(tiles_y), _p(start), _p(lst), ctypes.c_int64(max(m, 1)))
    assert got == m, (got, m)
    return start, lst[:m]


def render(scene, cam, opts=None, brute=False, proj=None):
    """Forward image of one camera: dict(image [H,W,3], tfinal, ncontrib, xflags, proj, bins)."""
    lib = _load()
    if proj is None:
        proj = project(scene, cam, opts)
    W, H = int(cam["width"]), int(cam["height"])
    tx, ty = tiles(cam)
    o = opts_array(opts)
    image = np.zeros((H, W, 3))
    tfin = np.zeros((H, W))
    ncon = np.zeros((H, W), np.int32)
    xf = np.zeros((H, W), np.int32)
    n = proj["valid"].shape[0]
    if brute:
        lib.orc_render_brute(ctypes.c_int(n), _p(proj["valid"]), _p(proj["key"]), _p(proj["mean2d"]),
                             _p(proj["conic"]), _p(proj["rgb"]), _p(proj["opacity"]), _p(proj["nu_c"]),
                             _p(proj["pflags"]), ctypes.c_int(W), ctypes.c_int(H), _p(o), _p(image),
                             _p(tfin), _p(ncon), _p(xf))
        bins = None
    else:
        start, lst = bin_tiles(proj["touched"], proj["rect"], proj["key"], tx, ty, proj=proj)
        lst_c = np.ascontiguousarray(lst if lst.size else np.zeros(1, np.int32))
        lib.orc_render_tiled(_p(proj["mean2d"]), _p(proj["conic"]), _p(proj["rgb"]), _p(proj["opacity"]),
                             _p(proj["nu_c"]), _p(proj["pflags"]), ctypes.c_int(W), ctypes.c_int(H),
                             _p(start), _p(lst_c), _p(o), _p(image), _p(tfin), _p(ncon), _p(xf))
        bins = (start, lst)
    return dict(image=image, tfinal=tfin, ncontrib=ncon, xflags=xf, proj=proj, bins=bins)


def render_backward(scene, cam, dl_dimage, opts=None, fwd=None):
    """Analytic gradients (FP64) of sum(dl_dimage * image) w.r.t. the scene.

    Returns dict with means, scales, quats, nu, opacity, sh and the
    per-component screen-space gradients (g_mean2d, g_conic, g_rgb, g_opac,
    g_nu)."""
    lib = _load()
    if fwd is None:
        fwd = render(scene, cam, opts)
    proj = fwd["proj"]
    start, lst = fwd["bins"]
    s = _scene64(scene)
    n = s["n"]
    W, H = int(cam["width"]), int(cam["height"])
    o = opts_array(opts)
    c = cam_array(cam)
    g = _f64(dl_dimage).reshape(H, W, 3)
    g2 = dict(g_mean2d=np.zeros((n, 2)), g_conic=np.zeros((n, 3)), g_rgb=np.zeros((n, 3)),
              g_opac=np.zeros(n), g_nu=np.zeros(n))
    lst_c = np.ascontiguousarray(lst if lst.size else np.zeros(1, np.int32))
    lib.orc_render_backward(ctypes.c_int(n), _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["rgb"]),
                            _p(proj["opacity"]), _p(proj["nu_c"]), _p(proj["pflags"]), ctypes.c_int(W),
                            ctypes.c_int(H), _p(start), _p(lst_c), _p(o), _p(g), _p(g2["g_mean2d"]),
                            _p(g2["g_conic"]), _p(g2["g_rgb"]), _p(g2["g_opac"]), _p(g2["g_nu"]))
    out = dict(means=np.zeros((n, 3)), scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
               nu=np.zeros(n), opacity=np.zeros(n), sh=np.zeros((n, s["K"], 3)))
    lib.orc_project_backward(ctypes.c_int(n), ctypes.c_int(s["deg"]), _p(s["means"]), _p(s["scales"]),
                             _p(s["quats"]), _p(s["nu"]), _p(s["opacity"]), _p(s["sh"]), _p(c), _p(o),
                             _p(proj["valid"]), _p(g2["g_mean2d"]), _p(g2["g_conic"]), _p(g2["g_rgb"]),
                             _p(g2["g_opac"]), _p(g2["g_nu"]), _p(out["means"]), _p(out["scales"]),
                             _p(out["quats"]), _p(out["nu"]), _p(out["opacity"]), _p(out["sh"]))
    out.update(g2)
    return out


def l1_grad(image, target):
    """dL/dC of the mean absolute error over all channels of all pixels."""
    image = np.asarray(image, np.float64)
    return np.sign(image - np.asarray(target, np.float64)) / image.size


# --------------------------------------------------------------------------
# sampler
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib.orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def normals3(i, seed, step):
    lib = _load()
    z = np.zeros(3)
    lib.orc_normals3(ctypes.c_uint64(i), ctypes.c_uint64(seed), ctypes.c_uint64(step), _p(z))
    return z


def sghmc_step(means, mom, grad, opacity, scales, quats, lr, friction=0.1, k=100.0, t=0.995,
               burn_in=False, noise=True, seed=0, step=0):
    """One SGHMC step on the means (in place on float64 copies, returned)."""
    lib = _load()
    means = _f64(means).copy().reshape(-1, 3)
    mom = _f64(mom).copy().reshape(-1, 3)
    n = means.shape[0]
    g = _f64(grad).reshape(n, 3)
    o = _f64(opacity).reshape(n)
    s = _f64(scales).reshape(n, 3)
    q = _f64(quats).reshape(n, 4)
    lib.orc_sghmc_step(ctypes.c_int(n), _p(means), _p(mom), _p(g), _p(o), _p(s), _p(q),
                       ctypes.c_double(lr), ctypes.c_double(friction), ctypes.c_double(k),
                       ctypes.c_double(t), ctypes.c_int(int(burn_in)), ctypes.c_int(int(noise)),
                       ctypes.c_uint64(seed), ctypes.c_uint64(step))
    return means, mom


def adam_step(param, grad, m, v, lr, b1=0.9, b2=0.999, eps=1e-15, t=1, lo=-np.inf, hi=np.inf):
    lib = _load()
    param = _f64(param).copy().reshape(-1)
    m = _f64(m).copy().reshape(-1)
    v = _f64(v).copy().reshape(-1)
    g = _f64(grad).reshape(-1)
    lib.orc_adam_step(ctypes.c_int64(param.size), _p(param), _p(g), _p(m), _p(v), ctypes.c_double(lr),
                      ctypes.c_double(b1), ctypes.c_double(b2), ctypes.c_double(eps), ctypes.c_int64(t),
                      ctypes.c_double(lo), ctypes.c_double(hi))
    return param, m, v


# --------------------------------------------------------------------------
# recycling
# --------------------------------------------------------------------------
def lnbeta(x, y):
    return float(_load().orc_lnbeta(x, y))


def relocate(o_old, nu_old, nu_new, N):
    """(o_new, Sigma_new / Sigma_old) for N components at one old component."""
    lib = _load()
    o = ctypes.c_double()
    f = ctypes.c_double()
    lib.orc_relocate(ctypes.c_double(o_old), ctypes.c_double(nu_old), ctypes.c_double(nu_new), ctypes.c_int(N),
                     ctypes.byref(o), ctypes.byref(f))
    return o.value, f.value


def relocate_step(scene, dead_opacity=0.005, max_fraction=0.05, seed=0, step=0, states=()):
    """One recycling step on float64 copies; returns (scene, states, dead, targets)."""
    lib = _load()
    s = _scene64(scene)
    n = s["n"]
    arrs = {k: s[k].copy() for k in ("means", "scales", "quats", "nu", "opacity", "sh")}
    st = [np.ascontiguousarray(np.asarray(a, np.float64).reshape(n, -1)).copy() for a in states]
    ptrs = (ctypes.c_void_p * max(1, len(st)))(*[a.ctypes.data for a in st])
    widths = (ctypes.c_int * max(1, len(st)))(*[a.shape[1] for a in st])
    dead = np.zeros(n, np.int64)
    targ = np.zeros(n, np.int64)
    nd = lib.orc_relocate_step(ctypes.c_int64(n), ctypes.c_int(s["deg"]), _p(arrs["means"]), _p(arrs["scales"]),
                               _p(arrs["quats"]), _p(arrs["nu"]), _p(arrs["opacity"]), _p(arrs["sh"]),
                               ctypes.c_double(dead_opacity), ctypes.c_double(max_fraction), ctypes.c_uint64(seed),
                               ctypes.c_uint64(step), ctypes.c_int(len(st)), ptrs, widths, _p(dead), _p(targ))
    arrs["sh_degree"] = s["deg"]
    return arrs, st, dead[:nd], targ[:nd]
