"""torch.autograd.Function around the rasterizer.

    image = render(means, scales, quats, nu, opacity, sh, cams, opts, mode="stored")

forward: sss_project -> sss_bin_sort -> sss_render_fwd; backward:
sss_render_bwd with the incoming dL/dimage.  mode "stored" keeps the
forward image and per-pixel list positions for the backward; "recompute"
keeps nothing per pixel and re-walks each tile's list in the backward, so
memory stays flat in the image size.  deterministic=True makes the backward
atomic-free: the gradients are bit-identical from run to run.  The inputs are the activated
parameters (opacity already in [-1, 1], scales positive); activations and
losses are ordinary torch operations around this function.

The returned image is [P, 3] with the views concatenated (see sss.h);
`split_views` reshapes it to a list of [H, W, 3].
"""
from __future__ import annotations

import torch

from . import sss

_PARAMS = ("means", "scales", "quats", "nu", "opacity", "sh")


def _degree(sh: torch.Tensor) -> int:
    K = sh.shape[1]
    d = int(round(K ** 0.5)) - 1
    if (d + 1) ** 2 != K or not 0 <= d <= 3:
        raise ValueError(f"sh must be [n, (d+1)^2, 3] with d <= 3, got {tuple(sh.shape)}")
    return d


class _Ctx:
    """Workspaces reused across calls.  Each forward keeps a pair list of its
    own (several renders may be alive before their backward passes run);
    the sort and backward workspaces are shared, since every call uses them
    only while it runs on the stream."""

    def __init__(self, deterministic: bool = False):
        self.binner = sss.BinSorter(0, keep_offsets=deterministic, own_pairs=True)
        self.deterministic = deterministic
        self.bwd_ws = None


_DEFAULT = _Ctx()
_DEFAULT_DET = _Ctx(deterministic=True)


class RenderFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, nu, opacity, sh, cams, opts, mode, state):
        scene = dict(means=means.contiguous(), scales=scales.contiguous(), quats=quats.contiguous(),
                     nu=nu.contiguous(), opacity=opacity.contiguous(), sh=sh.contiguous(), sh_degree=_degree(sh))
        n = means.shape[0]
        proj = sss.project(scene, cams, opts)
        bins = state.binner(proj, cams, n)
        image, _, n_contrib = sss.render_fwd(bins, cams, opts)
        ctx.scene = scene
        ctx.proj, ctx.bins, ctx.cams, ctx.opts, ctx.mode, ctx.state = proj, bins, cams, opts, mode, state
        # stored mode reads the forward image and list positions back: saved
        # through autograd, so an in-place change of the returned image is
        # reported instead of silently corrupting the gradients
        if mode == "stored":
            ctx.save_for_backward(image, n_contrib)
        return image

    @staticmethod
    def backward(ctx, dl_dimage):
        st = ctx.state
        n = ctx.scene["means"].shape[0]
        if st.deterministic:
            need = int(sss.lib().sss_render_bwd_workspace_det(n * len(ctx.cams), ctx.bins.n_pairs,
                                                              sss.total_tiles(ctx.cams)))
        else:
            need = int(sss.lib().sss_render_bwd_workspace(n * len(ctx.cams), sss.total_tiles(ctx.cams)))
        if st.bwd_ws is None or st.bwd_ws.numel() * 4 < need:
            st.bwd_ws = torch.empty(need // 4, dtype=torch.float32, device=dl_dimage.device)
        mode = sss.BWD_STORED if ctx.mode == "stored" else sss.BWD_RECOMPUTE
        image = n_contrib = None
        if ctx.mode == "stored":
            image, n_contrib = ctx.saved_tensors
        grads = sss.render_bwd(ctx.scene, ctx.proj, ctx.bins, ctx.cams, dl_dimage.contiguous().float(), ctx.opts,
                               mode=mode, loss=sss.LOSS_GRAD, image=image, n_contrib=n_contrib,
                               ws=st.bwd_ws, deterministic=st.deterministic)
        ctx.scene = ctx.proj = ctx.bins = None
        return tuple(grads[k] for k in _PARAMS) + (None, None, None, None)


def render(means, scales, quats, nu, opacity, sh, cams, opts=None, mode: str = "stored", state: _Ctx | None = None,
           deterministic: bool = False):
    """Differentiable render of all `cams` (list of camera dicts)."""
    if mode not in ("stored", "recompute"):
        raise ValueError(mode)
    if state is None:
        state = _DEFAULT_DET if deterministic else _DEFAULT
    return RenderFunction.apply(means, scales, quats, nu, opacity, sh, list(cams), opts, mode, state)


def split_views(image: torch.Tensor, cams):
    out, off = [], 0
    for c in cams:
        P = c["width"] * c["height"]
        out.append(image[off:off + P].view(c["height"], c["width"], 3))
        off += P
    return out
