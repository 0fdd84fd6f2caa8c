"""FP64 oracle of the photometric loss (Sec. 3.4):

    L = (1 - lambda) L1 + lambda (1 - SSIM)

L1 is the mean absolute difference over all channels and pixels; SSIM is the
mean over channels and pixels of the structural similarity index (Wang,
Bovik, Sheikh, Simoncelli 2004) with an 11 x 11 Gaussian window of standard
deviation 1.5, constants C1 = 0.01^2, C2 = 0.03^2, and zero padding at the
image border (the window/padding convention of the Gaussian rasterizer the
paper builds on; the paper does not state it).  The opacity and scale
regularisers of the paper's loss, eps_o sum_i |o_i| + eps_s sum_ij sqrt(lambda_ij)
with lambda the eigenvalues of Sigma_i, are sums over parameters and are not
part of the image gradient: `regulariser` computes them from that definition
(Sigma built from the quaternion and scales, eigenvalues by a symmetric
eigensolver).

TEST INFRASTRUCTURE ONLY.  Plain float64 PyTorch CPU operations; the
gradient dL/dimage is reverse-mode autograd of this definition.
"""
from __future__ import annotations

import math

import numpy as np
import torch

WINDOW, SIGMA, C1, C2 = 11, 1.5, 0.01 ** 2, 0.03 ** 2


def gaussian_window(size=WINDOW, sigma=SIGMA):
    x = torch.arange(size, dtype=torch.float64) - (size - 1) / 2.0
    g = torch.exp(-x * x / (2.0 * sigma * sigma))
    g = g / g.sum()
    return torch.outer(g, g)


def _blur(img):
    """img [C, H, W] -> window-weighted local means, zero padding."""
    C = img.shape[0]
    w = gaussian_window().expand(C, 1, WINDOW, WINDOW).contiguous()
    return torch.nn.functional.conv2d(img[None], w, padding=WINDOW // 2, groups=C)[0]


def ssim_map(x, y):
    """x, y: [C, H, W] float64 -> per-pixel SSIM [C, H, W]."""
    mx, my = _blur(x), _blur(y)
    sxx = _blur(x * x) - mx * mx
    syy = _blur(y * y) - my * my
    sxy = _blur(x * y) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def loss_and_grad(image, target, lam):
    """image, target: [H, W, 3] arrays.  Returns (L, dL/dimage [H, W, 3])."""
    x = torch.tensor(np.asarray(image, np.float64)).permute(2, 0, 1).contiguous().requires_grad_(True)
    y = torch.tensor(np.asarray(target, np.float64)).permute(2, 0, 1).contiguous()
    l1 = (x - y).abs().mean()
    ssim = ssim_map(x, y).mean()
    L = (1.0 - lam) * l1 + lam * (1.0 - ssim)
    L.backward()
    return float(L), x.grad.permute(1, 2, 0).numpy().copy()


def _sigma(scales, quats):
    """Sigma = R diag(s^2) R^T per component, R from the normalised quaternion (w, x, y, z)."""
    q = quats / torch.linalg.norm(quats, dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)], 1)
    return R @ torch.diag_embed(scales * scales) @ R.transpose(1, 2)


def regulariser(opacity, scales, quats, eps_o, eps_s):
    """Sec. 3.4 regularisers eps_o sum|o| + eps_s sum sqrt(eig Sigma).  Returns
    (value, d/d opacity [n], d/d scales [n, 3], d/d quats [n, 4]), FP64,
    gradient by reverse-mode autograd of the definition."""
    o = torch.tensor(np.asarray(opacity, np.float64)).requires_grad_(True)
    s = torch.tensor(np.asarray(scales, np.float64)).requires_grad_(True)
    q = torch.tensor(np.asarray(quats, np.float64)).requires_grad_(True)
    lam = torch.linalg.eigvalsh(_sigma(s, q)).clamp_min(0.0)
    R = eps_o * o.abs().sum() + eps_s * lam.sqrt().sum()
    R.backward()
    return float(R), o.grad.numpy().copy(), s.grad.numpy().copy(), q.grad.numpy().copy()
