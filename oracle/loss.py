"""FP64 oracle of the photometric loss (Sec. 3.4):

    L = (1 - lambda) L1 + lambda (1 - SSIM)

L1 is the mean absolute difference over all channels and pixels; SSIM is the
mean over channels and pixels of the structural similarity index (Wang,
Bovik, Sheikh, Simoncelli 2004) with an 11 x 11 Gaussian window of standard
deviation 1.5, constants C1 = 0.01^2, C2 = 0.03^2, and zero padding at the
image border (the window/padding convention of the Gaussian rasterizer the
paper builds on; the paper does not state it).  The opacity and scale
regularisers of the paper's loss are sums over parameters and are not part of
the image gradient.

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
