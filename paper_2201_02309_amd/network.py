"""Dual-domain network of Sec. III: sinogram-domain subnetwork -> Katsevich reconstruction
as the domain-transfer layer -> image-domain subnetwork, trained on the loss of eq. loss
with Adam.

The domain-transfer layer is the library's differentiable reconstruction (KatsevichFn:
katsevich_recon forward, its exact adjoint katsevich_recon_backward backward) on a plan of
one pitch: the sinogram window that reconstructs that pitch's slices goes in, the slices
come out.  The two subnetworks are PyTorch convolutions (MIOpen on ROCm); each 3x3x3
convolution runs as one 2-D convolution over the three depth-shifted copies of its input
stacked as channels, with depth folded into the batch: MIOpen's 3-D convolution backward
measured ~150x slower than this form on the network's shapes.
"""
from __future__ import annotations

import math

import torch
import torch.nn.functional as F
from torch import nn

from .katsevich import KatsevichFn, Plan


class Conv3x3x3(nn.Module):
    """3-D convolution with a 3x3x3 kernel and zero padding 1 (as nn.Conv3d(cin, cout, 3,
    padding=1)), computed as a 2-D convolution: output depth d sees input depths d-1, d,
    d+1 stacked as 3 cin channels."""

    def __init__(self, cin: int, cout: int):
        super().__init__()
        ref = nn.Conv3d(cin, cout, 3, padding=1)           # same initialisation as Conv3d
        self.weight = nn.Parameter(ref.weight.detach().clone())
        self.bias = nn.Parameter(ref.bias.detach().clone())

    def forward(self, x):                                   # x [B, C, D, H, W]
        B, C, D, H, W = x.shape
        xp = F.pad(x, (0, 0, 0, 0, 1, 1))
        stack = torch.cat([xp[:, :, k:k + D] for k in range(3)], dim=1)      # [B, 3C, D, H, W]
        stack = stack.permute(0, 2, 1, 3, 4).reshape(B * D, 3 * C, H, W)
        cout = self.weight.shape[0]
        w2 = self.weight.permute(0, 2, 1, 3, 4).reshape(cout, 3 * C, 3, 3)
        y = F.conv2d(stack, w2, self.bias, padding=1)
        return y.reshape(B, D, cout, H, W).permute(0, 2, 1, 3, 4)


class SubNet(nn.Module):
    """Subnetwork of Sec. III-A: `blocks` cascaded Conv3D(channels, 3x3x3) + PReLU blocks
    and one Conv3D(1, 3x3x3).  The output of every Conv3D+PReLU block is added to the last
    block's output before the final convolution, and the subnetwork's input is added to
    the final convolution's output (ResNet-style skips)."""

    def __init__(self, channels: int = 16, blocks: int = 7):
        super().__init__()
        self.convs = nn.ModuleList([Conv3x3x3(1 if i == 0 else channels, channels)
                                    for i in range(blocks)])
        self.acts = nn.ModuleList([nn.PReLU(channels) for _ in range(blocks)])
        self.out = Conv3x3x3(channels, 1)

    def forward(self, x):                          # x [B, 1, D, H, W]
        h = x
        outs = []
        for conv, act in zip(self.convs, self.acts):
            h = act(conv(h))
            outs.append(h)
        s = outs[-1]
        for o in outs[:-1]:
            s = s + o
        return x + self.out(s)


class DualDomainNet(nn.Module):
    """g (the window sinogram of one pitch, [B, views, rows, cols]) -> (denoised sinogram,
    denoised slices [B, nz, ny, nx])."""

    def __init__(self, plan: Plan, channels: int = 16, blocks: int = 7):
        super().__init__()
        self.plan = plan
        self.sino_net = SubNet(channels, blocks)
        self.image_net = SubNet(channels, blocks)

    def forward(self, g):
        gs = self.sino_net(g.unsqueeze(1)).squeeze(1)
        f0 = KatsevichFn.apply(gs.contiguous(), self.plan)
        f = self.image_net(f0.unsqueeze(1)).squeeze(1)
        return gs, f


def loss(g, f, g_gt, f_gt):
    """Eq. loss: squared L2 errors of the sinogram and of the image, averaged over the
    batch."""
    return ((g_gt - g) ** 2).sum(dim=(1, 2, 3)).mean() + ((f_gt - f) ** 2).sum(dim=(1, 2, 3)).mean()


def pitch_window_geometry(geom: dict, grid: dict):
    """(geometry of the views a pitch's slices use, index of its first view in geom): the
    scan restricted to the views the plan filters plus the derivative's neighbour on each
    side, at the same lambdas."""
    p = Plan(geom, grid, bind=False)
    a, b = int(p.info["first_view"]) - 1, int(p.info["last_view"]) + 1
    p.close()
    w = dict(geom)
    w["lambda_first"] = float(geom.get("lambda_first", 0.0)) + a * 2.0 * math.pi / int(
        geom["views_per_turn"])
    w["n_views"] = b - a + 1
    return w, a
