"""FP64 reference of the warm-start network (test infrastructure only).

Topology (fixed, widths configurable): trunk 1: 4 -> w1, 4x4 kernel, stride
4; trunk 2: w1 -> w2, 3x3, stride 2, padding 1; trunk 3: w2 -> w3, 3x3,
stride 2, padding 1; head k: trunk k -> out, 3x3, stride 1, padding 1.  ReLU
after the trunk layers.  Parameters are stored as one flat vector: for the
layers in the order trunk 1..3, head 1..3, the weights [co][ci][k][k] and
then the biases [co]; they are used after rounding to bfloat16 (nearest,
ties to even).  Loss: mean squared error over all head outputs.

Convolutions are torch.nn.functional.conv2d in float64 (a library routine);
the gradient is obtained by automatic differentiation.
"""
import numpy as np
import torch
import torch.nn.functional as F

DT = torch.float64


def layer_specs(w1, w2, w3, out_ch):
    """(co, ci, k, stride, padding, relu) of the six layers."""
    return [(w1, 4, 4, 4, 0, True), (w2, w1, 3, 2, 1, True), (w3, w2, 3, 2, 1, True),
            (out_ch, w1, 3, 1, 1, False), (out_ch, w2, 3, 1, 1, False), (out_ch, w3, 3, 1, 1, False)]


def n_params(specs):
    return sum(co * ci * k * k + co for co, ci, k, *_ in specs)


def bf16_round(x):
    """float32 values rounded to bfloat16 (nearest even), returned as float64."""
    return torch.as_tensor(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).to(DT)


def unpack(theta, specs):
    out, o = [], 0
    for co, ci, k, s, p, relu in specs:
        w = theta[o:o + co * ci * k * k].view(co, ci, k, k)
        o += co * ci * k * k
        b = theta[o:o + co]
        o += co
        out.append((w, b, s, p, relu))
    return out


def forward(theta, specs, img):
    """theta: float64 tensor (already bf16-rounded); img [B, 4, S, S]. Returns (acts, out)."""
    L = unpack(theta, specs)
    x = torch.as_tensor(img, dtype=DT)
    acts = []
    for w, b, s, p, relu in L[:3]:
        x = F.conv2d(x, w, b, stride=s, padding=p)
        x = torch.relu(x)
        acts.append(x)
    heads = [F.conv2d(a, w, b, stride=s, padding=p) for a, (w, b, s, p, _) in zip(acts, L[3:])]
    B = x.shape[0]
    out = torch.cat([h.reshape(B, -1) for h in heads], 1)
    act = torch.cat([a.reshape(B, -1) for a in acts], 1)
    return act, out


def loss_and_grad(theta, specs, img, target):
    """Mean squared error and its gradient with respect to theta (float64)."""
    t = torch.as_tensor(theta, dtype=DT).clone().requires_grad_(True)
    _, out = forward(t, specs, img)
    loss = ((out - torch.as_tensor(target, dtype=DT)) ** 2).mean()
    (g,) = torch.autograd.grad(loss, t)
    return float(loss), g.numpy()


def rasterize(size, idx, u, v, re, re_center, re_scale):
    """Image [B, 4, size, size]: u, v and 1 at observed cells, (Re - c) / s everywhere."""
    B = len(re)
    img = np.zeros((B, 4, size * size))
    for b in range(B):
        img[b, 0, idx[b]] = u[b]
        img[b, 1, idx[b]] = v[b]
        img[b, 2, idx[b]] = 1.0
        img[b, 3, :] = (re[b] - re_center) / re_scale
    return img.reshape(B, 4, size, size)
