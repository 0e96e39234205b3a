"""FP64 CPU reference of the learned corrector network (test infrastructure only).

TEST INFRASTRUCTURE ONLY (see the package docstring): only the tests, the smoke
check and the benchmark's CPU-baseline leg may call this module.

The corrector is a residual network on a real-space orientation volume
psi[N][H][W]: three 3x3 convolutions with circular (periodic) padding,
N -> 32 -> 32 -> N channels, ReLU after the first two, and the output added
to the input.  The network sees the volume divided by its root mean square
s (1 for an all-zero volume) and its output is scaled back by s, so it works
in the same units whatever the image's intensity.  Channels are carried
padded to 32: input channels N..31 are zero, as are the weights that read
them (layer 1) or write output channels N..31 (layer 3), so the padded
network computes exactly the N-channel one.

Definitions (written out, no blocking or reordering):

    conv(x, W, b)[o, y, x] = b[o] + sum_{c, dy, dx} W[o, c, dy+1, dx+1] x[c, y+dy, x+dx]

with indices taken modulo H and W, dy, dx in {-1, 0, 1};

    s = sqrt(mean(x^2)),  a0 = x/s padded to 32 channels,
    z1 = conv(a0, W1, b1),  a1 = relu(z1),  z2 = conv(a1, W2, b2),  a2 = relu(z2),
    r = conv(a2, W3, b3)[:N],  out = x + s r,
    loss = mean over (images, N, H, W) of ((out - target)/s)^2   (s per image).

Gradients follow from the chain rule:

    g3 = dloss/dr = 2 (out - target) / (s numel),
    dW3[o, c, dy, dx] = sum_{y, x} g3[o, y, x] a2[c, y+dy, x+dx],
    db3[o] = sum g3[o],  da2[c, y, x] = sum_{o, dy, dx} W3[o, c, dy, dx] g3[o, y-dy, x-dx],
    g2 = da2 * [a2 > 0],  and likewise for layers 2 and 1.

With ``bf16=True`` the values the GPU stores in bfloat16 are rounded to
bfloat16 at the same points (network input, weights, a1, a2, and the gradient
g3, g2, g1 handed from layer to layer), so that a comparison isolates the
accumulation order.  Rounding is to nearest, ties to even, of the float32
value.

Parameter vector (float64, 27744 values): for each layer l = 1, 2, 3 the
weights W_l[o][c][tap] (32 x 32 x 9, tap = (dy+1)*3 + (dx+1)) followed by the
bias b_l[o] (32).
"""
from __future__ import annotations

import numpy as np

CP = 32                     # padded channel count
NW = CP * CP * 9            # weights per layer
NL = NW + CP                # parameters per layer
NPARAM = 3 * NL


def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via float32; returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params: np.ndarray) -> list[tuple[np.ndarray, np.ndarray]]:
    """[(W_l [32][32][3][3], b_l [32]) for l = 1, 2, 3] from the flat vector."""
    p = np.asarray(params, dtype=np.float64)
    assert p.size == NPARAM
    out = []
    for l in range(3):
        w = p[l * NL:l * NL + NW].reshape(CP, CP, 3, 3)
        b = p[l * NL + NW:(l + 1) * NL]
        out.append((w, b))
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([w.reshape(-1), b]) for w, b in layers])


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Circular 3x3 convolution (cross-correlation) of x [C][H][W] with w [O][C][3][3]."""
    out = np.broadcast_to(b[:, None, None], (w.shape[0],) + x.shape[1:]).astype(np.float64).copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            shifted = np.roll(x, shift=(-dy, -dx), axis=(1, 2))  # shifted[c, y, x] = x[c, y+dy, x+dx]
            out += np.einsum("oc,chw->ohw", w[:, :, dy + 1, dx + 1], shifted)
    return out


def conv3x3_transpose(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of conv3x3 in its input: d[c, y, x] = sum_{o, dy, dx} w[o, c, dy, dx] g[o, y-dy, x-dx]."""
    out = np.zeros((w.shape[1],) + g.shape[1:])
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            shifted = np.roll(g, shift=(dy, dx), axis=(1, 2))  # shifted[o, y, x] = g[o, y-dy, x-dx]
            out += np.einsum("oc,ohw->chw", w[:, :, dy + 1, dx + 1], shifted)
    return out


def conv3x3_wgrad(g: np.ndarray, x: np.ndarray) -> np.ndarray:
    """dW[o, c, dy, dx] = sum_{y, x} g[o, y, x] x[c, y+dy, x+dx]."""
    dw = np.zeros((g.shape[0], x.shape[0], 3, 3))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            shifted = np.roll(x, shift=(-dy, -dx), axis=(1, 2))
            dw[:, :, dy + 1, dx + 1] = np.einsum("ohw,chw->oc", g, shifted)
    return dw


def _r(v, on):
    return bf16_round(v) if on else v


def forward(x: np.ndarray, params: np.ndarray, bf16: bool = False) -> dict:
    """x [N][H][W] -> the network's intermediate values and out = x + r."""
    N = x.shape[0]
    (w1, b1), (w2, b2), (w3, b3) = unpack(params)
    if bf16:
        w1, w2, w3 = bf16_round(w1), bf16_round(w2), bf16_round(w3)
    s = rms(x)
    a0 = np.zeros((CP,) + x.shape[1:])
    a0[:N] = _r(x / s, bf16)
    z1 = conv3x3(a0, w1, b1)
    a1 = _r(np.maximum(z1, 0.0), bf16)
    z2 = conv3x3(a1, w2, b2)
    a2 = _r(np.maximum(z2, 0.0), bf16)
    r = conv3x3(a2, w3, b3)[:N]
    return dict(s=s, a0=a0, a1=a1, a2=a2, r=r, out=x + s * r, w=(w1, w2, w3))


def rms(x) -> float:
    """Root mean square of a volume; 1 for an all-zero volume."""
    v = float(np.sqrt(np.mean(np.asarray(x, dtype=np.float64) ** 2)))
    return v if v > 0.0 else 1.0


def loss_and_grads(xs, targets, params: np.ndarray, bf16: bool = False) -> tuple[float, np.ndarray]:
    """Mean squared error of out against target, each image in units of its
    input's RMS, over a batch, and its gradient with respect to the parameter
    vector (chain rule as in the module docstring)."""
    xs = [np.asarray(x, dtype=np.float64) for x in xs]
    targets = [np.asarray(t, dtype=np.float64) for t in targets]
    numel = sum(x.size for x in xs)
    loss = 0.0
    grads = [[np.zeros((CP, CP, 3, 3)), np.zeros(CP)] for _ in range(3)]
    for x, t in zip(xs, targets):
        N = x.shape[0]
        fw = forward(x, params, bf16)
        w1, w2, w3 = fw["w"]
        diff = (fw["out"] - t) / fw["s"]
        loss += float(np.sum(diff * diff))
        g3 = np.zeros((CP,) + x.shape[1:])
        g3[:N] = _r(2.0 * diff / numel, bf16)
        grads[2][0] += conv3x3_wgrad(g3, fw["a2"])
        grads[2][1] += g3.sum(axis=(1, 2))
        g2 = _r(conv3x3_transpose(g3, w3) * (fw["a2"] > 0), bf16)
        grads[1][0] += conv3x3_wgrad(g2, fw["a1"])
        grads[1][1] += g2.sum(axis=(1, 2))
        g1 = _r(conv3x3_transpose(g2, w2) * (fw["a1"] > 0), bf16)
        grads[0][0] += conv3x3_wgrad(g1, fw["a0"])
        grads[0][1] += g1.sum(axis=(1, 2))
    return loss / numel, pack(grads)


def adam(params, grads, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step (Kingma and Ba), step number t >= 1, bias-corrected moments.
    Returns the new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grads
    v = beta2 * v + (1.0 - beta2) * grads * grads
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(N: int, seed: int) -> np.ndarray:
    """He-normal weights for layers 1 and 2, zero layer 3 (the network starts
    as the identity map), zero biases; padded entries zero."""
    rng = np.random.default_rng(seed)
    w1 = np.zeros((CP, CP, 3, 3))
    w1[:, :N] = rng.standard_normal((CP, N, 3, 3)) * np.sqrt(2.0 / (9 * N))
    w2 = rng.standard_normal((CP, CP, 3, 3)) * np.sqrt(2.0 / (9 * CP))
    w3 = np.zeros((CP, CP, 3, 3))
    z = np.zeros(CP)
    return pack([(w1, z), (w2, z.copy()), (w3, z.copy())])
