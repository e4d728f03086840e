"""CPU oracle of the learned initial guess (the network of fk_net_*).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg; the GPU library never uses it and shares no
code with it.  Plain numpy in FP64, written from the definitions:

  g = 2 u_m - u_{m-1};  x <- g;  repeat passes times: x <- x + N(b - A x)
  N: L layers of 3x3 cross-correlation with zero padding and no bias,
     1 -> C -> ... -> C -> 1 channels, ReLU (or the identity: linear)
     between layers
  training sample: r = b - A g and the target (u_next - g) divided by
  s = max|r|; loss = mean over the grid of (N - target)^2.

With ``bf16=True`` the oracle rounds to BF16 where the device stores BF16
(weights, the input plane, hidden activations, the output gradient and the
hidden gradients) and to FP32 where it stores FP32, so the two differ only
by accumulation order (FP32 matrix-core sums on the device, FP64 here).
The product A g uses the CSR oracle (rows summed left to right).
"""
from __future__ import annotations

import numpy as np

CH = 16
NIN = 1


def bf16(a) -> np.ndarray:
    """Round to FP32, then to BF16 (nearest, ties to even); returned as FP64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shapes(layers: int, ch: int = CH) -> list[tuple[int, int]]:
    """(cout, cin) of each layer."""
    return [(1 if l == layers - 1 else ch, NIN if l == 0 else ch) for l in range(layers)]


def num_weights(layers: int, ch: int = CH) -> int:
    return sum(co * ci * 9 for co, ci in shapes(layers, ch))


def split(w, layers: int, ch: int = CH) -> list[np.ndarray]:
    """Canonical weight vector -> per-layer arrays W[co][ci][ky][kx]."""
    w = np.asarray(w, dtype=np.float64)
    out, off = [], 0
    for co, ci in shapes(layers, ch):
        out.append(w[off: off + co * ci * 9].reshape(co, ci, 3, 3))
        off += co * ci * 9
    assert off == w.size
    return out


def conv(x: np.ndarray, W: np.ndarray) -> np.ndarray:
    """out[co][y][x] = sum_ci sum_ky,kx W[co][ci][ky][kx] * x[ci][y+ky-1][x+kx-1] (zeros outside)."""
    cin, ny, nx = x.shape
    xp = np.zeros((cin, ny + 2, nx + 2))
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((W.shape[0], ny, nx))
    for ky in range(3):
        for kx in range(3):
            out += np.tensordot(W[:, :, ky, kx], xp[:, ky: ky + ny, kx: kx + nx], axes=(1, 0))
    return out


def conv_adjoint(g: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Adjoint of conv with respect to its input: <conv(x, W), g> = <x, conv_adjoint(g, W)>."""
    _, ny, nx = g.shape
    xp = np.zeros((W.shape[1], ny + 2, nx + 2))
    for ky in range(3):
        for kx in range(3):
            xp[:, ky: ky + ny, kx: kx + nx] += np.tensordot(W[:, :, ky, kx], g, axes=(0, 0))
    return xp[:, 1:-1, 1:-1]


def conv_weight_grad(g: np.ndarray, x: np.ndarray) -> np.ndarray:
    """d<conv(x, W), g>/dW[co][ci][ky][kx] = sum_y,x g[co][y][x] x[ci][y+ky-1][x+kx-1]."""
    cin, ny, nx = x.shape
    xp = np.zeros((cin, ny + 2, nx + 2))
    xp[:, 1:-1, 1:-1] = x
    dw = np.zeros((g.shape[0], cin, 3, 3))
    for ky in range(3):
        for kx in range(3):
            dw[:, :, ky, kx] = np.tensordot(g, xp[:, ky: ky + ny, kx: kx + nx], axes=((1, 2), (1, 2)))
    return dw


def features(A, nx: int, ny: int, b, um, um1, unext=None, normalize: bool = False, bf: bool = True,
             spmv=None, base=None):
    """Input plane (1, ny, nx) r = b - A x for the base guess x (default the
    extrapolation g = 2 u_m - u_{m-1}), x itself, and (training) the target
    plane and the scale s.  spmv(A, v) is the CSR product (the oracle's by
    default)."""
    if spmv is None:
        from . import spmv as spmv  # the CSR oracle
    b, um, um1 = (np.asarray(v, dtype=np.float64) for v in (b, um, um1))
    g = 2.0 * um - um1 if base is None else np.asarray(base, dtype=np.float64)
    r = b - spmv(A, g)
    s = 1.0
    if normalize:
        s = float(np.max(np.abs(r)))
        if not s > 0.0:
            s = 1.0
    plane = (r / s).reshape(NIN, ny, nx)
    plane = bf16(plane) if bf else plane
    target = None
    if unext is not None:
        target = ((np.asarray(unext, dtype=np.float64) - g) / s).astype(np.float32).astype(np.float64)
    return plane, g, target, s


def forward(w, planes: np.ndarray, layers: int, bf: bool = True, linear: bool = False):
    """Network output y (ny, nx) and the input of every layer."""
    Ws = split(w, layers)
    if bf:
        Ws = [bf16(W) for W in Ws]
    acts = [planes]
    a = planes
    for l, W in enumerate(Ws):
        z = conv(a, W)
        if l < layers - 1:
            a = z if linear else np.maximum(z, 0.0)
            a = bf16(a) if bf else a
            acts.append(a)
        else:
            y = z[0].astype(np.float32).astype(np.float64) if bf else z[0]
    return y, acts


def loss_and_gradient(w, planes: np.ndarray, target: np.ndarray, layers: int, bf: bool = True,
                      linear: bool = False):
    """Mean squared error against target and its gradient (canonical order)."""
    Ws = split(w, layers)
    Wf = [bf16(W) for W in Ws] if bf else Ws
    y, acts = forward(w, planes, layers, bf, linear)
    n = y.size
    diff = y - target
    if bf:
        diff = diff.astype(np.float32).astype(np.float64)
        g = bf16(diff.astype(np.float32) * np.float32(2.0 / n))[None]
    else:
        g = (2.0 * diff / n)[None]
    loss = float(np.mean(diff * diff))
    grads = [None] * layers
    for l in range(layers - 1, -1, -1):
        grads[l] = conv_weight_grad(g, acts[l])
        if l > 0:
            g = conv_adjoint(g, Wf[l])
            g = g if linear else g * (acts[l] > 0)
            g = bf16(g) if bf else g
    return loss, np.concatenate([gr.ravel() for gr in grads])


def guess(w, A, nx: int, ny: int, b, um, um1, layers: int, passes: int = 1, bf: bool = True,
          spmv=None, linear: bool = False):
    """x0 after `passes` corrections, without the fallback."""
    x = None
    for _ in range(passes):
        plane, x, _, _ = features(A, nx, ny, b, um, um1, bf=bf, spmv=spmv, base=x)
        y, _ = forward(w, plane, layers, bf, linear)
        x = x + y.ravel()
    return x
