"""FP64 reference of the learned warm start: network, loss, gradients, Adam.

TEST INFRASTRUCTURE.  Same rule as the rest of ``oracle``: only tests/,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; it shares no code with the GPU library.

The paper has no network.  The learned warm start takes the first
multiplicative factor x of the EM-type update from the uniform start (Alg. 5
with f^0 = u everywhere, u = sum(y) / sum(b^(1)), b^(1) = A^T 1): the back
projection (the back projector of Alg. 3) of the count ratio y / (A f^0),
divided by b^(1) -- dimensionless, and u x is the first EM iterate.  As the
EM iterates are products of such factors, the network works on logarithms:
its input is log(x + delta), its last layer adds that input back (a residual),
its training target is log(f_T / u + delta) for a reconstruction f_T made by
Alg. 5 itself, and its output o gives the starting image through the inverse
map u max(exp(o) - delta, delta / 100) > 0, scaled to the total
sum(b^(1) f) = sum(y) that every unpenalised EM iterate carries (a regression
on logarithms estimates geometric means, biased low).  The definitions written out here
are the textbook ones:

* 3 x 3 cross-correlation with one pixel of zero padding, images stored
  height x width x channels (the q bins of an image [nz][nx][nq] are its
  channels), weights [tap][c_in][c_out] with tap = 3 dh + dw reading the input
  pixel (h + dh - 1, w + dw - 1);
* ReLU; squared error summed over elements and averaged over the images of a
  batch;
* gradients by the chain rule (pinned by central finite differences);
* Adam with bias correction (Kingma & Ba, 2015, Algorithm 1).

Precision model of the GPU network (``half=True``): every operand of a
convolution's products -- input activation, weight and, in the backward
passes, the output gradient -- is rounded to IEEE binary16 (nearest, ties to
even) before it is multiplied; products and sums are then exact here (the GPU
accumulates in binary32).  Bias terms, the residual, ReLU, the mask of the
ReLU backward, the head and Adam see unrounded values.

Parity status: pinned in tests/test_oracle_cnn.py (scipy.signal.correlate2d,
shifted-identity kernels, finite differences, Adam's closed-form first step,
binary16 rounding of known values).
"""
from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np

TAPS = [(dh, dw) for dh in range(3) for dw in range(3)]
O_CLAMP = 30.0        # upper bound of o before exponentiation
FLOOR = 0.01          # f^0 / u >= FLOOR * delta


def f16(a) -> np.ndarray:
    """Round to IEEE binary16 (nearest, ties to even) and widen back to float64."""
    return np.asarray(a, dtype=np.float64).astype(np.float16).astype(np.float64)


def _maybe16(a, half: bool) -> np.ndarray:
    return f16(a) if half else np.asarray(a, dtype=np.float64)


def _pad(x: np.ndarray) -> np.ndarray:
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))


def conv3x3(x, w, bias=None, relu: bool = False, half: bool = True, residual=None) -> np.ndarray:
    """y[b,h,w,o] = bias[o] + sum_{dh,dw,i} x[b,h+dh-1,w+dw-1,i] w[3dh+dw,i,o]
    (zero outside the image) (+ residual[b,h,w,o]), then max(., 0) if relu."""
    x = _maybe16(x, half)
    w = _maybe16(w, half)
    nb, H, W, _ = x.shape
    xp = _pad(x)
    y = np.zeros((nb, H, W, w.shape[2]))
    for t, (dh, dw) in enumerate(TAPS):
        y += xp[:, dh:dh + H, dw:dw + W, :] @ w[t]
    if bias is not None:
        y += np.asarray(bias, dtype=np.float64)
    if residual is not None:
        y += np.asarray(residual, dtype=np.float64)
    return np.maximum(y, 0.0) if relu else y


def conv3x3_backward_data(dy, w, mask=None, half: bool = True) -> np.ndarray:
    """dL/dx of conv3x3 given dL/dy: dx[b,p,i] = sum_t sum_o dy[b,p-off_t,o] w[t,i,o]
    with off_t = (dh-1, dw-1) and dy zero outside the image; multiplied by
    [mask > 0] if a mask (the layer's input activation after a ReLU) is given."""
    dy = _maybe16(dy, half)
    w = _maybe16(w, half)
    nb, H, W, _ = dy.shape
    dyp = _pad(dy)
    dx = np.zeros((nb, H, W, w.shape[1]))
    for t, (dh, dw) in enumerate(TAPS):
        # p - off_t + 1 (padded index) = p + 2 - dh
        dx += dyp[:, 2 - dh:2 - dh + H, 2 - dw:2 - dw + W, :] @ w[t].T
    if mask is not None:
        dx = dx * (np.asarray(mask) > 0)
    return dx


def conv3x3_backward_weights(x, dy, half: bool = True):
    """dL/dw[t,i,o] = sum_{b,p} x[b,p+off_t,i] dy[b,p,o] and dL/dbias[o] =
    sum_{b,p} dy[b,p,o] (the bias gradient uses the unrounded dy)."""
    xr = _maybe16(x, half)
    dyr = _maybe16(dy, half)
    nb, H, W, ci = xr.shape
    co = dyr.shape[3]
    xp = _pad(xr)
    d2 = dyr.reshape(-1, co)
    dw = np.zeros((9, ci, co))
    for t, (dh, dwd) in enumerate(TAPS):
        dw[t] = xp[:, dh:dh + H, dwd:dwd + W, :].reshape(-1, ci).T @ d2
    db = np.asarray(dy, dtype=np.float64).reshape(-1, co).sum(axis=0)
    return dw, db


def head(o, t, n_images: int):
    """Squared error of o against the target t, summed over elements and
    divided by the number of images; returns (loss, dL/do)."""
    r = np.asarray(o, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    return float(np.sum(r * r)) / n_images, 2.0 * r / n_images


def forward(params: List[Dict[str, np.ndarray]], x, half: bool = True) -> List[np.ndarray]:
    """Activations [x, a1, ..., o] of the network: every layer but the last is
    followed by a ReLU; the last adds the network input x (same channels)."""
    acts = [np.asarray(x, dtype=np.float64)]
    n = len(params)
    for k, lay in enumerate(params):
        acts.append(conv3x3(acts[-1], lay["w"], lay["b"], relu=k < n - 1, half=half,
                            residual=acts[0] if k == n - 1 else None))
    return acts


def loss(params, x, t, half: bool = True) -> float:
    o = forward(params, x, half)[-1]
    return head(o, t, o.shape[0])[0]


def backward(params, acts: List[np.ndarray], t, half: bool = True):
    """Loss and the gradients {w, b} of every layer (chain rule, the ReLU
    derivative taken as [activation > 0])."""
    o = acts[-1]
    L, d = head(o, t, o.shape[0])
    grads = [None] * len(params)
    for k in range(len(params) - 1, -1, -1):
        dw, db = conv3x3_backward_weights(acts[k], d, half)
        grads[k] = {"w": dw, "b": db}
        if k > 0:
            d = conv3x3_backward_data(d, params[k]["w"], mask=acts[k], half=half)
    return L, grads


def adam(w, m, v, g, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step (step counts from 1); returns (w, m, v)."""
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return np.asarray(w, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def warm_input(orc, y) -> np.ndarray:
    """Network input x = A^T (y / (u A 1)) / b^(1) of the scan modelled by the
    oracle ``orc`` (ratio 0 where A 1 = 0, x = 0 where b^(1) = 0)."""
    g = orc.geom
    y = np.asarray(y, dtype=np.float64).reshape(g.ndy, g.ndx)
    b1 = orc.sensitivity()
    u = uniform_value(y, b1)
    z0 = u * orc.forward(np.ones((g.nz, g.nx, g.nq)))
    rho = np.where(z0 > 0, y / np.where(z0 > 0, z0, 1.0), 0.0)
    b = orc.adjoint(rho)
    return np.where(b1 > 0, b / np.where(b1 > 0, b1, 1.0), 0.0)


def features(x, delta: float) -> np.ndarray:
    """Network input log(x + delta) of a first EM factor x."""
    return np.log(np.asarray(x, dtype=np.float64) + delta)


def target(f, u: float, delta: float) -> np.ndarray:
    """Training target log(f / u + delta) of a reconstruction f."""
    return np.log(np.asarray(f, dtype=np.float64) / u + delta)


def warm_output(o, u: float, delta: float) -> np.ndarray:
    """u max(exp(min(o, O_CLAMP)) - delta, FLOOR delta): the inverse of the
    target map, kept strictly positive and finite."""
    e = np.exp(np.minimum(np.asarray(o, dtype=np.float64), O_CLAMP))
    return u * np.maximum(e - delta, FLOOR * delta)


def mass_normalise(f, y, b1) -> np.ndarray:
    """f scaled so that sum(b^(1) f) = sum(y), the total that every
    unpenalised EM iterate of Alg. 5 carries (no background)."""
    f = np.asarray(f, dtype=np.float64)
    return f * (float(np.sum(y)) / float(np.sum(np.asarray(b1, dtype=np.float64) * f)))


def warm_start(orc, y, params, delta: float, half: bool = True) -> np.ndarray:
    """The starting image of the learned warm start for counts y."""
    g = orc.geom
    x = features(warm_input(orc, y), delta).reshape(1, g.nz, g.nx, g.nq)
    o = forward(params, x, half)[-1][0]
    b1 = orc.sensitivity()
    return mass_normalise(warm_output(o, uniform_value(y, b1), delta), y, b1)


def uniform_value(y, b1) -> float:
    """u = sum(y) / sum(b^(1)) (the value of the plain uniform start)."""
    return float(np.sum(y)) / float(np.sum(b1))
