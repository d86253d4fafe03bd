"""FP64 CPU oracle of the learned sketch.  Test infrastructure only: imported by the
tests, the smoke check and the benchmark's CPU baseline, never by the library path.

The sketch network is not part of the paper; it supplies the start matrix G of the
randomised eigendecompositions (Section 4, Algorithms 3-5, the Gaussian start block).
Definition (implemented independently by the HIP library):

  input A_0[i] (68 x n) for time level i: channels 0..63 are the Gaussian block the plain
      method would use, Omega[i n + j, c]; channel 64 is (x_i(j) - 2.3)/3.6 for a Lorenz-96
      trajectory (0 otherwise); 65 is 1 where point j is observed at time i; 66 is i/N;
      67 is exp(-(t_next(i) - i)/5) with t_next(i) the first observed time >= i (0 if none);
  layers l = 1..4: H_l[c, j] = b_l[c] + sum_{c', t=-2..2} W_l[c, c', t+2] A_{l-1}[c', (j+t) mod n],
      A_l = tanh(H_l) for l < 4, and the output G[i n + j, c] = H_4[c, j];
  weights and biases are used as their float16 roundings (round_fp16=True).
  Flat parameter order: per layer W_l (c_out, c_in, t) row-major, then b_l.

Loss on a start matrix G (n_A x m), with Y = A G, S = Y^T Y, P_w = U diag(w) U^T from
reference Ritz pairs (U, theta) of the method, w = 1 - 1/theta:
      f = -trace(S^{-1} Y^T P_w Y) / sum(w),
the weighted fraction of the reference subspace captured by range(A G) (the space the
three algorithms orthonormalise); its gradient is A (2/sum w)(Y S^{-1} T S^{-1} - P_w Y S^{-1}),
T = Y^T P_w Y.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

KW = 5          # kernel width
LAYERS = 4
CH = 64         # hidden and output channels
NF = 4          # feature channels
NZ = 64         # Gaussian input channels
C0 = NZ + NF    # input channels


def param_shapes(c0: int = C0, ch: int = CH, layers: int = LAYERS):
    shapes = []
    cin = c0
    for _ in range(layers):
        shapes.append(((ch, cin, KW), (ch,)))
        cin = ch
    return shapes


def unpack(theta: np.ndarray, c0: int = C0, ch: int = CH, layers: int = LAYERS):
    """Flat parameter vector -> [(W, b)] (W[c_out, c_in, t], b[c_out])."""
    out, off = [], 0
    for ws, bs in param_shapes(c0, ch, layers):
        nw = int(np.prod(ws))
        W = theta[off:off + nw].reshape(ws)
        off += nw
        b = theta[off:off + bs[0]]
        off += bs[0]
        out.append((W, b))
    return out


def n_params(c0: int = C0, ch: int = CH, layers: int = LAYERS) -> int:
    return sum(int(np.prod(w)) + b[0] for w, b in param_shapes(c0, ch, layers))


def features(n: int, N: int, pattern, traj=None) -> np.ndarray:
    """The four feature channels, (N+1, 4, n)."""
    F = np.zeros((N + 1, NF, n))
    if traj is not None:
        F[:, 0, :] = (np.asarray(traj) - 2.3) / 3.6
    obs_times = sorted(int(i) for i, idx in pattern if len(idx))
    for i, idx in pattern:
        F[int(i), 1, np.asarray(idx, dtype=np.int64)] = 1.0
    for i in range(N + 1):
        F[i, 2, :] = i / N
        nxt = [t for t in obs_times if t >= i]
        F[i, 3, :] = np.exp(-(nxt[0] - i) / 5.0) if nxt else 0.0
    return F


def net_input(F: np.ndarray, Omega: np.ndarray) -> np.ndarray:
    """A_0 (N+1, 68, n) from the features (N+1, 4, n) and Omega (n_A x 64)."""
    T, _, n = F.shape
    Z = np.asarray(Omega).reshape(T, n, -1).transpose(0, 2, 1)
    return np.concatenate([Z, F], axis=1)


def _conv(W: np.ndarray, b: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Periodic 1-D convolution over the last axis: A (T, c_in, n) -> (T, c_out, n)."""
    H = np.broadcast_to(b[None, :, None], (A.shape[0], W.shape[0], A.shape[2])).copy()
    for t in range(KW):
        shifted = np.roll(A, -(t - 2), axis=2)           # shifted[..., j] = A[..., j + t - 2]
        H += np.einsum("oc,Tcn->Ton", W[:, :, t], shifted)
    return H


def _rounded(theta, c0, round_fp16):
    ps = unpack(theta, c0)
    if not round_fp16:
        return ps
    return [(W.astype(np.float16).astype(np.float64), b.astype(np.float16).astype(np.float64)) for W, b in ps]


def forward(theta: np.ndarray, F: np.ndarray, round_fp16: bool = True):
    """F: net input (T, c0, n).  Returns (G (T n x 64), activations [A_0 .. A_3])."""
    params = _rounded(theta, F.shape[1], round_fp16)
    acts = [F]
    A = F
    for l, (W, b) in enumerate(params):
        H = _conv(W, b, A)
        if l < len(params) - 1:
            A = np.tanh(H)
            acts.append(A)
        else:
            out = H
    T, m, n = out.shape
    G = out.transpose(0, 2, 1).reshape(T * n, m)
    return G, acts


def backward(theta: np.ndarray, acts, dG: np.ndarray, round_fp16: bool = True) -> np.ndarray:
    """Gradient of sum(dG * G) with respect to the parameters (the float16-rounded ones
    when round_fp16: the rounding is treated as the identity)."""
    params = _rounded(theta, acts[0].shape[1], round_fp16)
    T, _, n = acts[0].shape
    m = params[-1][0].shape[0]
    dH = dG.reshape(T, n, m).transpose(0, 2, 1)
    grads = []
    for l in range(len(params) - 1, -1, -1):
        W, b = params[l]
        A = acts[l]
        dW = np.zeros_like(W)
        for t in range(KW):
            shifted = np.roll(A, -(t - 2), axis=2)
            dW[:, :, t] = np.einsum("Ton,Tcn->oc", dH, shifted)
        db = dH.sum(axis=(0, 2))
        grads.append((dW, db))
        if l == 0:
            break
        dA = np.zeros_like(A)
        for t in range(KW):
            # H[j] uses A[j + t - 2]: dA[j'] += W[:, :, t]^T dH[j' - (t - 2)]
            dA += np.roll(np.einsum("oc,Ton->Tcn", W[:, :, t], dH), (t - 2), axis=2)
        dH = dA * (1.0 - A * A)
    grads.reverse()
    return np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])


def capture_loss(applyA, G: np.ndarray, U: np.ndarray, theta: np.ndarray) -> Tuple[float, np.ndarray]:
    """f = -trace(S^{-1} Y^T P_w Y) / sum(w), Y = A G, and df/dG."""
    w = 1.0 - 1.0 / np.asarray(theta)
    Y = applyA(G)
    S = Y.T @ Y
    V = U.T @ Y                       # k x m
    T = V.T @ (w[:, None] * V)        # Y^T P_w Y
    Sinv = np.linalg.inv(S)
    f = -np.trace(Sinv @ T) / w.sum()
    PY = U @ (w[:, None] * V)         # P_w Y
    dY = (2.0 / w.sum()) * (Y @ (Sinv @ T @ Sinv) - PY @ Sinv)
    return f, applyA(dY)


def init_params(rng: np.random.Generator, c0: int = C0, ch: int = CH, layers: int = LAYERS) -> np.ndarray:
    """LeCun-normal weights, zero biases."""
    parts = []
    for ws, bs in param_shapes(c0, ch, layers):
        fan_in = ws[1] * ws[2]
        parts.append(rng.standard_normal(int(np.prod(ws))) / np.sqrt(fan_in))
        parts.append(np.zeros(bs[0]))
    return np.concatenate(parts)


def adam_step(theta, g, mom, vel, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), in place; step counts from 1."""
    mom[:] = b1 * mom + (1 - b1) * g
    vel[:] = b2 * vel + (1 - b2) * g * g
    mh = mom / (1 - b1 ** step)
    vh = vel / (1 - b2 ** step)
    theta -= lr * mh / (np.sqrt(vh) + eps)
    return theta
