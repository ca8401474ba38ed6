"""FP64 oracle of the unrolled, differentiable GoDec layer (test infrastructure).

The layer runs T iterations of Algorithm 1 (Sec. 3.1.3) and then treats the
supports it chose as fixed: with the masks M_t (the supports of S_t) frozen,
    S_0 = 0,  L_t = f(X - S_{t-1}),  S_t = M_t * (X - L_t),   t = 1..T,
is a smooth function of X, and the layer's backward pass gives the gradient of
a loss l(L_T, S_T) with respect to X.  f is the power-scheme BRP low-rank
update, here in the exact form of the restated oracle (``godec_ref.brp_power``:
Q2 = orth((D^T D)^p A1), B = L~ Q2, L = Q1 [R factor of B]^{1/p} Q2^T).

This module restates that forward in plain PyTorch FP64 on the CPU so that
autograd (PyTorch's own QR, SVD and product derivatives) supplies a reference
gradient independent of the library's hand-written adjoints.

Pinned by: central finite differences of the same forward on small inputs
(tests/test_oracle_layer.py).  Only the tests use it.
"""

import numpy as np
import torch


def _ltilde(D, Z, q):
    """L~ Z = (D D^T)^q D Z (reading R3)."""
    Y = D @ Z
    for _ in range(q):
        Y = D @ (D.T @ Y)
    return Y


def brp_power_torch(D, A1, q):
    """The restated BRP low-rank update of Algorithm 1 (as godec_ref.brp_power,
    full rank assumed), differentiable: returns L."""
    p = 2 * q + 1
    Z, _ = torch.linalg.qr(A1)
    for _ in range(p):
        Z, _ = torch.linalg.qr(D.T @ (D @ Z))
    Q2 = Z
    B = _ltilde(D, Q2, q)
    Q1, R1p = torch.linalg.qr(B)
    U, s, Vh = torch.linalg.svd(R1p)
    root = s ** (1.0 / p)
    return (Q1 @ (U * root)) @ (Q2 @ Vh.T).T


def layer_forward(X, A1, q, masks):
    """Frozen-mask forward: masks[t] is the linear-index support of S_{t+1}.
    Returns (L_T, S_T)."""
    m, n = X.shape
    S = torch.zeros_like(X)
    L = None
    for idx in masks:
        L = brp_power_torch(X - S, A1, q)
        M = torch.zeros(m * n, dtype=X.dtype)
        M[torch.as_tensor(idx, dtype=torch.int64)] = 1.0
        S = M.reshape(m, n) * (X - L)
    return L, S


def layer_grad(X, A1, q, masks, dL, dS):
    """d/dX of <dL, L_T> + <dS, S_T> by autograd (FP64)."""
    Xt = torch.tensor(np.asarray(X, np.float64), requires_grad=True)
    A = torch.tensor(np.asarray(A1, np.float64))
    L, S = layer_forward(Xt, A, q, masks)
    loss = torch.sum(torch.tensor(np.asarray(dL, np.float64)) * L) + \
        torch.sum(torch.tensor(np.asarray(dS, np.float64)) * S)
    (g,) = torch.autograd.grad(loss, Xt)
    return g.numpy()


def layer_value(X, A1, q, masks, dL, dS):
    """<dL, L_T> + <dS, S_T> (FP64) for finite differences."""
    with torch.no_grad():
        L, S = layer_forward(torch.tensor(np.asarray(X, np.float64)),
                             torch.tensor(np.asarray(A1, np.float64)), q, masks)
        return float(torch.sum(torch.tensor(dL) * L) + torch.sum(torch.tensor(dS) * S))
