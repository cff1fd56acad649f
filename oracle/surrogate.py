"""Learned frequency surrogate for the response (oracle; test infrastructure).

The paper computes the response at every frequency of the grid.  The
surrogate form computes it exactly only at a few anchor frequencies and
predicts it at the others; it is not in the paper, so every step here follows
the reading written down for it (anchor set, projection basis, interpolation
rule, network, fallback):

1. Anchors: n_a grid indices spread evenly over the grid, j (N_w - 1)/(n_a - 1)
   rounded half up (the same spreading as the Pade nodes).  A held-out index
   midway between the two middle anchors is also computed exactly; it is only
   used to judge the prediction.
2. Non-learned rule.  Every response element is a sum over transitions of
   the kernel g_D(w) = 2D/(D^2 + w^2) (Eq. chi0_matrix with the occupation
   factors), D in the transition window [D_lo, D_hi].  The rule predicts a
   value at w from the anchor values by weights c(w) that reproduce g_D for D
   on a log-spaced family over the window in the least-squares sense, with a
   small ridge term on the weights of unit-norm anchor columns:
   min_c sum_D (sum_l c_l g_D(w_l) - g_D(w))^2 + lam sum_l (c_l n_l)^2,
   n_l^2 = sum_D g_D(w_l)^2.
3. Projection basis U (N_aux x r): block subspace iteration on the positive
   semidefinite S = -chi(w_a0) (first anchor), orthonormalised by Cholesky QR
   at every step, from a caller-supplied start block.  U spans an
   approximation of the top-r eigenvectors of S.
4. The r x r Hermitian projection P(w) = U^H chi(w) U is stored as r^2 real
   series: entry (i, j) is Re P_ij for i <= j and Im P_ij for i > j.
5. Per series, the anchor values a (length n_a) are scaled by
   s = sign(a_0) |a|_2 (s = 0 for series at or below 1e-6 of the largest
   series norm of the q); the network maps a/s to the residual of the rule at
   every non-anchor index, in units of s.  The sign convention makes the
   prediction odd in the data and the scaling makes it homogeneous.
6. Prediction at a non-anchor w:
      chi_sur(w) = sum_l c_l(w) chi(w_l) + U R(w) U^H,
   R(w) the Hermitian matrix of the predicted residual series.
7. The prediction at the held-out index is compared with the exact response
   there (relative Frobenius error); above the threshold the q falls back to
   the exact response at every frequency.

The network: three affine layers, tanh after the first two,
  h1 = tanh(x W1 + b1),  h2 = tanh(h1 W2 + b2),  y = h2 W3 + b3,
loss = mean over rows and outputs of (y - target)^2, trained by Adam.
Parameters are one flat vector in the order W1 [n_in][H], b1, W2 [H][H], b2,
W3 [H][n_out], b3.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------- indices
def anchor_indices(n_freq: int, n_anchor: int):
    j = np.arange(n_anchor, dtype=np.int64)
    return (2 * j * (n_freq - 1) + (n_anchor - 1)) // (2 * (n_anchor - 1))


def holdout_index(anchors):
    m = len(anchors) // 2
    return int((anchors[m - 1] + anchors[m]) // 2)


def target_indices(n_freq: int, anchors):
    a = set(int(x) for x in anchors)
    return np.array([i for i in range(n_freq) if i not in a], dtype=np.int64)


# ---------------------------------------------------------------- rule
def kernel(D, w):
    D = np.asarray(D, dtype=np.float64)[:, None]
    w = np.asarray(w, dtype=np.float64)[None, :]
    return 2.0 * D / (D * D + w * w)


def delta_family(d_lo, d_hi, n_delta=256):
    return d_lo * (d_hi / d_lo) ** (np.arange(n_delta) / (n_delta - 1.0))


def rule_weights(omega, anchors, targets, d_lo, d_hi, n_delta=256, ridge=1e-12):
    """c[l][t]: weight of anchor l in the prediction at target t (step 2).
    The anchor columns of G = [g_D(w_l)] are scaled to unit norm (n_l) and the
    augmented least-squares problem [G/n; sqrt(ridge) I] c' = [g_D(w_t); 0] is
    solved; c_l = c'_l / n_l."""
    D = delta_family(d_lo, d_hi, n_delta)
    G = kernel(D, omega[anchors])                  # [n_D][n_a]
    na = len(anchors)
    nrm = np.linalg.norm(G, axis=0)
    Aug = np.vstack([G / nrm, np.sqrt(ridge) * np.eye(na)])
    out = np.zeros((na, len(targets)))
    for t, it in enumerate(targets):
        rhs = np.concatenate([kernel(D, [omega[it]])[:, 0], np.zeros(na)])
        out[:, t] = np.linalg.lstsq(Aug, rhs, rcond=None)[0] / nrm
    return out


# ---------------------------------------------------------------- basis
def cholesky_qr(Y):
    G = Y.conj().T @ Y
    L = np.linalg.cholesky(G)                       # G = L L^H
    return np.linalg.solve(L, Y.conj().T).conj().T  # Y L^{-H}


def subspace_basis(chi_a0, start, n_iter=4):
    """Step 3: Q_1 = cholqr(S start), Q_{i+1} = cholqr(S Q_i), S = -chi_a0."""
    S = -np.asarray(chi_a0)
    Q = cholesky_qr(S @ start.astype(np.complex128))
    for _ in range(n_iter - 1):
        Q = cholesky_qr(S @ Q)
    return Q


# ---------------------------------------------------------------- series
def to_series(P):
    """[..., r, r] Hermitian -> [..., r*r] real (step 4)."""
    r = P.shape[-1]
    up = np.triu(np.ones((r, r), dtype=bool))
    S = np.where(up, P.real, P.imag)
    return S.reshape(P.shape[:-2] + (r * r,))


def from_series(S, r):
    S = S.reshape(S.shape[:-1] + (r, r))
    up = np.triu(np.ones((r, r), dtype=bool), 1)
    diag = np.eye(r, dtype=bool)
    re = np.where(up, S, 0.0)
    im = np.where(up, -np.swapaxes(S, -1, -2), 0.0)
    U = re + 1j * im                                 # strict upper part
    D = np.where(diag, S, 0.0)
    return U + np.swapaxes(U, -1, -2).conj() + D


NOISE_FLOOR = 1e-6


def features(a):
    """a: [n_series][n_a] -> (x, s) with s = sign(a_0) |a|.  Series whose
    norm is at most NOISE_FLOOR times the largest series norm carry no
    frequency shape above rounding (for instance the imaginary parts at a
    time-reversal invariant q, which vanish exactly): they get s = 0, x = 0."""
    nrm = np.linalg.norm(a, axis=1)
    nrm = np.where(nrm > NOISE_FLOOR * (nrm.max() if nrm.size else 0.0), nrm, 0.0)
    s = np.where(a[:, 0] < 0, -nrm, nrm)
    x = np.zeros_like(a)
    nz = s != 0
    x[nz] = a[nz] / s[nz, None]
    return x, s


# ---------------------------------------------------------------- network
def dims_of(n_in, hidden, n_out):
    shapes = [(n_in, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, n_out), (n_out,)]
    return shapes


def n_params(n_in, hidden, n_out):
    return sum(int(np.prod(s)) for s in dims_of(n_in, hidden, n_out))


def unpack(theta, n_in, hidden, n_out):
    out, o = [], 0
    for s in dims_of(n_in, hidden, n_out):
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def forward(theta, X, n_in, hidden, n_out):
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, hidden, n_out)
    h1 = np.tanh(X @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    return h2 @ W3 + b3, (h1, h2)


def loss_grad(theta, X, Y, n_in, hidden, n_out):
    """Mean-squared loss and its gradient by the chain rule."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, hidden, n_out)
    X = np.asarray(X, dtype=np.float64)
    y, (h1, h2) = forward(theta, X, n_in, hidden, n_out)
    n = Y.size
    r = y - Y
    loss = np.sum(r * r) / n
    dy = 2.0 * r / n
    gW3 = h2.T @ dy
    gb3 = dy.sum(0)
    dz2 = (dy @ W3.T) * (1.0 - h2 * h2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * (1.0 - h1 * h1)
    gW1 = X.T @ dz1
    gb1 = dz1.sum(0)
    g = np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return loss, g


def adam_step(theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step count t >= 1), bias-corrected moments."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- data and prediction
def training_rows(chi, anchors, targets, C, U):
    """Rows (x, y) of every series of one q: chi [N_w][N][N] exact."""
    P = np.einsum('ia,wij,jb->wab', U.conj(), chi, U)
    S = to_series(P)                                 # [N_w][r*r]
    a = S[anchors].T                                 # [n_series][n_a]
    f = S[targets].T                                 # [n_series][n_t]
    x, s = features(a)
    base = a @ C                                     # rule at the targets
    y = np.zeros_like(f)
    nz = s != 0
    y[nz] = (f[nz] - base[nz]) / s[nz, None]
    return x, y


def anchor_series(chi_anchor, U):
    """Scaled anchor features (x, s) of every series: chi_anchor [n_a][N][N]."""
    P = np.einsum('ia,lij,jb->lab', U.conj(), chi_anchor, U)
    return features(to_series(P).T)


def predict_from_residual(chi_anchor, C, U, y, s):
    """Step 6 with the residual series y [r*r][n_t] (units of s) given."""
    r = U.shape[1]
    base = np.einsum('lt,lij->tij', C, chi_anchor)
    R = from_series((y * s[:, None]).T, r)           # [n_t][r][r]
    return base + np.einsum('ia,tab,jb->tij', U, R, U.conj())


def predict(chi_anchor, C, U, theta, hidden):
    """chi at every non-anchor index from the anchor responses [n_a][N][N]."""
    n_a, n_t = C.shape
    x, s = anchor_series(chi_anchor, U)
    y, _ = forward(theta, x, n_a, hidden, n_t)
    return predict_from_residual(chi_anchor, C, U, y, s)


def holdout_error(chi_pred, chi_exact):
    return np.linalg.norm(chi_pred - chi_exact) / np.linalg.norm(chi_exact)
