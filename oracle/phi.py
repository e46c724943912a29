"""phi-functions and the linear combination sum_k phi_k(tA) b_k (oracle).

Section 3 of the paper builds every ETD scheme out of the phi-functions
(eq. 3.4 gives the integral form, eq. 3.5 a recursion) and Section 3.3
reduces each scheme to one quantity, eq. 3.7: the linear combination
phi_0(A) v_0 + ... + phi_p(A) v_p, which is also the time-1 value of the
ODE y' = A y + v_1 + t v_2 + ... + t^{p-1}/(p-1)! v_p, y(0) = v_0.

Normalisation.  eq. 3.4 and eq. 3.5 as printed omit the 1/(k-1)! factor that
the ODE form of Section 3.3 carries; the two agree for k <= 2.  This module
uses the standard functions, phi_0(z) = e^z and
phi_k(z) = int_0^1 e^{(1-s) z} s^{k-1} / (k-1)! ds, which satisfy
phi_k(z) = (phi_{k-1}(z) - 1/(k-1)!) / z and phi_k(0) = 1/k!.

Three routes to the combination, deliberately independent of each other:

* ``phi_combination_dense``  -- exponential of the augmented matrix
  [[tA, W], [0, J]] (Al-Mohy & Higham 2011, Thm 2.1), via scipy expm.
* ``phi_combination_eigh``   -- A symmetric: A = Q diag(lam) Q^T and
  scalar phi_k on the eigenvalues.
* ``phi_combination_krylov`` -- Arnoldi (full reorthogonalisation) on the
  augmented *operator*, substeps exp(M) = exp(M/s)^s, s doubled until two
  successive results agree; for sizes where dense routes are too slow.

Pins (tests/test_oracle_phi.py): closed forms of phi_1..phi_3, phi_k(0)=1/k!,
the recurrence, the derivative identity phi_k' = phi_k - k phi_{k+1}
against finite differences, the integral definition by quadrature, and the
three routes against each other and against brute-force series on tiny
matrices.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla


def phi_scalar(k: int, z):
    """Standard phi_k(z) for real z (scalar or array), float64.

    |z| < 2: Taylor series sum_j z^j / (j+k)!  (40 terms, truncation < 1e-35).
    |z| >= 2: phi_0 = e^z and the recurrence phi_j = (phi_{j-1} - 1/(j-1)!)/z,
    whose cancellation stays below a few ulps once |z| >= 2 (k <= 5).
    """
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    small = np.abs(z) < 2.0
    if np.any(small):
        zs = z[small]
        acc = np.zeros_like(zs)
        for j in range(39, -1, -1):
            acc = acc * zs + 1.0 / math.factorial(j + k)
        out[small] = acc
    big = ~small
    if np.any(big):
        zb = z[big]
        val = np.exp(zb)
        for j in range(1, k + 1):
            val = (val - 1.0 / math.factorial(j - 1)) / zb
        out[big] = val
    return out if out.ndim else float(out)


def _eta(bs):
    """Power-of-two balancing factor for the W block (Al-Mohy & Higham 2011,
    Sec. 2): eta W has 1-norm near 1, and e_p is scaled by 1/eta instead."""
    p = len(bs) - 1
    if p == 0:
        return 1.0
    nw = max(float(np.abs(b).sum()) for b in bs[1:])
    if nw == 0.0:
        return 1.0
    return 2.0 ** (-math.ceil(math.log2(nw)))


def augmented_matrix(A, t: float, bs, eta: float = 1.0):
    """The (N+p) x (N+p) matrix [[tA, eta W], [0, J]] with W = [b_p, ..., b_1]
    and J the p x p upper shift, whose exponential applied to
    [b_0; e_p / eta] yields sum_k phi_k(tA) b_k in its first N entries
    (Al-Mohy & Higham 2011, Thm 2.1).  A dense or scipy sparse; returns dense."""
    A = A.toarray() if hasattr(A, "toarray") else np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    p = len(bs) - 1
    M = np.zeros((n + p, n + p))
    M[:n, :n] = t * A
    for j in range(p):
        # column n + j carries b_{p - j}
        M[:n, n + j] = eta * bs[p - j]
    for j in range(p - 1):
        M[n + j, n + j + 1] = 1.0
    return M


def phi_combination_dense(A, t: float, bs):
    """sum_{k=0}^{p} phi_k(tA) b_k by the dense augmented-matrix exponential."""
    bs = [np.asarray(b, dtype=np.float64) for b in bs]
    n = bs[0].shape[0]
    p = len(bs) - 1
    if p == 0:
        Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
        return sla.expm(t * Ad) @ bs[0]
    eta = _eta(bs)
    M = augmented_matrix(A, t, bs, eta)
    v = np.zeros(n + p)
    v[:n] = bs[0]
    v[n + p - 1] = 1.0 / eta
    return (sla.expm(M) @ v)[:n]


def phi_combination_eigh(A, t: float, bs):
    """sum_k phi_k(tA) b_k for symmetric A via its eigendecomposition."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A, dtype=np.float64)
    lam, Q = np.linalg.eigh(Ad)
    out = np.zeros(Ad.shape[0])
    for k, b in enumerate(bs):
        out += Q @ (phi_scalar(k, t * lam) * (Q.T @ np.asarray(b, dtype=np.float64)))
    return out


def phi_apply_eigh(A, t: float, k: int, b):
    """phi_k(tA) b for symmetric A (eigendecomposition)."""
    bs = [np.zeros_like(b)] * k + [b]
    return phi_combination_eigh(A, t, bs)


def _arnoldi_expv(matvec, v, m: int):
    """exp(M) v by one Arnoldi cycle of dimension m with full
    reorthogonalisation (modified Gram-Schmidt, twice).  Returns the vector."""
    beta = np.linalg.norm(v)
    if beta == 0.0:
        return np.zeros_like(v)
    n = v.shape[0]
    m = min(m, n)
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    V[:, 0] = v / beta
    mm = m
    for j in range(m):
        w = matvec(V[:, j])
        for _ in range(2):
            for i in range(j + 1):
                c = V[:, i] @ w
                H[i, j] += c
                w = w - c * V[:, i]
        h = np.linalg.norm(w)
        H[j + 1, j] = h
        if h <= 1e-14 * max(1.0, np.abs(H[: j + 2, : j + 1]).max()):
            mm = j + 1
            break
        V[:, j + 1] = w / h
    E = sla.expm(H[:mm, :mm])
    return beta * (V[:, :mm] @ E[:, 0])


def phi_combination_krylov(A, t: float, bs, m: int = 40, rtol: float = 1e-13,
                           s0: int = 1, s_max: int = 1 << 14):
    """sum_k phi_k(tA) b_k via Arnoldi on the augmented operator.

    The augmented operator M = [[tA, W], [0, J]] is applied matrix-free.
    exp(M) w0 = (exp(M/s))^s w0 with each factor approximated by one Arnoldi
    cycle of dimension m; s doubles until two successive results agree to
    rtol (relative, 2-norm).  A is a scipy sparse (or dense) N x N matrix.
    """
    bs = [np.asarray(b, dtype=np.float64) for b in bs]
    n = bs[0].shape[0]
    p = len(bs) - 1
    eta = _eta(bs)
    W = eta * np.stack([bs[p - j] for j in range(p)], axis=1) if p else np.zeros((n, 0))

    def make_mv(scale):
        def mv(x):
            y = np.empty_like(x)
            y[:n] = scale * t * (A @ x[:n])
            if p:
                y[:n] += scale * (W @ x[n:])
                y[n:] = 0.0
                y[n:n + p - 1] = scale * x[n + 1:n + p]
            return y
        return mv

    w0 = np.zeros(n + p)
    w0[:n] = bs[0]
    if p:
        w0[n + p - 1] = 1.0 / eta

    def run(s):
        mv = make_mv(1.0 / s)
        x = w0.copy()
        for _ in range(s):
            x = _arnoldi_expv(mv, x, m)
        return x[:n]

    s = s0
    prev = run(s)
    while True:
        s *= 2
        cur = run(s)
        den = max(np.linalg.norm(cur), 1e-300)
        if np.linalg.norm(cur - prev) <= rtol * den or s >= s_max:
            if np.linalg.norm(cur - prev) > rtol * den:
                raise RuntimeError("oracle Krylov route did not self-converge")
            return cur
        prev = cur


def phi_combination_at(A, t: float, bs, s: float, method: str = "auto"):
    """Value at time s of the ODE of Section 3.3 whose time-t value is
    sum_k phi_k(tA) b_k: y' = A y + sum_{k>=1} tau^{k-1}/(k-1)! b_k / t^k,
    y(0) = b_0, so y(s) = sum_k phi_k(sA) (s/t)^k b_k (intermediate output of
    one integration, as the simultaneous evaluation of Section 3.3 uses)."""
    return phi_combination(A, s, [(s / t) ** k * np.asarray(b) for k, b in enumerate(bs)], method)


def phi_combination(A, t: float, bs, method: str = "auto"):
    """Dispatch: dense augmented expm for small N, Krylov otherwise."""
    n = np.asarray(bs[0]).shape[0]
    if method == "auto":
        method = "dense" if n + len(bs) <= 2500 else "krylov"
    if n == 0:
        return np.zeros(0)
    if method == "dense":
        return phi_combination_dense(A, t, bs)
    if method == "eigh":
        return phi_combination_eigh(A, t, bs)
    if method == "krylov":
        return phi_combination_krylov(A, t, bs)
    raise ValueError(method)
