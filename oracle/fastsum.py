"""Fourier fast-summation chain of Sec. 5, evaluated directly in FP64 (TEST INFRASTRUCTURE).

This is what an NFFT-based fast summation computes when the NFFT itself makes
no error: the kernel is regularised and periodised, its Fourier coefficients are
taken, and the trigonometric sums of eq. (fastsum1) are evaluated directly
(the NDFT and adjoint NDFT of eqs. (ndft), (ndft*)), at O(M^d N) cost.

Readings of the paper used here (the paper's text is ambiguous or garbled at
these points):
  * kappa_B has degree 2p: derivatives r = 0..p match kappa at tau - eps_B and
    derivatives r = 1..p vanish at tau (2p+1 conditions).  With p = 1 this
    reproduces the polynomial printed in Fig. 1 exactly.
  * The forward NDFT uses exp(+i pi m.x / tau), as eq. (fastsum1) requires.
  * The result of eq. (fastsum1) is complex because the index set
    {-M, ..., M-1}^d is not symmetric; its real part is taken.
  * M is the half bandwidth: 2M coefficients per dimension.
"""
from __future__ import annotations

import math

import numpy as np


def kappa_derivatives(x, eta, rmax):
    """[kappa^(r)(x) for r = 0..rmax] for kappa(x) = exp(-x^2/eta), eq. (kappa).

    Uses d^r/dt^r exp(-t^2) = (-1)^r H_r(t) exp(-t^2) (physicists' Hermite
    polynomials, H_{r+1} = 2t H_r - 2r H_{r-1}) with t = x / sqrt(eta)."""
    t = x / math.sqrt(eta)
    e = math.exp(-t * t)
    H = [1.0, 2.0 * t]
    for r in range(1, rmax):
        H.append(2.0 * t * H[r] - 2.0 * r * H[r - 1])
    return [(-1.0) ** r * H[r] * e * eta ** (-0.5 * r) for r in range(rmax + 1)]


def kappa_B_shifted(eta, tau, eps_B, p):
    """Coefficients q_j of kappa_B(x) = sum_{j=0}^{2p} q_j (x - a)^j, a = tau - eps_B.

    Hermite conditions of eq. (Ker-reg) in the reading above:
      kappa_B^(r)(a) = kappa^(r)(a), r = 0..p;  kappa_B^(r)(tau) = 0, r = 1..p."""
    a = tau - eps_B
    deg = 2 * p
    A = np.zeros((deg + 1, deg + 1))
    rhs = np.zeros(deg + 1)
    der = kappa_derivatives(a, eta, p)
    row = 0
    for r in range(p + 1):  # at x = a the shifted monomial (x-a)^j has r-th derivative r! [j == r]
        A[row, r] = math.factorial(r)
        rhs[row] = der[r]
        row += 1
    for r in range(1, p + 1):  # at x = tau: d^r/dx^r (x-a)^j = j!/(j-r)! eps_B^(j-r)
        for j in range(r, deg + 1):
            A[row, j] = math.factorial(j) / math.factorial(j - r) * eps_B ** (j - r)
        rhs[row] = 0.0
        row += 1
    return np.linalg.solve(A, rhs)


def kappa_B_monomial(eta, tau, eps_B, p):
    """The same polynomial in the monomial basis sum_j c_j x^j (as printed in Fig. 1)."""
    q = kappa_B_shifted(eta, tau, eps_B, p)
    a = tau - eps_B
    c = np.zeros_like(q)
    for j, qj in enumerate(q):  # (x - a)^j = sum_i C(j,i) x^i (-a)^(j-i)
        for i in range(j + 1):
            c[i] += qj * math.comb(j, i) * (-a) ** (j - i)
    return c


def kappa_R(r, eta, tau, eps_B, p):
    """Regularised kernel of eq. (Ker-reg) at radius r >= 0 (vectorised)."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    a = tau - eps_B
    q = kappa_B_shifted(eta, tau, eps_B, p)
    poly = np.zeros_like(r)
    rr = np.minimum(r, tau) - a  # beyond tau the polynomial is frozen at kappa_B(tau)
    for j in range(len(q) - 1, -1, -1):
        poly = poly * rr + q[j]
    return np.where(r <= a, np.exp(-r * r / eta), poly)


def kappa_tilde(x, eta, tau, eps_B, p):
    """2 tau-periodic kernel of eq. (kappa_tilde): kappa_R(|x|) on [-tau, tau)^d."""
    x = np.asarray(x, dtype=np.float64)
    xr = np.mod(x + tau, 2.0 * tau) - tau
    return kappa_R(np.sqrt(np.sum(xr * xr, axis=-1)), eta, tau, eps_B, p)


def kappa_hat(d, M, eta, tau, eps_B, p):
    """Fourier coefficients of eq. (fft), as a real array of shape (2M,)*d.

    Entry [m_1+M, ..., m_d+M] holds kappa_hat(m) for m in {-M..M-1}^d:
      (2M)^-d sum_{x in (tau/M){-M..M-1}^d} kappa_tilde(x) exp(-i pi m.x / tau).
    The sum is taken one axis at a time with an explicit (2M x 2M) DFT matrix.
    The imaginary part vanishes (kappa_tilde is even and the sample set is
    symmetric modulo the period); it is checked and dropped."""
    idx = np.arange(-M, M)
    axis_pts = (tau / M) * idx
    grids = np.meshgrid(*([axis_pts] * d), indexing="ij")
    samples = kappa_tilde(np.stack(grids, axis=-1), eta, tau, eps_B, p).astype(np.complex128)
    E = np.exp(-1j * np.pi * np.outer(idx, axis_pts) / tau)  # E[m, x]
    out = samples
    for ax in range(d):
        out = np.moveaxis(np.tensordot(E, out, axes=([1], [ax])), 0, ax)
    out = out / (2 * M) ** d
    assert np.max(np.abs(out.imag)) <= 1e-12 * max(1.0, np.max(np.abs(out.real)))
    return out.real.copy()


def _phases(x, M, tau, sign):
    """exp(sign * i pi m x_c / tau) for every point, dimension and m in {-M..M-1}."""
    m = np.arange(-M, M)
    return np.exp(sign * 1j * np.pi * x[:, :, None] * m[None, None, :] / tau)  # (n, d, 2M)


def adjoint_ndft(xs, v, M, tau, chunk=2048):
    """[F*_l v]_m = sum_j v_j exp(-i pi m.y_j / tau), eq. (ndft*); shape (2M,)*d."""
    xs = np.asarray(xs, dtype=np.float64)
    d = xs.shape[1]
    out = np.zeros((2 * M,) * d, dtype=np.complex128)
    for s in range(0, xs.shape[0], chunk):
        ph = _phases(xs[s:s + chunk], M, tau, -1.0)
        w = np.asarray(v[s:s + chunk], dtype=np.float64)
        if d == 1:
            out += np.einsum("j,ja->a", w, ph[:, 0])
        elif d == 2:
            out += np.einsum("j,ja,jb->ab", w, ph[:, 0], ph[:, 1])
        else:
            A = np.einsum("j,ja,jb->jab", w, ph[:, 0], ph[:, 1])
            out += np.tensordot(A, ph[:, 2], axes=([0], [0]))
    return out


def ndft(xt, coef, M, tau, chunk=2048):
    """[F_k c]_i = sum_m c(m) exp(+i pi m.x_i / tau), eq. (ndft) with the sign of eq. (fastsum1)."""
    xt = np.asarray(xt, dtype=np.float64)
    d = xt.shape[1]
    out = np.zeros(xt.shape[0], dtype=np.complex128)
    for s in range(0, xt.shape[0], chunk):
        ph = _phases(xt[s:s + chunk], M, tau, +1.0)
        if d == 1:
            out[s:s + chunk] = ph[:, 0] @ coef
        elif d == 2:
            out[s:s + chunk] = np.einsum("ia,ab,ib->i", ph[:, 0], coef, ph[:, 1])
        else:
            B = np.tensordot(ph[:, 2], coef, axes=([1], [2]))  # (i, a, b)
            out[s:s + chunk] = np.einsum("ia,iab,ib->i", ph[:, 0], B, ph[:, 1])
    return out


def fastsum(xt, xs, v, eta, tau, eps_B, p, M):
    """Algorithm 4 with exact trigonometric sums: Re F_k (kappa_hat (.) F*_l v)."""
    d = np.asarray(xs).shape[1]
    kh = kappa_hat(d, M, eta, tau, eps_B, p)
    return ndft(xt, kh * adjoint_ndft(xs, v, M, tau), M, tau).real
